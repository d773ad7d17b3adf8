"""ctypes binding of libelph (include/elph.h): argument marshalling only.

Every computation runs in the HIP library; this module converts NumPy host
inputs and GPU tensors (device outputs, via their data pointers) into the C
ABI's plain pointers and turns nonzero status codes into ElphError.  It fails
loudly when the compiled library is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libelph.so")

ELPH_OK, ELPH_EINVAL, ELPH_ENOMEM, ELPH_EHIP, ELPH_ENOCONV, ELPH_ESTATE = range(6)
ELPH_FP64, ELPH_FP32, ELPH_BF16X3, ELPH_BF16X6, ELPH_FP16X3 = range(5)
ELPH_LEVEL_RTA, ELPH_LEVEL_PARTIAL, ELPH_LEVEL_DRAGLESS, ELPH_LEVEL_COUPLED = range(4)
PRECISIONS = {"fp64": ELPH_FP64, "fp32": ELPH_FP32, "bf16x3": ELPH_BF16X3, "bf16x6": ELPH_BF16X6,
              "fp16x3": ELPH_FP16X3}

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_f64p = ctypes.POINTER(ctypes.c_double)


class ElphWannier(ctypes.Structure):
    _fields_ = [("nwann", ctypes.c_int32), ("natom", ctypes.c_int32), ("nre", ctypes.c_int32),
                ("nrp", ctypes.c_int32), ("re", _c_i32p), ("rp", _c_i32p), ("wre", _c_f64p),
                ("wrp", _c_f64p), ("lat", _c_f64p), ("mass", _c_f64p), ("h_r", _c_f64p),
                ("d_r", _c_f64p), ("g_r", _c_f64p)]


class ElphParams(ctypes.Structure):
    _fields_ = [("mesh", ctypes.c_int32 * 3), ("precision", ctypes.c_int32), ("mu_eV", ctypes.c_double),
                ("window_eV", ctypes.c_double), ("sigma_eV", ctypes.c_double),
                ("omega_min_eV", ctypes.c_double)]


class ElphSizes(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int64), ("nkept", ctypes.c_int64), ("nstates", ctypes.c_int64),
                ("nwann", ctypes.c_int32), ("nbr", ctypes.c_int32), ("nterms", ctypes.c_int64),
                ("hw_max_eV", ctypes.c_double), ("ngroups", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTS = ("elph_create", "elph_destroy", "elph_last_error", "elph_reset", "elph_timing", "elph_sizes",
           "elph_batch_create", "elph_batch_destroy", "elph_batch_last_error", "elph_batch_scatt_rates",
           "elph_batch_tune", "elph_batch_set_shape", "elph_tables", "elph_timing_extra", "elph_set_refine", "elph_refine_info", "elph_save", "elph_load", "elph_set_memory_limit",
           "elph_memory_held", "elph_set_gemm_chunk",
           "elph_refine_estimates",
           "elph_interp_g", "elph_interp_g_noalloc", "elph_transition_probs", "elph_scatt_rates", "elph_iterate", "elph_ko_enforce", "elph_set_delta", "elph_set_polar",
           "elph_set_ifc3", "elph_phph_vertex", "elph_phph_rates", "elph_phph_inscatter", "elph_set_phph",
           "elph_mlp_create", "elph_mlp_destroy", "elph_mlp_last_error", "elph_mlp_nparams",
           "elph_mlp_get_params", "elph_mlp_set_params", "elph_mlp_forward", "elph_mlp_gradients",
           "elph_mlp_train_step", "elph_screen_nin", "elph_screen_samples", "elph_scatt_rates_screened")
_NO_STATUS = ("elph_destroy", "elph_last_error", "elph_batch_destroy", "elph_batch_last_error", "elph_mlp_destroy",
              "elph_mlp_last_error", "elph_mlp_nparams", "elph_screen_nin")
ELPH_SCREEN_NONE, ELPH_SCREEN_ENERGY, ELPH_SCREEN_MLP = range(3)

_lib = None


def load():
    """Load libelph.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libelph.so is not built; run __graft_entry__.build() or "
                           "python -m paper_2109_08547_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.elph_create.argtypes = [ctypes.POINTER(ElphWannier), ctypes.POINTER(ElphParams), vp,
                                ctypes.POINTER(vp)]
    lib.elph_destroy.argtypes = [vp]
    lib.elph_destroy.restype = None
    lib.elph_last_error.argtypes = [vp]
    lib.elph_last_error.restype = ctypes.c_char_p
    lib.elph_reset.argtypes = [vp, ctypes.c_int32]
    lib.elph_timing.argtypes = [vp, ctypes.c_int32, vp]
    lib.elph_timing_extra.argtypes = [vp, vp]
    lib.elph_set_refine.argtypes = [vp, ctypes.c_double]
    lib.elph_save.argtypes = [vp, ctypes.c_char_p]
    lib.elph_load.argtypes = [vp, ctypes.c_char_p]
    lib.elph_set_memory_limit.argtypes = [vp, ctypes.c_int64]
    lib.elph_memory_held.argtypes = [vp, vp]
    lib.elph_set_gemm_chunk.argtypes = [vp, ctypes.c_int64]
    lib.elph_refine_info.argtypes = [vp, vp, vp]
    lib.elph_refine_estimates.argtypes = [vp, vp]
    lib.elph_sizes.argtypes = [vp, ctypes.POINTER(ElphSizes)]
    lib.elph_tables.argtypes = [vp] * 7
    lib.elph_interp_g.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    lib.elph_interp_g_noalloc.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    lib.elph_transition_probs.argtypes = [vp, ctypes.c_double, vp, vp, ctypes.c_int32]
    lib.elph_scatt_rates.argtypes = [vp, ctypes.c_double, vp, vp]
    lib.elph_iterate.argtypes = [vp, ctypes.c_double, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                 vp, vp, vp, vp, vp, vp, vp]
    lib.elph_ko_enforce.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp, vp, vp, vp]
    lib.elph_set_delta.argtypes = [vp, ctypes.c_int32]
    lib.elph_set_polar.argtypes = [vp, vp, vp, vp]
    lib.elph_set_ifc3.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    lib.elph_phph_vertex.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    lib.elph_phph_rates.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp]
    lib.elph_phph_inscatter.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.elph_set_phph.argtypes = [vp, ctypes.c_double]
    lib.elph_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.elph_batch_destroy.argtypes = [vp]
    lib.elph_batch_destroy.restype = None
    lib.elph_batch_last_error.argtypes = [vp]
    lib.elph_batch_last_error.restype = ctypes.c_char_p
    lib.elph_batch_scatt_rates.argtypes = [vp, ctypes.c_double, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.c_int32]
    lib.elph_batch_tune.argtypes = [vp, ctypes.c_double, vp, vp]
    lib.elph_batch_set_shape.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.elph_mlp_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.POINTER(vp)]
    lib.elph_mlp_destroy.argtypes = [vp]
    lib.elph_mlp_destroy.restype = None
    lib.elph_mlp_last_error.argtypes = [vp]
    lib.elph_mlp_last_error.restype = ctypes.c_char_p
    lib.elph_mlp_nparams.argtypes = [vp]
    lib.elph_mlp_nparams.restype = ctypes.c_int64
    lib.elph_mlp_get_params.argtypes = [vp, vp]
    lib.elph_mlp_set_params.argtypes = [vp, vp]
    lib.elph_mlp_forward.argtypes = [vp, ctypes.c_int64, vp, vp]
    lib.elph_mlp_gradients.argtypes = [vp, ctypes.c_int64, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.elph_mlp_train_step.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_float, ctypes.POINTER(ctypes.c_double)]
    lib.elph_screen_nin.argtypes = [vp]
    lib.elph_screen_nin.restype = ctypes.c_int32
    lib.elph_screen_samples.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
    lib.elph_scatt_rates_screened.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, vp, vp, vp]
    for name in EXPORTS:
        if name not in _NO_STATUS:
            getattr(lib, name).restype = ctypes.c_int32
    _lib = lib
    return lib


class ElphError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("elph status %d: %s" % (status, message))
        self.status = status
        self.message = message


def _ptr(t):
    """Device pointer of a GPU tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns an elph_ctx handle; keeps the host input arrays alive while needed."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None):
            load().elph_destroy(self.handle)
            self.handle = None


def _check(ctx, status):
    if status != ELPH_OK:
        msg = load().elph_last_error(ctx.handle if ctx is not None else None)
        raise ElphError(status, msg.decode() if msg else "")


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def elph_create(mat, mesh, mu, window, sigma, omega_min=0.0, precision=ELPH_FP64, stream=None):
    """Create a context from a material dict (nwann, natom, re, rp, wre, wrp,
    lat, mass, h_r, d_r, g_r as NumPy arrays).  ``stream`` is a HIP stream
    handle (int) or None for the default stream."""
    lib = load()
    keep = {k: _arr(mat[k], np.int32) for k in ("re", "rp")}
    for k in ("wre", "wrp", "lat", "mass", "d_r"):
        keep[k] = _arr(mat[k], np.float64)
    for k in ("h_r", "g_r"):
        keep[k] = _arr(mat[k], np.complex128).view(np.float64)
    w = ElphWannier()
    w.nwann, w.natom = int(mat["nwann"]), int(mat["natom"])
    w.nre, w.nrp = keep["re"].shape[0], keep["rp"].shape[0]
    for k in ("re", "rp"):
        setattr(w, k, keep[k].ctypes.data_as(_c_i32p))
    for k in ("wre", "wrp", "lat", "mass", "h_r", "d_r", "g_r"):
        setattr(w, k, keep[k].ctypes.data_as(_c_f64p))
    p = ElphParams()
    m = [int(mesh)] * 3 if np.isscalar(mesh) else [int(x) for x in mesh]
    p.mesh[:] = m
    p.precision = PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision)
    p.mu_eV, p.window_eV, p.sigma_eV, p.omega_min_eV = float(mu), float(window), float(sigma), float(omega_min)
    h = ctypes.c_void_p()
    st = lib.elph_create(ctypes.byref(w), ctypes.byref(p), ctypes.c_void_p(stream) if stream else None,
                         ctypes.byref(h))
    _check(None, st)
    return Context(h)


def elph_destroy(ctx):
    ctx.close()


ELPH_RESET_ALL, ELPH_RESET_STORE, ELPH_RESET_TRIM = 0, 1, 2


def elph_reset(ctx, what=ELPH_RESET_ALL):
    _check(ctx, load().elph_reset(ctx.handle, int(what)))


def elph_timing(ctx, enable=True, read=False):
    """Turn event timing on/off; with read=True return the last durations (ms)
    of [tables, step1, step2, iterate] (-1 where none was recorded)."""
    ms = np.full(4, -1.0)
    _check(ctx, load().elph_timing(ctx.handle, int(bool(enable)),
                                   ms.ctypes.data_as(ctypes.c_void_p) if read else None))
    return dict(zip(("tables", "step1", "step2", "iterate"), ms)) if read else None


def elph_timing_extra(ctx):
    """Milliseconds of the last tetrahedron-delta scaling or Froehlich table (-1: none)."""
    ms = ctypes.c_double(-1.0)
    _check(ctx, load().elph_timing_extra(ctx.handle, ctypes.byref(ms)))
    return ms.value


def elph_save(ctx, path):
    _check(ctx, load().elph_save(ctx.handle, os.fsencode(path)))


def elph_load(ctx, path):
    _check(ctx, load().elph_load(ctx.handle, os.fsencode(path)))


def elph_set_memory_limit(ctx, nbytes):
    _check(ctx, load().elph_set_memory_limit(ctx.handle, int(nbytes)))


def elph_set_gemm_chunk(ctx, nbytes):
    _check(ctx, load().elph_set_gemm_chunk(ctx.handle, int(nbytes)))


def elph_memory_held(ctx):
    v = ctypes.c_int64(0)
    _check(ctx, load().elph_memory_held(ctx.handle, ctypes.byref(v)))
    return v.value


def elph_set_refine(ctx, theta):
    _check(ctx, load().elph_set_refine(ctx.handle, float(theta)))


def elph_refine_info(ctx):
    """Counters of the last FP64 refinement and its duration (ms, -1: none)."""
    st = np.zeros(8, dtype=np.int64)
    ms = ctypes.c_double(-1.0)
    _check(ctx, load().elph_refine_info(ctx.handle, st.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ms)))
    keys = ("rows_flagged", "modes_flagged", "pairs", "states", "qs", "overflow", "rows_unresolved",
            "modes_unresolved")
    out = dict(zip(keys, (int(v) for v in st)))
    out["ms"] = ms.value
    return out


def elph_refine_estimates(ctx, rel_err):
    _check(ctx, load().elph_refine_estimates(ctx.handle, _ptr(rel_err)))


def elph_sizes(ctx):
    s = ElphSizes()
    _check(ctx, load().elph_sizes(ctx.handle, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in ElphSizes._fields_ if f != "reserved"}


def elph_tables(ctx, state_k=None, state_m=None, eps=None, vel=None, hw=None, vph=None):
    _check(ctx, load().elph_tables(ctx.handle, _ptr(state_k), _ptr(state_m), _ptr(eps), _ptr(vel), _ptr(hw),
                                   _ptr(vph)))


def elph_interp_g(ctx, kidx, qidx, g_out):
    n = int(kidx.numel())
    _check(ctx, load().elph_interp_g(ctx.handle, n, _ptr(kidx), _ptr(qidx), _ptr(g_out)))


def elph_interp_g_noalloc(ctx, kidx, qidx, g_out):
    n = int(kidx.numel())
    _check(ctx, load().elph_interp_g_noalloc(ctx.handle, n, _ptr(kidx), _ptr(qidx), _ptr(g_out)))


def elph_transition_probs(ctx, T, Xp=None, Xm=None, store_B=False):
    _check(ctx, load().elph_transition_probs(ctx.handle, float(T), _ptr(Xp), _ptr(Xm), int(bool(store_B))))


def elph_scatt_rates(ctx, T, W_e=None, W_ph=None):
    _check(ctx, load().elph_scatt_rates(ctx.handle, float(T), _ptr(W_e), _ptr(W_ph)))


def elph_iterate(ctx, T, I, J, F, G, W_ph_ext=None, level=ELPH_LEVEL_COUPLED, tol=1e-8, maxit=200,
                 raise_on_noconv=True):
    """Returns dict(tensors [6,3,3] numpy, iters, ko_residual, status)."""
    tens = np.zeros(54)
    iters = ctypes.c_int32(0)
    ko = ctypes.c_double(0.0)
    st = load().elph_iterate(ctx.handle, float(T), _ptr(W_ph_ext), int(level), float(tol), int(maxit),
                             _ptr(I), _ptr(J), _ptr(F), _ptr(G), tens.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(iters), ctypes.byref(ko))
    if st != ELPH_OK and not (st == ELPH_ENOCONV and not raise_on_noconv):
        _check(ctx, st)
    names = ("sigma", "sigmaS", "alpha_el", "kappa0_el", "alpha_ph", "kappa_ph")
    return {"tensors": {n: tens[9 * a:9 * a + 9].reshape(3, 3).copy() for a, n in enumerate(names)},
            "iters": iters.value, "ko_residual": ko.value, "status": st}


ELPH_DELTA_GAUSS, ELPH_DELTA_TETRA, ELPH_DELTA_TRIANGLE = 0, 1, 2


def elph_set_delta(ctx, method):
    """Energy-conserving delta of Eq. 8: ELPH_DELTA_GAUSS, ELPH_DELTA_TETRA or ELPH_DELTA_TRIANGLE."""
    _check(ctx, load().elph_set_delta(ctx.handle, int(method)))


def elph_set_polar(ctx, zstar, eps_inf, tau=None):
    """Born charges zstar [natom][3][3], eps_inf [3][3] and atom positions tau
    [natom][3] (Angstrom; None: no Froehlich vertex) for Eqs. 4 and 7;
    zstar=None removes both."""
    if zstar is None:
        _check(ctx, load().elph_set_polar(ctx.handle, None, None, None))
        return
    z = np.ascontiguousarray(zstar, dtype=np.float64)
    e = np.ascontiguousarray(eps_inf, dtype=np.float64)
    t = None if tau is None else np.ascontiguousarray(tau, dtype=np.float64)
    _check(ctx, load().elph_set_polar(ctx.handle, z.ctypes.data_as(ctypes.c_void_p),
                                      e.ctypes.data_as(ctypes.c_void_p),
                                      None if t is None else t.ctypes.data_as(ctypes.c_void_p)))


def elph_set_ifc3(ctx, rj, rk, psi):
    """Third-order force constants: rj, rk [n][3] cells and psi
    [n][natom][natom][natom][3][3][3] (eV/A^3) of Eq. 13; psi=None removes them."""
    if psi is None:
        _check(ctx, load().elph_set_ifc3(ctx.handle, 0, None, None, None))
        return
    a = np.ascontiguousarray(rj, dtype=np.int32)
    b = np.ascontiguousarray(rk, dtype=np.int32)
    p = np.ascontiguousarray(psi, dtype=np.float64)
    _check(ctx, load().elph_set_ifc3(ctx.handle, int(a.shape[0]), a.ctypes.data_as(ctypes.c_void_p),
                                     b.ctypes.data_as(ctypes.c_void_p), p.ctypes.data_as(ctypes.c_void_p)))


def elph_phph_vertex(ctx, q, qp, V2):
    """|V-(q, q')|^2 of Eq. 13 for device int32 mesh-index lists q, qp into V2
    [npairs][nbr][nbr][nbr] (device FP64)."""
    _check(ctx, load().elph_phph_vertex(ctx.handle, int(q.numel()), _ptr(q), _ptr(qp), _ptr(V2)))


def elph_phph_rates(ctx, T, sigma, W_ph):
    """Three-phonon RTA rates (Eq. 26) of every mode into W_ph [Nq][nbr] (device FP64, 1/s)."""
    _check(ctx, load().elph_phph_rates(ctx.handle, float(T), float(sigma), _ptr(W_ph)))


def elph_phph_inscatter(ctx, T, sigma, F, S):
    """Three-phonon in-scattering of F [Nq][nbr][3] into S (device FP64, Eq. 26)."""
    _check(ctx, load().elph_phph_inscatter(ctx.handle, float(T), float(sigma), _ptr(F), _ptr(S)))


def elph_set_phph(ctx, sigma):
    """Three-phonon processes in elph_iterate with Gaussian width sigma (eV); 0 turns them off."""
    _check(ctx, load().elph_set_phph(ctx.handle, float(sigma)))


def elph_ko_enforce(ctx, T, I, J, F, G):
    """Kelvin-Onsager enforcement on device responses (I rewritten in place).
    Returns dict(tensors [6,3,3] numpy, lambda, ko_residual)."""
    tens = np.zeros(54)
    lam = ctypes.c_double(0.0)
    ko = ctypes.c_double(0.0)
    _check(ctx, load().elph_ko_enforce(ctx.handle, float(T), _ptr(I), _ptr(J), _ptr(F), _ptr(G),
                                       tens.ctypes.data_as(ctypes.c_void_p), ctypes.byref(lam), ctypes.byref(ko)))
    names = ("sigma", "sigmaS", "alpha_el", "kappa0_el", "alpha_ph", "kappa_ph")
    return {"tensors": {n: tens[9 * a:9 * a + 9].reshape(3, 3).copy() for a, n in enumerate(names)},
            "lambda": lam.value, "ko_residual": ko.value}


class Batch:
    """Owns an elph_batch handle (the contexts must outlive it)."""

    def __init__(self, ctxs):
        lib = load()
        self.ctxs = list(ctxs)
        arr = (ctypes.c_void_p * len(self.ctxs))(*[c.handle.value if hasattr(c.handle, "value") else c.handle
                                                 for c in self.ctxs])
        h = ctypes.c_void_p()
        st = lib.elph_batch_create(len(self.ctxs), arr, ctypes.byref(h))
        if st != ELPH_OK:
            raise ElphError(st, lib.elph_batch_last_error(None).decode())
        self.handle = h

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None):
            load().elph_batch_destroy(self.handle)
            self.handle = None

    def _check(self, st):
        if st != ELPH_OK:
            raise ElphError(st, load().elph_batch_last_error(self.handle).decode())


def elph_batch_create(ctxs):
    return Batch(ctxs)


def elph_batch_destroy(batch):
    batch.close()


def elph_batch_scatt_rates(batch, T, W_e=None, W_ph=None, use_graph=True):
    n = len(batch.ctxs)
    def arr(ts):
        if ts is None:
            return None
        return (ctypes.c_void_p * n)(*[t.data_ptr() if t is not None else None for t in ts])
    batch._check(load().elph_batch_scatt_rates(batch.handle, float(T), arr(W_e), arr(W_ph), int(bool(use_graph))))


def elph_batch_tune(batch, T):
    ch = np.zeros(3, dtype=np.int32)
    best = ctypes.c_double(0.0)
    batch._check(load().elph_batch_tune(batch.handle, float(T), ch.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(best)))
    return {"blocks_per_cu": int(ch[0]), "cost_ordered": bool(ch[1]), "tile_rows": int(ch[2]),
            "best_ms": best.value}


def elph_batch_set_shape(batch, blocks_per_cu, cost_ordered, tile_rows):
    batch._check(load().elph_batch_set_shape(batch.handle, int(blocks_per_cu), int(bool(cost_ordered)),
                                             int(tile_rows)))


# ---------------------------------------------------------------------------
# learned screen


class MLP:
    """Owns an elph_mlp handle (the screening network)."""

    def __init__(self, nin, width, depth, params, stream=None):
        lib = load()
        self.nin, self.width, self.depth = int(nin), int(width), int(depth)
        prm = _arr(params, np.float32)
        h = ctypes.c_void_p()
        st = lib.elph_mlp_create(self.nin, self.width, self.depth, prm.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != ELPH_OK:
            raise ElphError(st, lib.elph_mlp_last_error(None).decode())
        self.handle = h

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None):
            load().elph_mlp_destroy(self.handle)
            self.handle = None

    def _check(self, st):
        if st != ELPH_OK:
            raise ElphError(st, load().elph_mlp_last_error(self.handle).decode())


def elph_mlp_create(nin, width, depth, params, stream=None):
    return MLP(nin, width, depth, params, stream)


def elph_mlp_nparams(mlp):
    return int(load().elph_mlp_nparams(mlp.handle))


def elph_mlp_get_params(mlp):
    out = np.empty(elph_mlp_nparams(mlp), dtype=np.float32)
    mlp._check(load().elph_mlp_get_params(mlp.handle, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def elph_mlp_set_params(mlp, params):
    prm = _arr(params, np.float32)
    mlp._check(load().elph_mlp_set_params(mlp.handle, prm.ctypes.data_as(ctypes.c_void_p)))


def elph_mlp_forward(mlp, x, y):
    """x [n][nin], y [n]: FP32 GPU tensors."""
    mlp._check(load().elph_mlp_forward(mlp.handle, int(y.numel()), _ptr(x), _ptr(y)))


def elph_mlp_gradients(mlp, x, t, grad=None):
    loss = ctypes.c_double(0.0)
    mlp._check(load().elph_mlp_gradients(mlp.handle, int(t.numel()), _ptr(x), _ptr(t), _ptr(grad),
                                         ctypes.byref(loss)))
    return loss.value


def elph_mlp_train_step(mlp, x, t, lr):
    loss = ctypes.c_double(0.0)
    mlp._check(load().elph_mlp_train_step(mlp.handle, int(t.numel()), _ptr(x), _ptr(t), ctypes.c_float(lr),
                                          ctypes.byref(loss)))
    return loss.value


def elph_screen_nin(ctx):
    return int(load().elph_screen_nin(ctx.handle))


def elph_screen_samples(ctx, kidx, qidx, x, t):
    """kidx, qidx: int32 GPU tensors [npairs]; x [npairs*nbr*nb*nb][nin],
    t [npairs*nbr*nb*nb]: FP32 GPU tensors."""
    _check(ctx, load().elph_screen_samples(ctx.handle, int(kidx.numel()), _ptr(kidx), _ptr(qidx), _ptr(x),
                                           _ptr(t)))


def elph_scatt_rates_screened(ctx, mlp, mode, tau, T, W_e=None, W_ph=None, gauss_min=1e-30):
    stats = np.zeros(5, dtype=np.float64)
    _check(ctx, load().elph_scatt_rates_screened(ctx.handle, mlp.handle if mlp is not None else None, int(mode),
                                                 float(tau), float(gauss_min), float(T), _ptr(W_e), _ptr(W_ph),
                                                 stats.ctypes.data_as(ctypes.c_void_p)))
    return {"tiles": int(stats[0]), "tiles_computed": int(stats[1]), "tiles_energy": int(stats[2]),
            "terms_queried": int(stats[3]), "screen_ms": float(stats[4])}
