"""HIP path (through the C ABI) against the CPU oracle, element by element.

Tolerances: the plain FP64 path must match to relative 1e-10; elementwise
terms use |d| <= 1e-10 |x| + 1e-12 max|x| because tiny vertices carry the
absolute rounding of the phase sums.  Rates use the max-per-state relative
error over states with W_ref >= 1e-12 max W_ref (smaller ones absolutely).
"""
import numpy as np
import pytest

import ko_cases
import oracle
import synth
from synth import materials as sm

torch = pytest.importorskip("torch")
E = pytest.importorskip("paper_2109_08547_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rate_err(w, ref, floor=1e-12):
    w, ref = np.asarray(w).ravel(), np.asarray(ref).ravel()
    mx = np.abs(ref).max()
    big = np.abs(ref) >= floor * mx
    e_rel = (np.abs(w[big] - ref[big]) / np.abs(ref[big])).max() if big.any() else 0.0
    e_abs = (np.abs(w[~big] - ref[~big]) / mx).max() if (~big).any() else 0.0
    return max(e_rel, e_abs)


def term_ok(x, ref, rtol=1e-10, atol_rel=1e-12):
    x, ref = np.asarray(x), np.asarray(ref)
    bound = rtol * np.abs(ref) + atol_rel * np.abs(ref).max()
    return np.all(np.abs(x - ref) <= bound), (np.abs(x - ref) / (np.abs(ref) + 1e-300)).max()


def make_ctx(cfg, mat, precision="fp64", window=None, mu=None):
    return E.elph_create(mat, cfg["mesh"], cfg["mu"] if mu is None else mu,
                         cfg["window"] if window is None else window, cfg["sigma"], precision=precision)


def dtensor(n, dtype=torch.float64):
    return torch.empty(int(n), dtype=dtype, device=DEV)


class Case:
    """A workload with its oracle results on all rows (small meshes)."""

    def __init__(self, name, T=300.0, mat=None, cfg=None):
        self.cfg = cfg or synth.config(name)
        self.mat = mat or synth.material_for(self.cfg)
        self.T = T
        c = self.cfg
        self.prob = oracle.Problem(self.mat, c["mesh"], c["mu"], c["window"], c["sigma"])
        self.Xp, self.Xm = self.prob.transition_probs(T)
        self.we = self.prob.rates_e(T, self.Xp, self.Xm)
        self.wph = self.prob.rates_ph(T, self.Xp)


_cases = {}


def case(name):
    if name not in _cases:
        _cases[name] = Case(name)
    return _cases[name]


def _maxsize_case():
    """Largest band and branch counts the library supports: 16 bands, 5 atoms."""
    if "max16" not in _cases:
        mat = sm.make_material(16, 5, 41, sm.rset_cube(-1, 1), sm.rset_cube(0, 1), 2.0, 0.15, 0.6, 0.004)
        cfg = dict(mesh=3, mu=0.0, window=0.9, sigma=0.02, T=300.0)
        _cases["max16"] = Case("max16", mat=mat, cfg=cfg)
    return _cases["max16"]


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["tiny4", "plain8", "metal6"])
def test_tables(name):
    c = case(name)
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    p = c.prob
    assert sz["nstates"] == p.nstates and sz["nkept"] == p.kept.size and sz["nk"] == p.nk
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    sk, smm = dtensor(M, torch.int32), dtensor(M, torch.int32)
    eps, vel = dtensor(M), dtensor(3 * M)
    hw, vph = dtensor(nm), dtensor(3 * nm)
    E.elph_tables(ctx, sk, smm, eps, vel, hw, vph)
    torch.cuda.synchronize()
    assert np.array_equal(sk.cpu().numpy(), p.state_k)
    assert np.array_equal(smm.cpu().numpy(), p.state_m)
    assert np.abs(eps.cpu().numpy() - p.eps).max() < 1e-12 * max(1.0, np.abs(p.eps).max())
    v = vel.cpu().numpy().reshape(M, 3)
    assert np.abs(v - p.v_state).max() < 1e-9 * np.abs(p.v_state).max()
    # compare (hbar omega)^2: the zero modes at Gamma are square roots of rounding noise
    assert np.abs(hw.cpu().numpy().reshape(-1, sz["nbr"]) ** 2 - p.hw ** 2).max() < 1e-12 * p.hw.max() ** 2
    vp = vph.cpu().numpy().reshape(-1, sz["nbr"], 3)
    assert np.abs(vp - p.v_ph).max() < 1e-8 * np.abs(p.v_ph).max()
    assert abs(sz["hw_max_eV"] - p.hw.max()) < 1e-12
    ctx.close()


@pytest.mark.parametrize("name", ["tiny3", "tiny4", "plain8", "metal6"])
def test_transition_probs_full(name):
    c = case(name)
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    xp, xm = dtensor(sz["nterms"]), dtensor(sz["nterms"])
    E.elph_transition_probs(ctx, c.T, xp, xm)
    torch.cuda.synchronize()
    shape = c.Xp.shape
    ok_p, ep = term_ok(xp.cpu().numpy().reshape(shape), c.Xp)
    ok_m, em = term_ok(xm.cpu().numpy().reshape(shape), c.Xm)
    assert ok_p and ok_m, (ep, em)
    ctx.close()


@pytest.mark.parametrize("name", ["tiny3", "tiny4", "plain8", "metal6"])
def test_scatt_rates_full(name):
    c = case(name)
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
    E.elph_scatt_rates(ctx, c.T, we, wph)
    torch.cuda.synchronize()
    assert rate_err(we.cpu().numpy(), c.we) < 1e-10
    assert rate_err(wph.cpu().numpy(), c.wph) < 1e-10
    # the vertex store is reused at another temperature
    T2 = 200.0
    E.elph_scatt_rates(ctx, T2, we, wph)
    torch.cuda.synchronize()
    Xp2, Xm2 = c.prob.transition_probs(T2)
    assert rate_err(we.cpu().numpy(), c.prob.rates_e(T2, Xp2, Xm2)) < 1e-10
    assert rate_err(wph.cpu().numpy(), c.prob.rates_ph(T2, Xp2)) < 1e-10
    # transition probabilities from the retained store
    xp, xm = dtensor(sz["nterms"]), dtensor(sz["nterms"])
    E.elph_transition_probs(ctx, T2, xp, xm, store_B=True)
    torch.cuda.synchronize()
    assert term_ok(xp.cpu().numpy().reshape(Xp2.shape), Xp2)[0]
    assert term_ok(xm.cpu().numpy().reshape(Xm2.shape), Xm2)[0]
    ctx.close()


# every form at the largest band and branch counts (15 branches: the widest
# epilogues; the GEMM forms' row tiles end inside a block)
@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3", "bf16x6", "fp16x3"])
def test_maximum_sizes_16_bands_5_atoms(form):
    c = _maxsize_case()
    ctx = make_ctx(c.cfg, c.mat, precision=form)
    sz = E.elph_sizes(ctx)
    assert sz["nwann"] == 16 and sz["nbr"] == 15 and sz["nstates"] == c.prob.nstates
    we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
    E.elph_scatt_rates(ctx, c.T, we, wph)
    torch.cuda.synchronize()
    w1, w2 = we.cpu().numpy(), wph.cpu().numpy()
    if form == "fp64":
        assert rate_err(w1, c.we) < 1e-10
        assert rate_err(w2, c.wph) < 1e-10
    else:
        # the refined forms' strict bar, as in test_gemm_forms_refined_meet_the_strict_bar
        e1, e2 = rate_err(w1, c.we), rate_err(w2, c.wph)
        n1 = np.linalg.norm(w1 - c.we) / np.linalg.norm(c.we)
        n2 = np.linalg.norm(w2 - c.wph.ravel()) / np.linalg.norm(c.wph)
        print("%s at 16 bands, 5 atoms: strict %.2e %.2e, norm-wise %.2e %.2e, %s"
              % (form, e1, e2, n1, n2, E.elph_refine_info(ctx)))
        assert e1 <= 1e-5 and e2 <= 1e-5 and n1 < 1e-6 and n2 < 1e-6
    ctx.close()


@pytest.mark.parametrize("name", ["tiny4", "plain8"])
def test_interp_g_pairs(name):
    c = case(name)
    p = c.prob
    ctx = make_ctx(c.cfg, c.mat)
    rng = np.random.default_rng(17)
    npairs = 40
    kk = rng.integers(0, p.nk, npairs).astype(np.int32)
    qq = rng.integers(1, p.nk, npairs).astype(np.int32)  # q != Gamma (degenerate acoustic)
    g = torch.empty((npairs, p.nbr, p.nb, p.nb, 2), dtype=torch.float64, device=DEV)
    E.elph_interp_g(ctx, torch.from_numpy(kk).to(DEV), torch.from_numpy(qq).to(DEV), g)
    torch.cuda.synchronize()
    g2 = (g.cpu().numpy() ** 2).sum(-1)
    for t in range(npairs):
        k, q = p.kfrac[kk[t]], p.kfrac[qq[t]]
        gW = oracle.g_wannier_brute(c.mat, k, q) if name == "tiny4" else \
            oracle.g_wannier_factorised(c.mat, k, q[None])[0]
        _, Uk = oracle.electron_bands(c.mat, k[None])
        _, Ukq = oracle.electron_bands(c.mat, (k + q)[None])
        hw, u = oracle.phonon_modes(c.mat, q[None])
        ref = np.abs(oracle.g_bloch(c.mat, gW, Uk[0], Ukq[0], u[0], hw[0])) ** 2
        assert np.abs(g2[t] - ref).max() <= 1e-10 * ref.max(), t
    # an empty list is a no-op
    E.elph_interp_g(ctx, torch.empty(0, dtype=torch.int32, device=DEV),
                    torch.empty(0, dtype=torch.int32, device=DEV), g)
    ctx.close()


def test_determinism_plain8():
    c = case("plain8")
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    out = []
    for _ in range(2):
        E.elph_reset(ctx)
        we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
        xp = dtensor(sz["nterms"])
        E.elph_scatt_rates(ctx, c.T, we, wph)
        E.elph_transition_probs(ctx, c.T, xp, None, store_B=True)
        torch.cuda.synchronize()
        out.append((we.cpu().numpy(), wph.cpu().numpy(), xp.cpu().numpy()))
    # fixed-order reductions everywhere: bitwise equal
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    ctx.close()


# The GEMM forms (FP32 on the FP32 MFMA, the BF16 splits x3 / x6 and the
# FP16 split x3 on the BF16 / FP16 MFMA) accumulate in FP32: a vertex
# component carries an error of about 1e-7 of the root-sum-square of its
# products (2e-6 for BF16x3, whose operands keep 16 bits), so a term whose
# vertex nearly cancels has a far larger relative error, and a rate that such
# a term dominates inherits it.  With the FP64 refinement (on by default)
# every rate meets the strict bar: max over states of the relative error,
# rates below 1e-12 of the largest judged absolutely (1e-5), plus 1e-6
# norm-wise.  Without it the forms are held to what their arithmetic gives.
def _form_rates(name, form, theta=None):
    c = case(name)
    ctx = make_ctx(c.cfg, c.mat, precision=form)
    if theta is not None:
        E.elph_set_refine(ctx, theta)
    sz = E.elph_sizes(ctx)
    we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
    E.elph_scatt_rates(ctx, c.T, we, wph)
    torch.cuda.synchronize()
    info = E.elph_refine_info(ctx)
    ctx.close()
    w1, w2 = we.cpu().numpy(), wph.cpu().numpy()
    n1 = np.linalg.norm(w1 - c.we) / np.linalg.norm(c.we)
    n2 = np.linalg.norm(w2 - c.wph.ravel()) / np.linalg.norm(c.wph)
    return c, w1, w2, (rate_err(w1, c.we), rate_err(w2, c.wph)), (n1, n2), info


@pytest.mark.parametrize("name", ["plain8", "metal6"])
@pytest.mark.parametrize("form", ["fp32", "bf16x3", "bf16x6", "fp16x3"])
def test_gemm_forms_refined_meet_the_strict_bar(name, form):
    c, w1, w2, strict, norm, info = _form_rates(name, form)
    print("%s form %s refined: strict %.2e %.2e, norm-wise %.2e %.2e, %s" % (form, name, strict[0], strict[1],
                                                                           norm[0], norm[1], info))
    assert strict[0] <= 1e-5 and strict[1] <= 1e-5
    # BF16x3 leaves a diffuse error spread over every term of a rate, which
    # the selection (terms carrying theta/8 of a rate each) does not remove
    nbar = 5e-6 if form == "bf16x3" else 1e-6
    assert norm[0] <= nbar and norm[1] <= nbar
    assert info["overflow"] == 0


# Plain forms (refinement off): 1e-5 per rate above 1e-6 of the largest and
# 1e-6 norm-wise for FP32, BF16x6 and FP16x3; BF16x3 keeps products of total
# order <= 2^-8, a relative error of about 2 x 2^-16 per product, doubled by
# |g|^2, times a safety factor 3: 2e-4 per rate, 2e-5 norm-wise.
@pytest.mark.parametrize("form", ["fp32", "fp16x3"])
def test_gemm_forms_in_several_chunks(form):
    """The contractions' FP32 output in chunks of initial states (step 1 and
    step 2 each in at least three chunks through a small chunk size): the
    store is bitwise that of one chunk, and the rates meet the strict bar
    against the oracle."""
    c = case("plain8")
    M = c.prob.nstates
    ncol = c.prob.nbr * len(c.mat["rp"]) * c.prob.nb          # step-1 columns (x, R_p, n')
    out = []
    # step 1 in 4 chunks of M/3 rows, step 2 in chunks of 36 states
    for chunk in (None, 8 * ncol * (M // 3)):
        ctx = make_ctx(c.cfg, c.mat, precision=form)
        if chunk:
            E.elph_set_gemm_chunk(ctx, chunk)
        sz = E.elph_sizes(ctx)
        we, wph, xp = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"]), dtensor(sz["nterms"])
        E.elph_set_refine(ctx, 0.0)                     # the store itself, unrefined
        E.elph_transition_probs(ctx, c.T, xp, None, store_B=True)
        E.elph_set_refine(ctx, 2e-6)
        E.elph_reset(ctx, E.elph.ELPH_RESET_STORE)
        E.elph_scatt_rates(ctx, c.T, we, wph)
        torch.cuda.synchronize()
        out.append((xp.cpu().numpy(), we.cpu().numpy(), wph.cpu().numpy()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    for w in out:
        assert rate_err(w[1], c.we) <= 1e-5 and rate_err(w[2], c.wph) <= 1e-5
    with pytest.raises(E.ElphError):
        ctx = make_ctx(c.cfg, c.mat, precision=form)
        try:
            E.elph_set_gemm_chunk(ctx, 1000)
        finally:
            ctx.close()


@pytest.mark.parametrize("name", ["plain8", "metal6"])
@pytest.mark.parametrize("form", ["fp32", "bf16x3", "bf16x6", "fp16x3"])
def test_gemm_forms_plain(name, form):
    c, w1, w2, strict, norm, info = _form_rates(name, form, theta=0.0)
    e1, e2 = rate_err(w1, c.we, 1e-6), rate_err(w2, c.wph, 1e-6)
    print("%s form %s plain: strict %.2e %.2e, above 1e-6 max %.2e %.2e, norm-wise %.2e %.2e"
          % (form, name, strict[0], strict[1], e1, e2, norm[0], norm[1]))
    assert info["pairs"] == 0
    if form == "bf16x3":
        assert e1 < 2e-4 and e2 < 2e-4 and norm[0] < 2e-5 and norm[1] < 2e-5
    else:
        assert e1 < 1e-5 and e2 < 1e-5 and norm[0] < 1e-6 and norm[1] < 1e-6


@pytest.mark.parametrize("form", ["fp16x3", "fp32"])
def test_error_estimates_track_the_actual_term_errors(form):
    """The stored per-term estimates against the terms' actual relative errors
    (oracle, plain8, refinement effectively off): the median term sits below
    its estimate and no term exceeds it by more than an order of magnitude;
    refined terms carry code 0 and match the oracle to FP64 accuracy."""
    c = case("plain8")
    ctx = make_ctx(c.cfg, c.mat, precision=form)
    E.elph_set_refine(ctx, 1e30)          # estimates kept, no rate flagged
    sz = E.elph_sizes(ctx)
    we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
    E.elph_scatt_rates(ctx, c.T, we, wph)
    est = dtensor(sz["nterms"])
    E.elph_refine_estimates(ctx, est)
    xp = dtensor(sz["nterms"])
    E.elph_transition_probs(ctx, c.T, xp, None, store_B=True)
    torch.cuda.synchronize()
    est, xp = est.cpu().numpy(), xp.cpu().numpy()
    ref = c.Xp.reshape(-1)
    ok = ref > 1e-30 * ref.max()
    ratio = np.abs(xp[ok] - ref[ok]) / ref[ok] / est[ok]
    print("%s: actual/estimate median %.2f, p99.9 %.2f, max %.2f" % (form, np.median(ratio),
                                                                     np.quantile(ratio, 0.999), ratio.max()))
    assert np.all(est[ok] > 0)
    assert np.median(ratio) < 1.0 and ratio.max() < 12.0
    # now refine at the default threshold: refined terms are exact
    E.elph_set_refine(ctx, 2e-6)
    E.elph_reset(ctx, E.elph.ELPH_RESET_STORE)
    E.elph_scatt_rates(ctx, c.T, we, wph)
    info = E.elph_refine_info(ctx)
    est2 = dtensor(sz["nterms"])
    E.elph_refine_estimates(ctx, est2)
    E.elph_transition_probs(ctx, c.T, xp2 := dtensor(sz["nterms"]), None, store_B=True)
    torch.cuda.synchronize()
    est2, xp2 = est2.cpu().numpy(), xp2.cpu().numpy()
    exact = est2 == 0.0
    print("%s: refinement %s, %d exact terms" % (form, info, exact.sum()))
    assert info["pairs"] > 0 and exact.sum() >= info["pairs"]
    # exact terms: FP64 vertex, stored in FP32
    sel = exact & (ref > 1e-30 * ref.max())
    assert np.all(np.abs(xp2[sel] - ref[sel]) <= 2e-7 * ref[sel])
    ctx.close()


# 15 branches: the drag gathers take the branches in several passes.  All
# four levels; the oracle's plain inner substitution converges too slowly
# here when started cold (PARTIAL, DRAGLESS: its in-scattering operator has
# a spectral radius near 1), so the reference solves the electron step with
# its dense bordered solve (the same fixed point, pinned on metal6).
@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_iterate_16_bands_5_atoms(level):
    c = _maxsize_case()
    T = c.T
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    assert sz["nbr"] == 15
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    I, J, F, G = dtensor(3 * M), dtensor(3 * M), dtensor(3 * nm), dtensor(3 * nm)
    wext = oracle.default_w_ext(c.prob, T, gamma0=1e13)
    wext_d = torch.from_numpy(np.ascontiguousarray(wext.reshape(-1))).to(DEV)
    tol = 1e-12
    E.elph_iterate(ctx, T, I, J, F, G, W_ph_ext=wext_d, level=level, tol=tol, maxit=400)
    torch.cuda.synchronize()
    ref = oracle.iterate(c.prob, T, c.Xp, c.Xm, level, tol=tol, maxit=400, w_ext=wext, inner="direct")
    assert ref["converged"]
    got = dict(I=I.cpu().numpy().reshape(M, 3), J=J.cpu().numpy().reshape(M, 3),
               F=F.cpu().numpy().reshape(-1, sz["nbr"], 3), G=G.cpu().numpy().reshape(-1, sz["nbr"], 3))
    for key in ("I", "J", "F", "G"):
        scale = np.abs(ref[key]).max()
        if key == "G" and level in (0, 2):              # no drag: G stays 0
            assert scale == 0 and not np.any(got[key]), key
            continue
        assert scale > 0, key
        assert np.abs(got[key] - ref[key]).max() <= 1e-8 * scale, key
    ctx.close()


# polar material: the non-analytic term of Eq. 4 in the phonon tables and
# everything downstream
_polar = {}


def polar_case():
    if "metal6" not in _polar:
        cfg = synth.config("metal6")
        mat = dict(synth.material_for(cfg))
        mat["zstar"], mat["eps_inf"], mat["tau"] = synth.polar_params(int(mat["natom"]), 7, lat=mat["lat"])
        _polar["metal6"] = Case("metal6", mat=mat, cfg=cfg)
    return _polar["metal6"]


def test_polar_tables_and_rates():
    c = polar_case()
    p = c.prob
    ctx = make_ctx(c.cfg, c.mat)
    E.elph_set_polar(ctx, c.mat["zstar"], c.mat["eps_inf"], c.mat["tau"])
    sz = E.elph_sizes(ctx)
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    hw, vph = dtensor(nm), dtensor(3 * nm)
    E.elph_tables(ctx, None, None, None, None, hw, vph)
    we, wph = dtensor(M), dtensor(nm)
    E.elph_scatt_rates(ctx, c.T, we, wph)
    torch.cuda.synchronize()
    assert np.abs(hw.cpu().numpy().reshape(-1, sz["nbr"]) ** 2 - p.hw ** 2).max() < 1e-12 * p.hw.max() ** 2
    vp = vph.cpu().numpy().reshape(-1, sz["nbr"], 3)
    assert np.abs(vp - p.v_ph).max() < 1e-8 * np.abs(p.v_ph).max()
    assert rate_err(we.cpu().numpy(), c.we) < 1e-10
    assert rate_err(wph.cpu().numpy(), c.wph) < 1e-10
    # the vertex at arbitrary pairs carries the Froehlich part too
    rng = np.random.default_rng(9)
    kk = rng.integers(0, p.nk, 12).astype(np.int32)
    qq = rng.integers(1, p.nk, 12).astype(np.int32)
    g = torch.empty((12, p.nbr, p.nb, p.nb, 2), dtype=torch.float64, device=DEV)
    E.elph_interp_g(ctx, torch.from_numpy(kk).to(DEV), torch.from_numpy(qq).to(DEV), g)
    torch.cuda.synchronize()
    g2 = (g.cpu().numpy() ** 2).sum(-1)
    for t in range(12):
        k, q = p.kfrac[kk[t]], p.kfrac[qq[t]]
        gW = oracle.g_wannier_factorised(c.mat, k, q[None])[0]
        _, Uk = oracle.electron_bands(c.mat, k[None])
        _, Ukq = oracle.electron_bands(c.mat, (k + q)[None])
        hwq, u = oracle.phonon_modes(c.mat, q[None])
        ref = oracle.g_bloch(c.mat, gW, Uk[0], Ukq[0], u[0], hwq[0]) + p.frohlich_g(Uk[0], Ukq[0], qq[t])
        ref = np.abs(ref) ** 2
        assert np.abs(g2[t] - ref).max() <= 1e-9 * ref.max(), t
    # the terms change the phonons (LO-TO splitting) and are removed again
    plain = case("metal6")
    assert np.abs(p.hw - plain.prob.hw).max() > 1e-4
    E.elph_set_polar(ctx, None, None)
    E.elph_tables(ctx, None, None, None, None, hw, vph)
    torch.cuda.synchronize()
    assert np.abs(hw.cpu().numpy().reshape(-1, sz["nbr"]) ** 2 - plain.prob.hw ** 2).max() < 1e-12 * plain.prob.hw.max() ** 2
    with pytest.raises(E.ElphError):
        E.elph_set_polar(ctx, c.mat["zstar"], -np.eye(3))
    ctx.close()


# analytic tetrahedron delta: the store, X+- and the rates against the oracle
_tetra_ref = {}


DELTA = {"tetra": 1, "triangle": 2}


def tetra_ref(name, method="tetra"):
    if (name, method) not in _tetra_ref:
        c = case(name)
        Xp, Xm = c.prob.transition_probs(c.T, delta=method)
        _tetra_ref[(name, method)] = (Xp, Xm, c.prob.rates_e(c.T, Xp, Xm), c.prob.rates_ph(c.T, Xp))
    return _tetra_ref[(name, method)]


@pytest.mark.parametrize("method", ["tetra", "triangle"])
@pytest.mark.parametrize("name", ["tiny4", "metal6"])
def test_tetra_delta_transition_probs_and_rates(name, method):
    c = case(name)
    Xp_ref, Xm_ref, we_ref, wph_ref = tetra_ref(name, method)
    ctx = make_ctx(c.cfg, c.mat)
    E.elph_set_delta(ctx, DELTA[method])
    sz = E.elph_sizes(ctx)
    xp, xm = dtensor(sz["nterms"]), dtensor(sz["nterms"])
    E.elph_transition_probs(ctx, c.T, xp, xm, 1)
    we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
    E.elph_scatt_rates(ctx, c.T, we, wph)
    torch.cuda.synchronize()
    # the tetrahedron (triangle) weights divide by energy differences of the
    # corners, which magnify the 1e-15 differences of the two sides'
    # eigenvalues: bars 1e-8 (1e-10 of the largest term absolutely).  Where
    # the level passes within ~1e-10 eV of a triangle's corner (mirror
    # corners of the symmetric model bands), the two energy differences of a
    # triangle weight leave those differences at ~1e-7: bar 1e-6 there
    rtol = 1e-8 if method == "tetra" else 1e-6
    assert np.count_nonzero(Xp_ref) > 0.01 * Xp_ref.size
    ok_p, ep = term_ok(xp.cpu().numpy().reshape(Xp_ref.shape), Xp_ref, rtol=rtol, atol_rel=1e-10)
    ok_m, em = term_ok(xm.cpu().numpy().reshape(Xm_ref.shape), Xm_ref, rtol=rtol, atol_rel=1e-10)
    assert ok_p and ok_m, (ep, em)
    assert rate_err(we.cpu().numpy(), we_ref) < 1e-8
    assert rate_err(wph.cpu().numpy(), wph_ref) < 1e-8
    # switching back gives the Gaussian store again
    E.elph_set_delta(ctx, E.elph.ELPH_DELTA_GAUSS)
    E.elph_transition_probs(ctx, c.T, xp, xm, 0)
    torch.cuda.synchronize()
    ok, e = term_ok(xp.cpu().numpy().reshape(c.Xp.shape), c.Xp)
    assert ok, e
    with pytest.raises(E.ElphError):
        E.elph_set_delta(ctx, 7)
    ctx.close()


# the FP64 refinement applies to the Gaussian delta only, so the
# tetrahedron delta keeps the plain forms' bars
@pytest.mark.parametrize("method", ["tetra", "triangle"])
@pytest.mark.parametrize("form", ["fp32", "fp16x3"])
def test_tetra_delta_forms(form, method):
    c = case("metal6")
    _, _, we_ref, wph_ref = tetra_ref("metal6", method)
    ctx = make_ctx(c.cfg, c.mat, precision=form)
    E.elph_set_delta(ctx, DELTA[method])
    sz = E.elph_sizes(ctx)
    we, wph = dtensor(sz["nstates"]), dtensor(sz["nk"] * sz["nbr"])
    E.elph_scatt_rates(ctx, c.T, we, wph)
    torch.cuda.synchronize()
    w1, w2 = we.cpu().numpy(), wph.cpu().numpy()
    e1, e2 = rate_err(w1, we_ref, 1e-6), rate_err(w2, wph_ref, 1e-6)
    n1 = np.linalg.norm(w1 - we_ref) / np.linalg.norm(we_ref)
    n2 = np.linalg.norm(w2 - wph_ref.ravel()) / np.linalg.norm(wph_ref)
    assert e1 < 1e-5 and e2 < 1e-5 and n1 < 1e-6 and n2 < 1e-6, (e1, e2, n1, n2)
    ctx.close()


def _iterate_against_oracle(ctx, c, Xp, Xm, prob):
    T = c.T
    sz = E.elph_sizes(ctx)
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    I, J, F, G = dtensor(3 * M), dtensor(3 * M), dtensor(3 * nm), dtensor(3 * nm)
    wext = oracle.default_w_ext(prob, T, gamma0=1e13)
    wext_d = torch.from_numpy(np.ascontiguousarray(wext.reshape(-1))).to(DEV)
    E.elph_iterate(ctx, T, I, J, F, G, W_ph_ext=wext_d, level=3, tol=1e-12, maxit=400)
    torch.cuda.synchronize()
    ref = oracle.iterate(prob, T, Xp, Xm, 3, tol=1e-12, maxit=400, w_ext=wext)
    assert ref["converged"]
    got = dict(I=I.cpu().numpy().reshape(M, 3), J=J.cpu().numpy().reshape(M, 3),
               F=F.cpu().numpy().reshape(-1, sz["nbr"], 3), G=G.cpu().numpy().reshape(-1, sz["nbr"], 3))
    for key in ("I", "J", "F", "G"):
        scale = np.abs(ref[key]).max()
        assert scale > 0, key
        assert np.abs(got[key] - ref[key]).max() <= 1e-7 * scale, key


@pytest.mark.parametrize("method", ["tetra", "triangle"])
def test_tetra_delta_coupled_iteration(method):
    c = case("metal6")
    Xp, Xm, _, _ = tetra_ref("metal6", method)
    ctx = make_ctx(c.cfg, c.mat)
    E.elph_set_delta(ctx, DELTA[method])
    _iterate_against_oracle(ctx, c, Xp, Xm, c.prob)
    ctx.close()


def test_polar_coupled_iteration():
    c = polar_case()
    ctx = make_ctx(c.cfg, c.mat)
    E.elph_set_polar(ctx, c.mat["zstar"], c.mat["eps_inf"], c.mat["tau"])
    _iterate_against_oracle(ctx, c, c.Xp, c.Xm, c.prob)
    ctx.close()


@pytest.mark.parametrize("method", ["tetra", "triangle"])
def test_tetra_delta_is_refused_by_batches(method):
    c = case("tiny4")
    ctx = make_ctx(c.cfg, c.mat, precision="fp32")
    E.elph_set_delta(ctx, DELTA[method])
    with pytest.raises(Exception):
        E.Batch([ctx])
    ctx.close()


def test_ko_enforce_planted_lambda():
    # responses for which Eq. 35 holds at lambda = 0.8 (built from the oracle)
    c = case("metal6")
    ctx = make_ctx(c.cfg, c.mat)
    E.elph_sizes(ctx)
    T = c.T
    I, J, F, G = ko_cases.planted_ko_case(c.prob, T, 0.8)
    I_ref, lam_ref, tens_ref = oracle.ko_enforce(c.prob, T, I, J, F, G)
    dev = [torch.from_numpy(np.ascontiguousarray(a.reshape(-1))).to(DEV) for a in (I, J, F, G)]
    r = E.elph_ko_enforce(ctx, T, *dev)
    torch.cuda.synchronize()
    assert abs(r["lambda"] - 0.8) < 1e-9 and abs(lam_ref - 0.8) < 1e-12
    assert r["ko_residual"] < 1e-9
    got = dev[0].cpu().numpy().reshape(I.shape)
    assert np.abs(got - I_ref).max() <= 1e-10 * np.abs(I_ref).max()
    for key, val in tens_ref.items():
        assert np.abs(r["tensors"][key] - val).max() <= 1e-10 * max(np.abs(val).max(), 1e-300), key
    with pytest.raises(E.ElphError):
        E.elph_ko_enforce(ctx, T, dev[0], None, dev[2], dev[3])
    ctx.close()


def test_ko_enforce_on_the_coupled_solution():
    c = case("metal6")
    T = c.T
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    I, J, F, G = dtensor(3 * M), dtensor(3 * M), dtensor(3 * nm), dtensor(3 * nm)
    wext = oracle.default_w_ext(c.prob, T, gamma0=1e13)
    wext_d = torch.from_numpy(np.ascontiguousarray(wext.reshape(-1))).to(DEV)
    E.elph_iterate(ctx, T, I, J, F, G, W_ph_ext=wext_d, level=3, tol=1e-12, maxit=400)
    r = E.elph_ko_enforce(ctx, T, I, J, F, G)
    torch.cuda.synchronize()
    ref = oracle.iterate(c.prob, T, c.Xp, c.Xm, 3, tol=1e-12, maxit=400, w_ext=wext)
    I_ref, lam_ref, tens_ref = oracle.ko_enforce(c.prob, T, ref["I"], ref["J"], ref["F"], ref["G"])
    assert abs(r["lambda"] - lam_ref) <= 1e-6 * abs(lam_ref)
    got = I.cpu().numpy().reshape(M, 3)
    assert np.abs(got - I_ref).max() <= 1e-7 * np.abs(I_ref).max()
    for key, val in tens_ref.items():
        assert np.abs(r["tensors"][key] - val).max() <= 1e-7 * max(np.abs(val).max(), 1e-300), key
    assert abs(r["ko_residual"] - oracle.ko_residual(tens_ref, T)) < 1e-6
    ctx.close()


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_iterate_metal6(level):
    c = case("metal6")
    T = c.T
    ctx = make_ctx(c.cfg, c.mat)
    sz = E.elph_sizes(ctx)
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    I, J, F, G = dtensor(3 * M), dtensor(3 * M), dtensor(3 * nm), dtensor(3 * nm)
    wext = oracle.default_w_ext(c.prob, T, gamma0=1e13)
    wext_d = torch.from_numpy(np.ascontiguousarray(wext.reshape(-1))).to(DEV)
    tol = 1e-12
    res = E.elph_iterate(ctx, T, I, J, F, G, W_ph_ext=wext_d, level=level, tol=tol, maxit=400)
    torch.cuda.synchronize()
    ref = oracle.iterate(c.prob, T, c.Xp, c.Xm, level, tol=tol, maxit=400, w_ext=wext)
    assert ref["converged"]
    got = dict(I=I.cpu().numpy().reshape(M, 3), J=J.cpu().numpy().reshape(M, 3),
               F=F.cpu().numpy().reshape(-1, sz["nbr"], 3), G=G.cpu().numpy().reshape(-1, sz["nbr"], 3))
    for key in ("I", "J", "F", "G"):
        scale = np.abs(ref[key]).max()
        if scale == 0:
            assert np.abs(got[key]).max() == 0
            continue
        assert np.abs(got[key] - ref[key]).max() <= 1e-8 * scale, key
    tens = oracle.transport_tensors(c.prob, T, ref["I"], ref["J"], ref["F"], ref["G"])
    for key, val in tens.items():
        assert np.abs(res["tensors"][key] - val).max() <= 1e-8 * max(np.abs(val).max(), 1e-300), key
    assert abs(res["ko_residual"] - oracle.ko_residual(tens, T)) < 1e-6
    ctx.close()


_branch_cases = {}


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("na", [1, 3, 4])
def test_iterate_coupled_3_9_12_branches(na, form):
    """The coupled iteration with 3, 9 and 12 phonon branches (metal6's
    settings with 1, 3 and 4 atoms) against the oracle: the drag kernels and
    the LDS-staged drag gather at the branch counts the metal6 and 16-band
    cases leave out, with the FP64 and the FP32 store."""
    if na not in _branch_cases:
        cfg = dict(synth.config("metal6"))
        cfg.update(na=na)
        _branch_cases[na] = Case("metal6", mat=synth.material_for(cfg), cfg=cfg)
    c = _branch_cases[na]
    T = c.T
    ctx = make_ctx(c.cfg, c.mat, precision=form)
    sz = E.elph_sizes(ctx)
    assert sz["nbr"] == 3 * na
    M, nm = sz["nstates"], sz["nk"] * sz["nbr"]
    I, J, F, G = dtensor(3 * M), dtensor(3 * M), dtensor(3 * nm), dtensor(3 * nm)
    wext = oracle.default_w_ext(c.prob, T, gamma0=1e13)
    wext_d = torch.from_numpy(np.ascontiguousarray(wext.reshape(-1))).to(DEV)
    E.elph_iterate(ctx, T, I, J, F, G, W_ph_ext=wext_d, level=3, tol=1e-12, maxit=400)
    torch.cuda.synchronize()
    ref = oracle.iterate(c.prob, T, c.Xp, c.Xm, 3, tol=1e-12, maxit=400, w_ext=wext)
    assert ref["converged"]
    got = dict(I=I.cpu().numpy().reshape(M, 3), J=J.cpu().numpy().reshape(M, 3),
               F=F.cpu().numpy().reshape(-1, sz["nbr"], 3), G=G.cpu().numpy().reshape(-1, sz["nbr"], 3))
    # FP32 store: each X carries ~1e-7 of its vertex scale, which the solve
    # carries into the deviations at the same relative order
    bar = 1e-8 if form == "fp64" else 1e-5
    for key in ("I", "J", "F", "G"):
        scale = np.abs(ref[key]).max()
        assert scale > 0, key
        assert np.abs(got[key] - ref[key]).max() <= bar * scale, key
    ctx.close()


def test_window_excluding_everything_is_einval():
    c = case("plain8")
    ctx = make_ctx(c.cfg, c.mat, window=1e-9, mu=50.0)
    with pytest.raises(E.ElphError) as ei:
        E.elph_sizes(ctx)
    assert ei.value.status == E.elph.ELPH_EINVAL
    ctx.close()
