"""Seeded synthetic Wannier-space materials.

Recipe (simple-cubic lattice, a = 5.40 Angstrom, the silicon lattice constant
of the paper's Methods section reused as a length scale):

* H(R_e): complex normal CN(0,1) * s_H * exp(-|R|/L), made Hermitian in the
  lattice sense, H(R) <- (H(R) + H(-R)^dagger)/2, plus an on-site offset
  -delta on the lower half of the bands and +delta on the upper half.
* Force constants (mass-weighted, eV / (Angstrom^2 amu)), real: a Gram form
  D(R) = sum_R' B(R')^T B(R' + R) with B(R) real normal * exp(-|R|/L) on a
  half-radius set, translations projected out of sum_R B(R) so that the
  acoustic sum rule holds exactly, then scaled by c_D.
* g(R_e, R_p) in eV/Angstrom, layout [R_e][R_p][3*natom][final][initial]:
  CN(0,1) * s_g * exp(-(|R_e|+|R_p|)/L) on the support R_p - R_e in the
  phonon set, then g_ij(R_e,R_p) <- (g_ij(R_e,R_p) + conj(g_ji(-R_e,R_p-R_e)))/2,
  which is the Wannier-space form of the hermiticity of the perturbing
  potential (dV_q^dagger = dV_{-q}).

Draw order from numpy's PCG64 ``default_rng(seed)``: H (real part, then
imaginary part), B, g (real, then imaginary).
"""
import json
import itertools
import os

import numpy as np

LATTICE_A = 5.40  # Angstrom
MASS_CYCLE = (28.0855, 12.011, 69.723, 74.9216, 14.007)  # amu
_HERE = os.path.dirname(os.path.abspath(__file__))
_CONFIGS_JSON = os.path.join(_HERE, "configs.json")


def _sort_vectors(vs):
    vs = sorted(set(tuple(int(x) for x in v) for v in vs),
                key=lambda v: (v[0] ** 2 + v[1] ** 2 + v[2] ** 2, v))
    return np.array(vs, dtype=np.int32).reshape(-1, 3)


def rset_cube(lo, hi):
    """All integer vectors with every component in [lo, hi]."""
    return _sort_vectors(itertools.product(range(lo, hi + 1), repeat=3))


def rset_sphere(r2):
    """All integer vectors with |R|^2 <= r2 (lattice units)."""
    m = int(np.ceil(np.sqrt(r2))) + 1
    return _sort_vectors(v for v in itertools.product(range(-m, m + 1), repeat=3)
                         if v[0] ** 2 + v[1] ** 2 + v[2] ** 2 <= r2)


def _rset(spec):
    kind = spec[0]
    if kind == "cube":
        return rset_cube(spec[1], spec[2])
    if kind == "sphere":
        return rset_sphere(spec[1])
    raise ValueError(spec)


def _index_map(rs):
    return {tuple(int(x) for x in v): i for i, v in enumerate(rs)}


def _cnormal(rng, shape):
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def make_material(nb, na, seed, rset_e, rset_b, L, s_H, delta, c_D, s_g=1.0,
                  masses=None, lattice_a=LATTICE_A, dtype_g=np.complex128, with_g=True):
    """Assemble one synthetic material; returns a dict of numpy arrays.

    ``rset_e`` is used for both R_e and R_p; ``rset_b`` is the half-radius
    set that carries the Gram factor B(R).  All sets must be closed under
    R -> -R.
    """
    rs = np.asarray(rset_e, dtype=np.int32)
    rb = np.asarray(rset_b, dtype=np.int32)
    nr = rs.shape[0]
    nbr = 3 * na
    if masses is None:
        masses = np.array([MASS_CYCLE[t % len(MASS_CYCLE)] for t in range(na)])
    masses = np.asarray(masses, dtype=np.float64)
    rmap = _index_map(rs)
    neg = np.array([rmap[tuple(-v)] for v in rs])
    rnorm = np.sqrt((rs.astype(np.float64) ** 2).sum(1))
    rng = np.random.default_rng(seed)

    # --- H(R_e)
    h = _cnormal(rng, (nr, nb, nb)) * np.exp(-rnorm / L)[:, None, None]
    h = 0.5 * (h + np.conj(np.transpose(h[neg], (0, 2, 1))))
    h *= s_H
    i0 = rmap[(0, 0, 0)]
    onsite = np.array([-delta if b < nb // 2 else delta for b in range(nb)])
    h[i0] += np.diag(onsite)

    # --- force constants via the Gram form
    nbB = rb.shape[0]
    bnorm = np.sqrt((rb.astype(np.float64) ** 2).sum(1))
    B = rng.standard_normal((nbB, nbr, nbr)) * np.exp(-bnorm / L)[:, None, None]
    # orthonormal mass-weighted translation vectors t_alpha[(tau,beta)]
    T = np.zeros((nbr, 3))
    for tau in range(na):
        for a in range(3):
            T[3 * tau + a, a] = np.sqrt(masses[tau])
    T /= np.sqrt(masses.sum())
    PT = T @ T.T
    Bsum = B.sum(0)
    B = B - (Bsum @ PT)[None] / nbB
    bmap = _index_map(rb)
    d = np.zeros((nr, nbr, nbr))
    for ia, ra in enumerate(rb):
        for ib, rbv in enumerate(rb):
            dr = tuple(int(x) for x in (rbv - ra))  # R = R'' - R'
            if dr not in rmap:
                raise ValueError("Gram support exceeds the phonon R set")
            d[rmap[dr]] += B[ia].T @ B[ib]
    d *= c_D
    del bmap

    lat = lattice_a * np.eye(3)
    if not with_g:  # band and phonon calibration only (g is drawn last)
        return {"nwann": nb, "natom": na, "re": rs.copy(), "rp": rs.copy(), "wre": np.ones(nr),
                "wrp": np.ones(nr), "lat": lat, "mass": masses, "h_r": h, "d_r": d, "g_r": None}

    # --- g(R_e, R_p)
    decay = np.exp(-(rnorm[:, None] + rnorm[None, :]) / L)  # [Re, Rp]
    support = np.zeros((nr, nr), dtype=bool)
    pair_img = np.full((nr, nr, 2), -1, dtype=np.int64)
    for ie, re_ in enumerate(rs):
        for ip, rp_ in enumerate(rs):
            diff = tuple(int(x) for x in (rp_ - re_))
            if diff in rmap:
                support[ie, ip] = True
                pair_img[ie, ip] = (neg[ie], rmap[diff])
    g = _cnormal(rng, (nr, nr, nbr, nb, nb)).astype(np.complex128)
    g *= (s_g * decay * support)[:, :, None, None, None]
    ie_img = pair_img[..., 0]
    ip_img = pair_img[..., 1]
    ie_img = np.where(support, ie_img, 0)
    ip_img = np.where(support, ip_img, 0)
    partner = np.conj(np.swapaxes(g[ie_img, ip_img], -1, -2))
    g = 0.5 * (g + partner * support[:, :, None, None, None])
    g = g.astype(dtype_g, copy=False)

    lat = lattice_a * np.eye(3)
    return {
        "nwann": nb, "natom": na, "re": rs.copy(), "rp": rs.copy(),
        "wre": np.ones(nr), "wrp": np.ones(nr), "lat": lat, "mass": masses,
        "h_r": h, "d_r": d, "g_r": g,
    }


# --------------------------------------------------------------------------
# Named workloads.  Static definitions live here; calibrated scales come from
# configs.json (band-gap offset delta, Hamiltonian scale s_H where bisected,
# force-constant scale c_D and the chemical potential mu).

_STATIC = {
    # 4 Wannier bands, 2 atoms, R sets {-1,0,1}^3, 8^3 meshes, all k kept.
    "plain8": dict(seed=1, nb=4, na=2, rset=("cube", -1, 1), rset_b=("cube", 0, 1),
                   L=2.0, s_H=0.25, mesh=8, window=float("inf"), sigma=0.010,
                   T=300.0, mu_rule="midgap+0.1"),
    # 8 bands, 2 atoms, |R|^2 <= 13 (203 vectors), 48^3 meshes, ~3% of k kept.
    "mixed48": dict(seed=2, nb=8, na=2, rset=("sphere", 13), rset_b=("sphere", 3.25),
                    L=3.0, mesh=48, window=0.4, sigma=0.010, T=300.0,
                    mu_rule="cbm-0.1", kept_target=0.03),
    # 16 bands, 5 atoms, |R|^2 <= 20 (389 vectors), 100^3 meshes, ~1% kept.
    "large100": dict(seed=5, nb=16, na=5, rset=("sphere", 20), rset_b=("sphere", 5),
                     L=3.0, mesh=100, window=0.4, sigma=0.010, T=300.0,
                     mu_rule="cbm-0.1", kept_target=0.01),
    # tiny materials for tests: brute force is affordable on these
    "tiny3": dict(seed=11, nb=2, na=1, rset=("cube", -1, 1), rset_b=("cube", 0, 1),
                  L=2.0, s_H=0.25, mesh=3, window=float("inf"), sigma=0.010,
                  T=300.0, mu_rule="midgap+0.1"),
    "tiny4": dict(seed=12, nb=3, na=2, rset=("cube", -1, 1), rset_b=("cube", 0, 1),
                  L=2.0, s_H=0.25, mesh=4, window=float("inf"), sigma=0.020,
                  T=300.0, mu_rule="midgap+0.1"),
    # a metal (mu at the median band energy, no gap offset): the coupled
    # iteration converges quickly here, and it is small enough for a dense solve
    "metal6": dict(seed=21, nb=2, na=2, rset=("cube", -1, 1), rset_b=("cube", 0, 1),
                   L=2.0, s_H=0.05, delta_fixed=0.0, mesh=6, window=float("inf"),
                   sigma=0.030, T=300.0, mu_rule="median"),
}


def _batched_static():
    """32 materials for the batched workload; sizes drawn from seed 3000."""
    rng = np.random.default_rng(3000)
    out = {}
    for j in range(32):
        nb = int(rng.integers(4, 17))
        na = int(rng.integers(2, 5))
        mesh = int(rng.integers(24, 41))
        kept = float(rng.uniform(0.01, 0.10))
        out["batch%02d" % j] = dict(seed=300 + j, nb=nb, na=na, rset=("sphere", 13),
                                    rset_b=("sphere", 3.25), L=3.0, mesh=mesh,
                                    window=0.4, sigma=0.010, T=300.0,
                                    mu_rule="cbm-0.1", kept_target=kept)
    return out


_STATIC.update(_batched_static())


def config_names():
    return list(_STATIC)


def _load_calibration():
    if not os.path.exists(_CONFIGS_JSON):
        return {}
    with open(_CONFIGS_JSON) as fh:
        return json.load(fh)


def config(name, calibrated=True):
    """Static definition merged with the stored calibration of ``name``."""
    if name not in _STATIC:
        raise KeyError(name)
    cfg = dict(_STATIC[name])
    cfg["name"] = name
    if calibrated:
        cal = _load_calibration().get(name)
        if cal is None:
            raise KeyError("config %r has no calibration in %s" % (name, _CONFIGS_JSON))
        cfg.update(cal)
    return cfg


def material_for(cfg, **overrides):
    """Build the material that ``cfg`` (from :func:`config`) describes."""
    c = dict(cfg)
    c.update(overrides)
    return make_material(nb=c["nb"], na=c["na"], seed=c["seed"], rset_e=_rset(c["rset"]),
                         rset_b=_rset(c["rset_b"]), L=c["L"], s_H=c["s_H"],
                         delta=c["delta"], c_D=c["c_D"], with_g=c.get("with_g", True))


def polar_params(na, seed, z0=2.0, eps0=8.0, lat=None):
    """Seeded Born effective charges Z*[na][3][3] (random anisotropic parts,
    sum over atoms zero: charge neutrality) and a symmetric positive definite
    high-frequency dielectric tensor near eps0 (a polar material's inputs);
    with lat [3][3] (rows a_i, Angstrom) also Cartesian atom positions
    [na][3] at seeded fractional coordinates."""
    rng = np.random.default_rng(seed)
    if lat is not None:
        frac = rng.uniform(0.0, 1.0, (na, 3))
        frac[0] = 0.0
        tau = frac @ np.asarray(lat, dtype=np.float64)
    Z = np.zeros((na, 3, 3))
    for t in range(na):
        Z[t] = (z0 if t % 2 == 0 else -z0) * np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    Z -= Z.mean(axis=0, keepdims=True)
    A = 0.5 * rng.standard_normal((3, 3))
    eps = eps0 * np.eye(3) + 0.5 * (A + A.T)
    if lat is not None:
        return Z, eps, tau
    return Z, eps


def ifc3_params(na, seed, cells=None, scale=2.0, L=1.0, sweeps=200):
    """Seeded third-order force constants Psi (eV/Angstrom^3) on the cell
    triples {0, Rj, Rk} whose pairwise differences lie in ``cells`` (default
    the cube {-1, 0, 1}^3).

    Returns (rj [n][3] int32, rk [n][3] int32, psi [n][na][na][na][3][3][3]):
    entry e holds Psi(0 ti a, rj_e tj b, rk_e tk c) for the atom triple
    (ti, tj, tk) and Cartesian triple (a, b, c).  The tensor is made
    symmetric under every permutation of its three legs (with the triple
    recentred on the first leg's cell) and obeys the acoustic sum rule
    sum_{Rk, tk} Psi = 0, by alternating the two orthogonal projections from
    a seeded normal draw damped as exp(-(|Rj| + |Rk| + |Rj - Rk|) / L)."""
    cells = rset_cube(-1, 1) if cells is None else np.asarray(cells, dtype=np.int32)
    cset = {tuple(int(x) for x in v) for v in cells}
    keys = [(a, b) for a in sorted(cset) for b in sorted(cset)
            if tuple(bb - aa for aa, bb in zip(a, b)) in cset]
    idx = {k: i for i, k in enumerate(keys)}
    rng = np.random.default_rng(seed)
    n = len(keys)
    rj = np.array([k[0] for k in keys], dtype=np.int32)
    rk = np.array([k[1] for k in keys], dtype=np.int32)
    damp = np.exp(-(np.linalg.norm(rj, axis=1) + np.linalg.norm(rk, axis=1)
                    + np.linalg.norm(rk - rj, axis=1)) / L)
    psi = rng.standard_normal((n, na, na, na, 3, 3, 3)) * (scale * damp)[:, None, None, None, None, None, None]

    # the six leg orders: entry (Rj, Rk) viewed from leg p[0]; cells of the legs
    # are (0, Rj, Rk), recentred on the new first leg
    perms = list(itertools.permutations(range(3)))
    maps = []
    for p in perms:
        tgt = np.empty(n, dtype=np.int64)
        for e, (a, b) in enumerate(keys):
            c = ((0, 0, 0), a, b)
            o = c[p[0]]
            na_ = tuple(x - y for x, y in zip(c[p[1]], o))
            nb_ = tuple(x - y for x, y in zip(c[p[2]], o))
            tgt[e] = idx[(na_, nb_)]
        axes = (0,) + tuple(1 + q for q in p) + tuple(4 + q for q in p)
        maps.append((tgt, axes))
    # groups of entries sharing (Rj) for the sum rule over (Rk, tk)
    rj_groups = {}
    for e, (a, b) in enumerate(keys):
        rj_groups.setdefault(a, []).append(e)
    rj_groups = [np.array(v) for v in rj_groups.values()]

    def symmetrise(x):
        out = np.zeros_like(x)
        for tgt, axes in maps:
            np.add.at(out, tgt, np.transpose(x, axes))
        return out / len(maps)

    def sum_rule(x):
        y = x.copy()
        for g in rj_groups:
            m = y[g].sum(axis=(0, 3), keepdims=True) / (g.size * na)
            y[g] -= m
        return y

    for _ in range(sweeps):
        psi = symmetrise(sum_rule(psi))
    return rj, rk, psi
