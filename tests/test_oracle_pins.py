"""Pins of the CPU oracle to facts other than itself.

Each test fixes a part of the oracle against mathematics the paper's method
must obey: exact inverse transforms on a coarse mesh, closed-form band and
phonon models, finite differences, a quadrature of the delta function,
identities of the Fermi/Bose factors, analytic eigenvectors, detailed
balance between absorption and emission, closed-form rates of a flat-band /
Einstein-phonon model, brute force on tiny meshes and a dense direct solve of
the coupled BTEs.
"""
import numpy as np
import pytest

import ko_cases
import oracle
import synth
from synth import materials as sm


# ---------------------------------------------------------------------------
# helpers: hand-built materials

def _material(nb, na, re, rp, h_r, d_r, g_r, masses, a=5.4):
    re = np.asarray(re, dtype=np.int32).reshape(-1, 3)
    rp = np.asarray(rp, dtype=np.int32).reshape(-1, 3)
    return dict(nwann=nb, natom=na, re=re, rp=rp, wre=np.ones(len(re)),
                wrp=np.ones(len(rp)), lat=a * np.eye(3), mass=np.asarray(masses, float),
                h_r=np.asarray(h_r, complex), d_r=np.asarray(d_r, float),
                g_r=np.asarray(g_r, complex))


def _tiny(name):
    cfg = synth.config(name)
    return cfg, synth.material_for(cfg)


# ---------------------------------------------------------------------------
# Eqs. 1, 3, 6: Fourier sums

def test_coarse_mesh_exactness_hamiltonian():
    """R = {-1,0,1}^3 is dual to a 3^3 mesh: H(R) obtained from random Bloch
    matrices on that mesh by an FFT must interpolate back to them exactly."""
    rng = np.random.default_rng(7)
    n, nb = 3, 3
    kf = oracle.mesh_points(n)
    hk = rng.standard_normal((n, n, n, nb, nb)) + 1j * rng.standard_normal((n, n, n, nb, nb))
    hk = hk + np.conj(np.swapaxes(hk, -1, -2))
    # H(R) = (1/N) sum_k exp(-2 pi i k.R) H(k): numpy's forward FFT, divided by N
    hR_grid = np.fft.fftn(hk, axes=(0, 1, 2)) / n ** 3
    rs = sm.rset_cube(-1, 1)
    h_r = np.stack([hR_grid[tuple(np.mod(r, n))] for r in rs])
    mat = _material(nb, 1, rs, rs, h_r, np.zeros((27, 3, 3)), np.zeros((27, 27, 3, nb, nb)), [1.0])
    got = oracle.bloch_hamiltonian(mat, kf)
    assert np.abs(got - hk.reshape(-1, nb, nb)).max() < 1e-13


def test_coarse_mesh_exactness_dynamical_matrix():
    rng = np.random.default_rng(8)
    n, nbr = 3, 6
    # real force constants with D(-R) = D(R)^T give Hermitian D(q)
    rs = sm.rset_cube(-1, 1)
    idx = {tuple(r): i for i, r in enumerate(rs)}
    d = rng.standard_normal((27, nbr, nbr))
    d = 0.5 * (d + np.transpose(d[[idx[tuple(-r)] for r in rs]], (0, 2, 1)))
    mat = _material(1, 2, rs, rs, np.zeros((27, 1, 1)), d, np.zeros((27, 27, nbr, 1, 1)), [1.0, 2.0])
    dq = oracle.dynamical_matrix(mat, oracle.mesh_points(n))
    # back to real space with numpy's inverse FFT and compare
    grid = dq.reshape(n, n, n, nbr, nbr)
    back = np.fft.fftn(grid, axes=(0, 1, 2)) / n ** 3
    for r in rs:
        assert np.abs(back[tuple(np.mod(r, n))] - d[idx[tuple(r)]]).max() < 1e-13
    assert np.abs(dq - np.conj(np.swapaxes(dq, -1, -2))).max() < 1e-13


def test_coarse_mesh_exactness_vertex():
    """g(Re, Rp) from random g(k, q) on a 3^3 x 3^3 grid by a 6-d FFT must
    interpolate back to g(k, q) exactly (both the brute double sum and the
    factorised sum)."""
    rng = np.random.default_rng(9)
    n, nb, nbr = 3, 2, 3
    shape = (n, n, n, n, n, n, nbr, nb, nb)
    gkq = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    gR = np.fft.fftn(gkq, axes=tuple(range(6))) / n ** 6
    rs = sm.rset_cube(-1, 1)
    g_r = np.empty((27, 27, nbr, nb, nb), complex)
    for ie, re_ in enumerate(rs):
        for ip, rp_ in enumerate(rs):
            g_r[ie, ip] = gR[tuple(np.mod(re_, n)) + tuple(np.mod(rp_, n))]
    mat = _material(nb, 1, rs, rs, np.zeros((27, nb, nb)), np.zeros((27, 3, 3)), g_r, [1.0])
    kf = oracle.mesh_points(n)
    for a in (0, 5, 13, 26):
        ka = tuple(np.rint(kf[a] * n).astype(int))
        qs = kf
        fac = oracle.g_wannier_factorised(mat, kf[a], qs)
        want = gkq[ka].reshape(n ** 3, nbr, nb, nb)
        assert np.abs(fac - want).max() < 1e-12
        for b in (0, 7, 20):
            br = oracle.g_wannier_brute(mat, kf[a], kf[b])
            assert np.abs(br - want[b]).max() < 1e-12


@pytest.mark.parametrize("name", ["tiny3", "tiny4"])
def test_brute_equals_factorised_rates(name):
    """Transition probabilities from the literal double sum equal the
    factorised sum on tiny meshes."""
    cfg, mat = _tiny(name)
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    rows = np.arange(0, prob.nstates, max(1, prob.nstates // 5))
    xb = prob.transition_probs(300.0, rows, brute=True)
    xf = prob.transition_probs(300.0, rows, brute=False)
    for a, b in zip(xb, xf):
        assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()


# ---------------------------------------------------------------------------
# eigensolves and velocities (Eqs. 1-2, 3, 5)

def test_cosine_band_and_velocity():
    """One band with nearest-neighbour hopping t: eps = e0 + 2t sum cos(2 pi k_i),
    v_i = -(2 t a / hbar) sin(2 pi k_i)."""
    e0, t, a = 0.3, -0.7, 5.4
    rs = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    h = np.array([e0, t, t, t, t, t, t], complex).reshape(-1, 1, 1)
    mat = _material(1, 1, rs, rs[:1], h, np.zeros((1, 3, 3)), np.zeros((7, 1, 3, 1, 1)), [1.0], a)
    rng = np.random.default_rng(1)
    k = rng.random((50, 3))
    eps, U = oracle.electron_bands(mat, k)
    want = e0 + 2 * t * np.cos(2 * np.pi * k).sum(1)
    assert np.abs(eps[:, 0] - want).max() < 1e-13
    v = oracle.electron_velocities(mat, k, eps, U)
    vw = -(2 * t * a / oracle.HBAR_EVS) * np.sin(2 * np.pi * k) * oracle.ANG_M
    assert np.abs(v[:, 0, :] - vw).max() < 1e-10 * np.abs(vw).max()


def test_scalar_springs_phonons():
    """D(0) = 6K/M, D(+-e_i) = -K/M (times I3): (hw)^2 = C (4K/M) sum sin^2(pi q_i),
    triply degenerate; v = a C K sin(2 pi q)/(M hw) /hbar."""
    K, M, a = 2.5, 28.0855, 5.4
    rs = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    d = np.stack([6 * K / M * np.eye(3)] + [-K / M * np.eye(3)] * 6)
    mat = _material(1, 1, rs[:1], rs, np.zeros((1, 1, 1)), d, np.zeros((1, 7, 3, 1, 1)), [M], a)
    rng = np.random.default_rng(2)
    q = rng.random((40, 3))
    hw, u = oracle.phonon_modes(mat, q)
    want = np.sqrt(oracle.C_PHONON * 4 * K / M * (np.sin(np.pi * q) ** 2).sum(1))
    assert np.abs(hw - want[:, None]).max() < 1e-13
    v = oracle.phonon_velocities(mat, q, hw, u)
    vw = a * oracle.C_PHONON * K * np.sin(2 * np.pi * q) / (M * want[:, None]) \
        * oracle.ANG_M / oracle.HBAR_EVS
    for s in range(3):
        assert np.abs(v[:, s, :] - vw).max() < 1e-9 * np.abs(vw).max()
    # acoustic sum rule: zero modes at Gamma
    hw0, _ = oracle.phonon_modes(mat, np.zeros((1, 3)))
    assert hw0.max() < 1e-6


@pytest.mark.parametrize("name", ["plain8", "tiny4"])
def test_eigensolves_hermitian_residuals(name):
    cfg, mat = _tiny(name)
    k = np.random.default_rng(3).random((30, 3))
    H = oracle.bloch_hamiltonian(mat, k)
    assert np.abs(H - np.conj(np.swapaxes(H, -1, -2))).max() < 1e-13
    eps, U = oracle.electron_bands(mat, k)
    nrm = np.abs(H).max()
    assert np.abs(H @ U - U * eps[:, None, :]).max() < 1e-12 * nrm
    assert np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - np.eye(U.shape[-1])).max() < 1e-13
    D = oracle.dynamical_matrix(mat, k)
    lam, u = np.linalg.eigh(D)
    assert np.abs(D @ u - u * lam[:, None, :]).max() < 1e-12 * np.abs(D).max()
    assert lam.min() > -1e-12 * np.abs(D).max()          # Gram form: PSD
    hw0, _ = oracle.phonon_modes(mat, np.zeros((1, 3)))
    assert np.sort(hw0[0])[:3].max() < 1e-6               # ASR: 3 zero modes at Gamma


@pytest.mark.parametrize("name", ["plain8", "tiny4"])
def test_velocities_match_finite_differences(name):
    """Eq. 2 and Eq. 5 against central differences of the eigenvalues."""
    cfg, mat = _tiny(name)
    rng = np.random.default_rng(4)
    k = rng.random((6, 3))
    a = mat["lat"][0, 0]
    h = 1e-5
    eps, U = oracle.electron_bands(mat, k)
    v = oracle.electron_velocities(mat, k, eps, U)
    hw, u = oracle.phonon_modes(mat, k)
    vp = oracle.phonon_velocities(mat, k, hw, u)
    for c in range(3):
        dk = np.zeros(3)
        dk[c] = h
        ep, _ = oracle.electron_bands(mat, k + dk)
        em, _ = oracle.electron_bands(mat, k - dk)
        # d eps / d k_cart = (a / 2 pi) d eps / d k_frac
        fd = (ep - em) / (2 * h) * a / (2 * np.pi) * oracle.ANG_M / oracle.HBAR_EVS
        assert np.abs(fd - v[..., c]).max() < 1e-6 * np.abs(v).max()
        hp, _ = oracle.phonon_modes(mat, k + dk)
        hm, _ = oracle.phonon_modes(mat, k - dk)
        fdp = (hp - hm) / (2 * h) * a / (2 * np.pi) * oracle.ANG_M / oracle.HBAR_EVS
        assert np.abs(fdp - vp[..., c]).max() < 1e-5 * np.abs(vp).max()


# ---------------------------------------------------------------------------
# delta and thermal factors (Eq. 8)

def test_gaussian_delta_normalised_and_symmetric():
    s = 0.01
    x = np.linspace(-12 * s, 12 * s, 200001)
    d = oracle.gaussian_delta(x, s)
    integral = np.trapezoid(d, x)
    assert abs(integral - 1.0) < 1e-12
    assert np.abs(d - oracle.gaussian_delta(-x, s)).max() == 0.0


def test_thermal_identities():
    x = np.linspace(-3, 3, 101)
    T = 250.0
    f, omf = oracle.fermi_pair(x, 0.0, T)
    f2, omf2 = oracle.fermi_pair(-x, 0.0, T)
    assert np.abs(f + f2 - 1).max() < 1e-15
    assert np.abs(omf - f2).max() < 1e-15
    y = np.linspace(1e-3, 0.2, 50)
    n, onp = oracle.bose_pair(y, T)
    nm, _ = oracle.bose_pair(-y, T)
    assert np.abs(onp + nm).max() < 1e-12 * np.abs(nm).max()
    # at exact energy conservation eps_n = eps_m + hw:
    # (1 - f_n) n / (1 - f_m) = n + f_n
    em = np.linspace(-0.2, 0.2, 21)
    for hw in (0.005, 0.03, 0.06):
        _, omf_m = oracle.fermi_pair(em, 0.0, T)
        f_n, omf_n = oracle.fermi_pair(em + hw, 0.0, T)
        nn, _ = oracle.bose_pair(hw, T)
        lhs = omf_n * nn / omf_m
        assert np.abs(lhs - (nn + f_n)).max() < 1e-13 * lhs.max()


# ---------------------------------------------------------------------------
# Eq. 6: Bloch rotation

def test_gauge_invariance_of_g2():
    cfg, mat = _tiny("tiny4")
    rng = np.random.default_rng(5)
    k, q = rng.random(3), rng.random(3)
    gW = oracle.g_wannier_factorised(mat, k, q[None])[0]
    _, Uk = oracle.electron_bands(mat, k[None])
    _, Ukq = oracle.electron_bands(mat, (k + q)[None])
    hw, u = oracle.phonon_modes(mat, q[None])
    g1 = oracle.g_bloch(mat, gW, Uk[0], Ukq[0], u[0], hw[0])
    ph = lambda n: np.exp(2j * np.pi * rng.random(n))  # noqa: E731
    g2 = oracle.g_bloch(mat, gW, Uk[0] * ph(mat["nwann"]), Ukq[0] * ph(mat["nwann"]),
                        u[0] * ph(3 * mat["natom"]), hw[0])
    assert np.abs(np.abs(g1) ** 2 - np.abs(g2) ** 2).max() < 1e-13 * (np.abs(g1) ** 2).max()


def test_rotation_index_order_analytic_eigenvectors():
    """Two bands, H(k) = [[D, t(k)], [t(k)*, -D]] with t(k) = t0 exp(2 pi i k_x),
    one atom with an Einstein spring, g^W = c_x * identity.  Summed over the
    degenerate branches, |g^{nm}|^2 = l^2 |c|^2 |<n,k+q|m,k>|^2 with the
    closed-form eigenvectors; the final band n sits at k+q."""
    Dl, t0, K, M = 0.4, 0.3 + 0.2j, 1.7, 12.011
    rs_e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0]])
    h = np.zeros((3, 2, 2), complex)
    h[0] = np.diag([Dl, -Dl])
    h[1, 0, 1] = t0
    h[2, 1, 0] = np.conj(t0)
    d = (K / M * np.eye(3))[None]
    c = np.array([0.7 - 0.1j, -0.2 + 0.5j, 0.3j])
    g = np.zeros((3, 1, 3, 2, 2), complex)
    for x in range(3):
        g[0, 0, x] = c[x] * np.eye(2)
    mat = _material(2, 1, rs_e, [[0, 0, 0]], h, d, g, [M])
    hw0 = np.sqrt(oracle.C_PHONON * K / M)
    l2 = oracle.C_PHONON / (2 * M * hw0)

    def vecs(k):
        tk = t0 * np.exp(2j * np.pi * k[0])
        E = np.sqrt(Dl ** 2 + abs(tk) ** 2)
        lo = np.array([-tk, Dl + E])
        hi = np.array([Dl + E, np.conj(tk)])
        return np.stack([lo / np.linalg.norm(lo), hi / np.linalg.norm(hi)], 1)

    rng = np.random.default_rng(6)
    for _ in range(5):
        k, q = rng.random(3), rng.random(3)
        Vk, Vkq = vecs(k), vecs(k + q)
        gW = oracle.g_wannier_factorised(mat, k, q[None])[0]
        _, Uk = oracle.electron_bands(mat, k[None])
        _, Ukq = oracle.electron_bands(mat, (k + q)[None])
        hw, u = oracle.phonon_modes(mat, q[None])
        gb = oracle.g_bloch(mat, gW, Uk[0], Ukq[0], u[0], hw[0])
        got = (np.abs(gb) ** 2).sum(0)                       # [n, m]
        ov = np.abs(np.conj(Vkq).T @ Vk) ** 2                 # [n, m] = |<n,k+q|m,k>|^2
        want = l2 * np.vdot(c, c).real * ov
        assert np.abs(got - want).max() < 1e-12 * want.max()


def test_hermitian_pair_identity():
    """|g^s_{nm}(k,q)|^2 = |g^s_{mn}(k+q,-q)|^2 for the generated materials."""
    cfg, mat = _tiny("plain8")
    rng = np.random.default_rng(10)
    for _ in range(4):
        k, q = rng.random(3), rng.random(3)
        gW = oracle.g_wannier_factorised(mat, k, q[None])[0]
        gR = oracle.g_wannier_factorised(mat, k + q, -q[None])[0]
        _, Uk = oracle.electron_bands(mat, k[None])
        _, Ukq = oracle.electron_bands(mat, (k + q)[None])
        hw, u = oracle.phonon_modes(mat, q[None])
        hwm, um = oracle.phonon_modes(mat, -q[None])
        a = np.abs(oracle.g_bloch(mat, gW, Uk[0], Ukq[0], u[0], hw[0])) ** 2
        b = np.abs(oracle.g_bloch(mat, gR, Ukq[0], Uk[0], um[0], hwm[0])) ** 2
        assert np.abs(a - np.swapaxes(b, -1, -2)).max() < 1e-12 * a.max()


# ---------------------------------------------------------------------------
# Eq. 8: transition probabilities

@pytest.fixture(scope="module")
def plain8():
    cfg, mat = _tiny("plain8")
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    rows = np.arange(0, prob.nstates, 37)
    Xp, Xm = prob.transition_probs(cfg["T"], rows)
    return cfg, prob, rows, Xp, Xm


def test_detailed_balance_per_term(plain8):
    """X^+_{i->j|s,q} exp(-beta(eps_j - eps_i - hw)) = X^-_{j->i|s,-q}."""
    cfg, prob, rows, Xp, Xm = plain8
    T = cfg["T"]
    cols = np.arange(0, prob.nstates, 53)
    _, XmT = prob.transition_probs(T, cols)
    beta = 1.0 / (oracle.KB_EVK * T)
    worst = 0.0
    for r, i in enumerate(rows):
        for c, j in enumerate(cols):
            q = prob.q_index(prob.state_k[i], prob.state_k[j])
            hw = prob.hw[q]
            lhs = Xp[r, j] * np.exp(-beta * (prob.eps[j] - prob.eps[i] - hw))
            rhs = XmT[c, i]
            scale = max(lhs.max(), rhs.max(), 1e-300)
            worst = max(worst, np.abs(lhs - rhs).max() / scale)
    assert worst < 1e-10


def _flat_einstein(nk_mesh, eps0, K, M, g0, sigma):
    rs = np.array([[0, 0, 0]])
    g = np.zeros((1, 1, 3, 1, 1), complex)
    g[0, 0, :, 0, 0] = g0
    mat = _material(1, 1, rs, rs, np.full((1, 1, 1), eps0), (K / M * np.eye(3))[None], g, [M])
    return mat


def test_flat_band_einstein_closed_forms():
    """Flat band, Einstein phonon, local vertex g0: W_e = (2pi/hbar) l^2 |g0|^2
    (2n+1) delta(hw0) and sum_s W_ph = d_s (2pi/hbar)(N_k/N_q) l^2 |g0|^2
    f(1-f) delta(hw0) / (1+n)."""
    eps0, K, M, sigma, T, mu = 0.05, 0.9, 28.0855, 0.02, 300.0, 0.0
    g0 = np.array([0.4 + 0.1j, -0.3j, 0.25])
    mat = _flat_einstein(3, eps0, K, M, g0, sigma)
    prob = oracle.Problem(mat, 3, mu, np.inf, sigma)
    Xp, Xm = prob.transition_probs(T)
    W = prob.rates_e(T, Xp, Xm)
    hw0 = np.sqrt(oracle.C_PHONON * K / M)
    l2 = oracle.C_PHONON / (2 * M * hw0)
    n, onp = oracle.bose_pair(hw0, T)
    d = oracle.gaussian_delta(hw0, sigma)
    g2 = np.vdot(g0, g0).real
    want = 2 * np.pi / oracle.HBAR_EVS * l2 * g2 * (2 * n + 1) * d
    assert np.abs(W - want).max() < 1e-12 * want
    Wph = prob.rates_ph(T, Xp)
    f, omf = oracle.fermi_pair(eps0, mu, T)
    want_ph = oracle.SPIN_DEG * 2 * np.pi / oracle.HBAR_EVS * l2 * g2 * f * omf * d / onp
    assert np.abs(Wph.sum(1) - want_ph).max() < 1e-12 * want_ph


def test_e_side_equals_ph_side(plain8):
    """sum of all X^+ (electron side) = (N_q/N_k) sum of all Y (phonon side)."""
    cfg, prob, rows, Xp, Xm = plain8
    T = cfg["T"]
    Xp_all, _ = prob.transition_probs(T)
    Wph = prob.rates_ph(T, Xp_all)
    n, onp = oracle.bose_pair(prob.hw, T)
    ysum = np.where(prob.mode_on, Wph * n * onp, 0.0).sum() / oracle.SPIN_DEG
    assert abs(ysum * prob.nq / prob.nk - Xp_all.sum()) < 1e-12 * Xp_all.sum()


# ---------------------------------------------------------------------------
# Eqs. 19-31: the coupled BTEs

def _bordered_solve(prob, T, Xp, Xm, w_ext):
    """Dense direct solve of the coupled linear system with the carrier-number
    constraint: (1 - Aee - Aep Ape) I + alpha 1 = I0 + Aep F0, w.I = 0."""
    M, nbr, nq = prob.nstates, prob.nbr, prob.nq
    f, omf = oracle.fermi_pair(prob.eps, prob.mu, T)
    ff = f * omf
    We = (Xp + Xm).sum((1, 2)) / ff
    Wphe = prob.rates_ph(T, Xp)
    Wp = Wphe + w_ext
    n, onp = oracle.bose_pair(prob.hw, T)
    on = prob.mode_on
    qij = prob.q_index(prob.state_k[:, None], prob.state_k[None, :])
    nqij = prob.neg_q(qij)
    row = 1.0 / (ff * We)
    Aee = (Xp + Xm).sum(2) * row[:, None]
    P = nq * nbr
    Aep = np.zeros((M, P))
    for i in range(M):
        for j in range(M):
            for s in range(nbr):
                Aep[i, qij[i, j] * nbr + s] -= Xp[i, j, s] * row[i]
                Aep[i, nqij[i, j] * nbr + s] += Xm[i, j, s] * row[i]
    Ape = np.zeros((P, M))
    pn = np.where(on, oracle.SPIN_DEG * (prob.nk / prob.nq) / (Wp * n * onp), 0.0).reshape(-1)
    for i in range(M):
        for j in range(M):
            for s in range(nbr):
                p = qij[i, j] * nbr + s
                Ape[p, j] += pn[p] * Xp[i, j, s]
                Ape[p, i] -= pn[p] * Xp[i, j, s]
    v = prob.v_state
    I0 = ((prob.eps - prob.mu) / T / We)[:, None] * v
    J0 = (1.0 / We)[:, None] * v
    inv_wp = np.where(on, 1.0 / Wp, 0.0)
    F0 = ((prob.hw / T * inv_wp)[..., None] * prob.v_ph).reshape(P, 3)
    grp = oracle.energy_groups(prob.eps, prob.hw.max(), prob.sigma)
    C = grp.max() + 1
    A = np.zeros((M + C, M + C))
    A[:M, :M] = np.eye(M) - Aee - Aep @ Ape
    for c in range(C):
        A[:M, M + c] = (grp == c)
        A[M + c, :M] = ff * (grp == c)
    rhsI = np.zeros((M + C, 3))
    rhsI[:M] = I0 + Aep @ F0
    rhsJ = np.zeros((M + C, 3))
    rhsJ[:M] = J0
    I = np.linalg.solve(A, rhsI)[:M]
    J = np.linalg.solve(A, rhsJ)[:M]
    F = F0 + Ape @ I
    G = Ape @ J
    return I, J, F.reshape(nq, nbr, 3), G.reshape(nq, nbr, 3)


def test_iteration_matches_dense_direct_solve():
    cfg = synth.config("metal6")
    mat = synth.material_for(cfg)
    T = 300.0
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    Xp, Xm = prob.transition_probs(T)
    w_ext = oracle.default_w_ext(prob, T, gamma0=1e13)
    res = oracle.iterate(prob, T, Xp, Xm, oracle.LEVEL_COUPLED, tol=1e-12, maxit=500, w_ext=w_ext)
    assert res["converged"]
    I, J, F, G = _bordered_solve(prob, T, Xp, Xm, w_ext)
    for got, want in ((res["I"], I), (res["J"], J), (res["F"], F), (res["G"], G)):
        assert np.abs(got - want).max() < 1e-8 * np.abs(want).max()
    # drag actually couples the systems here
    assert np.abs(res["G"]).max() > 1e-6 * np.abs(res["F"]).max()


def test_rta_level_reproduces_eqs_20_24_and_kelvin_onsager():
    cfg = synth.config("metal6")
    mat = synth.material_for(cfg)
    T = 300.0
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    Xp, Xm = prob.transition_probs(T)
    res = oracle.iterate(prob, T, Xp, Xm, oracle.LEVEL_RTA)
    f, omf = oracle.fermi_pair(prob.eps, prob.mu, T)
    We = (Xp + Xm).sum((1, 2)) / (f * omf)
    I0 = ((prob.eps - prob.mu) / T / We)[:, None] * prob.v_state
    J0 = (1 / We)[:, None] * prob.v_state
    assert np.abs(res["I"] - I0).max() <= 1e-14 * np.abs(I0).max()
    assert np.abs(res["J"] - J0).max() <= 1e-14 * np.abs(J0).max()
    tens = oracle.transport_tensors(prob, T, res["I"], res["J"], res["F"], res["G"])
    # at RTA the phonon Peltier term vanishes and sigma S = alpha_el / T exactly
    assert oracle.ko_residual(tens, T) < 1e-12
    assert np.all(np.linalg.eigvalsh(0.5 * (tens["sigma"] + tens["sigma"].T)) > 0)


# ---------------------------------------------------------------------------
# Kelvin-Onsager enforcement (Eqs. 32-35)

def _ko_problem():
    cfg = synth.config("metal6")
    mat = synth.material_for(cfg)
    return oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"]), 300.0


def test_ko_diffusion_part_is_alpha_el_over_T():
    # Eq. 34: sigma S of I_diff = (eps - mu)/T J equals alpha_el / T
    prob, T = _ko_problem()
    rng = np.random.default_rng(3)
    J = rng.standard_normal((prob.nstates, 3))
    I_diff = ((prob.eps - prob.mu) / T)[:, None] * J
    zero = np.zeros_like(prob.v_ph)
    t = oracle.transport_tensors(prob, T, I_diff, J, zero, zero)
    assert np.abs(t["sigmaS"] - t["alpha_el"] / T).max() <= 1e-13 * np.abs(t["sigmaS"]).max()


@pytest.mark.parametrize("c", [0.8, 1.0, -0.3])
def test_ko_enforce_recovers_a_planted_lambda(c):
    prob, T = _ko_problem()
    I, J, F, G = ko_cases.planted_ko_case(prob, T, c)
    I_ko, lam, tens = oracle.ko_enforce(prob, T, I, J, F, G)
    assert abs(lam - c) <= 1e-12 * max(1.0, abs(c))
    assert oracle.ko_residual(tens, T) < 1e-12
    I_diff = ((prob.eps - prob.mu) / T)[:, None] * J
    assert np.abs(I_ko - (I_diff + c * (I - I_diff))).max() <= 1e-12 * np.abs(I).max()
    if c == 1.0:
        assert np.abs(I_ko - I).max() <= 1e-12 * np.abs(I).max()


def test_ko_enforce_minimises_the_mismatch_on_a_coupled_solution():
    # the numerator of Eq. 31 after enforcement is the least-squares minimum
    # over lambda: no other scale of the drag part does better
    prob, T = _ko_problem()
    Xp, Xm = prob.transition_probs(T)
    w_ext = oracle.default_w_ext(prob, T, gamma0=1e13)
    res = oracle.iterate(prob, T, Xp, Xm, oracle.LEVEL_COUPLED, tol=1e-12, maxit=500, w_ext=w_ext)
    assert res["converged"]
    I, J, F, G = res["I"], res["J"], res["F"], res["G"]
    _, lam, tens = oracle.ko_enforce(prob, T, I, J, F, G)

    def mismatch(t):
        return np.linalg.norm(t["sigmaS"] - (t["alpha_el"] + t["alpha_ph"]) / T)

    best = mismatch(tens)
    I_diff = ((prob.eps - prob.mu) / T)[:, None] * J
    for l2 in (lam * 0.9, lam * 1.1, 1.0, 0.0):
        t2 = oracle.transport_tensors(prob, T, I_diff + l2 * (I - I_diff), J, F, G)
        assert best <= mismatch(t2) * (1 + 1e-12)
    assert best <= mismatch(oracle.transport_tensors(prob, T, I, J, F, G))


# ---------------------------------------------------------------------------
# Analytic tetrahedron delta

def _dos_closed_form(e):
    """Density of states at 0 of one tetrahedron of volume 1/6 with linear E
    (the standard piecewise closed forms of the linear tetrahedron method)."""
    e1, e2, e3, e4 = np.sort(e)
    V = 1.0 / 6.0
    if 0 <= e1 or 0 >= e4:
        return 0.0
    if e2 >= 0:
        return V * 3 * e1 ** 2 / ((e2 - e1) * (e3 - e1) * (e4 - e1))
    if e3 <= 0:
        return V * 3 * e4 ** 2 / ((e4 - e1) * (e4 - e2) * (e4 - e3))
    return V / ((e3 - e1) * (e4 - e1)) * (3 * (e2 - e1) - 6 * e2
                                          - 3 * (e3 - e1 + e4 - e2) * e2 ** 2 / ((e3 - e2) * (e4 - e2)))


def test_tetra_weights_sum_to_the_tetrahedron_dos():
    rng = np.random.default_rng(11)
    e = rng.standard_normal((4000, 4))
    w = oracle.tetra_delta_weights(e)
    ref = np.array([_dos_closed_form(x) for x in e])
    assert np.all(w >= 0)
    assert np.abs(w.sum(1) - ref).max() <= 1e-13 * ref.max()
    assert np.count_nonzero(ref) > 2000          # all three cases occur


def test_tetra_corner_weights_against_quadrature():
    # integral of a narrow Gaussian of E times the barycentric coordinate, on a
    # fine midpoint grid of the reference tetrahedron (corners 0, x, y, z)
    n = 240
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    x, y, z = np.meshgrid(c, c, c, indexing="ij")
    inside = x + y + z < 1.0
    x, y, z = x[inside], y[inside], z[inside]
    lam = np.stack([1 - x - y - z, x, y, z])
    for e in ([-0.9, 0.4, 1.1, 2.0], [-1.3, -0.2, 0.7, 1.5], [-2.0, -1.1, -0.4, 0.8]):
        e = np.array(e)
        E = e[0] * lam[0] + e[1] * lam[1] + e[2] * lam[2] + e[3] * lam[3]
        sig = 0.02
        d = np.exp(-0.5 * (E / sig) ** 2) / (np.sqrt(2 * np.pi) * sig)
        quad = (d[None, :] * lam).sum(1) * h ** 3
        w = oracle.tetra_delta_weights(e)
        assert np.abs(w - quad).max() <= 0.01 * w.max(), (e, w, quad)


@pytest.mark.parametrize("axis,sign,t", [(0, 1, 0.0), (0, 1, 0.3), (1, -1, 0.55), (2, 1, 0.8), (2, -1, 0.1)])
def test_tetra_neighbourhood_integrates_the_hat_function(axis, sign, t):
    # for E = sign * x_axis - t (mesh units), the 24 corner weights of the
    # centre add up to the integral of the centre's hat function over the
    # plane E = 0, which is 1 - t for a plane at distance t from the centre
    corners, centre = oracle.tetra_neighbourhood()
    off = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], dtype=float)
    E = sign * off[:, axis] - t
    w = oracle.tetra_delta_weights(E[corners])
    D = w[np.arange(24), centre].sum()
    assert abs(D - (1.0 - t)) <= 1e-13


# ---------------------------------------------------------------------------
# The triangle delta: a triangle of area 1/2 over which E is linear

def _tri_dos_closed_form(e):
    """Length of the level-0 segment over |grad E| for a triangle of area 1/2:
    the piecewise closed form of the linear triangle method (2 A (0 - e1) /
    ((e2 - e1)(e3 - e1)) below the middle corner, 2 A (e3 - 0) / ((e3 - e1)
    (e3 - e2)) above it, A = 1/2)."""
    e1, e2, e3 = np.sort(e)
    if 0 <= e1 or 0 >= e3:
        return 0.0
    if e2 >= 0:
        return -e1 / ((e2 - e1) * (e3 - e1))
    return e3 / ((e3 - e1) * (e3 - e2))


def test_triangle_weights_sum_to_the_triangle_dos():
    rng = np.random.default_rng(12)
    e = rng.standard_normal((4000, 3))
    w = oracle.triangle_delta_weights(e)
    ref = np.array([_tri_dos_closed_form(x) for x in e])
    assert np.all(w >= 0)
    assert np.abs(w.sum(1) - ref).max() <= 1e-13 * ref.max()
    assert np.count_nonzero(ref) > 2000          # both cases occur


def test_triangle_corner_weights_against_quadrature():
    # integral of a narrow Gaussian of E times the barycentric coordinate, on a
    # fine midpoint grid of the reference triangle (corners 0, x, y)
    n = 2000
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    x, y = np.meshgrid(c, c, indexing="ij")
    inside = x + y < 1.0
    x, y = x[inside], y[inside]
    lam = np.stack([1 - x - y, x, y])
    for e in ([-0.9, 0.4, 1.1], [-1.3, -0.2, 0.7], [0.5, -2.0, 0.9]):
        e = np.array(e)
        E = e[0] * lam[0] + e[1] * lam[1] + e[2] * lam[2]
        sig = 0.01
        d = np.exp(-0.5 * (E / sig) ** 2) / (np.sqrt(2 * np.pi) * sig)
        quad = (d[None, :] * lam).sum(1) * h ** 2
        w = oracle.triangle_delta_weights(e)
        assert np.abs(w - quad).max() <= 0.005 * w.max(), (e, w, quad)


def test_triangle_corner_weight_integrates_to_a_third_of_the_area():
    # over every level, the corner weight integrates to the integral of the
    # barycentric coordinate over the triangle: (1/2) / 3
    e = np.array([0.2, 1.0, 1.7])
    lev = np.linspace(-0.5, 2.5, 300001)
    w = oracle.triangle_delta_weights(e[None, :] - lev[:, None])
    integ = w.sum(0) * (lev[1] - lev[0])
    assert np.abs(integ - 1.0 / 6.0).max() <= 1e-5


@pytest.mark.parametrize("axis,sign,t", [(0, 1, 0.0), (0, 1, 0.3), (1, -1, 0.55), (1, 1, 0.8), (0, -1, 0.1)])
def test_triangle_neighbourhood_integrates_the_hat_function(axis, sign, t):
    # for E = sign * x_axis - t (mesh units), the 6 corner weights of the
    # centre add up to the integral of the centre's hat function over the
    # line E = 0, which is 1 - t for a line at distance t from the centre
    corners, centre = oracle.triangle_neighbourhood()
    off = np.array([[a, b] for a in (-1, 0, 1) for b in (-1, 0, 1)], dtype=float)
    E = sign * off[:, axis] - t
    w = oracle.triangle_delta_weights(E[corners])
    D = w[np.arange(6), centre].sum()
    assert abs(D - (1.0 - t)) <= 1e-13


def test_triangle_neighbourhood_is_the_diagonal_split():
    # the 6 triangles around the centre of the split along the main diagonal:
    # the centre's neighbours (+-1, 0), (0, +-1) and (1, 1), (-1, -1), never
    # the anti-diagonal corners
    corners, centre = oracle.triangle_neighbourhood()
    assert corners.shape == (6, 3) and np.all(corners[np.arange(6), centre] == 4)
    used = set(corners.ravel()) - {4}
    assert used == {1, 3, 5, 7, 0, 8}                     # (dx+1)*3 + (dy+1)


# ---------------------------------------------------------------------------
# Non-analytic (dipole-dipole) term of polar materials (Eq. 4)

def _polar_mat(isotropic=False):
    cfg = synth.config("metal6")
    mat = dict(synth.material_for(cfg))
    Z, eps = synth.polar_params(int(mat["natom"]), 7)
    if isotropic:
        Z = np.stack([(2.0 if t % 2 == 0 else -2.0) * np.eye(3) for t in range(int(mat["natom"]))])
        eps = 6.0 * np.eye(3)
    mat["zstar"], mat["eps_inf"] = Z, eps
    return mat


def test_nac_lo_to_splitting_of_a_diatomic_ionic_model():
    # isotropic Z = +-z, eps_inf = e I: the dipole term moves one mode (the
    # longitudinal optical one, displacements +-q_hat / sqrt(m)) by
    # (e^2 / (eps_0 V)) z^2 (1/m1 + 1/m2) / e, whatever the direction of q
    mat = _polar_mat(isotropic=True)
    assert int(mat["natom"]) == 2
    m1, m2 = mat["mass"]
    V = abs(np.linalg.det(np.asarray(mat["lat"])))
    want = oracle.NAC_EV_A / V * 4.0 * (1 / m1 + 1 / m2) / 6.0
    rng = np.random.default_rng(2)
    q = rng.uniform(-0.4, 0.4, (6, 3))
    D, _ = oracle.nac_term(mat, q)
    for k in range(q.shape[0]):
        lam = np.sort(np.linalg.eigvalsh(D[k]))
        assert abs(lam[-1] - want) <= 1e-12 * want
        assert np.abs(lam[:-1]).max() <= 1e-12 * want
    # unchanged by the length of q and by q -> -q; zero at Gamma
    assert np.allclose(oracle.nac_term(mat, 0.5 * q)[0], D, rtol=1e-12, atol=0)
    assert np.allclose(oracle.nac_term(mat, -q)[0], D, rtol=1e-12, atol=0)
    assert not np.any(oracle.nac_term(mat, np.zeros((1, 3)))[0])


def test_nac_gradient_against_finite_differences():
    mat = _polar_mat()
    lat = np.asarray(mat["lat"])
    rng = np.random.default_rng(4)
    q = rng.uniform(-0.3, 0.3, (4, 3))
    _, G = oracle.nac_term(mat, q)
    h = 1e-6
    for c in range(3):
        dq = np.zeros(3)
        dq[c] = h
        # a Cartesian step h is the fractional step h a_c / (2 pi)
        df = dq @ lat.T / (2.0 * np.pi)
        Dp, _ = oracle.nac_term(mat, q + df)
        Dm, _ = oracle.nac_term(mat, q - df)
        fd = (Dp - Dm) / (2 * h)
        assert np.abs(G[:, c] - fd).max() <= 1e-6 * np.abs(G).max()


def test_polar_phonons_keep_time_reversal_and_the_acoustic_sum():
    # D(-q) = D(q)^* still holds with the term; at Gamma it adds nothing, so
    # the three acoustic modes stay at zero
    mat = _polar_mat()
    q = np.array([[0.25, -0.125, 0.375], [0.5, 0.25, -0.125], [0.5, 0.5, 0.375], [0.0, 0.0, 0.0]])
    D = oracle.dynamical_matrix(mat, q)
    Dm = oracle.dynamical_matrix(mat, -q)
    assert np.abs(Dm - np.conj(D)).max() <= 1e-12 * np.abs(D).max()
    hw, _ = oracle.phonon_modes(mat, q[3:])
    assert np.sort(hw[0])[:3].max() < 1e-5


def test_frohlich_factor_small_q_limit_and_periodicity():
    # |q| F_s(q) tends to the G = 0 term i (e^2/eps_0 V) sum_t (q^.Z_t.lu_t,s)/(q^.eps.q^)
    # as q -> 0 along q^ (the other terms stay bounded), and F is periodic
    mat = _polar_mat()
    mat["tau"] = np.array([[0.0, 0.0, 0.0], [1.3, 2.1, 0.7]])
    na = int(mat["natom"])
    rng = np.random.default_rng(6)
    lu = rng.standard_normal((1, 3 * na, 3 * na)) + 1j * rng.standard_normal((1, 3 * na, 3 * na))
    lat = np.asarray(mat["lat"])
    V = abs(np.linalg.det(lat))
    B = 2 * np.pi * np.linalg.inv(lat).T
    d = np.array([0.3, -0.2, 0.5])
    qhat = d @ B / np.linalg.norm(d @ B)
    lim = np.zeros(3 * na, dtype=complex)
    for t in range(na):
        lim += (qhat @ mat["zstar"][t]) @ lu[0, 3 * t:3 * t + 3, :]
    lim = 1j * oracle.NAC_EV_A / V * lim / (qhat @ mat["eps_inf"] @ qhat)
    errs = []
    for h in (1e-3, 1e-4):
        F = oracle.frohlich_factor(mat, h * d[None, :], lu)[0]
        errs.append(np.abs(np.linalg.norm(h * d @ B) * F - lim).max() / np.abs(lim).max())
    assert errs[1] < 1e-3 and errs[1] < 0.2 * errs[0]
    q = np.array([[0.25, -0.125, 0.375]])
    F0 = oracle.frohlich_factor(mat, q, lu)
    F1 = oracle.frohlich_factor(mat, q + np.array([[1.0, -2.0, 0.0]]), lu)
    assert np.abs(F1 - F0).max() <= 1e-12 * np.abs(F0).max()


# ---------------------------------------------------------------------------
# three-phonon processes (Eqs. 13, 14, 26)

def _phph_problem(name="tiny4", seed=5):
    cfg, mat = _tiny(name)
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    return prob, synth.ifc3_params(mat["natom"], seed, scale=0.3)


def _leg_vertex(prob, ifc3, q1, q2, q3):
    """V with legs at the mesh points q1, q2, q3 (first leg in the central cell)."""
    E = oracle.eigendisplacements(prob.mat, prob.u)
    return oracle.phph_vertex(ifc3, prob.kfrac[[q2]], prob.kfrac[[q3]], E[q1], E[[q2]], E[[q3]])[0]


def test_ifc3_generator_is_symmetric_with_sum_rule():
    """The synthetic Psi is symmetric under exchange of its legs (recentred on
    the new first leg's cell) and sums to zero over the third leg's atoms and
    cells."""
    rj, rk, psi = synth.ifc3_params(2, 9)
    key = {(tuple(a), tuple(b)): e for e, (a, b) in enumerate(zip(rj.tolist(), rk.tolist()))}
    for e, (a, b) in enumerate(zip(rj.tolist(), rk.tolist())):
        # swap legs j and k
        f = key[(tuple(b), tuple(a))]
        assert np.allclose(psi[e], psi[f].transpose(0, 2, 1, 3, 5, 4), atol=1e-14)
        # swap legs i and j: cells (0, a, b) -> (a, 0, b) recentred on a
        g = key[(tuple(-x for x in a), tuple(y - x for x, y in zip(a, b)))]
        assert np.allclose(psi[e], psi[g].transpose(1, 0, 2, 4, 3, 5), atol=1e-14)
    for a in set(map(tuple, rj.tolist())):
        sel = [e for e in range(len(rj)) if tuple(rj[e]) == a]
        assert np.abs(psi[sel].sum(axis=(0, 3))).max() <= 1e-13 * np.abs(psi).max()


@pytest.mark.parametrize("leg", [0, 1, 2])
def test_phph_vertex_vanishes_for_a_uniform_translation(leg):
    """Eq. 13 with the acoustic sum rule of Psi: a mode that translates the
    crystal rigidly (acoustic at Gamma) on any one leg gives V = 0.  For the
    central-cell leg this holds only through translation invariance, so it
    fixes the signs and cells of the other two legs' phases."""
    prob, ifc3 = _phph_problem()
    ac = np.nonzero(prob.hw[0] < prob.omega_min)[0]
    assert ac.size == 3
    big = 0.0
    for q in range(1, prob.nq, 5):
        mq = prob.neg_q(q)
        legs = [(0, q, mq), (q, 0, mq), (q, mq, 0)][leg]
        V = _leg_vertex(prob, ifc3, *legs)
        big = max(big, np.abs(V).max())
        zero = np.take(V, ac, axis=leg)
        assert np.abs(zero).max() <= 1e-12 * np.abs(V).max()
    assert big > 0


def test_phph_vertex_is_symmetric_in_its_legs():
    """With a leg-symmetric Psi the vertex of Eq. 13 is symmetric under
    exchange of (wave vector, branch) between legs, although each ordering
    puts a different leg in the central cell."""
    prob, ifc3 = _phph_problem()
    rng = np.random.default_rng(3)
    for _ in range(6):
        q1, q2 = rng.integers(0, prob.nq, 2)
        q3 = mesh = oracle.mesh_linear(-(prob.ijk[q1] + prob.ijk[q2]), prob.n)
        V = _leg_vertex(prob, ifc3, q1, q2, q3)
        assert np.abs(V).max() > 0
        assert np.allclose(_leg_vertex(prob, ifc3, q2, q1, q3).transpose(1, 0, 2), V,
                           rtol=0, atol=1e-12 * np.abs(V).max())
        assert np.allclose(_leg_vertex(prob, ifc3, q3, q2, q1).transpose(2, 1, 0), V,
                           rtol=0, atol=1e-12 * np.abs(V).max())
        assert np.allclose(_leg_vertex(prob, ifc3, q1, q3, q2).transpose(0, 2, 1), V,
                           rtol=0, atol=1e-12 * np.abs(V).max())


def test_phph_vertex_against_explicit_loops():
    """Eq. 13 summed term by term (cells, atoms, Cartesian directions) on a
    few pairs equals the vectorised oracle."""
    prob, ifc3 = _phph_problem("tiny3")
    rj, rk, psi = ifc3
    na = psi.shape[1]
    E = oracle.eigendisplacements(prob.mat, prob.u)
    for q, qp in [(1, 2), (4, 7), (8, 3)]:
        qpp = oracle.mesh_linear(prob.ijk[q] - prob.ijk[qp], prob.n)
        l2, l3 = prob.neg_q(qp), prob.neg_q(qpp)
        ref = oracle.phph_vertex(ifc3, prob.kfrac[[l2]], prob.kfrac[[l3]], E[q], E[[l2]], E[[l3]])[0]
        V = np.zeros((3 * na,) * 3, complex)
        for e in range(len(rj)):
            p2 = np.exp(2j * np.pi * np.dot(prob.kfrac[l2], rj[e]))
            p3 = np.exp(2j * np.pi * np.dot(prob.kfrac[l3], rk[e]))
            for ti in range(na):
                for tj in range(na):
                    for tk in range(na):
                        for a in range(3):
                            for b in range(3):
                                for c in range(3):
                                    w = psi[e, ti, tj, tk, a, b, c] * p2 * p3
                                    if w == 0:
                                        continue
                                    V += w * np.einsum("s,t,u->stu", E[q][3 * ti + a], E[l2][3 * tj + b],
                                                       E[l3][3 * tk + c])
        assert np.abs(V - ref).max() <= 1e-12 * np.abs(ref).max()


def test_phph_absorption_and_decay_sums_agree():
    """Every three-phonon event a + b -> c appears twice among the absorption
    terms (first leg a or b) and twice among the decay terms (first leg c,
    the products in either order); with Eq. 13's leg symmetry and a symmetric
    delta the bare sums of |V|^2 delta / (E E' E'') over both kinds agree."""
    prob, ifc3 = _phph_problem()
    W, Sp, Sm = oracle.phph_rates(prob, ifc3, 300.0, 0.004, parts=True)
    assert Sp > 0
    assert abs(Sp - Sm) <= 1e-12 * Sp
    assert np.all(W >= 0) and np.all(np.isfinite(W))
    assert np.all(W[0][prob.hw[0] < prob.omega_min] == 0)


def test_phph_rate_prefactor_in_si_units():
    """The prefactor of Eq. 14 evaluated with SI quantities (hbar in J s,
    omega in rad/s, the vertex in J m^-3 kg^-3/2, the delta in s) equals the
    eV form the oracle uses."""
    N, V2, E, d = 512, 3.7, np.array([0.021, 0.013, 0.034]), 11.0   # eV^2/(A^6 amu^3), eV, 1/eV
    w_ev = np.pi / (4 * N) * oracle.C_PHPH * V2 * d / E.prod()
    hbar = 1.054571817e-34                                            # J s
    omega = E * 1.602176634e-19 / hbar
    v2_si = V2 * (1.602176634e-19 / (1e-30 * 1.66053906660e-27 ** 1.5)) ** 2
    d_si = d / 1.602176634e-19 * hbar                                 # delta(omega) in s
    w_si = np.pi * hbar / (4 * N) * v2_si / omega.prod() * d_si
    assert abs(w_ev - w_si) <= 1e-8 * w_si


@pytest.mark.parametrize("sigma", [0.004, 0.002])
def test_phph_inscatter_conserves_energy(sigma):
    """Each three-phonon event conserves energy up to the width of the delta,
    so the in-scattering of the field F_sq = hbar omega_sq (Eq. 26) returns
    hbar omega_sq times the RTA rate of the mode, up to the Gaussian-weighted
    energy mismatch of its terms (a few sigma): a wrong sign of the W+ term,
    a missing half on W- or a wrong partner index misses by about hbar omega."""
    prob, ifc3 = _phph_problem()
    W = oracle.phph_rates(prob, ifc3, 300.0, sigma)
    F = np.repeat(prob.hw[:, :, None], 3, axis=2)
    S = oracle.phph_inscatter(prob, ifc3, 300.0, sigma, F)
    on = prob.mode_on & (W > 0)
    assert on.sum() > 100
    assert np.all(np.abs(S[..., 0] - prob.hw * W)[on] <= 3.0 * sigma * W[on])
    assert np.allclose(S[..., 1], S[..., 0]) and np.all(S[~prob.mode_on] == 0)


def test_phph_operator_matches_inscatter():
    """The dense in-scattering matrix the oracle's iteration uses applies the
    same terms as the row-by-row in-scattering."""
    prob, ifc3 = _phph_problem()
    F = np.random.default_rng(4).standard_normal((prob.nq, prob.nbr, 3))
    S = oracle.phph_inscatter(prob, ifc3, 300.0, 0.004, F)
    M = oracle.phph_operator(prob, ifc3, 300.0, 0.004)
    assert np.abs((M @ F.reshape(-1, 3)).reshape(S.shape) - S).max() <= 1e-13 * np.abs(S).max()


def _einstein_triad(mesh=3):
    """One atom, no dispersion, branches at hbar w_a (twice) and exactly
    2 hbar w_a: the only three-phonon events are b -> a + a' and its reverse,
    and they conserve energy exactly."""
    hwa = 0.020                                           # eV
    lam = hwa ** 2 / oracle.C_PHONON                      # mass-weighted eV / (A^2 amu)
    d0 = np.diag([lam, lam, 4.0 * lam])[None]
    mat = _material(1, 1, [[0, 0, 0]], [[0, 0, 0]], np.zeros((1, 1, 1)), d0, np.zeros((1, 1, 3, 1, 1)), [28.0855])
    prob = oracle.Problem(mat, mesh, 0.0, np.inf, 0.01)
    return prob, hwa


def test_phph_rates_equal_the_golden_rule_on_exact_resonance():
    """With every event exactly on shell, the paper's W/(n(1+n)) of Eq. 26
    must reduce to the golden-rule lifetimes: (n' - n'') for absorption
    a + a' -> b and (1 + n' + n'')/2 for decay b -> a + a' (the Bose
    identities (n'+1) n'' = n (n' - n'') and n' n'' = n (1 + n' + n'') at
    w'' = w + w' and w = w' + w''), with the same vertex and delta.  A wrong
    occupation factor or a missing half changes the rates at order one."""
    prob, hwa = _einstein_triad()
    assert np.allclose(prob.hw, [hwa, hwa, 2 * hwa], rtol=1e-12)
    ifc3 = synth.ifc3_params(1, 21, scale=0.3)
    T, sigma = 300.0, hwa / 40.0
    W = oracle.phph_rates(prob, ifc3, T, sigma)
    E = oracle.eigendisplacements(prob.mat, prob.u)
    nB, _ = oracle.bose_pair(prob.hw, T)
    pref = np.pi / (4.0 * prob.nq) * oracle.C_PHPH
    d0 = 1.0 / (np.sqrt(2.0 * np.pi) * sigma)            # the delta at zero mismatch
    ref = np.zeros_like(W)
    allq = np.arange(prob.nq)
    for q in range(prob.nq):
        for sign in (+1, -1):
            l2 = oracle.mesh_linear(sign * prob.ijk[allq], prob.n)
            qpp = oracle.mesh_linear(prob.ijk[q] + sign * prob.ijk[allq], prob.n)
            l3 = oracle.mesh_linear(-prob.ijk[qpp], prob.n)
            V2 = np.abs(oracle.phph_vertex(ifc3, prob.kfrac[l2], prob.kfrac[l3], E[q], E[l2], E[l3])) ** 2
            for s1 in range(3):
                for s2 in range(3):
                    for s3 in range(3):
                        w1, w2, w3 = prob.hw[q, s1], prob.hw[allq, s2], prob.hw[qpp, s3]
                        if not np.allclose(w1 + sign * w2, w3, rtol=0, atol=1e-12):
                            continue
                        n2, n3 = nB[allq, s2], nB[qpp, s3]
                        occ = (n2 - n3) if sign > 0 else 0.5 * (1.0 + n2 + n3)
                        ref[q, s1] += (pref * d0 * V2[:, s1, s2, s3] * occ / (w1 * w2 * w3)).sum()
    assert ref.min() > 0
    assert np.abs(W - ref).max() <= 1e-9 * ref.max()
