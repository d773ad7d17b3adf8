"""Pins of the oracle's assembled quantities to facts other than itself.

* The tetrahedron delta of Eq. 8 summed over every final state of a band is
  the mesh's linear-tetrahedron density of states at the energy the process
  reaches (absorption lands at eps_i + hw, emission at eps_i - hw), built
  here cell by cell from the closed form of one tetrahedron.
* The Bloch rotation of Eq. 6 and the Froehlich vertex of Eq. 7 carry the
  overlap <n, k+q | m, k> of the final and the initial state, checked on a
  three-band model whose eigenvectors are known in closed form (with three
  bands the overlap matrix is not symmetric in modulus, so a transposed
  index order fails).
* The transport tensors of Eqs. 28-30 (section on transport coefficients)
  obey the effective-mass sum rules of a cosine band and the mode heat
  capacity of the phonon gas, which fix every normalisation (spin
  degeneracy, charge, cell volume, k_B T, 1/N_k, 1/N_q).
* The coupled iteration with three-phonon scattering (Eq. 26's in-scattering
  Delta F^S) converges to a dense direct solve of the same linear systems.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _material(nb, na, re, rp, h_r, d_r, g_r, masses, a=5.4):
    re = np.asarray(re, dtype=np.int32).reshape(-1, 3)
    rp = np.asarray(rp, dtype=np.int32).reshape(-1, 3)
    return dict(nwann=nb, natom=na, re=re, rp=rp, wre=np.ones(len(re)),
                wrp=np.ones(len(rp)), lat=a * np.eye(3), mass=np.asarray(masses, float),
                h_r=np.asarray(h_r, complex), d_r=np.asarray(d_r, float),
                g_r=np.asarray(g_r, complex))


NN = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])


def _cosine_bands(onsite, hop):
    """H(R) of independent cosine bands: H(0) = diag(onsite), H(+-e_i) = diag(hop)."""
    nb = len(onsite)
    h = np.zeros((7, nb, nb), complex)
    h[0] = np.diag(onsite)
    for r in range(1, 7):
        h[r] = np.diag(hop)
    return h


def _scalar_springs(K, M):
    """Force constants of one atom with nearest-neighbour scalar springs."""
    return np.stack([6 * K / M * np.eye(3)] + [-K / M * np.eye(3)] * 6)


# ---------------------------------------------------------------------------
# tetrahedron delta: the mesh density of states

def _tet_dos(e):
    """Density of states at level 0 of one tetrahedron of volume 1/6 (mesh-cell
    units) over which the energy is linear with corner values e: the
    piecewise closed forms of the linear tetrahedron method."""
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


def _mesh_dos(values, n, level):
    """Linear-tetrahedron DOS of a function given on the n^3 mesh: every mesh
    cell split into six tetrahedra along its main diagonal (the paths
    corner -> +e_a -> +e_a+e_b -> opposite corner), each contributing the
    closed form above."""
    vals = np.asarray(values).reshape(n, n, n)
    total = 0.0
    for a, b, c in itertools.product(range(n), repeat=3):
        for perm in itertools.permutations(range(3)):
            p = np.array([a, b, c])
            es = [vals[tuple(p % n)]]
            for ax in perm:
                p = p.copy()
                p[ax] += 1
                es.append(vals[tuple(p % n)])
            total += _tet_dos(np.array(es) - level)
    return total


def test_tetra_delta_sums_to_the_band_dos_at_the_final_energy():
    """Two cosine bands, an Einstein phonon hw0: summed over every final state
    of band n, the absorption weight is DOS_n(eps_i + hw0) and the emission
    weight DOS_n(eps_i - hw0).  Swapping the signs, the bands or the energies
    of the neighbours changes the sums."""
    n = 6
    onsite, hop = [-0.5, 0.45], [0.1, 0.07]
    K, M = 2.4, 28.0855
    mat = _material(2, 1, NN, [[0, 0, 0]], _cosine_bands(onsite, hop), (K / M * np.eye(3))[None],
                    np.zeros((7, 1, 3, 2, 2)), [M])
    hw0 = np.sqrt(oracle.C_PHONON * K / M)
    prob = oracle.Problem(mat, n, 0.0, np.inf, 0.01)
    assert prob.nstates == 2 * n ** 3 and np.allclose(prob.hw, hw0)
    checked = 0
    for target in (-0.72, -0.18, 0.02):
        i = int(np.argmin(np.abs(prob.eps - target) + 10 * (prob.state_m != 0)))
        Dp, Dm = prob.tetra_delta(i)
        for band in range(2):
            sel = prob.state_m == band
            want_p = _mesh_dos(prob.eps_all[:, band], n, prob.eps[i] + hw0)
            want_m = _mesh_dos(prob.eps_all[:, band], n, prob.eps[i] - hw0)
            for s in range(3):
                assert abs(Dp[sel, s].sum() - want_p) <= 1e-11 * max(want_p, 1.0)
                assert abs(Dm[sel, s].sum() - want_m) <= 1e-11 * max(want_m, 1.0)
            if abs(want_p - want_m) > 0.05 * max(want_p, want_m):
                checked += 1
    assert checked >= 3          # the two signs are told apart


def test_tetra_delta_uses_the_phonon_energies_at_the_neighbours():
    """Two flat bands Delta apart and dispersive phonons: absorption from the
    lower to the upper band sums to the phonon DOS at hw = Delta (the phonon
    energies at q'' - k_i enter every corner), emission from the upper band
    to the lower one likewise, and the other two processes to zero."""
    n = 6
    ea, eb = 0.0, 0.021
    K, M = 1.3, 12.011
    h = np.zeros((1, 2, 2), complex)
    h[0] = np.diag([ea, eb])
    mat = _material(2, 1, [[0, 0, 0]], NN, h, _scalar_springs(K, M), np.zeros((1, 7, 3, 2, 2)), [M])
    prob = oracle.Problem(mat, n, 0.0, np.inf, 0.01)
    want = _mesh_dos(prob.hw[:, 0], n, eb - ea)          # three degenerate branches
    assert want > 0.05 * n ** 3 / 0.05                    # Delta lies inside the phonon band
    lower = np.nonzero(prob.state_m == 0)[0]
    upper = np.nonzero(prob.state_m == 1)[0]
    for i in (lower[0], lower[37], lower[101]):
        Dp, Dm = prob.tetra_delta(i)
        for s in range(3):
            assert abs(Dp[upper, s].sum() - want) <= 1e-11 * want
            assert Dm[upper, s].sum() == 0.0
    for i in (upper[5], upper[77]):
        Dp, Dm = prob.tetra_delta(i)
        for s in range(3):
            assert abs(Dm[lower, s].sum() - want) <= 1e-11 * want
            assert Dp[lower, s].sum() == 0.0


def _tri_dos(e):
    """Density of states at level 0 of one triangle of area 1/2 (mesh-cell
    units) over which the energy is linear with corner values e: the
    piecewise closed forms of the linear triangle method."""
    e1, e2, e3 = np.sort(e)
    if 0 <= e1 or 0 >= e3:
        return 0.0
    if e2 >= 0:
        return -e1 / ((e2 - e1) * (e3 - e1))
    return e3 / ((e3 - e1) * (e3 - e2))


def _plane_dos(values, n, level):
    """Linear-triangle DOS of a function on the n^3 mesh, plane by plane
    normal to the third axis: every cell (a, b) of a plane split into two
    triangles along its main diagonal (the paths corner -> +e_x -> +e_x+e_y
    and corner -> +e_y -> +e_x+e_y), each contributing the closed form."""
    vals = np.asarray(values).reshape(n, n, n)
    total = 0.0
    for a, b, c in itertools.product(range(n), repeat=3):
        for first in (0, 1):
            es = [vals[a, b, c]]
            p = [a, b]
            p[first] += 1
            es.append(vals[p[0] % n, p[1] % n, c])
            es.append(vals[(a + 1) % n, (b + 1) % n, c])
            total += _tri_dos(np.array(es) - level)
    return total


def test_triangle_delta_sums_to_the_plane_dos_at_the_final_energy():
    """Two cosine bands, an Einstein phonon hw0: summed over every final state
    of band n, the absorption weight is the plane-by-plane triangle DOS of
    band n at eps_i + hw0 and the emission weight at eps_i - hw0."""
    n = 6
    onsite, hop = [-0.5, 0.45], [0.1, 0.07]
    K, M = 2.4, 28.0855
    mat = _material(2, 1, NN, [[0, 0, 0]], _cosine_bands(onsite, hop), (K / M * np.eye(3))[None],
                    np.zeros((7, 1, 3, 2, 2)), [M])
    hw0 = np.sqrt(oracle.C_PHONON * K / M)
    prob = oracle.Problem(mat, n, 0.0, np.inf, 0.01)
    checked = 0
    for target in (-0.72, -0.18, 0.02):
        i = int(np.argmin(np.abs(prob.eps - target) + 10 * (prob.state_m != 0)))
        Dp, Dm = prob.triangle_delta(i)
        for band in range(2):
            sel = prob.state_m == band
            want_p = _plane_dos(prob.eps_all[:, band], n, prob.eps[i] + hw0)
            want_m = _plane_dos(prob.eps_all[:, band], n, prob.eps[i] - hw0)
            for s in range(3):
                assert abs(Dp[sel, s].sum() - want_p) <= 1e-11 * max(want_p, 1.0)
                assert abs(Dm[sel, s].sum() - want_m) <= 1e-11 * max(want_m, 1.0)
            if abs(want_p - want_m) > 0.05 * max(want_p, want_m):
                checked += 1
    assert checked >= 3          # the two signs are told apart


def test_triangle_delta_uses_the_phonon_energies_at_the_neighbours():
    """Two flat bands Delta apart and dispersive phonons: absorption from the
    lower to the upper band sums to the plane-by-plane phonon DOS at
    hw = Delta, emission from the upper band likewise, the other two
    processes to zero."""
    n = 6
    ea, eb = 0.0, 0.021
    K, M = 1.3, 12.011
    h = np.zeros((1, 2, 2), complex)
    h[0] = np.diag([ea, eb])
    mat = _material(2, 1, [[0, 0, 0]], NN, h, _scalar_springs(K, M), np.zeros((1, 7, 3, 2, 2)), [M])
    prob = oracle.Problem(mat, n, 0.0, np.inf, 0.01)
    want = _plane_dos(prob.hw[:, 0], n, eb - ea)
    assert want > 0.05 * n ** 3 / 0.05
    lower = np.nonzero(prob.state_m == 0)[0]
    upper = np.nonzero(prob.state_m == 1)[0]
    for i in (lower[0], lower[37], lower[101]):
        Dp, Dm = prob.triangle_delta(i)
        for s in range(3):
            assert abs(Dp[upper, s].sum() - want) <= 1e-11 * want
            assert Dm[upper, s].sum() == 0.0
    for i in (upper[5], upper[77]):
        Dp, Dm = prob.triangle_delta(i)
        for s in range(3):
            assert abs(Dm[lower, s].sum() - want) <= 1e-11 * want
            assert Dp[lower, s].sum() == 0.0


def test_triangle_delta_resolves_in_plane_only():
    """A band that disperses along the third axis only: E is constant on every
    mesh plane, so no triangle carries a level crossing and every weight is
    zero unless the level sits exactly on a plane's energy."""
    n = 6
    K, M = 2.4, 28.0855
    h = np.zeros((3, 1, 1), complex)
    h[0, 0, 0] = 0.1
    h[1, 0, 0] = h[2, 0, 0] = 0.2
    mat = _material(1, 1, [[0, 0, 0], [0, 0, 1], [0, 0, -1]], [[0, 0, 0]], h, (K / M * np.eye(3))[None],
                    np.zeros((3, 1, 3, 1, 1)), [M])
    prob = oracle.Problem(mat, n, 0.0, np.inf, 0.01)
    hw0 = np.sqrt(oracle.C_PHONON * K / M)
    levels = np.unique(np.round(prob.eps_all[:, 0], 12))
    assert levels.size == n // 2 + 1                       # one energy per plane pair
    for i in (0, 5, 40):
        for shifted in (prob.eps[i] + hw0, prob.eps[i] - hw0):
            assert np.min(np.abs(levels - shifted)) > 1e-6  # no level on a plane
        Dp, Dm = prob.triangle_delta(i)
        assert np.all(Dp == 0.0) and np.all(Dm == 0.0)


# ---------------------------------------------------------------------------
# the overlap <n, k+q | m, k> in the Bloch rotation (Eq. 6) and in the
# Froehlich vertex (Eq. 7)

A_W = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]])        # cell offsets of the three orbitals


def _phase_gauge_bands(seed):
    """H(k) = W(k) H0 W(k)^+, W(k) = diag(exp(2 pi i k.a_w)): eigenvalues of H0
    at every k and eigenvectors W(k) V0 in closed form.  H(R)[a][b] = H0[a][b]
    for R = a_a - a_b."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    H0 = 0.3 * (A + A.conj().T)
    rs, hs = [], []
    for a in range(3):
        for b in range(3):
            R = A_W[a] - A_W[b]
            for t, r in enumerate(rs):
                if np.array_equal(r, R):
                    hs[t][a, b] += H0[a, b]
                    break
            else:
                rs.append(R)
                m = np.zeros((3, 3), complex)
                m[a, b] = H0[a, b]
                hs.append(m)
    return H0, np.array(rs), np.array(hs)


def _overlap2(V0, q):
    """|<n, k+q | m, k>|^2 = |sum_w conj(V0[w, n]) exp(-2 pi i q.a_w) V0[w, m]|^2."""
    ph = np.exp(-2j * np.pi * (A_W @ q))
    return np.abs(np.conj(V0).T @ (ph[:, None] * V0)) ** 2


def test_rotation_carries_the_final_initial_overlap_three_bands():
    """g^W_x = c_x * identity (one cell, one atom with an Einstein spring):
    summed over branches |g^{s}_{nm}|^2 = l^2 |c|^2 |<n,k+q|m,k>|^2; with three
    bands |<n,k+q|m,k>| != |<m,k+q|n,k>|, so the index order of Eq. 6 is
    fixed."""
    H0, rs, hs = _phase_gauge_bands(3)
    _, V0 = np.linalg.eigh(H0)
    K, M = 1.7, 12.011
    c = np.array([0.7 - 0.1j, -0.2 + 0.5j, 0.3j])
    g = np.zeros((len(rs), 1, 3, 3, 3), complex)
    i0 = int(np.nonzero((rs == 0).all(1))[0][0])
    for x in range(3):
        g[i0, 0, x] = c[x] * np.eye(3)
    mat = _material(3, 1, rs, [[0, 0, 0]], hs, (K / M * np.eye(3))[None], g, [M])
    hw0 = np.sqrt(oracle.C_PHONON * K / M)
    l2 = oracle.C_PHONON / (2 * M * hw0)
    rng = np.random.default_rng(8)
    asym = 0.0
    for _ in range(5):
        k, q = rng.random(3), rng.random(3)
        gW = oracle.g_wannier_factorised(mat, k, q[None])[0]
        _, Uk = oracle.electron_bands(mat, k[None])
        _, Ukq = oracle.electron_bands(mat, (k + q)[None])
        hw, u = oracle.phonon_modes(mat, q[None])
        gb = oracle.g_bloch(mat, gW, Uk[0], Ukq[0], u[0], hw[0])
        got = (np.abs(gb) ** 2).sum(0)
        want = l2 * np.vdot(c, c).real * _overlap2(V0, q)
        assert np.abs(got - want).max() <= 1e-12 * want.max()
        asym = max(asym, np.abs(want - want.T).max() / want.max())
    assert asym > 0.05


def test_frohlich_vertex_carries_the_final_initial_overlap():
    """sum_s |g^Fr_{s n m}(k, q)|^2 = (sum_s |F_s(q)|^2) |<n,k+q|m,k>|^2 for the
    closed-form eigenvectors of the three-band model (Eq. 7's [U_k' U_k^+]_nm
    with n the final band at k' = k + q)."""
    H0, rs, hs = _phase_gauge_bands(4)
    _, V0 = np.linalg.eigh(H0)
    masses = [12.011, 28.0855]
    d = np.zeros((1, 6, 6))
    d[0, :3, :3] = 1.7 / masses[0] * np.eye(3)
    d[0, 3:, 3:] = 2.3 / masses[1] * np.eye(3)
    mat = _material(3, 2, rs, [[0, 0, 0]], hs, d, np.zeros((len(rs), 1, 6, 3, 3)), masses)
    Z, eps = synth.polar_params(2, 7)
    mat["zstar"], mat["eps_inf"], mat["tau"] = Z, eps, np.array([[0.0, 0.0, 0.0], [1.3, 2.1, 0.7]])
    n = 4
    prob = oracle.Problem(mat, n, 0.0, np.inf, 0.01)
    rng = np.random.default_rng(9)
    asym = 0.0
    for _ in range(6):
        ki, kj = rng.integers(0, prob.nk, 2)
        if ki == kj:
            continue
        a, b = prob.kidx_of_mesh[ki], prob.kidx_of_mesh[kj]
        qm = prob.q_index(ki, kj)
        gfr = prob.frohlich_g(prob.U_kept[a], prob.U_kept[b], qm)     # [nbr, n, m]
        F2 = (np.abs(prob._frohlich[qm]) ** 2).sum()
        assert F2 > 0
        want = F2 * _overlap2(V0, prob.kfrac[kj] - prob.kfrac[ki])
        got = (np.abs(gfr) ** 2).sum(0)
        assert np.abs(got - want).max() <= 1e-11 * want.max()
        asym = max(asym, np.abs(want - want.T).max() / want.max())
    assert asym > 0.05


# ---------------------------------------------------------------------------
# Eqs. 28-30: absolute normalisation of the transport tensors

def _cosine_problem(n, T, e0=0.0, t=0.05, mu=-0.1, a=5.4):
    K, M = 1.3, 28.0855
    mat = _material(1, 1, NN, NN, _cosine_bands([e0], [t]), _scalar_springs(K, M),
                    np.zeros((7, 7, 3, 1, 1)), [M], a)
    return oracle.Problem(mat, n, mu, np.inf, 0.01), t, a


def test_electron_tensors_obey_the_effective_mass_sum_rules():
    """Cosine band eps = e0 + 2t sum cos(k_i a), constant rate W0 (J = v/W0,
    I = (eps - mu)/T J).  Integration by parts over the zone turns
    sum f(1-f)/kT (eps - mu)^p (d eps/dk)^2 into sums of f times derivatives of
    eps (p = 0: the Drude weight sum f eps''; p = 1, 2 likewise), exact for the
    mesh sum of a smooth periodic band up to exponentially small terms:
      sigma   = d_s e^2/(V N_k W0 hbar^2) sum f eps''
      alpha   = -d_s e/(V N_k W0 hbar^2) [sum f eps'^2 + sum (eps-mu) f eps'']
      kappa0  = d_s/(V N_k W0 T hbar^2) [2 sum (eps-mu) f eps'^2 + sum (eps-mu)^2 f eps'']
    (energies in J, k in 1/m, V in m^3)."""
    T, W0 = 900.0, 3.0e13
    prob, t, a_A = _cosine_problem(32, T)
    e, hbar = oracle.E_CHARGE, oracle.HBAR_EVS * oracle.E_CHARGE
    a = a_A * oracle.ANG_M
    V = a ** 3
    f, _ = oracle.fermi_pair(prob.eps, prob.mu, T)
    kx = 2 * np.pi * prob.kfrac[prob.state_k, 0]             # k_x a
    d1 = -2 * t * e * a * np.sin(kx)                         # d eps / dk_x, J m
    d2 = -2 * t * e * a ** 2 * np.cos(kx)                    # d^2 eps / dk_x^2, J m^2
    de = (prob.eps - prob.mu) * e
    J = prob.v_state / W0
    I = ((prob.eps - prob.mu) / T)[:, None] * J
    zero = np.zeros((prob.nq, prob.nbr, 3))
    tens = oracle.transport_tensors(prob, T, I, J, zero, zero)
    pre = oracle.SPIN_DEG / (V * prob.nk * W0 * hbar ** 2)
    want = {
        "sigma": pre * e ** 2 * (f * d2).sum(),
        "alpha_el": -pre * e * ((f * d1 ** 2).sum() + (de * f * d2).sum()),
        "sigmaS": -pre * e * ((f * d1 ** 2).sum() + (de * f * d2).sum()) / T,
        "kappa0_el": pre / T * (2 * (de * f * d1 ** 2).sum() + (de ** 2 * f * d2).sum()),
    }
    for key, w in want.items():
        got = tens[key]
        assert abs(got[0, 0] - w) <= 1e-9 * abs(w), (key, got[0, 0], w)
        # cubic: isotropic
        assert abs(got[1, 1] - got[0, 0]) <= 1e-9 * abs(w) and abs(got[0, 1]) <= 1e-9 * abs(w)


def test_phonon_tensors_obey_the_mode_heat_capacity():
    """F = (hw/T) v/W0 and G = v/W0 (constant rate): kappa_ph = (1/(V N_q W0))
    sum_qs C_qs v^2 with the mode heat capacity C = d(hw n)/dT, and
    alpha_ph = -(e T/(V N_q W0)) sum_qs (dn/dT) v^2; both derivatives taken
    here by central differences in T."""
    T, W0 = 250.0, 2.0e12
    prob, _, a_A = _cosine_problem(10, T)
    e = oracle.E_CHARGE
    V = (a_A * oracle.ANG_M) ** 3
    on = prob.mode_on
    v = np.where(on[..., None], prob.v_ph, 0.0)
    F = (prob.hw / T)[..., None] * v / W0
    G = v / W0
    zero = np.zeros((prob.nstates, 3))
    tens = oracle.transport_tensors(prob, T, zero, zero, F, G)
    h = 1e-3 * T
    hwJ = np.where(on, prob.hw, 0.0) * e

    def occ(TT):
        return np.where(on, oracle.bose_pair(prob.hw, TT)[0], 0.0)

    dn = (occ(T + h) - occ(T - h)) / (2 * h)                  # dn/dT, 1/K
    C = hwJ * dn                                              # J/K
    vx2 = v[..., 0] ** 2
    want_k = (C * vx2).sum() / (V * prob.nq * W0)
    want_a = -e * T * (dn * vx2).sum() / (V * prob.nq * W0)
    assert abs(tens["kappa_ph"][0, 0] - want_k) <= 1e-6 * want_k
    assert abs(tens["alpha_ph"][0, 0] - want_a) <= 1e-6 * abs(want_a)
    # the classical limit of the mode heat capacity is k_B per mode
    assert abs(C.max() / (oracle.KB_EVK * e) - 1.0) < 0.05


# ---------------------------------------------------------------------------
# the iteration with three-phonon scattering against dense solves

@pytest.fixture(scope="module")
def phph_system():
    cfg = synth.config("metal6")
    mat = synth.material_for(cfg)
    T, sig = 300.0, 0.004
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    Xp, Xm = prob.transition_probs(T)
    ifc3 = synth.ifc3_params(mat["natom"], 5, scale=3.0)
    Mph = oracle.phph_operator(prob, ifc3, T, sig)
    Wpp = oracle.phph_rates(prob, ifc3, T, sig)
    return prob, T, sig, Xp, Xm, ifc3, Mph, Wpp


def _dense_coupled(prob, T, Xp, Xm, Wp, Mph):
    """Dense solve of Eqs. 19-27 with the three-phonon in-scattering: the
    phonon equations F = F0 + Ape I + D Mph F (D = 1/W^RTA) are solved for F,
    F = R (F0 + Ape I) with R = (1 - D Mph)^-1, and the electrons then satisfy
    (1 - Aee - Aep R Ape) I = I0 + Aep R F0 with one carrier-number
    constraint per energy group (a bordered system)."""
    M, nbr, nq = prob.nstates, prob.nbr, prob.nq
    f, omf = oracle.fermi_pair(prob.eps, prob.mu, T)
    ff = f * omf
    We = (Xp + Xm).sum((1, 2)) / ff
    n, onp = oracle.bose_pair(prob.hw, T)
    on = prob.mode_on
    qij = prob.q_index(prob.state_k[:, None], prob.state_k[None, :])
    nqij = prob.neg_q(qij)
    row = 1.0 / (ff * We)
    Aee = (Xp + Xm).sum(2) * row[:, None]
    P = nq * nbr
    Aep = np.zeros((M, P))
    Ape = np.zeros((P, M))
    pn = np.where(on, oracle.SPIN_DEG * (prob.nk / prob.nq) / (Wp * n * onp), 0.0).reshape(-1)
    for s in range(nbr):
        np.add.at(Aep, (np.arange(M)[:, None].repeat(M, 1), qij * nbr + s), -Xp[:, :, s] * row[:, None])
        np.add.at(Aep, (np.arange(M)[:, None].repeat(M, 1), nqij * nbr + s), Xm[:, :, s] * row[:, None])
        p = qij * nbr + s
        np.add.at(Ape, (p, np.arange(M)[None, :].repeat(M, 0)), pn[p] * Xp[:, :, s])
        np.add.at(Ape, (p, np.arange(M)[:, None].repeat(M, 1)), -pn[p] * Xp[:, :, s])
    inv_wp = np.where(on, 1.0 / Wp, 0.0).reshape(-1)
    R = np.linalg.inv(np.eye(P) - inv_wp[:, None] * Mph)
    v = prob.v_state
    I0 = ((prob.eps - prob.mu) / T / We)[:, None] * v
    J0 = (1.0 / We)[:, None] * v
    F0 = ((prob.hw / T * inv_wp.reshape(nq, nbr))[..., None] * prob.v_ph).reshape(P, 3)
    grp = oracle.energy_groups(prob.eps, prob.hw.max(), prob.sigma)
    C = grp.max() + 1
    A = np.zeros((M + C, M + C))
    A[:M, :M] = np.eye(M) - Aee - Aep @ R @ Ape
    for c in range(C):
        A[:M, M + c] = (grp == c)
        A[M + c, :M] = ff * (grp == c)
    rhsI = np.zeros((M + C, 3))
    rhsI[:M] = I0 + Aep @ R @ F0
    rhsJ = np.zeros((M + C, 3))
    rhsJ[:M] = J0
    I = np.linalg.solve(A, rhsI)[:M]
    J = np.linalg.solve(A, rhsJ)[:M]
    F = R @ (F0 + Ape @ I)
    G = R @ (Ape @ J)
    return I, J, F.reshape(nq, nbr, 3), G.reshape(nq, nbr, 3), F0.reshape(nq, nbr, 3), R


def test_dragless_phonons_with_three_phonon_inscattering_match_a_dense_solve(phph_system):
    """Level DRAGLESS with three-phonon processes: the phonons solve their own
    BTE F = F0 + Delta F^S[F] (Eq. 26); its fixed point is (1 - D Mph)^-1 F0."""
    prob, T, sig, Xp, Xm, ifc3, Mph, Wpp = phph_system
    res = oracle.iterate(prob, T, Xp, Xm, oracle.LEVEL_DRAGLESS, tol=1e-13, maxit=2000, phph=(ifc3, sig))
    assert res["converged"]
    Wp = prob.rates_ph(T, Xp) + Wpp
    _, _, _, _, F0, R = _dense_coupled(prob, T, Xp, Xm, Wp, Mph)
    F = (R @ F0.reshape(-1, 3)).reshape(F0.shape)
    assert np.abs(res["F"] - F).max() <= 1e-9 * np.abs(F).max()
    # the in-scattering really changes the answer here
    assert np.abs(F - F0).max() > 1e-3 * np.abs(F).max()


def test_coupled_iteration_with_three_phonon_inscattering_matches_a_dense_solve(phph_system):
    prob, T, sig, Xp, Xm, ifc3, Mph, Wpp = phph_system
    res = oracle.iterate(prob, T, Xp, Xm, oracle.LEVEL_COUPLED, tol=1e-12, maxit=2000, phph=(ifc3, sig))
    assert res["converged"]
    Wp = prob.rates_ph(T, Xp) + Wpp
    I, J, F, G, F0, _ = _dense_coupled(prob, T, Xp, Xm, Wp, Mph)
    for got, want in ((res["I"], I), (res["J"], J), (res["F"], F), (res["G"], G)):
        assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    assert np.abs(G).max() > 1e-6 * np.abs(F).max()


@pytest.mark.parametrize("level", [1, 2, 3])
def test_direct_electron_solve_equals_the_substitution(level):
    """The dense bordered electron solve (inner="direct") reaches the fixed
    point the plain substitution reaches (metal6, where it converges), at
    every level of the scheme."""
    cfg = synth.config("metal6")
    mat = synth.material_for(cfg)
    T = 300.0
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    Xp, Xm = prob.transition_probs(T)
    w_ext = oracle.default_w_ext(prob, T, gamma0=1e13)
    a = oracle.iterate(prob, T, Xp, Xm, level, tol=1e-13, maxit=3000, w_ext=w_ext)
    b = oracle.iterate(prob, T, Xp, Xm, level, tol=1e-13, maxit=3000, w_ext=w_ext, inner="direct")
    assert a["converged"] and b["converged"]
    for k in ("I", "J", "F", "G"):
        scale = np.abs(a[k]).max()
        if scale == 0:
            assert not np.any(b[k])
            continue
        assert np.abs(a[k] - b[k]).max() <= 1e-9 * scale, k


@pytest.mark.parametrize("name", ["tiny4", "plain8"])
def test_sampled_rows_equal_the_whole_problem(name):
    """rates_e_rows (phonons only at the q the rows need) equals
    Problem.rates_e on Problem.transition_probs for the same rows."""
    cfg = synth.config(name)
    mat = synth.material_for(cfg)
    prob = oracle.Problem(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"])
    rows = np.random.default_rng(3).choice(prob.nstates, 6, replace=False)
    Xp, Xm = prob.transition_probs(cfg["T"], rows)
    want = prob.rates_e(cfg["T"], Xp, Xm, rows)
    got, M = oracle.rates_e_rows(mat, cfg["mesh"], cfg["mu"], cfg["window"], cfg["sigma"], cfg["T"], rows)
    assert M == prob.nstates
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
