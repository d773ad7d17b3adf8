"""Plain FP64 NumPy oracle of the e-ph transition-probability path.

Test infrastructure only (tests, smoke check and the benchmark's CPU leg); the
product library never imports it and shares no code with it.

Every function cites the passage of the paper it follows (section and
equation of "The elphbolt ab initio solver for the coupled electron-phonon
Boltzmann transport equations").  Equation numbers count the displayed
equations in order of appearance: Eq. 1 H(k), Eq. 2 electron velocity,
Eq. 3 D(q), Eq. 4 non-analytic term, Eq. 5 phonon velocity, Eq. 6 e-ph
vertex, Eq. 7 Froehlich term, Eq. 8 X^{+/-}, Eq. 12 Y^{ph-e}, Eqs. 17-18
deviation functions, Eq. 19 coupled BTEs, Eqs. 20-27 RTA / self / drag
terms, Eqs. 28-31 transport tensors and the Kelvin-Onsager relation.

Readings of the paper used here (where it is silent, garbled or ambiguous):

* Normalisations 1/N_e, 1/N_ph of Eqs. 1, 3, 6 are absorbed into the
  Wannier-space inputs; optional per-vector weights w_R multiply each term.
* Phases are exp(+2 pi i k_frac . n) with integer cell vectors n (Eqs. 1, 3,
  6 show cell phases only, no atom-position phases).
* Eq. 6 index order: U columns are eigenvectors; m is the initial band at k,
  n the final band at k' = k + q:
  g_x[n,m] = sum_{n',m'} conj(U_{k'}[n',n]) gW_x[n',m'] U_k[m',m], and the
  phonon projection is g_s = sum_x l_{x,s} u_q[x,s] g_x with the mass of
  the atom of x inside the sum.
* Eq. 6 prefactor: l = sqrt(hbar^2 / (2 M hbar*omega)) =
  sqrt(C / (2 M[amu] hbar*omega[eV])) Angstrom with C = hbar^2/(amu A^2).
* Modes with hbar*omega < omega_min (the acoustic modes at Gamma) are
  dropped: their g, X and rates are zero.
* The energy-conserving delta of Eq. 8 is a Gaussian of standard deviation
  sigma, never truncated.
* Emission in Eq. 8 uses n and omega at -q; the force constants are real so
  omega(-q) = omega(q).
* Y = (N_k/N_q) X^+ on the same term (Eq. 12 vs Eq. 8), spin degeneracy 2.
* Electron states enter through an energy window |eps - mu| <= w (per state);
  k is kept if any band is active; initial and final states are active
  states.  N_k is the full mesh count.
* Transport tensors (Eqs. 28-30) carry 1/N_k (electrons) and 1/N_q
  (phonons); V is the cell volume.
* The e-ph collision operator conserves carrier number: the in-scattering
  matrix of Eq. 22 has every group-constant vector as an eigenvector with
  eigenvalue 1, one per group of states that the Gaussian-broadened
  interaction couples.  Groups are the maximal runs of active states, sorted
  by energy, with no gap wider than hw_max + 12 sigma (beyond which the
  coupling is below 1e-31 of the peak).  Iterated electron responses are
  constrained to sum_{i in group} f_i (1 - f_i) I_i = 0 for every group (no
  change of carrier number), applied after every electron sweep; for
  materials with inversion or time-reversal symmetry this holds by itself.
* Phonon scattering other than ph-e enters the iteration as an external rate
  per mode (default model gamma0 (hw/hw_max)^2 (T/300 K), gamma0 = 1e12/s).
  Without three-phonon processes the phonon in-scattering Delta F^S is zero;
  iterate(..., phph=(ifc3, sigma)) adds the three-phonon RTA rate of Eq. 26
  (phph_rates) to W^RTA, with w_ext then holding only the remaining channels
  (none when None), and Delta F^S = S[F] / W^RTA (phph_operator) to every
  phonon update.
"""
import numpy as np

# CODATA 2018
HBAR_EVS = 6.582119569e-16        # eV s
KB_EVK = 8.617333262e-5           # eV / K
E_CHARGE = 1.602176634e-19        # C  (= J per eV)
AMU_KG = 1.66053906660e-27        # kg
ANG_M = 1.0e-10                   # m per Angstrom
HBAR_JS = HBAR_EVS * E_CHARGE
# (hbar omega)^2 [eV^2] = C_PHONON [eV] * lambda [eV / (A^2 amu)]
C_PHONON = HBAR_JS ** 2 / (AMU_KG * ANG_M ** 2) / E_CHARGE
SPIN_DEG = 2.0
OMEGA_MIN_DEFAULT = 1.0e-4        # eV
DEGEN_TOL = 1.0e-6                # eV, degenerate-group tolerance

LEVEL_RTA, LEVEL_PARTIAL, LEVEL_DRAGLESS, LEVEL_COUPLED = 0, 1, 2, 3

__all__ = [
    "HBAR_EVS", "KB_EVK", "E_CHARGE", "AMU_KG", "ANG_M", "C_PHONON", "SPIN_DEG",
    "OMEGA_MIN_DEFAULT", "NAC_EV_A", "nac_images", "nac_term", "frohlich_factor", "LEVEL_RTA", "LEVEL_PARTIAL", "LEVEL_DRAGLESS", "LEVEL_COUPLED",
    "mesh_points", "mesh_linear", "phases", "rates_e_rows", "bloch_hamiltonian", "bloch_hamiltonian_grad",
    "electron_bands", "electron_velocities", "dynamical_matrix", "dynamical_matrix_grad",
    "phonon_modes", "phonon_velocities", "fermi_pair", "bose_pair", "gaussian_delta",
    "g_wannier_brute", "g_wannier_factorised", "g_bloch", "Problem", "default_w_ext",
    "tetra_delta_weights", "tetra_neighbourhood", "triangle_delta_weights", "triangle_neighbourhood",
    "iterate", "transport_tensors", "ko_residual", "ko_enforce", "energy_groups",
    "C_PHPH", "eigendisplacements", "ifc3_matrix", "phph_vertex", "phph_rates", "phph_inscatter", "phph_operator",
]


# ----------------------------------------------------------------------------
# meshes and phases

def mesh_points(n):
    """Gamma-centred n^3 mesh in fractional coordinates, linear index
    (a*n + b)*n + c for k = (a, b, c)/n."""
    a = np.arange(n)
    g = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3)
    return g.astype(np.float64) / n


def mesh_linear(ijk, n):
    ijk = np.mod(np.asarray(ijk, dtype=np.int64), n)
    return (ijk[..., 0] * n + ijk[..., 1]) * n + ijk[..., 2]


def phases(kfrac, R, w=None):
    """w_R exp(2 pi i k . R) for fractional k and integer R -> [nk, nR]."""
    arg = 2.0 * np.pi * (np.atleast_2d(kfrac) @ np.asarray(R, dtype=np.float64).T)
    ph = np.exp(1j * arg)
    if w is not None:
        ph = ph * np.asarray(w)[None, :]
    return ph


# ----------------------------------------------------------------------------
# electrons: Eq. 1 (H(k)), Eq. 2 (velocity)

def bloch_hamiltonian(mat, kfrac):
    """Eq. 1: H(k) = sum_Re w exp(i k.Re) H(Re)."""
    return np.einsum("kr,rab->kab", phases(kfrac, mat["re"], mat["wre"]), mat["h_r"])


def _cart(mat, R):
    return np.asarray(R, dtype=np.float64) @ np.asarray(mat["lat"])  # Angstrom


def bloch_hamiltonian_grad(mat, kfrac):
    """Cartesian gradient of Eq. 1: sum_Re i Re_cart w exp(i k.Re) H(Re), eV*A."""
    ph = phases(kfrac, mat["re"], mat["wre"])
    rc = _cart(mat, mat["re"])
    return np.einsum("kr,rc,rab->kcab", 1j * ph, rc, mat["h_r"])


def electron_bands(mat, kfrac):
    """Diagonalise H(k) (after Eq. 1): eigenvalues ascending, U columns."""
    return np.linalg.eigh(bloch_hamiltonian(mat, kfrac))


def _group_average(values, energies, tol=DEGEN_TOL):
    """Average per-state values over groups of (sorted) degenerate states."""
    out = values.copy()
    nk, nb = energies.shape
    for k in range(nk):
        start = 0
        for b in range(1, nb + 1):
            if b == nb or energies[k, b] - energies[k, b - 1] >= tol:
                if b - start > 1:
                    out[k, start:b] = values[k, start:b].mean(0)
                start = b
    return out


def electron_velocities(mat, kfrac, eps, U):
    """Eq. 2: v = (1/hbar) <mk| grad_k H |mk>, m/s, degenerate groups averaged."""
    dh = bloch_hamiltonian_grad(mat, kfrac)
    diag = np.einsum("kam,kcab,kbm->kmc", np.conj(U), dh, U).real  # eV*A
    v = diag * ANG_M / HBAR_EVS
    return _group_average(v, eps)


# ----------------------------------------------------------------------------
# phonons: Eq. 3 (D(q), short-range part), Eq. 5 (velocity)

# e^2 / (eps_0 V) in eV / Angstrom^2 for V in Angstrom^3 is NAC_EV_A / V
EPS0_SI = 8.8541878128e-12        # F / m
NAC_EV_A = E_CHARGE / EPS0_SI / ANG_M   # e / eps_0 in eV Angstrom


def nac_images(mat, qf):
    """Cartesian images (1/Angstrom, 2 pi included) nearest Gamma of one
    fractional q: coordinates folded into [-1/2, 1/2), and a coordinate of
    exactly 1/2 taken at both +1/2 and -1/2 (reading: Eq. 4 is averaged over
    the equally near images, which keeps it even in q)."""
    f = np.asarray(qf, dtype=np.float64) - np.floor(np.asarray(qf, dtype=np.float64) + 0.5)
    B = np.linalg.inv(np.asarray(mat["lat"], dtype=np.float64)).T     # rows b_i, a_i . b_j = delta_ij
    imgs = [f]
    for d in range(3):
        if f[d] == -0.5:
            imgs = imgs + [g + np.eye(3)[d] for g in imgs]
    return [2.0 * np.pi * g @ B for g in imgs]


def nac_term(mat, qfrac):
    """Eq. 4, the non-analytic (dipole-dipole) part of D(q) for polar
    materials, in the units of D (eV / (Angstrom^2 amu)):
    (e^2 / (eps_0 V)) (q.Z_t)_a (q.Z_t')_b / (q.eps_inf.q) / sqrt(m_t m_t'),
    with (q.Z_t)_b = sum_a q_a Z_t[a][b], at the image of q nearest Gamma
    (averaged over equally near images, see nac_images).  Zero at Gamma
    (reading: the direction-dependent limit is not taken on the mesh).
    Returns (D_nac [nq, nbr, nbr], dD_nac/dq_cart [nq, 3, nbr, nbr])."""
    Z = np.asarray(mat["zstar"], dtype=np.float64)               # [na, 3, 3]
    eps = np.asarray(mat["eps_inf"], dtype=np.float64)
    m = np.repeat(np.asarray(mat["mass"], dtype=np.float64), 3)    # per x
    V = abs(np.linalg.det(np.asarray(mat["lat"], dtype=np.float64)))
    qfrac = np.atleast_2d(np.asarray(qfrac, dtype=np.float64))
    nq, na = qfrac.shape[0], Z.shape[0]
    dZ = np.transpose(Z, (1, 0, 2)).reshape(3, 3 * na)             # d(q.Z)_x / dq_c
    scale = NAC_EV_A / V / np.sqrt(np.outer(m, m))
    D = np.zeros((nq, 3 * na, 3 * na))
    G = np.zeros((nq, 3, 3 * na, 3 * na))
    for k in range(nq):
        imgs = nac_images(mat, qfrac[k])
        for q in imgs:
            Q = q @ eps @ q
            if Q <= 0.0:
                continue
            A = (q @ Z.reshape(na, 3, 3).transpose(1, 0, 2).reshape(3, 3 * na))   # (q.Z_t)_b at x = 3t + b
            epsq = eps @ q
            D[k] += scale * np.outer(A, A) / Q / len(imgs)
            for c in range(3):
                G[k, c] += scale * ((np.outer(dZ[c], A) + np.outer(A, dZ[c])) / Q
                                    - 2.0 * epsq[c] * np.outer(A, A) / Q ** 2) / len(imgs)
    return D, G


def dynamical_matrix(mat, qfrac):
    """Eq. 3: D(q) = sum_Rp w exp(i q.Rp) D(Rp), plus the non-analytic term
    of Eq. 4 when the material carries Born charges ("zstar", "eps_inf")."""
    D = np.einsum("kr,rab->kab", phases(qfrac, mat["rp"], mat["wrp"]), mat["d_r"])
    if mat.get("zstar") is not None:
        D = D + nac_term(mat, qfrac)[0]
    return D


def dynamical_matrix_grad(mat, qfrac):
    ph = phases(qfrac, mat["rp"], mat["wrp"])
    rc = _cart(mat, mat["rp"])
    G = np.einsum("kr,rc,rab->kcab", 1j * ph, rc, mat["d_r"])
    if mat.get("zstar") is not None:
        G = G + nac_term(mat, qfrac)[1]
    return G


def phonon_modes(mat, qfrac):
    """Diagonalise D(q): hbar*omega = sqrt(C max(lambda, 0)) eV, u columns."""
    lam, u = np.linalg.eigh(dynamical_matrix(mat, qfrac))
    hw = np.sqrt(C_PHONON * np.maximum(lam, 0.0))
    return hw, u


def phonon_velocities(mat, qfrac, hw, u, omega_min=OMEGA_MIN_DEFAULT):
    """Eq. 5: v = <sq| grad_q D |sq> / (2 omega), m/s; zero below omega_min."""
    dd = dynamical_matrix_grad(mat, qfrac)
    diag = np.einsum("kas,kcab,kbs->ksc", np.conj(u), dd, u).real  # eV/(A amu)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = C_PHONON * diag / (2.0 * hw[..., None]) * ANG_M / HBAR_EVS
    v = np.where((hw >= omega_min)[..., None], v, 0.0)
    return _group_average(v, hw)


# ----------------------------------------------------------------------------
# thermal factors and the delta function (Eq. 8)

def fermi_pair(eps, mu, T):
    """(f, 1 - f) of the Fermi-Dirac distribution, each from its own logistic."""
    x = (np.asarray(eps) - mu) / (KB_EVK * T)
    f = np.exp(-np.logaddexp(0.0, x))
    omf = np.exp(-np.logaddexp(0.0, -x))
    return f, omf


def bose_pair(hw, T):
    """(n, 1 + n) of the Bose-Einstein distribution."""
    y = np.asarray(hw) / (KB_EVK * T)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        n = 1.0 / np.expm1(y)
        onp = -1.0 / np.expm1(-y)
    return n, onp


def gaussian_delta(x, sigma):
    """Normalised Gaussian of standard deviation sigma (eV^-1)."""
    return np.exp(-0.5 * (np.asarray(x) / sigma) ** 2) / (np.sqrt(2.0 * np.pi) * sigma)


# ----------------------------------------------------------------------------
# The analytic tetrahedron delta (the alternative to smearing that the paper
# provides beside the triangle method; section on the program's workflow)

def tetra_delta_weights(e):
    """e [..., 4]: energies (level 0) at the corners of tetrahedra over which
    E is linear -> w [..., 4]: the integral over the tetrahedron of
    delta(E(x)) lambda_c(x), lambda_c the barycentric coordinate of corner c,
    for a tetrahedron of volume 1/6 (one sixth of a mesh cell in mesh units).
    By the coarea formula this is the area integral of lambda_c over the
    section E = 0 divided by |grad E|; lambda_c is linear on each triangle of
    the section, so a triangle contributes its area times the mean of
    lambda_c over its corners.  The integral depends only on the corner
    energies and the volume, so the sorted corners are placed at 0, x, y, z."""
    e = np.asarray(e, dtype=np.float64)
    shp = e.shape[:-1]
    e = e.reshape(-1, 4)
    order = np.argsort(e, axis=1, kind="stable")
    es = np.take_along_axis(e, order, axis=1)
    P = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    grad = np.stack([es[:, 1] - es[:, 0], es[:, 2] - es[:, 0], es[:, 3] - es[:, 0]], axis=1)
    gn = np.linalg.norm(grad, axis=1)
    ws = np.zeros_like(es)
    nneg = (es < 0).sum(axis=1)

    def cross(a, b, rows):
        # point of edge (a, b) where E = 0: position and barycentric coordinates
        ea, eb = es[rows, a], es[rows, b]
        t = ea / (ea - eb)
        X = P[a][None, :] + t[:, None] * (P[b] - P[a])[None, :]
        lam = np.zeros((rows.size, 4))
        lam[:, a] = 1.0 - t
        lam[:, b] = t
        return X, lam

    def add_triangle(rows, A, B, C):
        (Xa, la), (Xb, lb), (Xc, lc) = A, B, C
        area = 0.5 * np.linalg.norm(np.cross(Xb - Xa, Xc - Xa), axis=1)
        ws[rows] += (area / gn[rows])[:, None] * (la + lb + lc) / 3.0

    ok = gn > 0
    r1 = np.nonzero(ok & (nneg == 1))[0]
    if r1.size:
        add_triangle(r1, cross(0, 1, r1), cross(0, 2, r1), cross(0, 3, r1))
    r3 = np.nonzero(ok & (nneg == 3))[0]
    if r3.size:
        add_triangle(r3, cross(0, 3, r3), cross(1, 3, r3), cross(2, 3, r3))
    r2 = np.nonzero(ok & (nneg == 2))[0]
    if r2.size:
        q02, q03, q13, q12 = cross(0, 2, r2), cross(0, 3, r2), cross(1, 3, r2), cross(1, 2, r2)
        add_triangle(r2, q02, q03, q13)   # the section's corners in cyclic order
        add_triangle(r2, q02, q13, q12)
    w = np.empty_like(ws)
    np.put_along_axis(w, order, ws, axis=1)
    return w.reshape(shp + (4,))


def tetra_neighbourhood():
    """The 24 tetrahedra of the mesh that have a given point as a corner, in
    the six-tetrahedra split of every mesh cell along its main diagonal (the
    paths 0 -> e_a -> e_a + e_b -> (1,1,1)).  Points of the 3x3x3
    neighbourhood are numbered (dx+1)*9 + (dy+1)*3 + (dz+1); returns
    (corners [24, 4], index of the centre point 13 among them [24])."""
    import itertools
    corners, centre = [], []
    for o in itertools.product((0, 1), repeat=3):
        for perm in itertools.permutations(range(3)):
            path = [np.array(o)]
            for ax in perm:
                nxt = path[-1].copy()
                nxt[ax] += 1
                path.append(nxt)
            ids = [int(p[0] * 9 + p[1] * 3 + p[2]) for p in path]
            if 13 in ids:
                corners.append(ids)
                centre.append(ids.index(13))
    return np.array(corners), np.array(centre)


# ----------------------------------------------------------------------------
# The triangle delta (the paper's default method for the energy-conserving
# delta, its only one in two dimensions; section on the program's workflow).
# Reading: a 2-D mesh (one point along the third axis) is split into
# triangles; a 3-D mesh is taken as its planes normal to the third mesh axis,
# each triangulated the same way, the delta resolved within a plane and the
# planes summed as mesh points.

def triangle_delta_weights(e):
    """e [..., 3]: energies (level 0) at the corners of triangles over which
    E is linear -> w [..., 3]: the integral over the triangle of
    delta(E(x)) lambda_c(x), lambda_c the barycentric coordinate of corner c,
    for a triangle of area 1/2 (half a mesh cell in mesh units).  By the
    coarea formula this is the integral of lambda_c along the segment E = 0
    divided by |grad E|; lambda_c is linear along the segment, so it gives
    the segment's length times the mean of lambda_c at its two ends.  The
    integral depends only on the corner energies and the area, so the sorted
    corners are placed at (0, 0), (1, 0), (0, 1)."""
    e = np.asarray(e, dtype=np.float64)
    shp = e.shape[:-1]
    e = e.reshape(-1, 3)
    order = np.argsort(e, axis=1, kind="stable")
    es = np.take_along_axis(e, order, axis=1)
    P = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    grad = np.stack([es[:, 1] - es[:, 0], es[:, 2] - es[:, 0]], axis=1)
    gn = np.linalg.norm(grad, axis=1)
    ws = np.zeros_like(es)
    nneg = (es < 0).sum(axis=1)

    def cross(a, b, rows):
        ea, eb = es[rows, a], es[rows, b]
        t = ea / (ea - eb)
        X = P[a][None, :] + t[:, None] * (P[b] - P[a])[None, :]
        lam = np.zeros((rows.size, 3))
        lam[:, a] = 1.0 - t
        lam[:, b] = t
        return X, lam

    def add_segment(rows, A, B):
        (Xa, la), (Xb, lb) = A, B
        length = np.linalg.norm(Xb - Xa, axis=1)
        ws[rows] += (length / gn[rows])[:, None] * (la + lb) / 2.0

    ok = gn > 0
    r1 = np.nonzero(ok & (nneg == 1))[0]
    if r1.size:
        add_segment(r1, cross(0, 1, r1), cross(0, 2, r1))
    r2 = np.nonzero(ok & (nneg == 2))[0]
    if r2.size:
        add_segment(r2, cross(0, 2, r2), cross(1, 2, r2))
    w = np.empty_like(ws)
    np.put_along_axis(w, order, ws, axis=1)
    return w.reshape(shp + (3,))


def triangle_neighbourhood():
    """The 6 triangles of a mesh plane that have a given point as a corner,
    in the split of every cell of the plane along its main diagonal (the
    paths 0 -> e_a -> e_a + e_b).  Points of the 3x3 in-plane neighbourhood
    are numbered (dx+1)*3 + (dy+1) (the third mesh axis fixed); returns
    (corners [6, 3], index of the centre point 4 among them [6])."""
    import itertools
    corners, centre = [], []
    for o in itertools.product((0, 1), repeat=2):
        for perm in itertools.permutations(range(2)):
            path = [np.array(o)]
            for ax in perm:
                nxt = path[-1].copy()
                nxt[ax] += 1
                path.append(nxt)
            ids = [int(p[0] * 3 + p[1]) for p in path]
            if 4 in ids:
                corners.append(ids)
                centre.append(ids.index(4))
    return np.array(corners), np.array(centre)


# ----------------------------------------------------------------------------
# Eq. 6: the e-ph vertex

def g_wannier_brute(mat, k, q):
    """Wannier part of Eq. 6 as the literal double sum over (Re, Rp):
    gW_x = sum_{Re,Rp} w_e w_p exp(i(k.Re + q.Rp)) g(Re, Rp)_x  -> [nbr, nb, nb]."""
    re, rp = np.asarray(mat["re"], float), np.asarray(mat["rp"], float)
    k = np.asarray(k, float)
    q = np.asarray(q, float)
    nbr = 3 * mat["natom"]
    nb = mat["nwann"]
    out = np.zeros((nbr, nb, nb), dtype=np.complex128)
    for ie in range(re.shape[0]):
        for ip in range(rp.shape[0]):
            ph = mat["wre"][ie] * mat["wrp"][ip] * np.exp(
                2j * np.pi * (k @ re[ie] + q @ rp[ip]))
            out += ph * mat["g_r"][ie, ip]
    return out


def g_wannier_factorised(mat, k, qs):
    """Same sum as :func:`g_wannier_brute`, the exponential split into its
    R_e and R_p factors: first sum over R_e at fixed k, then over R_p for
    every q in ``qs`` -> [nq, nbr, nb, nb]."""
    g = mat["g_r"]
    ne, npr = g.shape[0], g.shape[1]
    phk = phases(k, mat["re"], mat["wre"])[0]                          # [Re]
    gk = (phk @ g.reshape(ne, -1)).reshape((npr,) + g.shape[2:])       # [Rp, x, n', m']
    phq = phases(np.atleast_2d(qs), mat["rp"], mat["wrp"])             # [nq, Rp]
    return (phq @ gk.reshape(npr, -1)).reshape((phq.shape[0],) + g.shape[2:])


def phonon_lengths(mat, hw, omega_min=OMEGA_MIN_DEFAULT):
    """Eq. 6 prefactor l_{x,s} = sqrt(C / (2 M_tau(x) hbar omega_s)) in A,
    zero for modes below omega_min -> [..., nbr(x), nbr(s)]."""
    mass_x = np.repeat(np.asarray(mat["mass"], float), 3)
    hw = np.asarray(hw)
    with np.errstate(divide="ignore", invalid="ignore"):
        l = np.sqrt(C_PHONON / (2.0 * mass_x[:, None] * hw[..., None, :]))
    return np.where((hw >= omega_min)[..., None, :], l, 0.0)


def g_bloch(mat, gW, Uk, Ukq, u_q, hw_q, omega_min=OMEGA_MIN_DEFAULT):
    """Eq. 6 Bloch vertex g[..., s, n, m] from the Wannier-gauge gW[..., x, n', m']:
    rotate with the electron eigenvectors at k (initial) and k+q (final), then
    project on the phonon eigenvectors with the length prefactor."""
    gh = np.einsum("...ab,...xac,...cd->...xbd", np.conj(Ukq), gW, Uk)
    lu = phonon_lengths(mat, hw_q, omega_min) * u_q                   # [..., x, s]
    return np.einsum("...xs,...xnm->...snm", lu, gh)


BOHR_A = 0.529177210903           # Angstrom
EWALD_ALPHA = 1.0 / BOHR_A ** 2    # 1 Bohr^-2 in Angstrom^-2
EWALD_CUT = 40.0                   # terms with (q+G).eps.(q+G) / (4 alpha) above this are dropped


def frohlich_factor(mat, qfrac, lu):
    """Eq. 7 without its electron overlap: F_s(q) such that
    g^Fr_{smn}(k, q) = F_s(q) [U_k' U_k^+]_{nm}, for the phonon factors
    lu[q, x, s] = l_{x,s} u_{x,s}(q) (Angstrom) ->  [nq, nbr] complex, eV:
    F_s(q) = i (e^2 / (eps_0 V)) sum_t sum_{G != -q} ((q+G).Z_t.lu_t,s)
    / ((q+G).eps_inf.(q+G)) exp(-i (q+G).r_t) exp(-(q+G).eps_inf.(q+G) / (4 alpha)),
    alpha = 1 Bohr^-2, over every G with (q+G).eps_inf.(q+G)/(4 alpha) <= 40
    (reading: the Ewald-damped sum taken to where the damping is below
    e^-40), q at its fractional coordinates (the sum over G makes it periodic)."""
    Z = np.asarray(mat["zstar"], dtype=np.float64)
    eps = np.asarray(mat["eps_inf"], dtype=np.float64)
    tau = np.asarray(mat["tau"], dtype=np.float64)                # [na, 3] Angstrom
    lat = np.asarray(mat["lat"], dtype=np.float64)
    V = abs(np.linalg.det(lat))
    B = 2.0 * np.pi * np.linalg.inv(lat).T                        # rows 2 pi b_i
    na = Z.shape[0]
    qfrac = np.atleast_2d(np.asarray(qfrac, dtype=np.float64))
    lam_min = np.linalg.eigvalsh(eps).min()
    gmax = np.sqrt(4.0 * EWALD_ALPHA * EWALD_CUT / lam_min)       # |q+G| bound
    nmax = [int(np.ceil((gmax + np.linalg.norm(B, axis=1).sum()) * np.linalg.norm(lat[i]) / (2 * np.pi))) + 1
            for i in range(3)]
    grid = np.stack(np.meshgrid(*[np.arange(-n, n + 1) for n in nmax], indexing="ij"), -1).reshape(-1, 3)
    out = np.zeros((qfrac.shape[0], lu.shape[-1]), dtype=np.complex128)
    for k in range(qfrac.shape[0]):
        qg = (qfrac[k][None, :] + grid) @ B                        # q + G, Cartesian
        Q = np.einsum("ga,ab,gb->g", qg, eps, qg)
        keep = (Q > 0.0) & (Q / (4.0 * EWALD_ALPHA) <= EWALD_CUT)
        qg, Q = qg[keep], Q[keep]
        damp = np.exp(-Q / (4.0 * EWALD_ALPHA)) / Q
        acc = np.zeros(lu.shape[-1], dtype=np.complex128)
        for t in range(na):
            qZ = qg @ Z[t]                                         # [nG, 3]: (q+G).Z_t
            proj = qZ @ lu[k, 3 * t:3 * t + 3, :]                  # [nG, nbr]
            ph = np.exp(-1j * (qg @ tau[t])) * damp
            acc += ph @ proj
        out[k] = 1j * NAC_EV_A / V * acc
    return out


# ----------------------------------------------------------------------------
# the whole problem on a mesh

class Problem:
    """Tables and transition probabilities of one material on an n^3 mesh
    (equal k and q meshes, so q = k' - k mod 1 lies on the q mesh)."""

    def __init__(self, mat, mesh, mu, window, sigma, omega_min=OMEGA_MIN_DEFAULT):
        self.mat = mat
        self.n = int(mesh)
        self.mu = float(mu)
        self.window = float(window)
        self.sigma = float(sigma)
        self.omega_min = float(omega_min)
        self.nb = int(mat["nwann"])
        self.nbr = 3 * int(mat["natom"])
        self.kfrac = mesh_points(self.n)
        self.nk = self.kfrac.shape[0]
        self.nq = self.nk
        self.ijk = np.rint(self.kfrac * self.n).astype(np.int64)

        # electrons on the whole mesh: energies decide the window (Eq. 1)
        eps_all = np.empty((self.nk, self.nb))
        for s in range(0, self.nk, 65536):
            eps_all[s:s + 65536] = np.linalg.eigvalsh(
                bloch_hamiltonian(mat, self.kfrac[s:s + 65536]))
        self.eps_all = eps_all
        act = np.abs(eps_all - self.mu) <= self.window
        self.active = act
        self.kept = np.nonzero(act.any(1))[0]                 # mesh indices, ascending
        self.kidx_of_mesh = np.full(self.nk, -1, dtype=np.int64)
        self.kidx_of_mesh[self.kept] = np.arange(self.kept.size)
        st_k, st_m = np.nonzero(act[self.kept])
        self.state_k = self.kept[st_k]                        # mesh index of each state
        self.state_kidx = st_k
        self.state_m = st_m
        self.nstates = st_k.size
        self.nact = act[self.kept].sum(1)
        self.state_off = np.concatenate([[0], np.cumsum(self.nact)])

        kk = self.kfrac[self.kept]
        self.eps_kept, self.U_kept = electron_bands(mat, kk)
        self.v_kept = electron_velocities(mat, kk, self.eps_kept, self.U_kept)
        self.eps = self.eps_kept[st_k, st_m]
        self.v_state = self.v_kept[st_k, st_m]

        # phonons on the whole q mesh (Eqs. 3, 5)
        self.hw, self.u = phonon_modes(mat, self.kfrac)
        self.v_ph = phonon_velocities(mat, self.kfrac, self.hw, self.u, self.omega_min)
        self.mode_on = self.hw >= self.omega_min

    # ---- index helpers
    def q_index(self, kmesh_from, kmesh_to):
        return mesh_linear(self.ijk[kmesh_to] - self.ijk[kmesh_from], self.n)

    def neg_q(self, qmesh):
        return mesh_linear(-self.ijk[qmesh], self.n)

    # ---- Eq. 6 for one initial kept k and every kept k'
    def g2_row(self, kidx, brute=False):
        """|g^{s n m}_{k q}|^2 for the kept k number ``kidx`` (initial) and every
        kept k' (final) -> [nK', nbr(s), nb(n), nb(m)]."""
        kmesh = self.kept[kidx]
        k = self.kfrac[kmesh]
        qmesh = self.q_index(np.full(self.kept.size, kmesh), self.kept)
        qs = self.kfrac[qmesh]
        if brute:
            gW = np.stack([g_wannier_brute(self.mat, k, q) for q in qs])
        else:
            gW = g_wannier_factorised(self.mat, k, qs)
        g = g_bloch(self.mat, gW, self.U_kept[kidx][None], self.U_kept,
                    self.u[qmesh], self.hw[qmesh], self.omega_min)
        if self.mat.get("zstar") is not None and self.mat.get("tau") is not None:
            # Eq. 7: the long-range Froehlich part, F_s(q) [U_k' U_k^+]_{nm}
            g = g + self.frohlich_g(self.U_kept[kidx][None], self.U_kept, qmesh)
        return np.abs(g) ** 2, qmesh

    def frohlich_g(self, Uk, Ukq, qmesh):
        """Eq. 7 for initial eigenvectors Uk and final Ukq [..., nb, nb] (columns)
        at mesh q -> [..., nbr, nb(n), nb(m)]: F_s(q) times the overlap
        sum_w conj(Ukq[w, n]) Uk[w, m] (the [U_k' U_k^+]_{nm} of the paper)."""
        if not hasattr(self, "_frohlich"):
            lu = phonon_lengths(self.mat, self.hw, self.omega_min) * self.u   # [nq, x, s]
            self._frohlich = frohlich_factor(self.mat, self.kfrac, lu)
        ov = np.einsum("...wn,...wm->...nm", np.conj(Ukq), Uk)
        return self._frohlich[qmesh][..., :, None, None] * ov[..., None, :, :]

    # ---- Eq. 8
    def tetra_delta(self, i):
        """Delta of Eq. 8 by the analytic tetrahedron method for initial state
        i and every final state j and branch s -> (Dp, Dm) [nstates, nbr],
        1/eV: at the final k_j, the sum over the 24 mesh tetrahedra with
        corner k_j of the corner weight of k_j for
        E(k'') = eps_n(k'') -+ hw_s(k'' - k_i) - eps_i (n the band of j),
        linear in each tetrahedron.  Replaces the Gaussian's delta(E(k_j))."""
        corners, centre = tetra_neighbourhood()
        off = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
        kj = self.ijk[self.state_k]                                   # [M, 3]
        nbr_mesh = mesh_linear(kj[:, None, :] + off[None, :, :], self.n)  # [M, 27]
        eps_n = self.eps_all[nbr_mesh, self.state_m[:, None]]       # [M, 27]
        ki = self.ijk[self.state_k[i]]
        q_mesh = mesh_linear(kj[:, None, :] + off[None, :, :] - ki, self.n)  # [M, 27]
        hw = self.hw[q_mesh]                                          # [M, 27, nbr]
        out = []
        for sign in (-1.0, 1.0):                                      # absorption, emission
            E = eps_n[:, :, None] + sign * hw - self.eps[i]           # [M, 27, nbr]
            Ec = E[:, corners, :]                                     # [M, 24, 4, nbr]
            w = tetra_delta_weights(np.moveaxis(Ec, 2, -1))           # [M, 24, nbr, 4]
            out.append(np.take_along_axis(w, centre[None, :, None, None], axis=3)[..., 0].sum(axis=1))
        return out[0], out[1]

    def triangle_delta(self, i):
        """Delta of Eq. 8 by the triangle method for initial state i and every
        final state j and branch s -> (Dp, Dm) [nstates, nbr], 1/eV: at the
        final k_j, the sum over the 6 triangles of its mesh plane (normal to
        the third mesh axis) with corner k_j of the corner weight of k_j for
        E(k'') = eps_n(k'') -+ hw_s(k'' - k_i) - eps_i, linear in each
        triangle.  Replaces the Gaussian's delta(E(k_j))."""
        corners, centre = triangle_neighbourhood()
        off = np.array([[a, b, 0] for a in (-1, 0, 1) for b in (-1, 0, 1)])
        kj = self.ijk[self.state_k]                                   # [M, 3]
        nbr_mesh = mesh_linear(kj[:, None, :] + off[None, :, :], self.n)  # [M, 9]
        eps_n = self.eps_all[nbr_mesh, self.state_m[:, None]]       # [M, 9]
        ki = self.ijk[self.state_k[i]]
        q_mesh = mesh_linear(kj[:, None, :] + off[None, :, :] - ki, self.n)  # [M, 9]
        hw = self.hw[q_mesh]                                          # [M, 9, nbr]
        out = []
        for sign in (-1.0, 1.0):                                      # absorption, emission
            E = eps_n[:, :, None] + sign * hw - self.eps[i]           # [M, 9, nbr]
            Ec = E[:, corners, :]                                     # [M, 6, 3, nbr]
            w = triangle_delta_weights(np.moveaxis(Ec, 2, -1))        # [M, 6, nbr, 3]
            out.append(np.take_along_axis(w, centre[None, :, None, None], axis=3)[..., 0].sum(axis=1))
        return out[0], out[1]

    def transition_probs(self, T, rows=None, brute=False, delta="gauss"):
        """X^+ and X^- of Eq. 8 for initial states ``rows`` (all when None) and
        every final active state -> (Xp, Xm) of shape [len(rows), nstates, nbr].
        delta: "gauss" (Gaussian of width sigma), "tetra" (analytic
        tetrahedron weights, see tetra_delta) or "triangle" (triangle
        weights, see triangle_delta)."""
        rows = np.arange(self.nstates) if rows is None else np.asarray(rows)
        f, omf = fermi_pair(self.eps, self.mu, T)
        pref = 2.0 * np.pi / (HBAR_EVS * self.nk)
        Xp = np.zeros((rows.size, self.nstates, self.nbr))
        Xm = np.zeros_like(Xp)
        by_k = {}
        for r, i in enumerate(rows):
            by_k.setdefault(int(self.state_kidx[i]), []).append((r, i))
        jk = self.state_kidx                      # kept-k number of each final state
        jm = self.state_m
        for kidx, lst in by_k.items():
            g2, qmesh = self.g2_row(kidx, brute)  # [nK', s, n, m]
            hw = self.hw[qmesh]                   # [nK', s]
            on = self.mode_on[qmesh]
            nq, onq = bose_pair(hw, T)
            for r, i in lst:
                m = self.state_m[i]
                g2j = g2[jk, :, jm, m]             # [nstates, s]
                if delta == "tetra":
                    dp, dm = self.tetra_delta(i)
                elif delta == "triangle":
                    dp, dm = self.triangle_delta(i)
                else:
                    de = (self.eps - self.eps[i])[:, None]      # eps_j - eps_i
                    dp = gaussian_delta(de - hw[jk], self.sigma)
                    dm = gaussian_delta(de + hw[jk], self.sigma)
                occ = f[i] * omf                               # f_i (1 - f_j)
                with np.errstate(invalid="ignore"):
                    xp = pref * g2j * occ[:, None] * nq[jk] * dp
                    xm = pref * g2j * occ[:, None] * onq[jk] * dm
                Xp[r] = np.where(on[jk], xp, 0.0)
                Xm[r] = np.where(on[jk], xm, 0.0)
        return Xp, Xm

    # ---- Eq. 21 (e-ph part)
    def rates_e(self, T, Xp, Xm, rows=None):
        rows = np.arange(self.nstates) if rows is None else np.asarray(rows)
        f, omf = fermi_pair(self.eps, self.mu, T)
        tot = (Xp + Xm).sum(axis=(1, 2))
        return tot / (f[rows] * omf[rows])

    # ---- Eqs. 12, 25 (ph-e part) from the full X^+ array
    def rates_ph(self, T, Xp):
        """W_sq = d_s/(n(1+n)) sum_{mnk} Y, Y = (N_k/N_q) X^+  -> [nq, nbr]."""
        qij = self.q_index(self.state_k[:, None], self.state_k[None, :])   # [i, j]
        acc = _scatter_q(qij, Xp, self.nq)
        n, onp = bose_pair(self.hw, T)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = SPIN_DEG * (self.nk / self.nq) * acc / (n * onp)
        return np.where(self.mode_on, w, 0.0)

    def rates_ph_at(self, T, qmesh_list):
        """W_sq of Eq. 25 (ph-e part) at selected q, each summed over its pairs
        (k, k+q) directly from Eq. 12 -> [len(q), nbr]."""
        f, omf = fermi_pair(self.eps, self.mu, T)
        pref = 2.0 * np.pi / (HBAR_EVS * self.nq)
        out = np.zeros((len(qmesh_list), self.nbr))
        for t, qm in enumerate(qmesh_list):
            hw = self.hw[qm]
            if not self.mode_on[qm].any():
                continue
            n, onp = bose_pair(hw, T)
            acc = np.zeros(self.nbr)
            for kidx, kmesh in enumerate(self.kept):
                kp = mesh_linear(self.ijk[kmesh] + self.ijk[qm], self.n)
                kpidx = self.kidx_of_mesh[kp]
                if kpidx < 0:
                    continue
                gW = g_wannier_factorised(self.mat, self.kfrac[kmesh], self.kfrac[qm][None])[0]
                g = g_bloch(self.mat, gW, self.U_kept[kidx], self.U_kept[kpidx],
                            self.u[qm], hw, self.omega_min)
                g2 = np.abs(g) ** 2                                  # [s, n, m]
                for i in range(self.state_off[kidx], self.state_off[kidx + 1]):
                    for j in range(self.state_off[kpidx], self.state_off[kpidx + 1]):
                        m, nn = self.state_m[i], self.state_m[j]
                        d = gaussian_delta(self.eps[j] - self.eps[i] - hw, self.sigma)
                        acc += pref * g2[:, nn, m] * f[i] * omf[j] * n * d
            with np.errstate(divide="ignore", invalid="ignore"):
                w = SPIN_DEG * acc / (n * onp)
            out[t] = np.where(self.mode_on[qm], w, 0.0)
        return out


def rates_e_rows(mat, mesh, mu, window, sigma, T, rows, omega_min=OMEGA_MIN_DEFAULT, progress=None):
    """W_e of Eq. 21 (e-ph part) for the initial active states ``rows`` (indices
    in the (kept k, band) order of Problem), each against every final active
    state, with the Gaussian delta of Eq. 8.  The same definition as
    Problem.rates_e on Problem.transition_probs, but the phonon modes (Eq. 3)
    are diagonalised only at the q = k' - k that the rows need, so that it
    runs on meshes whose whole-mesh phonon tables would not fit (100^3).
    Returns (W [len(rows)], nstates).  Non-polar materials only.  progress,
    if given, is called as progress(rows done, rows) before the first row and
    after each row (it only reports)."""
    if mat.get("zstar") is not None:
        raise ValueError("rates_e_rows: polar materials need Problem")
    n = int(mesh)
    kfrac = mesh_points(n)
    nk = kfrac.shape[0]
    ijk = np.rint(kfrac * n).astype(np.int64)
    nb = int(mat["nwann"])
    eps_all = np.empty((nk, nb))
    for s in range(0, nk, 32768):
        eps_all[s:s + 32768] = np.linalg.eigvalsh(bloch_hamiltonian(mat, kfrac[s:s + 32768]))
    act = np.abs(eps_all - mu) <= window                     # window per state (section on the workflow)
    kept = np.nonzero(act.any(1))[0]
    st_k, st_m = np.nonzero(act[kept])
    state_k = kept[st_k]
    nstates = st_k.size
    eps = eps_all[state_k, st_m]
    _, U_kept = electron_bands(mat, kfrac[kept])
    f, omf = fermi_pair(eps, mu, T)
    pref = 2.0 * np.pi / (HBAR_EVS * nk)
    out = np.empty(len(rows))
    if progress is not None:
        progress(0, len(rows))
    for r, i in enumerate(np.asarray(rows)):
        kidx = st_k[i]
        kmesh = kept[kidx]
        qmesh = mesh_linear(ijk[kept] - ijk[kmesh], n)       # q of every final kept k'
        hw, u = phonon_modes(mat, kfrac[qmesh])
        gW = g_wannier_factorised(mat, kfrac[kmesh], kfrac[qmesh])
        g = g_bloch(mat, gW, U_kept[kidx][None], U_kept, u, hw, omega_min)
        g2 = np.abs(g) ** 2                                   # [nK', s, n, m]
        on = hw >= omega_min
        nq, onq = bose_pair(hw, T)
        g2j = g2[st_k, :, st_m, st_m[i]]                     # final states j, all s
        de = (eps - eps[i])[:, None]
        dp = gaussian_delta(de - hw[st_k], sigma)
        dm = gaussian_delta(de + hw[st_k], sigma)
        occ = (f[i] * omf)[:, None]
        with np.errstate(invalid="ignore"):
            x = pref * g2j * occ * (nq[st_k] * dp + onq[st_k] * dm)
        x = np.where(on[st_k], x, 0.0)
        out[r] = x.sum() / (f[i] * omf[i])
        if progress is not None:
            progress(r + 1, len(rows))
    return out, nstates


def _scatter_q(qij, vals, nq):
    """sum of vals[i, j, s] into out[q_ij, s] (a plain bin count per branch)."""
    nbr = vals.shape[-1]
    key = qij.reshape(-1)
    out = np.empty((nq, nbr))
    for s in range(nbr):
        out[:, s] = np.bincount(key, weights=vals[..., s].reshape(-1), minlength=nq)
    return out


# ----------------------------------------------------------------------------
# Eqs. 19-27: the coupled BTEs, unified iteration

def default_w_ext(prob, T, gamma0=1.0e12):
    """External (non ph-e) phonon rate per mode, s^-1: gamma0 (hw/hw_max)^2 T/300."""
    hwmax = prob.hw.max()
    w = gamma0 * (prob.hw / hwmax) ** 2 * (T / 300.0)
    return np.where(prob.mode_on, w, 0.0)


def energy_groups(eps, hw_max, sigma):
    """Group label of each state: runs of sorted energies split at gaps wider
    than hw_max + 12 sigma."""
    eps = np.asarray(eps)
    order = np.argsort(eps, kind="stable")
    brk = np.concatenate([[0], np.cumsum(np.diff(eps[order]) > hw_max + 12.0 * sigma)])
    grp = np.empty(eps.size, dtype=np.int64)
    grp[order] = brk
    return grp


def _rel_change(new, old):
    nn = np.linalg.norm(new)
    return np.linalg.norm(new - old) / max(nn, 1e-300)


def iterate(prob, T, Xp, Xm, level=LEVEL_COUPLED, tol=1e-8, maxit=200, w_ext=None, phph=None,
            inner="substitution"):
    """Solve Eq. 19 with the unified scheme: each phonon (outer) iteration
    brings the electrons (inner) to self-consistency with the current phonons.
    ``inner`` = "substitution" iterates the electron equations to tol/10;
    "direct" solves them (with the carrier-number constraints) by one dense
    bordered solve, which reaches the same fixed point where the substitution
    converges slowly (an in-scattering operator with spectral radius near 1).
    ``Xp``/``Xm`` are the full [nstates, nstates, nbr] arrays of Eq. 8.
    ``phph`` = (ifc3, sigma) adds three-phonon scattering (Eq. 26): its RTA
    rate joins W^RTA (``w_ext`` then holds the remaining channels, none when
    None) and Delta F^S = S[F] / W^RTA joins every phonon update; at level
    DRAGLESS the phonons then solve their own BTE F = F0 + Delta F^S[F].
    Returns dict(I, J, F, G, W_e, W_ph, iters, converged)."""
    M, nbr = prob.nstates, prob.nbr
    f, omf = fermi_pair(prob.eps, prob.mu, T)
    ff = f * omf
    W_e = (Xp + Xm).sum(axis=(1, 2)) / ff
    if w_ext is None:
        w_ext = default_w_ext(prob, T) if phph is None else np.zeros((prob.nq, nbr))
    W_phe = prob.rates_ph(T, Xp)
    W_p = W_phe + w_ext                                     # [nq, nbr]
    Mph = None
    if phph is not None:
        W_p = W_p + phph_rates(prob, phph[0], T, phph[1])
        Mph = phph_operator(prob, phph[0], T, phph[1])
    n, onp = bose_pair(prob.hw, T)
    on = prob.mode_on

    v = prob.v_state
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_we = np.where(W_e > 0, 1.0 / W_e, 0.0)
        inv_wp = np.where(on & (W_p > 0), 1.0 / W_p, 0.0)
    I0 = ((prob.eps - prob.mu) / T * inv_we)[:, None] * v      # eV m / K
    J0 = inv_we[:, None] * v                                   # m (per unit charge)
    F0 = (prob.hw / T * inv_wp)[..., None] * prob.v_ph         # eV m / K
    G0 = np.zeros_like(F0)

    qij = prob.q_index(prob.state_k[:, None], prob.state_k[None, :])
    nqij = prob.neg_q(qij)
    # normalised kernels
    with np.errstate(divide="ignore", invalid="ignore"):
        row = np.where(W_e > 0, 1.0 / (ff * W_e), 0.0)
    Kp = Xp * row[:, None, None]
    Km = Xm * row[:, None, None]
    Kself = (Kp + Km).sum(2)                                   # [i, j]
    with np.errstate(divide="ignore", invalid="ignore"):
        ph_norm = np.where(on, SPIN_DEG * (prob.nk / prob.nq) * inv_wp / (n * onp), 0.0)
    w = ff
    grp = energy_groups(prob.eps, prob.hw.max(), prob.sigma)
    ngrp = grp.max() + 1
    wsum = np.bincount(grp, weights=w, minlength=ngrp)

    def project(x):
        out = x.copy()
        for c in range(x.shape[1]):
            mean = np.bincount(grp, weights=w * x[:, c], minlength=ngrp) / wsum
            out[:, c] -= mean[grp]
        return out

    def drag_e(phon):
        """Eq. 23 for fixed phonon responses: sum_{j,s} (-F_{s,q} X^+ + F_{s,-q} X^-)."""
        acc = np.zeros((M, 3))
        for c in range(3):
            acc[:, c] = (-(Kp * phon[qij, :, c]).sum((1, 2))
                         + (Km * phon[nqij, :, c]).sum((1, 2)))
        return acc

    def ph_drag(x, phon0):
        """Eq. 27: phon0 + d_s/(n(1+n)W) sum Y (x_j - x_i), Y = (N_k/N_q) X^+."""
        acc = np.zeros(phon0.shape)
        for c in range(3):
            diff = x[None, :, c] - x[:, None, c]               # x_j - x_i  [i, j]
            acc[..., c] = _scatter_q(qij, Xp * diff[:, :, None], prob.nq)
        return phon0 + ph_norm[..., None] * acc

    def ph_self(phon):
        """Delta F^S of Eq. 26: the three-phonon in-scattering over W^RTA."""
        if Mph is None:
            return 0.0
        S = (Mph @ phon.reshape(-1, 3)).reshape(phon.shape)
        return S * inv_wp[..., None]

    if inner == "direct":
        # x = project(x0 + K x): (1 - K) x + sum_g c_g 1_g = x0 with
        # sum_{i in g} w_i x_i = 0 for every group g
        A = np.zeros((M + ngrp, M + ngrp))
        A[:M, :M] = np.eye(M) - Kself
        for c in range(ngrp):
            A[:M, M + c] = (grp == c)
            A[M + c, :M] = w * (grp == c)

    def solve_e(x0, x):
        """Electron BTE (Eqs. 19, 22) to self-consistency for a fixed drive x0."""
        if inner == "direct":
            rhs = np.zeros((M + ngrp, x0.shape[1]))
            rhs[:M] = x0
            return np.linalg.solve(A, rhs)[:M], 1, True
        for it in range(1, maxit + 1):
            xn = project(x0 + Kself @ x)
            r = _rel_change(xn, x)
            x = xn
            if r < tol * 0.1:
                return x, it, True
        return x, maxit, False

    out = dict(W_e=W_e, W_ph=W_phe, W_p=W_p, I0=I0, J0=J0, F0=F0)
    if level == LEVEL_RTA:
        out.update(I=I0.copy(), J=J0.copy(), F=F0.copy(), G=G0.copy(), iters=0, converged=True)
        return out
    if level == LEVEL_DRAGLESS:
        I, itI, cI = solve_e(I0, I0.copy())
        J, itJ, cJ = solve_e(J0, J0.copy())
        F, itF, cF = F0.copy(), 0, True
        if Mph is not None:
            cF = False
            for itF in range(1, maxit + 1):
                Fn = F0 + ph_self(F)
                r = _rel_change(Fn, F)
                F = Fn
                if r < tol:
                    cF = True
                    break
        out.update(I=I, J=J, F=F, G=G0.copy(), iters=max(itI, itJ, itF), converged=cI and cJ and cF)
        return out

    I, J, F, G = I0.copy(), J0.copy(), F0.copy(), G0.copy()
    converged = False
    it = 0
    for it in range(1, maxit + 1):
        In, _, c1 = solve_e(I0 + drag_e(F), I)
        Jn, _, c2 = solve_e(J0 + drag_e(G), J)
        Fn = ph_drag(In, F0) + ph_self(F)
        Gn = ph_drag(Jn, G0) + ph_self(G)
        r = max(_rel_change(In, I), _rel_change(Jn, J), _rel_change(Fn, F), _rel_change(Gn, G))
        I, J, F, G = In, Jn, Fn, Gn
        if level == LEVEL_PARTIAL:
            converged = c1 and c2
            break
        if r < tol and c1 and c2:
            converged = True
            break
    out.update(I=I, J=J, F=F, G=G, iters=it, converged=converged)
    return out


# ----------------------------------------------------------------------------
# Eqs. 28-31: transport tensors

def transport_tensors(prob, T, I, J, F, G):
    """sigma, sigma*S, alpha_el, kappa0_el, alpha_ph, kappa_ph (SI units) from
    Eqs. 28-30 with 1/N_k and 1/N_q normalisations."""
    V = abs(np.linalg.det(np.asarray(prob.mat["lat"]))) * ANG_M ** 3
    kT = KB_EVK * T * E_CHARGE                              # J
    f, omf = fermi_pair(prob.eps, prob.mu, T)
    ff = f * omf
    v = prob.v_state
    I_si, J_si = I * E_CHARGE, J * E_CHARGE
    F_si, G_si = F * E_CHARGE, G * E_CHARGE
    de = (prob.eps - prob.mu) * E_CHARGE
    ce = SPIN_DEG / (V * kT * prob.nk)
    sigma = ce * E_CHARGE * np.einsum("i,ia,ib->ab", ff, v, J_si)
    sigmaS = ce * E_CHARGE * np.einsum("i,ia,ib->ab", ff, v, -I_si)
    alpha_el = -ce * np.einsum("i,i,ia,ib->ab", de, ff, v, J_si)
    kappa0_el = -ce * np.einsum("i,i,ia,ib->ab", de, ff, v, -I_si)
    n, onp = bose_pair(prob.hw, T)
    wgt = np.where(prob.mode_on, prob.hw * E_CHARGE * n * onp, 0.0)
    cp = 1.0 / (V * kT * prob.nq)
    alpha_ph = cp * np.einsum("qs,qsa,qsb->ab", wgt, prob.v_ph, -G_si)
    kappa_ph = cp * np.einsum("qs,qsa,qsb->ab", wgt, prob.v_ph, F_si)
    return dict(sigma=sigma, sigmaS=sigmaS, alpha_el=alpha_el, kappa0_el=kappa0_el,
                alpha_ph=alpha_ph, kappa_ph=kappa_ph)


def ko_residual(tens, T):
    """Eq. 31: |sigma S - (alpha_el + alpha_ph)/T| / |sigma S| (Frobenius)."""
    d = tens["sigmaS"] - (tens["alpha_el"] + tens["alpha_ph"]) / T
    return np.linalg.norm(d) / max(np.linalg.norm(tens["sigmaS"]), 1e-300)


def ko_enforce(prob, T, I, J, F, G, bisect_steps=200):
    """Kelvin-Onsager enforcement (Eqs. 32-35, section on the coupled BTEs).

    sigma S and alpha are split into diffusion and drag parts (Eq. 32) and I
    into I_diff + I_drag (Eq. 33).  Demanding sigma S_diff[I_diff] =
    alpha_el / T gives I_diff = (eps - mu) / (e T) J (Eq. 34; e = 1 in the
    units of I and J here); the drag part is rescaled by the scalar lambda
    that satisfies sigma S_drag[lambda I_drag] = alpha_ph / T (Eq. 35).
    Reading: the tensor condition is taken in the least-squares sense
    (Frobenius norm), the scalar condition being d/dlambda of
    |sigma S_drag[lambda I_drag] - alpha_ph/T|^2 = 0, whose root is found by
    bisection as the paper says.  Returns (I_ko, lambda, tensors of I_ko)."""
    I_diff = ((prob.eps - prob.mu) / T)[:, None] * J
    I_drag = I - I_diff
    S_drag = transport_tensors(prob, T, I_drag, J, F, G)["sigmaS"]
    target = transport_tensors(prob, T, I, J, F, G)["alpha_ph"] / T
    if not np.any(S_drag):
        raise ValueError("no drag part of sigma S to rescale")

    def cond(lam):
        # half the derivative of the squared residual; increasing in lambda
        return float(np.sum(S_drag * (lam * S_drag - target)))

    lo, hi = 0.0, 2.0
    while cond(lo) > 0:
        lo = 2.0 * lo - 1.0 if lo < 0 else -1.0
    while cond(hi) < 0:
        hi = 2.0 * hi
    for _ in range(bisect_steps):
        mid = 0.5 * (lo + hi)
        if cond(mid) < 0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4e-16 * max(abs(lo), abs(hi), 1.0):
            break
    lam = 0.5 * (lo + hi)
    I_ko = I_diff + lam * I_drag
    return I_ko, lam, transport_tensors(prob, T, I_ko, J, F, G)


# ----------------------------------------------------------------------------
# Three-phonon processes: the vertex of Eq. 13, the transition rates of
# Eq. 14 and the ph-ph part of the phonon RTA rate of Eq. 26.
#
# Readings: the eigendisplacement e_j(Q) of Eq. 13 is exp(2 pi i Q.R_j) times
# the mass-weighted eigenvector column u(Q) of D(Q) (the phase convention of
# Eq. 3; no atom-position phase), and the explicit 1/sqrt(m m m) turns the
# three columns into u/sqrt(M).  The occupations of Eq. 14 are those of the
# modes s'q' and s''q'' (the printed branch labels are garbled).  The delta
# is the Gaussian of standard deviation sigma in hbar*omega, and modes below
# omega_min take no part (as in the e-ph path).

# hbar^5 e^3 / (amu^3 Angstrom^6): |V|^2 in eV^2 / (A^6 amu^3), energies in eV
# and the delta in 1/eV give W of Eq. 14 in 1/s
C_PHPH = HBAR_EVS ** 5 * E_CHARGE ** 3 / (AMU_KG ** 3 * ANG_M ** 6)


def eigendisplacements(mat, u):
    """u_{x,s} / sqrt(M_x) for every column of u (..., nbr, nbr)."""
    mx = np.repeat(np.asarray(mat["mass"], dtype=np.float64), 3)
    return u / np.sqrt(mx)[:, None]


def ifc3_matrix(ifc3):
    """Psi entries as [n_entries][x_i][x_j][x_k] with x = 3 * atom + Cartesian."""
    rj, rk, psi = ifc3
    n, na = psi.shape[0], psi.shape[1]
    return psi.transpose(0, 1, 4, 2, 5, 3, 6).reshape(n, 3 * na, 3 * na, 3 * na)


def phph_vertex(ifc3, q2, q3, E1, E2, E3):
    """Eq. 13 for one first leg and many second/third legs:
    V[n][s1][s2][s3] = sum_{x_i, (R_j, x_j), (R_k, x_k)} Psi
        E1[x_i, s1] exp(2 pi i q2_n.R_j) E2_n[x_j, s2] exp(2 pi i q3_n.R_k) E3_n[x_k, s3],
    where the first leg's atom sits in the central cell (its phase is 1),
    q2, q3 are [n][3] fractional wave vectors of the second and third legs
    (the three legs' wave vectors sum to a reciprocal lattice vector) and
    E* are eigendisplacement columns u / sqrt(M)."""
    rj, rk, _ = ifc3
    P = ifc3_matrix(ifc3)
    nent, nbr = P.shape[0], P.shape[1]
    ph = np.exp(2j * np.pi * (np.atleast_2d(q2) @ rj.T.astype(np.float64)
                              + np.atleast_2d(q3) @ rk.T.astype(np.float64)))
    A = (ph @ P.reshape(nent, -1)).reshape(-1, nbr, nbr, nbr)
    return np.einsum("nabc,as,nbt,ncu->nstu", A, E1, E2, E3, optimize=True)


def phph_rates(prob, ifc3, T, sigma, rows=None, parts=False):
    """Eq. 26's three-phonon part W_sq = sum_{s'q's''} (W+ + W-/2) / (n (1 + n))
    with W+- of Eq. 14 (absorption q + q' -> q'' = q + q', decay
    q -> q' + q'' with q'' = q - q'), each vertex from Eq. 13 with the second
    leg at +-q' and the third at -q''.  Returns W [len(rows)][nbr] in 1/s; with
    parts=True also the bare sums S+- = sum |V+-|^2 delta / (E E' E'') over
    the same terms."""
    n = prob.n
    nq, nbr = prob.nq, prob.nbr
    E = eigendisplacements(prob.mat, prob.u)
    nB, onB = bose_pair(prob.hw, T)
    on = prob.mode_on
    pref = np.pi / (4.0 * nq) * C_PHPH
    rows = np.arange(nq) if rows is None else np.asarray(rows)
    W = np.zeros((rows.size, nbr))
    S = {+1: 0.0, -1: 0.0}
    allq = np.arange(nq)
    with np.errstate(divide="ignore", invalid="ignore"):
        for r, q in enumerate(rows):
            for sign in (+1, -1):
                leg2 = mesh_linear(sign * prob.ijk[allq], n)                 # +-q'
                qpp = mesh_linear(prob.ijk[q] + sign * prob.ijk[allq], n)    # q''
                leg3 = mesh_linear(-prob.ijk[qpp], n)                        # -q''
                V = phph_vertex(ifc3, prob.kfrac[leg2], prob.kfrac[leg3], E[q], E[leg2], E[leg3])
                e1 = prob.hw[q][None, :, None, None]
                e2 = prob.hw[allq][:, None, :, None]
                e3 = prob.hw[qpp][:, None, None, :]
                mask = (on[q][None, :, None, None] & on[allq][:, None, :, None]
                        & on[qpp][:, None, None, :])
                bare = np.abs(V) ** 2 * gaussian_delta(e1 + sign * e2 - e3, sigma) / (e1 * e2 * e3)
                bare = np.where(mask, bare, 0.0)
                S[sign] += bare.sum()
                n1, on1 = nB[q][None, :, None, None], onB[q][None, :, None, None]
                n2, on2 = nB[allq][:, None, :, None], onB[allq][:, None, :, None]
                n3 = nB[qpp][:, None, None, :]
                if sign > 0:
                    w = pref * bare * on1 * on2 * n3                 # Eq. 14, +
                else:
                    w = 0.5 * pref * bare * on1 * n2 * n3            # Eq. 14, - (half in Eq. 26)
                w = np.where(mask, w, 0.0)
                W[r] += w.sum(axis=(0, 2, 3)) / np.where(on[q], nB[q] * onB[q], 1.0)
    if parts:
        return W, S[+1], S[-1]
    return W


def phph_operator(prob, ifc3, T, sigma):
    """The in-scattering of phph_inscatter as a dense matrix M [nq*nbr][nq*nbr]
    (S = M F for each Cartesian column), assembled from the same W+- terms,
    for small meshes."""
    n = prob.n
    nq, nbr = prob.nq, prob.nbr
    E = eigendisplacements(prob.mat, prob.u)
    nB, onB = bose_pair(prob.hw, T)
    on = prob.mode_on
    pref = np.pi / (4.0 * nq) * C_PHPH
    M = np.zeros((nq, nbr, nq, nbr))
    allq = np.arange(nq)
    with np.errstate(divide="ignore", invalid="ignore"):
        for q in range(nq):
            for sign in (+1, -1):
                leg2 = mesh_linear(sign * prob.ijk[allq], n)
                qpp = mesh_linear(prob.ijk[q] + sign * prob.ijk[allq], n)
                leg3 = mesh_linear(-prob.ijk[qpp], n)
                V = phph_vertex(ifc3, prob.kfrac[leg2], prob.kfrac[leg3], E[q], E[leg2], E[leg3])
                e1 = prob.hw[q][None, :, None, None]
                e2 = prob.hw[allq][:, None, :, None]
                e3 = prob.hw[qpp][:, None, None, :]
                mask = (on[q][None, :, None, None] & on[allq][:, None, :, None]
                        & on[qpp][:, None, None, :])
                bare = np.abs(V) ** 2 * gaussian_delta(e1 + sign * e2 - e3, sigma) / (e1 * e2 * e3)
                on1 = onB[q][None, :, None, None]
                n2, on2 = nB[allq][:, None, :, None], onB[allq][:, None, :, None]
                n3 = nB[qpp][:, None, None, :]
                if sign > 0:
                    w = np.where(mask, pref * bare * on1 * on2 * n3, 0.0)          # W+ (F'' - F')
                else:
                    w = np.where(mask, 0.5 * pref * bare * on1 * n2 * n3, 0.0)     # W-/2 (F'' + F')
                M[q][:, qpp, :] += w.sum(axis=2).transpose(1, 0, 2)
                M[q][:, allq, :] += -sign * w.sum(axis=3).transpose(1, 0, 2)
            M[q] /= np.where(on[q], nB[q] * onB[q], 1.0)[:, None, None]
    return M.reshape(nq * nbr, nq * nbr)


def phph_inscatter(prob, ifc3, T, sigma, F, rows=None):
    """The three-phonon in-scattering of a phonon deviation field F [nq][nbr][3]
    (the self term of Eq. 26 before its division by the RTA rate):
    S_sq = sum_{s'q's''} [W+ (F_s''q'' - F_s'q') + W-/2 (F_s''q'' + F_s'q')] / (n (1 + n)),
    W+ for q'' = q + q', W- for q'' = q - q' (Eq. 14), terms as in phph_rates."""
    n = prob.n
    nq, nbr = prob.nq, prob.nbr
    E = eigendisplacements(prob.mat, prob.u)
    nB, onB = bose_pair(prob.hw, T)
    on = prob.mode_on
    pref = np.pi / (4.0 * nq) * C_PHPH
    rows = np.arange(nq) if rows is None else np.asarray(rows)
    out = np.zeros((rows.size, nbr, 3))
    allq = np.arange(nq)
    with np.errstate(divide="ignore", invalid="ignore"):
        for r, q in enumerate(rows):
            for sign in (+1, -1):
                leg2 = mesh_linear(sign * prob.ijk[allq], n)
                qpp = mesh_linear(prob.ijk[q] + sign * prob.ijk[allq], n)
                leg3 = mesh_linear(-prob.ijk[qpp], n)
                V = phph_vertex(ifc3, prob.kfrac[leg2], prob.kfrac[leg3], E[q], E[leg2], E[leg3])
                e1 = prob.hw[q][None, :, None, None]
                e2 = prob.hw[allq][:, None, :, None]
                e3 = prob.hw[qpp][:, None, None, :]
                mask = (on[q][None, :, None, None] & on[allq][:, None, :, None]
                        & on[qpp][:, None, None, :])
                bare = np.abs(V) ** 2 * gaussian_delta(e1 + sign * e2 - e3, sigma) / (e1 * e2 * e3)
                on1 = onB[q][None, :, None, None]
                n2, on2 = nB[allq][:, None, :, None], onB[allq][:, None, :, None]
                n3 = nB[qpp][:, None, None, :]
                if sign > 0:
                    w = np.where(mask, pref * bare * on1 * on2 * n3, 0.0)          # W+
                    # sum_{q', s', s''} W+ (F_{s''q''} - F_{s'q'})
                    out[r] += (np.einsum("nsab,nbc->sc", w, F[qpp])
                               - np.einsum("nsab,nac->sc", w, F[allq]))
                else:
                    w = np.where(mask, 0.5 * pref * bare * on1 * n2 * n3, 0.0)     # W-/2
                    out[r] += (np.einsum("nsab,nbc->sc", w, F[qpp])
                               + np.einsum("nsab,nac->sc", w, F[allq]))
            out[r] /= np.where(on[q], nB[q] * onB[q], 1.0)[:, None]
    return out
