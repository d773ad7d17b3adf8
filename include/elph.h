/*
 * elph.h -- C ABI of libelph: the electron-phonon transition-probability path
 * (Wannier-interpolated e-ph vertices, transition probabilities, RTA
 * scattering rates and the coupled e-ph drag iteration) on AMD MI355X.
 *
 * Physics follows "The elphbolt ab initio solver for the coupled
 * electron-phonon Boltzmann transport equations": section "Electrons,
 * phonons, and interactions" (Eqs. 1-3, 5, 6, 8, 12), section "Coupled and
 * decoupled BTEs" (Eqs. 17-27) and section "Transport coefficients"
 * (Eqs. 28-31).  Equation numbers count displayed equations in order.
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: energies eV, lengths Angstrom, masses amu, temperatures K, rates
 * 1/s, velocities m/s.  Complex numbers are interleaved (re, im) doubles.
 * All arrays are row-major.
 *
 * Meshes: the k mesh and the q mesh are the same Gamma-centred
 * N0 x N1 x N2 mesh, k = (a/N0, b/N1, c/N2), linear index (a*N1 + b)*N2 + c.
 * q = k' - k is reduced modulo the mesh.
 *
 * Active states (the transport window): state (k, m) is active when
 * |eps_mk - mu| <= window; k is "kept" when any band is active.  Active
 * states are numbered 0..nstates-1 in increasing mesh index of k, then
 * increasing band index m (bands ascending in energy).
 *
 * Term store: transition probabilities are returned as dense arrays
 * X[i][j][s] over initial active state i, final active state j and phonon
 * branch s (0..3*natom-1, ascending in energy at q = k_j - k_i).  Branches
 * with hbar*omega < omega_min (the acoustic modes at Gamma) carry zeros.
 *
 * Pointers: unless stated otherwise, output arrays are DEVICE pointers
 * allocated by the caller (for example the data pointer of a GPU tensor),
 * written asynchronously on the context's stream.  Input descriptions
 * (elph_wannier, elph_params) are host memory, copied at elph_create; the
 * caller keeps ownership of everything it passes.
 *
 * Errors: every call returns an elph_status.  On error, outputs are
 * unspecified and the context stays usable, except after ELPH_EHIP (a HIP
 * runtime failure), after which only elph_destroy is allowed.
 * elph_last_error() returns a message for the last failing call, valid
 * until the next call on that context.  A context is not thread-safe;
 * separate contexts are independent.
 */
#ifndef ELPH_H
#define ELPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct elph_ctx_s* elph_ctx;
typedef int32_t elph_status;

enum {
  ELPH_OK = 0,
  ELPH_EINVAL = 1,   /* malformed input or argument */
  ELPH_ENOMEM = 2,   /* device or host allocation failed */
  ELPH_EHIP = 3,     /* HIP runtime error; the context is unusable */
  ELPH_ENOCONV = 4,  /* iteration did not reach the tolerance; results are the last iterate */
  ELPH_ESTATE = 5    /* call not valid in the context's current state */
};

/* Arithmetic of the two Wannier contractions (Eq. 6).  Eigensolves and the
 * thermal/delta factors and all rate accumulations stay FP64 in every form. */
enum {
  ELPH_FP64 = 0,     /* FP64 MFMA contractions (plain path) */
  ELPH_FP32 = 1,     /* FP32 MFMA contractions, FP32 accumulation */
  ELPH_BF16X3 = 2,   /* BF16 split a = hi + lo, 3 products, FP32 accumulation */
  ELPH_BF16X6 = 3,   /* BF16 split a = hi + mid + lo, 6 products, FP32 accumulation */
  ELPH_FP16X3 = 4    /* FP16 split a = hi + lo (22 significant bits), 3 products, FP32
                        accumulation; operands scaled by powers of two derived from the
                        largest Wannier weight and |g| so that both parts stay normal
                        FP16 numbers (exact inverse scaling in the epilogues) */
};

/* Energy-conserving delta of Eq. 8 (see elph_set_delta). */
enum {
  ELPH_DELTA_GAUSS = 0,    /* Gaussian of standard deviation sigma (elph_create's sigma) */
  ELPH_DELTA_TETRA = 1,    /* analytic tetrahedron weights on the mesh (no smearing parameter) */
  ELPH_DELTA_TRIANGLE = 2  /* triangle weights on the mesh planes (no smearing parameter) */
};

/* Solution levels of the coupled BTEs (section "Coupled and decoupled BTEs"). */
enum {
  ELPH_LEVEL_RTA = 0,       /* Eqs. 20, 24 only */
  ELPH_LEVEL_PARTIAL = 1,   /* first phonon iteration of the unified scheme */
  ELPH_LEVEL_DRAGLESS = 2,  /* self terms only (Eq. 22), no drag */
  ELPH_LEVEL_COUPLED = 3    /* full dragged solution (Eq. 19) */
};

/* Wannier-space inputs (section "Electrons, phonons, and interactions" and
 * the workflow section: Hamiltonian, dynamical matrix and e-ph vertex in the
 * Wannier basis with their real-space cell lists and weights). */
typedef struct {
  int32_t nwann;          /* Wannier bands nb, 1..16 */
  int32_t natom;          /* atoms per cell; branches nbr = 3*natom, 1..16 */
  int32_t nre, nrp;       /* number of electron / phonon cell vectors */
  const int32_t* re;      /* [nre][3] integer cell vectors R_e (lattice units) */
  const int32_t* rp;      /* [nrp][3] integer cell vectors R_p */
  const double* wre;      /* [nre] weights of R_e, or NULL for all 1 */
  const double* wrp;      /* [nrp] weights of R_p, or NULL for all 1 */
  const double* lat;      /* [3][3] lattice vectors as rows, Angstrom */
  const double* mass;     /* [natom] amu */
  const double* h_r;      /* [nre][nb][nb] complex, eV (Eq. 1); H(-R) = H(R)^dagger */
  const double* d_r;      /* [nrp][nbr][nbr] real, mass-weighted eV/(A^2 amu) (Eq. 3) */
  const double* g_r;      /* [nre][nrp][nbr][nb][nb] complex, eV/A (Eq. 6);
                             index order [..][x = 3*atom + cart][final n'][initial m'] */
} elph_wannier;

typedef struct {
  int32_t mesh[3];        /* N0, N1, N2 of the common k and q mesh */
  int32_t precision;      /* ELPH_FP64 / ELPH_FP32 / ELPH_BF16X3 / ELPH_BF16X6 / ELPH_FP16X3 */
  double mu_eV;           /* chemical potential */
  double window_eV;       /* half-width of the transport window; INFINITY keeps all */
  double sigma_eV;        /* standard deviation of the Gaussian delta (Eq. 8) */
  double omega_min_eV;    /* modes below this are dropped; 0 selects 1e-4 eV */
} elph_params;

typedef struct {
  int64_t nk;             /* mesh points (= nq) */
  int64_t nkept;          /* kept k */
  int64_t nstates;        /* active states */
  int32_t nwann, nbr;
  int64_t nterms;         /* nstates * nstates * nbr: length of one term array */
  double hw_max_eV;       /* largest phonon energy on the mesh */
  int32_t ngroups;        /* energy groups of active states (see elph_iterate); 0 until it ran */
  int32_t reserved;
} elph_sizes_t;

/* Create a context on a HIP stream (hipStream_t passed as void*, NULL = the
 * default stream).  Validates the inputs: finite values, nb and nbr in 1..16,
 * lattice Hermiticity H(-R) = H(R)^dagger, real D(-R) = D(R)^T, and the
 * acoustic sum rule sum_R D(R) t = 0 on mass-weighted translations t
 * (relative tolerance 1e-8); violations return ELPH_EINVAL.  Copies all
 * inputs to the device.  Tables are built lazily by the first call needing
 * them. */
elph_status elph_create(const elph_wannier* w, const elph_params* p, void* hip_stream,
                        elph_ctx* out);

/* Free every device and host resource of the context; NULL is a no-op. */
void elph_destroy(elph_ctx ctx);

/* Message of the last failing call on ctx ("" if none); ctx may be NULL for
 * errors of elph_create. */
const char* elph_last_error(elph_ctx ctx);

/* what = ELPH_RESET_ALL: drop every derived table, contraction operand, the
 * vertex store and the cached rates; their device blocks stay in the
 * context's pool and are reused by later allocations of the same size.
 * ELPH_RESET_STORE: only mark the vertex store (and the cached rates) stale
 * so that the next rate call recomputes the vertices.  ELPH_RESET_TRIM: as
 * ELPH_RESET_ALL, then return the pool's memory to the device.  The next
 * call rebuilds what it needs (inputs stay on the device).  Used to time the
 * path and to release memory.  Do not reset a context that belongs to a live
 * batch. */
enum { ELPH_RESET_ALL = 0, ELPH_RESET_STORE = 1, ELPH_RESET_TRIM = 2 };
elph_status elph_reset(elph_ctx ctx, int32_t what);

/* Kernel timing with HIP events recorded on the context's stream around
 * the table build, the step-1 contraction (with its epilogue), the step-2
 * contraction (FP64/FP32 forms: the kernel fused with the rate epilogue;
 * BF16 split forms: the GEMM kernel alone, its per-q epilogue follows) and
 * the whole iteration.  enable = 1 turns recording on
 * for later calls, 0 turns it off.  ms (host, may be NULL) receives the
 * durations of the most recent recorded launches in milliseconds:
 * [tables, step1, step2, iterate] (-1 where nothing was recorded);
 * synchronises the stream when ms is given. */
elph_status elph_timing(elph_ctx ctx, int32_t enable, double* ms);

/* With timing on (elph_timing): the duration in milliseconds of the most
 * recent tetrahedron-delta scaling of a vertex store (k_tetra_scale,
 * elph_set_delta) or Froehlich table (k_frohlich, elph_set_polar), whichever
 * ran last; -1 when none was recorded.  ms: one host double.  Synchronises
 * the stream. */
elph_status elph_timing_extra(elph_ctx ctx, double* ms);

/* Save the context's temperature-independent state to a file: its tables
 * (active states, energies, velocities, phonon energies and velocities,
 * eigenvectors of the kept k) and its vertex store B+/- of Eq. 8 with the
 * error codes of the GEMM forms, so that temperature and carrier sweeps can
 * resume without recomputing the vertices (the workflow section stores
 * vertices and rates for reuse).  The file also holds the sizes, parameters
 * and a hash of the inputs, and a checksum.  ESTATE without a vertex store,
 * EINVAL when the file cannot be written.  Synchronises the stream. */
elph_status elph_save(elph_ctx ctx, const char* path);

/* Restore a state saved by elph_save into a context created from the same
 * inputs and parameters (same sizes, mesh, mu, window, sigma, omega_min,
 * precision form, delta method and polar terms, checked against the file):
 * the tables are rebuilt and must equal the saved ones bit for bit, then the
 * vertex store and its codes are taken from the file and the cached rates
 * are dropped; later calls give bitwise the results an uninterrupted context
 * would.  EINVAL for a missing, truncated or corrupt file, another material
 * or parameters, or tables that differ (another library version or device);
 * the store is then left invalid.  Synchronises the stream. */
elph_status elph_load(elph_ctx ctx, const char* path);

/* Device-memory budget of the context in bytes (inputs, tables, operands,
 * vertex store, work buffers and released blocks kept for reuse; 0 = none,
 * the default).  Setting a budget first returns the released blocks to the
 * device.  An allocation beyond it fails like an exhausted device:
 * the call returns ELPH_ENOMEM, and after every ELPH_ENOMEM the context
 * releases its derived tables, operands, store and work buffers (the inputs
 * stay) and remains usable (a batch built over it must be created again).
 * EINVAL for a negative budget. */
elph_status elph_set_memory_limit(elph_ctx ctx, int64_t bytes);

/* Largest FP32 output buffer of a GEMM form's contraction in bytes (default
 * 2 GiB, at least 1 MiB): the step-1 rows and the step-2 output [i][j][x]
 * are produced in chunks of initial states that fit it (step 2: whole kept k
 * and at least 16 states per chunk).  Results do not depend on it; a smaller
 * chunk lowers peak memory at the cost of more launches.  Applies to later
 * vertex evaluations.  EINVAL below 1 MiB. */
elph_status elph_set_gemm_chunk(elph_ctx ctx, int64_t bytes);

/* Bytes of device memory the context holds (live and kept for reuse). */
elph_status elph_memory_held(elph_ctx ctx, int64_t* bytes);

/* FP64 refinement of ill-conditioned vertices in the GEMM forms (FP32 and
 * the BF16 / FP16 splits; Eq. 6 evaluated as FP32-accumulated MFMA sums).
 * A vertex component is a sum of N_Rp * nb products accumulated with an
 * error of about u times the root-sum-square of those products plus v times
 * the component's own magnitude (FP32 partial sums; u = 1.2e-7, v = 1e-7 for
 * FP32, FP16x3 and BF16x6, u = 6e-6, v = 2e-6 for BF16x3); where |g| is far
 * below that scale (a near-cancellation) |g|^2 is only accurate to a few
 * digits.  With the refinement on, the vertex store of a GEMM form keeps for
 * every term a log-coded estimate of the relative error of its |g|^2, and
 * every rate reduction (elph_scatt_rates, elph_iterate) sums each term's
 * contribution times its estimate: for a rate (W_e of Eq. 21 or a mode of
 * Eq. 25) whose estimated relative error exceeds theta, the terms that carry
 * at least theta/8 of the rate are recomputed in FP64 (the
 * same contraction with FP64 MFMA step-1 rows of their initial states),
 * written back to the store as exact, and the affected rates reduced again.
 * theta: default 2e-6; 0 turns the refinement off (the stored terms keep the
 * form's plain accuracy).  Applies with the Gaussian delta and without a
 * screen's tile mask; other evaluations keep the plain form.  Marks the
 * cached rates stale.  EINVAL for a negative or non-finite theta. */
elph_status elph_set_refine(elph_ctx ctx, double theta);

/* Counters of the last refinement (host int64[8], may be NULL): rates
 * flagged (W_e rows, phonon modes), pairs (i, j) recomputed in FP64, their
 * distinct initial states, their distinct wave vectors, pairs beyond the
 * per-call capacity of 4194304, rows and modes still above theta after it.
 * ms (host, may be NULL): duration of the refinement with timing on (-1:
 * none recorded).  Synchronises the stream. */
elph_status elph_refine_info(elph_ctx ctx, int64_t* stats, double* ms);

/* The estimates themselves: rel_err [nterms] device FP64, the relative error
 * estimate of every stored |g|^2 in the term-store layout (0 for terms
 * recomputed in FP64; estimates are coded to within a factor 2^(1/6)).
 * ESTATE unless the context holds the store of a GEMM form computed with the
 * refinement on.  Synchronises the stream. */
elph_status elph_refine_estimates(elph_ctx ctx, double* rel_err);

/* Build the electron and phonon tables if needed (Eqs. 1-3, 5 and the
 * window) and report sizes; synchronises the stream. */
elph_status elph_sizes(elph_ctx ctx, elph_sizes_t* out);

/* Copy tables to caller device buffers (any pointer may be NULL to skip):
 * state_k [nstates] mesh index, state_m [nstates] band, eps [nstates] eV,
 * vel [nstates][3] m/s (Eq. 2, averaged over degenerate groups),
 * hw [nk][nbr] eV and vph [nk][nbr][3] m/s (Eq. 5, zero below omega_min). */
elph_status elph_tables(elph_ctx ctx, int32_t* state_k, int32_t* state_m, double* eps,
                        double* vel, double* hw, double* vph);

/* Eq. 6 for arbitrary mesh pairs (k, q), all bands and branches:
 * kidx, qidx [npairs] device int32 mesh indices; g_out [npairs][nbr][nb][nb]
 * complex = g^{s n m}_{k q} with n the final band at k+q and m the initial
 * band at k, eV.  The result depends on the eigenvector gauge; |g|^2 and
 * sums over degenerate groups do not.  Branches below omega_min give 0. */
elph_status elph_interp_g(elph_ctx ctx, int64_t npairs, const int32_t* kidx,
                          const int32_t* qidx, double* g_out);

/* elph_interp_g for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, layout and result, but no device allocation, no free and
 * no synchronisation; the work is queued on the context's stream.  Its work
 * buffers (phases, H(k), eigenvectors of k, k+q and q, the two Wannier
 * stages of Eq. 6) live in one static device array of 64 MiB per GPU,
 * resident until the process ends, and pairs are processed in chunks that
 * fit it (about 50 pairs per chunk for 8 bands, 2 atoms and 203 R_p; 2 for
 * 16 bands, 5 atoms and 389 R_p).  Every call on a GPU shares that array:
 * calls that overlap on one GPU (two streams, two threads) race and must be
 * serialised by the caller; nothing in it needs to start at zero.  The first
 * call on a device must have that device current (ESTATE otherwise).
 * EINVAL when one pair needs more work space than the array holds
 * (nbr * N_Rp * nb^2 * 16 bytes dominate) or for an invalid pair list. */
elph_status elph_interp_g_noalloc(elph_ctx ctx, int64_t npairs, const int32_t* kidx,
                                  const int32_t* qidx, double* g_out);

/* Polar materials.  Eq. 4: the non-analytic dipole-dipole term
 * (e^2 / (eps_0 V)) (q.Z_t)_a (q.Z_t')_b / (q.eps_inf.q) / sqrt(m_t m_t') is
 * added to D(q) (and its gradient to the velocities of Eq. 5), with
 * (q.Z_t)_b = sum_a q_a Z_t[a][b] and q the Cartesian image of the mesh
 * point nearest Gamma (averaged over the two images of a fractional
 * coordinate of exactly 1/2); nothing is added at Gamma.  Eq. 7 (when tau
 * is given): the long-range Froehlich vertex F_s(q) [U_k' U_k^+]_{nm} is
 * added to g of Eq. 6 (store, rates, iteration and elph_interp_g), with
 * F_s(q) = i (e^2 / (eps_0 V)) sum_t sum_{G != -q} ((q+G).Z_t.l u_t,s)
 * / ((q+G).eps_inf.(q+G)) exp(-i (q+G).r_t) exp(-(q+G).eps_inf.(q+G) / (4 alpha)),
 * alpha = 1 Bohr^-2, summed over every G with (q+G).eps_inf.(q+G)/(4 alpha)
 * <= 40, and [U_k' U_k^+]_{nm} the overlap of the two states' eigenvectors
 * in the Wannier basis.  zstar [natom][3][3] (units of e), eps_inf [3][3]
 * (symmetric positive definite) and tau [natom][3] (Cartesian atom
 * positions, Angstrom; NULL: Eq. 4 only) are host arrays, copied;
 * zstar = NULL removes both terms.  Drops every derived table and the
 * vertex store (as ELPH_RESET_ALL).  EINVAL for non-finite input or an
 * eps_inf that is not symmetric positive definite. */
elph_status elph_set_polar(elph_ctx ctx, const double* zstar, const double* eps_inf, const double* tau);

/* Three-phonon processes (Eqs. 13, 14 and the three-phonon part of Eq. 26).
 * Third-order force constants: n entries, entry e holding
 * Psi(0 t_i a, rj_e t_j b, rk_e t_k c) in eV/Angstrom^3 for the atom in the
 * central cell, the atoms in cells rj_e and rk_e (integer lattice vectors,
 * host int32 [n][3]) and Cartesian directions (a, b, c); psi is a host array
 * [n][natom][natom][natom][3][3][3] (t_i, t_j, t_k, a, b, c), copied.  At
 * most 256 distinct rj and 4 atoms.  n = 0 or psi = NULL removes them.
 * EINVAL for non-finite input.  Nothing else is changed. */
elph_status elph_set_ifc3(elph_ctx ctx, int32_t n, const int32_t* rj, const int32_t* rk, const double* psi);

/* |V-(q s, q' s', q'' s'')|^2 of Eq. 13, q'' = q - q', for npairs mesh
 * pairs (q[p], qp[p]) (device int32 mesh indexes), into V2 (device FP64
 * [npairs][nbr(s)][nbr(s')][nbr(s'')], eV^2 / (Angstrom^6 amu^3)), with the
 * second leg at -q', the third at -q'' and the eigendisplacements u / sqrt(M)
 * of the context's phonon tables; a mode below omega_min contributes a zero
 * eigendisplacement.  |V+(q, -q', q'')|^2 is the same number.  A pair with
 * an index outside the mesh gets NaN.  ESTATE without force constants. */
elph_status elph_phph_vertex(elph_ctx ctx, int64_t npairs, const int32_t* q, const int32_t* qp, double* V2);

/* The three-phonon RTA rate of every mode at T (the ph-ph bracket of Eq. 26
 * divided by n (1 + n)):
 *   W_sq = sum_{s'q's''} (W+ + W-/2) / (n_sq (1 + n_sq)),
 * W+ = (pi hbar / (4 N_q)) |V+|^2 / (w w' w'') (n + 1)(n' + 1) n'' delta(w + w' - w'')
 * for q + q' -> q'' = q + q', and W- the same with n' in place of n' + 1 and
 * delta(w - w' - w'') for q -> q' + q'' (Eq. 14), delta the Gaussian of
 * standard deviation sigma_eV in hbar w; modes below omega_min take no
 * part.  W_ph: device FP64 [Nq][nbr], 1/s; it can be passed to
 * elph_iterate as W_ph_ext.  Synchronous.  With timing on, the row kernel
 * (the pair sums) is reported in the step2 slot of elph_timing.  ESTATE
 * without force constants, EINVAL for T or sigma not positive. */
elph_status elph_phph_rates(elph_ctx ctx, double T_K, double sigma_eV, double* W_ph);

/* The three-phonon in-scattering of a phonon deviation field (the self term
 * of Eq. 26 before its division by the RTA rate):
 *   S_sq = sum_{s'q's''} [W+ (F_s''q'' - F_s'q') + W-/2 (F_s''q'' + F_s'q')] / (n_sq (1 + n_sq))
 * with W+- as in elph_phph_rates (q'' = q + q' for W+, q - q' for W-), so
 * that Delta F^S = S / W^RTA.  F and S: device FP64 [Nq][nbr][3] (S in
 * units of F times 1/s; zero for modes below omega_min).  Synchronous.
 * ESTATE without force constants, EINVAL for T or sigma not positive or F
 * null. */
elph_status elph_phph_inscatter(elph_ctx ctx, double T_K, double sigma_eV, const double* F, double* S);

/* Three-phonon processes in elph_iterate (Eq. 26): with sigma_eV > 0 (the
 * Gaussian width of elph_phph_rates) every later elph_iterate adds the
 * three-phonon RTA rate to the phonons' W^RTA (W_ph_ext then supplies the
 * remaining channels; NULL means none instead of the model rate) and
 * Delta F^S = S[F] / W^RTA (elph_phph_inscatter, for F and G) to every phonon
 * update of levels PARTIAL and COUPLED; at level DRAGLESS the phonons then
 * solve their own BTE F = F0 + Delta F^S[F] (G = 0) to tol.  sigma_eV = 0
 * turns this off (the default).  Needs force constants (elph_set_ifc3) at
 * iterate time (ESTATE there).  EINVAL for a negative or non-finite sigma. */
elph_status elph_set_phph(elph_ctx ctx, double sigma_eV);

/* Select the energy-conserving delta of Eq. 8 for this context's later
 * vertex stores (the paper offers the triangle and the analytic
 * tetrahedron methods beside smearing; section on the program's workflow).
 * ELPH_DELTA_TETRA: every mesh cell is split into six tetrahedra along its
 * main diagonal, E(k'') = eps_n(k'') -+ hbar omega_s(k'' - k) - eps_m(k)
 * (bands and branches by index) is interpolated linearly in each, and the
 * delta at the final k' becomes the sum, over the 24 tetrahedra with corner
 * k', of the integral of delta(E) times the barycentric coordinate of k'
 * (mesh-cell units, 1/eV).  ELPH_DELTA_TRIANGLE: the same on the mesh planes
 * normal to the third mesh axis (a 2-D mesh has one point along it): every
 * cell of a plane is split into two triangles along its main diagonal and
 * the delta at k' is the sum over the 6 triangles of its plane with corner
 * k' (a 3-D sum then adds the planes as mesh points).  Marks the vertex
 * store and the cached rates stale.  EINVAL for an unknown method.  The batch and screened calls
 * accept only ELPH_DELTA_GAUSS. */
elph_status elph_set_delta(elph_ctx ctx, int32_t method);

/* Eq. 8 over the window at temperature T: Xp, Xm [nterms] FP64 (term-store
 * layout, absorption + and emission -).  Either may be NULL.  When store_B
 * is nonzero the temperature-independent terms are also retained in the
 * context (the "vertex store" reused by elph_scatt_rates and elph_iterate
 * at any temperature). */
elph_status elph_transition_probs(elph_ctx ctx, double T_K, double* Xp, double* Xm,
                                  int32_t store_B);

/* RTA scattering rates at T: W_e [nstates] (Eq. 21, e-ph part) and
 * W_ph [nk][nbr] (Eq. 25, ph-e part with Y of Eq. 12, spin degeneracy 2),
 * s^-1.  Either may be NULL.  Reuses the vertex store if present,
 * otherwise recomputes the vertices (and keeps them). */
elph_status elph_scatt_rates(elph_ctx ctx, double T_K, double* W_e, double* W_ph);

/* Coupled e-ph BTEs with the unified single-iterator scheme (Eq. 19,
 * Eqs. 20-27): each phonon iteration brings the electron equations to
 * self-consistency with the current phonons (relative residual tol/10, or
 * tol/100 at level COUPLED).
 * W_ph_ext [nk][nbr] device: phonon rates from other channels (ph-ph,
 * isotopes), s^-1, added to the ph-e rate (Eq. 25); NULL selects the model
 * 1e12 (hw/hw_max)^2 (T/300).  Without elph_set_phph the phonon
 * in-scattering Delta F^S is zero.  After elph_set_phph(sigma > 0) the
 * three-phonon RTA rate of Eq. 26 is added to W^RTA as well (W_ph_ext then
 * holds only the channels other than ph-e and three-phonon, and NULL means
 * none, not the model rate, so no channel is counted twice) and Delta F^S of
 * Eq. 26 joins every phonon update.
 * Electron responses are constrained to carry no change of carrier number
 * in each energy group (sorted active energies split at gaps wider than
 * hw_max + 12 sigma), which removes the conserved modes of the e-ph
 * collision operator.
 * Outputs (device): I, J [nstates][3] (I in eV m/K, J in m per unit charge),
 * F, G [nk][nbr][3].  tensors (host, may be NULL): 6 row-major 3x3 tensors
 * sigma (S/m), sigma*S (A/(m K)), alpha_el (A/m), kappa0_el (W/(m K)),
 * alpha_ph (A/m), kappa_ph (W/(m K)) of Eqs. 28-30 with 1/N_k, 1/N_q.
 * iters (host, may be NULL): phonon iterations used.  ko_residual (host,
 * may be NULL): |sigma S - (alpha_el + alpha_ph)/T| / |sigma S| (Eq. 31).
 * Residual = max over I, J, F, G of |x_new - x_old| / |x_new| (2-norms),
 * where for F, G x_new is the phonon map applied to x_old.  At level
 * COUPLED the phonon iterates are Anderson-accelerated (history 6, per
 * Cartesian column): the converged pair is the fixed point of the scheme,
 * reached in fewer phonon iterations than by plain substitution.
 * Returns ELPH_ENOCONV (with the last iterate) if maxit is reached. */
elph_status elph_iterate(elph_ctx ctx, double T_K, const double* W_ph_ext, int32_t level,
                         double tol, int32_t maxit, double* I, double* J, double* F,
                         double* G, double* tensors, int32_t* iters, double* ko_residual);

/* Kelvin-Onsager enforcement (Eqs. 32-35) on responses at temperature T_K,
 * normally those elph_iterate returned.  sigma*S and alpha split into
 * diffusion and drag parts; with I_diff = (eps - mu)/T J (Eq. 34, I in eV m/K,
 * J in m per unit charge) the diffusion part of sigma*S equals alpha_el/T
 * identically, and the drag part I_drag = I - I_diff is rescaled:
 * I <- I_diff + lambda I_drag, lambda being the scalar that brings
 * sigma*S_drag[lambda I_drag] closest to alpha_ph/T (Eq. 35; least squares
 * over the nine tensor components, the root of the scalar condition that the
 * method finds by bisection, here in closed form).
 * I [nstates][3] device, rewritten in place; J [nstates][3] and F, G
 * [nk][nbr][3] device, read only.  tensors (host, may be NULL): the 54 values
 * of elph_iterate after the correction; lambda and ko_residual (host, may be
 * NULL): lambda and Eq. 31's residual after the correction.  Synchronises the
 * context's stream.  EINVAL if a pointer is NULL, or if I has no drag part
 * (I = I_diff, as at level RTA). */
elph_status elph_ko_enforce(elph_ctx ctx, double T_K, double* I, const double* J,
                            const double* F, const double* G, double* tensors,
                            double* lambda, double* ko_residual);

/* ---- Batches: many independent materials evaluated together ------------
 * The vertex contractions of all materials run in persistent launches that
 * pull (material, tile) work items from a queue, longest contraction first
 * (one step-1 launch, one step-2 launch per branch count), and the whole
 * per-temperature sequence can be captured in a HIP graph and replayed.
 * Results are identical to elph_scatt_rates on each context.  Contexts must
 * share one precision form; while a batch call runs, their work goes to the
 * batch's own stream.  The batch does not own the contexts (destroy the
 * batch first). */
typedef struct elph_batch_s* elph_batch;

/* n >= 1 contexts (host array of handles). */
elph_status elph_batch_create(int32_t n, const elph_ctx* ctxs, elph_batch* out);
void elph_batch_destroy(elph_batch b);
/* Message of the last failing batch call; b may be NULL for create errors. */
const char* elph_batch_last_error(elph_batch b);

/* Eqs. 21 and 25 for every material: W_e[m] [nstates_m], W_ph[m] [nk_m][nbr_m]
 * are device pointers in host arrays of length n (either array, or any entry,
 * may be NULL).  use_graph != 0 captures the sequence in a HIP graph on the
 * first call for a given temperature and set of output pointers and replays
 * it afterwards.  Synchronises the batch stream.  The vertex stores of all
 * contexts are left valid.  Batches compute the plain form of their
 * precision: the FP64 refinement of elph_set_refine is not applied (the
 * results equal those of elph_scatt_rates on each context with the
 * refinement off). */
elph_status elph_batch_scatt_rates(elph_batch b, double T_K, double* const* W_e, double* const* W_ph,
                                   int32_t use_graph);

/* Autotuner: times each launch shape of the persistent contractions (blocks
 * per compute unit 1, 2, 4, 8 x work items in cost order or in natural
 * order x, in FP32 batches, GEMM tiles of 64 or 128 rows by 64 columns) on
 * this batch, keeps the fastest, and caches it for batches of the same
 * signature (precision and each material's states, branches and contraction
 * lengths).  The vertex epilogues of all materials run as persistent
 * launches too.  Every shape gives bit-identical results.
 * choice (host, may be NULL) receives [blocks_per_cu, cost_ordered,
 * tile_rows]; best_ms (host, may be NULL) the per-evaluation time of the
 * winner. */
elph_status elph_batch_tune(elph_batch b, double T_K, int32_t* choice, double* best_ms);

/* Sets a launch shape explicitly (as one of the tuner's candidates):
 * blocks_per_cu 1, 2, 4 or 8; cost_ordered 0 or 1; tile_rows 64 or 128 (FP32
 * batches; FP64 batches take 128).  EINVAL otherwise. */
elph_status elph_batch_set_shape(elph_batch b, int32_t blocks_per_cu, int32_t cost_ordered, int32_t tile_rows);

/* ---------------------------------------------------------------------------
 * Learned screen of negligible terms.  A small MLP predicts log10 |g|^2
 * (|g^{s n m}_{k q}|^2 of Eq. 6 in eV^2) of a term from its features; with
 * the exact Gaussian delta and occupations of Eq. 8 this gives a predicted
 * X of every term, and the step-2 tiles whose predicted terms all lie below
 * tau times the largest predicted term of their initial state are skipped.
 * The exact path remains the reference: callers compare the screened rates
 * with elph_scatt_rates.
 *
 * Network: depth hidden layers of `width` units, z = a W + b, a = GELU(z)
 * (z Phi(z), Phi the normal CDF), output y = a w + b; loss = mean squared
 * error.  Products run on BF16 copies of the weights with FP32 accumulation;
 * FP32 master weights are updated by Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * params (host, FP32): for each layer in order W [fan_in][fan_out] row-major
 * then b [fan_out]; elph_mlp_nparams gives the length. */
typedef struct elph_mlp_s* elph_mlp;

/* 1 <= nin <= 1024; width a multiple of 64 in [64, 1024]; 1 <= depth <= 8.
 * hip_stream: NULL = default stream.  Errors: EINVAL (sizes, non-finite
 * params), ENOMEM. */
elph_status elph_mlp_create(int32_t nin, int32_t width, int32_t depth, const float* params,
                            void* hip_stream, elph_mlp* out);
void elph_mlp_destroy(elph_mlp m);
const char* elph_mlp_last_error(elph_mlp m);
int64_t elph_mlp_nparams(elph_mlp m);
/* FP32 master parameters to / from the host; setting resets Adam. */
elph_status elph_mlp_get_params(elph_mlp m, float* params);
elph_status elph_mlp_set_params(elph_mlp m, const float* params);
/* y [n] = network(x [n][nin]); x, y device FP32. */
elph_status elph_mlp_forward(elph_mlp m, int64_t n, const float* x, float* y);
/* Gradient of the loss over a batch (n a positive multiple of 64) into grad
 * [nparams] (device FP32, may be NULL); loss (host, may be NULL). */
elph_status elph_mlp_gradients(elph_mlp m, int64_t n, const float* x, const float* t, float* grad,
                               double* loss);
/* One Adam step of learning rate lr on the batch; loss before the step. */
elph_status elph_mlp_train_step(elph_mlp m, int64_t n, const float* x, const float* t, float lr,
                                double* loss);

/* Number of screen features of a context: 9 + 2 nwann + nbr, in the order
 * k (3 fractional coordinates), q (3), eps_{m k}, eps_{n k+q} (eV, relative
 * to mu), hbar omega_{q s} / hbar omega_max, one-hot m (nwann), one-hot n
 * (nwann), one-hot s (nbr). */
int32_t elph_screen_nin(elph_ctx ctx);

/* Training samples from the exact vertex (Eq. 6): for every mesh pair
 * (kidx[p], qidx[p]) (device int32) and every (s, n, m), a feature row of
 * x [npairs * nbr * nwann^2][nin] and the target t = log10(max(|g|^2, 1e-12))
 * (device FP32), ordered like elph_interp_g. */
elph_status elph_screen_samples(elph_ctx ctx, int64_t npairs, const int32_t* kidx,
                                const int32_t* qidx, float* x, float* t);

enum { ELPH_SCREEN_NONE = 0, ELPH_SCREEN_ENERGY = 1, ELPH_SCREEN_MLP = 2 };
/* Screened RTA rates at T (outputs as elph_scatt_rates), the skip rule of
 * the learned screen applied to whole step-2 tiles.  The states are ranked by
 * energy (ties by state index) and a tile is 32 consecutive ranks of final
 * states x 32 of initial states.  Mode ENERGY keeps a tile when one of its
 * terms has a Gaussian factor exp(-(dE -/+ hw)^2 / 2 sigma^2) of at least
 * gauss_min (0 < gauss_min < 1; m may be NULL; tau unused).  Mode MLP runs
 * that stage first, then evaluates the network on every term of the kept
 * tiles and keeps a tile when one of its terms has a predicted X+ + X- of at
 * least tau (0 < tau < 1) times the largest of its initial state, or a
 * predicted X+ of at least tau times the largest of its phonon mode (the sums
 * of Eqs. 21 and 25), maxima over the evaluated terms.  Mode NONE computes every tile.  Tiles not kept have
 * zero vertex-store entries; the store is not reused as the exact one by
 * later calls.  stats (host, may be NULL) [5]: tiles, tiles computed, tiles
 * kept by the energy stage, terms evaluated by the network, screen time (ms,
 * both stages, before the vertex evaluation).  EINVAL on a bad mode,
 * threshold, temperature, network size or a non-Gaussian delta. */
elph_status elph_scatt_rates_screened(elph_ctx ctx, elph_mlp m, int32_t mode, double tau, double gauss_min,
                                      double T_K, double* W_e, double* W_ph, double* stats);

#ifdef __cplusplus
}
#endif

#endif /* ELPH_H */
