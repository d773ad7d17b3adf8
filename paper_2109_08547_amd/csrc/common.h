// Internal declarations of libelph (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/elph.h"

namespace elph {

// CODATA 2018.
constexpr double kHbarEVs = 6.582119569e-16;     // eV s
constexpr double kBoltzEVK = 8.617333262e-5;     // eV / K
constexpr double kCharge = 1.602176634e-19;      // C = J/eV
constexpr double kAmuKg = 1.66053906660e-27;     // kg
constexpr double kAngM = 1.0e-10;                // m / Angstrom
constexpr double kSpinDeg = 2.0;
constexpr double kPi = 3.14159265358979323846;
constexpr double kEps0 = 8.8541878128e-12;         // F / m
// (hbar omega)^2 [eV^2] = kPhononC [eV] * lambda [eV/(A^2 amu)]
constexpr double kHbarJs = kHbarEVs * kCharge;
constexpr double kPhononC = kHbarJs * kHbarJs / (kAmuKg * kAngM * kAngM) / kCharge;

constexpr int kMaxBands = 16;
constexpr int64_t kMaxPairKept = 46340;  // nkept^2 below 2^31

// ---------------------------------------------------------------- complex
struct cd {
  double x, y;
};
__host__ __device__ inline cd cmake(double a, double b) { return cd{a, b}; }
__host__ __device__ inline cd cadd(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cd csub(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cd cmul(cd a, cd b) {
  return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline cd cmulc(cd a, cd b) {  // a * conj(b)
  return cd{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__host__ __device__ inline cd cconj(cd a) { return cd{a.x, -a.y}; }
__host__ __device__ inline cd cscale(cd a, double s) { return cd{a.x * s, a.y * s}; }
__host__ __device__ inline double cabs2(cd a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------- launch helpers
// Dynamic LDS that a kernel leaves unused, sized so that at most `per_cu`
// of its blocks (each also holding own_lds bytes of static LDS) are resident
// on a CU: for row kernels whose rows each sweep their own window of a
// table, so that the windows of the rows running together stay in L2.
inline size_t lds_pad_for(int per_cu, int own_lds) {
  int dev = 0, cu = 0, blk = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int64_t margin = 1024;  // allocation granularity
  int64_t pad = (int64_t)cu / per_cu - own_lds - margin;
  if (pad > (int64_t)blk - own_lds - margin) pad = (int64_t)blk - own_lds - margin;
  return pad > 0 ? (size_t)(pad / 1024 * 1024) : 0;
}

inline unsigned blocks_for(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}

}  // namespace elph

// ---------------------------------------------------------------- context
struct elph_ctx_s {
  // status
  std::string err;
  bool hip_dead = false;
  hipStream_t stream = nullptr;
  int device = 0;

  // inputs (host copies of scalars)
  int nb = 0, na = 0, nbr = 0, nre = 0, nrp = 0;
  int mesh[3] = {0, 0, 0};
  int64_t nk = 0;
  int precision = ELPH_FP64;
  int delta = ELPH_DELTA_GAUSS;  // energy-conserving delta of Eq. 8
  double mu = 0, window = 0, sigma = 0, omega_min = 1e-4;
  // operand scales of the FP16 split form (powers of two; 1 in the other
  // forms): A_e, A_p, gR, B2
  double sc_ae = 1, sc_ap = 1, sc_g = 1, sc_b2 = 1;
  double lat[9];
  double volume_A3 = 0;
  std::vector<double> mass;

  // device inputs
  int32_t* d_re = nullptr;   // [nre][3]
  int32_t* d_rp = nullptr;   // [nrp][3]
  double* d_wre = nullptr;   // [nre]
  double* d_wrp = nullptr;   // [nrp]
  double* d_hr = nullptr;    // [nre][nb][nb] complex
  double* d_dr = nullptr;    // [nrp][nbr][nbr]
  double* d_gr = nullptr;    // [nre][nrp][nbr][nb][nb] complex (as given)
  double* d_mass_x = nullptr;  // [nbr] mass of the atom of each x
  double* d_lat = nullptr;   // [9]
  double* d_nac = nullptr;   // polar materials: Z* [na][3][3], eps_inf [3][3], 2 pi b_i rows [3][3] (null: none)
  double nac_coef = 0;       // e^2 / (eps_0 V), eV / Angstrom^2
  bool frohlich = false;     // polar with atom positions: the Froehlich vertex of Eq. 7 (d_nac then ends with tau [na][3])
  int fr_box[3] = {0, 0, 0}; // half widths of the G box of its Ewald sum
  double* d_frohlich = nullptr;  // [nk][nbr] complex F_s(q) of Eq. 7 (eV)
  double* d_ustate = nullptr;    // [nstates][nb] complex eigenvector of each active state (its column of U)
  // third-order force constants (three-phonon processes, Eq. 13): entries
  // grouped by their second cell R_j
  int n3 = 0, ng3 = 0;
  int32_t* d_i3_rj = nullptr;   // [ng3][3] distinct R_j
  int32_t* d_i3_off = nullptr;  // [ng3 + 1] first entry of each R_j
  int32_t* d_i3_rk = nullptr;   // [n3][3]
  double* d_i3_psi = nullptr;   // [n3][nbr][nbr][nbr] eV / Angstrom^3, x = 3 atom + Cartesian
  void* d_i3_fold = nullptr;     // fold table of the force constants over the phonon tables (derived; cached)
  double phph_sigma = 0;        // > 0: three-phonon processes in elph_iterate (Gaussian width, eV)
  double2* d_tab[3] = {nullptr, nullptr, nullptr};  // per-axis exp(2 pi i j / N)
  int32_t* d_qrep = nullptr;                          // mesh points q with q <= -q (one of each +-q pair)
  int64_t nqrep = 0;

  // tables
  bool tables_ready = false;
  int64_t nkept = 0, nstates = 0;
  int ngroups = 0;
  double hw_max = 0;
  double* d_eps_all = nullptr;    // [nk][nb]
  int32_t* d_kidx = nullptr;      // [nk] kept index or -1
  int32_t* d_kept = nullptr;      // [nkept] mesh index
  int32_t* d_soff = nullptr;      // [nkept+1] first state of each kept k
  int32_t* d_state_k = nullptr;   // [nstates] mesh index
  int32_t* d_state_kidx = nullptr;  // [nstates] kept index
  int32_t* d_state_m = nullptr;   // [nstates] band
  double* d_eps = nullptr;        // [nstates]
  double* d_vel = nullptr;        // [nstates][3]
  int32_t* d_group = nullptr;     // [nstates] energy group
  double* d_U = nullptr;          // [nkept][nb][nb] complex, columns = eigenvectors
  double* d_hw = nullptr;         // [nk][nbr]
  double* d_Lq = nullptr;         // [nk][nbr(x)][nbr(s)] complex, l_{x,s} u[x][s]
  double* d_vph = nullptr;        // [nk][nbr][3]
  double* d_Ee = nullptr;         // [nkept][nre] complex  w_e exp(2 pi i k.Re)
  double* d_Ep = nullptr;         // [nkept][nrp] complex  exp(2 pi i k.Rp)

  // contraction operands (precision dependent)
  int64_t m_pad = 0;              // nstates padded
  int64_t ke = 0, kp = 0;         // padded contraction lengths
  void* d_Ae = nullptr;           // [m_pad][ke]
  void* d_Ap = nullptr;           // [m_pad][kp]
  void* d_gR = nullptr;           // [nbr*nrp*nb][ke]
  void* d_B2 = nullptr;           // [m_pad*nbr][kp]
  bool operands_ready = false;

  // vertex store (temperature independent), FP64 or FP32 by precision
  void* d_Bp = nullptr;
  void* d_Bm = nullptr;
  bool store_ready = false;
  bool store_f32 = false;

  // scratch
  double* d_we_part = nullptr;    // [n_jtiles][m_pad]
  int64_t we_part_len = 0;

  // FP64 refinement of ill-conditioned vertices in the GEMM forms: every
  // stored |g|^2 carries an estimate of its relative error; rates whose
  // estimated relative error exceeds refine_theta have their dominant terms
  // recomputed in FP64 (0 turns the refinement off)
  double refine_theta = 2.0e-6;
  uint8_t* d_rho = nullptr;       // [nstates][nstates][rho_stride] log-coded error estimate of each |g|^2 (0: exact)
  int rho_stride = 8;             // bytes per pair (i, j): 8 for up to 8 branches, else 16
  bool rho_valid = false;         // d_rho describes the current vertex store
  float* d_b2n = nullptr;         // [nstates][nbr] mean over n' of sum_Rp w_p^2 |B2[(i,x)][(Rp,n')]|^2
  double* d_gR64 = nullptr;       // [nbr*nrp*nb][ke64] FP64 vertex operand of the refinement (built on demand)
  int64_t ke64 = 0, kp64 = 0;     // FP64 padded contraction lengths
  int64_t ref_stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // last refinement: see elph_refine_info

  // event timing: [0,1] tables, [2,3] step 1, [4,5] step 2, [6,7] iterate,
  // [8,9] tetrahedron weights / Froehlich table, [10,11] refinement
  bool timing = false;
  hipEvent_t ev[12] = {};
  bool ev_recorded[6] = {false, false, false, false, false, false};

  // caches reused across calls (dropped with the tables)
  int32_t* d_order = nullptr;     // [nstates] states sorted by energy
  int32_t* d_goff = nullptr;      // [ngroups+1] offsets of the energy groups in d_order
  bool groups_ready = false;
  int32_t* d_poff = nullptr;      // [nk+1] offsets of the pair lists by q
  int32_t* d_plist = nullptr;     // [nkept^2] kept index t of each pair (k_t, k_t + q)
  uint64_t* d_ppk = nullptr;      // [nkept^2] the pair's state ranges, packed (pack_pair), list order
  bool pairs_ready = false;
  bool pairs_failed = false;      // lists not allocatable: q-gathers walk the kept set
  double* d_we_cache = nullptr;   // [nstates] W_e of the last full elph_scatt_rates
  double* d_wph_cache = nullptr;  // [nk][nbr] W_ph of the same call
  double rates_T = -1.0;
  bool rates_valid = false;
  double* h_pin = nullptr;        // pinned host words for solver status reads
  const uint8_t* d_tile_keep = nullptr;  // step-2 tile mask of a screened evaluation (else null)
  const int32_t* d_tile_perm = nullptr;  // state at each tile position of that evaluation (null = identity)

  // device memory: live blocks (pointer, bytes) and released blocks kept for
  // reuse by later allocations of the same size (freed by elph_destroy or
  // ELPH_RESET_TRIM); mem_limit > 0 caps the bytes of both together
  std::vector<std::pair<void*, size_t>> allocs;
  std::vector<std::pair<void*, size_t>> pool;
  size_t mem_limit = 0;
  // largest FP32 output buffer of a GEMM form's contraction (rows in chunks)
  size_t gemm_chunk = (size_t)1 << 31;
};

namespace elph {

// Record timing event e (0..7) on the context stream when timing is on.
inline void mark(elph_ctx ctx, int e) {
  if (!ctx->timing) return;
  (void)hipEventRecord(ctx->ev[e], ctx->stream);
  if (e & 1) ctx->ev_recorded[e >> 1] = true;
}

// Device allocation through the context pool: a released block of exactly
// the requested size is reused, otherwise hipMalloc.  dev_free returns the
// block to the pool; pool_trim releases the pool.
hipError_t dev_alloc(elph_ctx ctx, void** p, size_t bytes);
void dev_free(elph_ctx ctx, void* p);
void pool_trim(elph_ctx ctx);
// After a failed allocation: release every derived table, operand, store and
// work buffer (the inputs stay) so that the context can start over.
void recover_after_enomem(elph_ctx ctx);

// Host-side error plumbing of functions that take `elph_ctx ctx` and return
// elph_status.
#define HIPCHK(x)                                                       \
  do {                                                                  \
    hipError_t e_ = (x);                                                \
    if (e_ != hipSuccess) {                                             \
      ctx->err = std::string("HIP error ") + hipGetErrorString(e_) +    \
                 " at " + __FILE__ + ":" + std::to_string(__LINE__);    \
      ctx->hip_dead = true;                                             \
      return ELPH_EHIP;                                                 \
    }                                                                   \
  } while (0)

#define ALLOC(ptr, bytes)                                                          \
  do {                                                                             \
    void* p_ = nullptr;                                                            \
    hipError_t e_ = dev_alloc(ctx, &p_, (size_t)(bytes));                          \
    if (e_ != hipSuccess) {                                                        \
      ctx->err = "device allocation of " + std::to_string((size_t)(bytes)) + " bytes failed"; \
      (void)hipGetLastError();                                                     \
      return ELPH_ENOMEM;                                                          \
    }                                                                              \
    ptr = (decltype(ptr))p_;                                                       \
  } while (0)

}  // namespace elph
