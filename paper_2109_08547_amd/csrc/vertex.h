// Internal: vertex contractions (vertex.hip) and rate / iteration kernels (rates.hip).
#pragma once
#include "common.h"

namespace elph {

// Per-temperature factor tables (device).
struct Thermal {
  double* f = nullptr;      // [nstates] Fermi-Dirac f
  double* omf = nullptr;    // [nstates] 1 - f
  double* lomf = nullptr;   // [nstates] log(1 - f)
  double* nocc = nullptr;   // [nk][nbr] Bose-Einstein n (0 below omega_min)
};

elph_status build_operands(elph_ctx ctx);
elph_status run_vertex(elph_ctx ctx, void* Bp, void* Bm, bool store_f64, const Thermal* th, double* we_out,
                       double* wph_acc);

// Error-estimate options of the rate reductions (null rho: none).  With rho
// set, a rate whose estimated relative error (sum of term contributions
// times their codes over the rate) exceeds theta is appended to list (count
// in *cnt).  idx (optional) restricts the reduction to n listed rows or
// wave vectors.
struct RateErr {
  const uint8_t* rho = nullptr;   // [nstates][nstates][RhoStride<nbr>] codes
  double theta = 0.0;
  int32_t* cnt = nullptr;
  int32_t* list = nullptr;
  const int32_t* idx = nullptr;
  int64_t n = 0;
};

elph_status make_thermal(elph_ctx ctx, double T, Thermal* th);
elph_status alloc_thermal(elph_ctx ctx, Thermal* th);
void fill_thermal(elph_ctx ctx, double T, const Thermal& th, hipStream_t s);
template <typename ST, int NV>
void launch_q_gather(elph_ctx ctx, const ST* Bp, const double* f, const double* omf, const double* x, double* acc,
                     const RateErr* err = nullptr);
void free_thermal(elph_ctx ctx, Thermal* th);
elph_status ensure_store(elph_ctx ctx);
// pair lists by q used by the q-gathers (built once per table build)
elph_status ensure_pairs(elph_ctx ctx);
elph_status rates_from_store(elph_ctx ctx, const Thermal& th, double* we, double* wph);
// W_e[i] = sum_{j,s} (B+ n + B- (1 + n)) (1 - f_j) / (1 - f_i) from a finished store
template <typename ST>
void launch_we_rows(elph_ctx ctx, const ST* Bp, const ST* Bm, const double* lomf, const double* nocc, double* we,
                    const RateErr* err = nullptr);

// saved state of a context: tables and vertex store (io.hip)
elph_status save_state(elph_ctx ctx, const char* path);
elph_status load_state(elph_ctx ctx, const char* path);

// FP64 refinement of ill-conditioned vertices in the GEMM forms (refine.hip)
bool refine_applicable(elph_ctx ctx);
// error-estimate buffers for the next vertex store (d_rho, d_b2n)
elph_status refine_prepare(elph_ctx ctx);
// sum_Rp w_p^2 |B2|^2 of states [i0, i0 + ni) from the step-1 GEMM rows C1
void refine_b2_norms(elph_ctx ctx, int64_t i0, int64_t ni, const float* C1);
// contraction error units of the context's form: relative to the
// root-sum-square of a component's products (coherent = false) or to the
// component's magnitude (coherent = true)
double refine_unit(elph_ctx ctx, bool coherent);
// After the rate reductions at a temperature flagged rows / modes (err_e,
// err_ph): recompute their dominant terms in FP64, update the store and the
// codes, recompute the affected W_e rows and phonon accumulators.
elph_status refine_terms(elph_ctx ctx, const Thermal& th, double* we, double* acc, const RateErr& err_e,
                         const RateErr& err_ph, int32_t* cnt);
// FP64 operands of the refinement (vertex.hip): the permuted vertex and
// step-1 rows B2[(s, x)][(Rp, n')] of listed states
elph_status ensure_gR64(elph_ctx ctx);
elph_status step1_fp64_rows(elph_ctx ctx, int64_t ns, const int32_t* st_kidx, const int32_t* st_m, double* Ae64,
                            double* B2_64);
elph_status x_from_store(elph_ctx ctx, const Thermal& th, double* Xp, double* Xm);
elph_status finalize_wph(elph_ctx ctx, const Thermal& th, double* acc, double* wph);
elph_status interp_g(elph_ctx ctx, int64_t npairs, const int32_t* kidx, const int32_t* qidx, double* g_out);
// the same through the static work array (no device allocation)
constexpr size_t kInterpScratchBytes = (size_t)64 << 20;
elph_status interp_g_noalloc(elph_ctx ctx, int64_t npairs, const int32_t* kidx, const int32_t* qidx, double* g_out);
elph_status iterate(elph_ctx ctx, double T, const double* wext, int level, double tol, int maxit, double* I,
                    double* J, double* F, double* G, double* tensors, int* iters, double* ko);
// three-phonon processes (Eqs. 13, 14, 26)
elph_status phph_set_ifc3(elph_ctx ctx, int32_t n, const int32_t* rj, const int32_t* rk, const double* psi);
elph_status phph_vertex(elph_ctx ctx, int64_t npairs, const int32_t* q, const int32_t* qp, double* V2);
elph_status phph_rates(elph_ctx ctx, double T_K, double sigma_eV, double* W);
elph_status phph_inscatter(elph_ctx ctx, double T_K, double sigma_eV, const double* F, double* S);
elph_status ko_enforce(elph_ctx ctx, double T, double* I, const double* J, const double* F, const double* G,
                       double* tensors, double* lambda, double* ko);

// electron self-consistency solver (solve.hip)
struct SelfSolver {
  void* KT = nullptr;                   // [M][ldk] transposed, group-projected self operator (FP64 or FP32)
  bool kt_f32 = false;
  double *b = nullptr, *r = nullptr, *rh = nullptr, *s = nullptr, *t = nullptr;
  double *p = nullptr, *p2 = nullptr, *v = nullptr, *v2 = nullptr;  // p and v alternate between two buffers
  double* part = nullptr;               // [S][M][6] split partials of the matrix-vector product
  double* dpart = nullptr;              // [nblk][12] dot partials
  double* dxr = nullptr;                // [nblk][12] dot partials of the x, r update
  double* sc = nullptr;                 // device scalars
  int S = 1, nblk = 1, nt = 1;          // j splits, vector-kernel blocks, row tiles
  int64_t jlen = 1, ldk = 1;            // rows per split; row stride of K^T
};
size_t self_solver_doubles(int64_t M, bool kt_f32);
void self_solver_carve(int64_t M, bool kt_f32, double* base, SelfSolver* sv);
template <typename ST>
elph_status build_self_operator(elph_ctx ctx, const ST* Bp, const ST* Bm, const double* lomf, const double* nocc,
                                const double* we, const int32_t* order, const int32_t* goff, const double* wff,
                                const SelfSolver& sv);
// Solves L x = b (b in sv.b, projected; x projected on entry) to relative
// residual thr per column; *ok when all six columns reached it.
elph_status self_solve(elph_ctx ctx, const SelfSolver& sv, double* x, double thr, int maxit, bool* ok, int* iters);

// batches of materials in persistent launches (vertex.hip)
struct BatchImpl;
BatchImpl* batch_new(const std::vector<elph_ctx>& ctxs, std::string* err);
void batch_free(BatchImpl* b);
elph_status batch_rates(BatchImpl* b, double T_K, double* const* we, double* const* wph, bool use_graph);
elph_status batch_tune(BatchImpl* b, double T_K, int* choice, double* best_ms);
elph_status batch_set_shape(BatchImpl* b, int bpc, bool sorted, int wr);
const std::string& batch_error(BatchImpl* b);

}  // namespace elph
