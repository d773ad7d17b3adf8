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

elph_status make_thermal(elph_ctx ctx, double T, Thermal* th);
elph_status alloc_thermal(elph_ctx ctx, Thermal* th);
void fill_thermal(elph_ctx ctx, double T, const Thermal& th, hipStream_t s);
template <typename ST, int NV>
void launch_q_gather(elph_ctx ctx, const ST* Bp, const double* f, const double* omf, const double* x, double* acc);
void free_thermal(elph_ctx ctx, Thermal* th);
elph_status ensure_store(elph_ctx ctx);
elph_status rates_from_store(elph_ctx ctx, const Thermal& th, double* we, double* wph);
elph_status x_from_store(elph_ctx ctx, const Thermal& th, double* Xp, double* Xm);
elph_status finalize_wph(elph_ctx ctx, const Thermal& th, double* acc, double* wph);
elph_status interp_g(elph_ctx ctx, int64_t npairs, const int32_t* kidx, const int32_t* qidx, double* g_out);
elph_status iterate(elph_ctx ctx, double T, const double* wext, int level, double tol, int maxit, double* I,
                    double* J, double* F, double* G, double* tensors, int* iters, double* ko);

// batches of materials in persistent launches (vertex.hip)
struct BatchImpl;
BatchImpl* batch_new(const std::vector<elph_ctx>& ctxs, std::string* err);
void batch_free(BatchImpl* b);
elph_status batch_rates(BatchImpl* b, double T_K, double* const* we, double* const* wph, bool use_graph);
elph_status batch_tune(BatchImpl* b, double T_K, int* choice, double* best_ms);
const std::string& batch_error(BatchImpl* b);

}  // namespace elph
