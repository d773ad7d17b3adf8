// C ABI of libelph (declared in include/elph.h): context lifecycle, input
// validation and orchestration of the table, vertex, rate and iteration
// kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "common.h"
#include "tables.h"
#include "vertex.h"
#include "devutil.h"

using namespace elph;

namespace elph {

static size_t held_bytes(elph_ctx ctx) {
  size_t t = 0;
  for (auto& b : ctx->allocs) t += b.second;
  for (auto& b : ctx->pool) t += b.second;
  return t;
}

hipError_t dev_alloc(elph_ctx ctx, void** p, size_t bytes) {
  *p = nullptr;
  const size_t n = bytes > 0 ? bytes : 1;
  for (size_t k = 0; k < ctx->pool.size(); ++k)
    if (ctx->pool[k].second == n) {
      *p = ctx->pool[k].first;
      ctx->pool.erase(ctx->pool.begin() + k);
      ctx->allocs.push_back({*p, n});
      return hipSuccess;
    }
  if (ctx->mem_limit > 0 && held_bytes(ctx) + n > ctx->mem_limit) {
    pool_trim(ctx);
    if (held_bytes(ctx) + n > ctx->mem_limit) return hipErrorOutOfMemory;  // the context's budget
  }
  hipError_t e = hipMalloc(p, n);
  if (e != hipSuccess) {
    // give the pool back to the device and try once more
    (void)hipGetLastError();
    pool_trim(ctx);
    e = hipMalloc(p, n);
  }
  if (e == hipSuccess) ctx->allocs.push_back({*p, n});
  return e;
}

void dev_free(elph_ctx ctx, void* p) {
  if (!p) return;
  for (size_t k = 0; k < ctx->allocs.size(); ++k)
    if (ctx->allocs[k].first == p) {
      ctx->pool.push_back(ctx->allocs[k]);
      ctx->allocs.erase(ctx->allocs.begin() + k);
      return;
    }
}

void pool_trim(elph_ctx ctx) {
  if (ctx->pool.empty()) return;
  if (!ctx->hip_dead) (void)hipStreamSynchronize(ctx->stream);
  for (auto& b : ctx->pool) (void)hipFree(b.first);
  ctx->pool.clear();
}

}  // namespace elph

static void drop_derived(elph_ctx ctx);

namespace elph {

void recover_after_enomem(elph_ctx ctx) {
  if (ctx->hip_dead) return;
  (void)hipStreamSynchronize(ctx->stream);
  drop_derived(ctx);
  ctx->d_gR64 = nullptr;
  // the inputs (and what is built from them alone at create or by the
  // set_* calls) stay; every other live block, including the work buffers
  // of the failed call, is freed
  const void* keep[] = {ctx->d_re,     ctx->d_rp,     ctx->d_wre,    ctx->d_wrp,    ctx->d_hr,     ctx->d_dr,
                        ctx->d_gr,     ctx->d_mass_x, ctx->d_lat,    ctx->d_nac,    ctx->d_tab[0], ctx->d_tab[1],
                        ctx->d_tab[2], ctx->d_qrep,   ctx->d_i3_rj,  ctx->d_i3_off, ctx->d_i3_rk,  ctx->d_i3_psi};
  std::vector<std::pair<void*, size_t>> live;
  for (auto& b : ctx->allocs) {
    bool k = false;
    for (const void* q : keep) k |= (q && q == b.first);
    if (k) live.push_back(b);
    else (void)hipFree(b.first);
  }
  ctx->allocs.swap(live);
  pool_trim(ctx);
  (void)hipGetLastError();
}

}  // namespace elph

static thread_local std::string g_create_err;

#define CHECK_CTX(ctx)                                          \
  do {                                                          \
    if (!(ctx)) return ELPH_EINVAL;                             \
    if ((ctx)->hip_dead) {                                      \
      (ctx)->err = "context unusable after a HIP error";        \
      return ELPH_ESTATE;                                       \
    }                                                           \
    (ctx)->err.clear();                                         \
  } while (0)


// A failed device allocation leaves the context usable: its derived tables,
// operands, store and work buffers are released (the inputs stay) and the
// next call starts over.
static elph_status enomem_guard(elph_ctx ctx, elph_status st) {
  if (st == ELPH_ENOMEM && ctx) {
    const std::string e = ctx->err;
    recover_after_enomem(ctx);
    ctx->err = e + "; the context released its derived tables and vertex store";
  }
  return st;
}

static bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static elph_status fail_create(const std::string& msg) {
  g_create_err = msg;
  return ELPH_EINVAL;
}

// Checks of the Wannier inputs: Hermiticity in the lattice sense, real
// symmetric force constants and the acoustic sum rule.
static elph_status validate(const elph_wannier* w, const elph_params* p) {
  if (!w || !p) return fail_create("null input");
  if (w->nwann < 1 || w->nwann > kMaxBands) return fail_create("nwann must be in 1..16");
  if (w->natom < 1 || 3 * w->natom > 15) return fail_create("natom must be in 1..5");
  if (w->nre < 1 || w->nrp < 1) return fail_create("empty cell-vector list");
  if (!w->re || !w->rp || !w->lat || !w->mass || !w->h_r || !w->d_r || !w->g_r)
    return fail_create("null array in elph_wannier");
  for (int d = 0; d < 3; ++d)
    if (p->mesh[d] < 1 || p->mesh[d] > 4096) return fail_create("mesh sizes must be in 1..4096");
  if ((int64_t)p->mesh[0] * p->mesh[1] * p->mesh[2] > (int64_t)1 << 31) return fail_create("mesh too large");
  if (!(p->sigma_eV > 0) || !std::isfinite(p->sigma_eV)) return fail_create("sigma must be positive");
  if (!(p->window_eV > 0)) return fail_create("window must be positive (INFINITY keeps all)");
  if (!std::isfinite(p->mu_eV)) return fail_create("mu must be finite");
  if (p->omega_min_eV < 0 || !std::isfinite(p->omega_min_eV)) return fail_create("omega_min must be >= 0");
  if (p->precision < ELPH_FP64 || p->precision > ELPH_FP16X3) return fail_create("unknown precision form");
  const int nb = w->nwann, nbr = 3 * w->natom;
  const size_t nn = (size_t)nb * nb, mm = (size_t)nbr * nbr;
  if (!all_finite(w->lat, 9) || !all_finite(w->mass, w->natom)) return fail_create("non-finite lattice or mass");
  for (int a = 0; a < w->natom; ++a)
    if (!(w->mass[a] > 0)) return fail_create("masses must be positive");
  if (!all_finite(w->h_r, 2 * nn * w->nre)) return fail_create("non-finite H(R)");
  if (!all_finite(w->d_r, mm * w->nrp)) return fail_create("non-finite D(R)");
  if (!all_finite(w->g_r, 2 * (size_t)w->nre * w->nrp * nbr * nn)) return fail_create("non-finite g(Re, Rp)");
  if ((w->wre && !all_finite(w->wre, w->nre)) || (w->wrp && !all_finite(w->wrp, w->nrp)))
    return fail_create("non-finite weights");

  // H(-R) = H(R)^dagger
  std::map<std::tuple<int, int, int>, int> re, rp;
  for (int r = 0; r < w->nre; ++r) re[{w->re[3 * r], w->re[3 * r + 1], w->re[3 * r + 2]}] = r;
  for (int r = 0; r < w->nrp; ++r) rp[{w->rp[3 * r], w->rp[3 * r + 1], w->rp[3 * r + 2]}] = r;
  double hmax = 0;
  for (size_t t = 0; t < 2 * nn * w->nre; ++t) hmax = std::max(hmax, std::fabs(w->h_r[t]));
  for (int r = 0; r < w->nre; ++r) {
    auto it = re.find({-w->re[3 * r], -w->re[3 * r + 1], -w->re[3 * r + 2]});
    if (it == re.end()) return fail_create("R_e list is not closed under R -> -R");
    const int m = it->second;
    const double wr = w->wre ? w->wre[r] : 1.0, wm = w->wre ? w->wre[m] : 1.0;
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) {
        const double* x = w->h_r + 2 * ((size_t)r * nn + a * nb + b);
        const double* y = w->h_r + 2 * ((size_t)m * nn + b * nb + a);
        if (std::fabs(wr * x[0] - wm * y[0]) > 1e-8 * hmax || std::fabs(wr * x[1] + wm * y[1]) > 1e-8 * hmax)
          return fail_create("H(R) is not Hermitian: H(-R) != H(R)^dagger");
      }
  }
  // D(-R) = D(R)^T and the acoustic sum rule on mass-weighted translations
  double dmax = 0;
  for (size_t t = 0; t < mm * w->nrp; ++t) dmax = std::max(dmax, std::fabs(w->d_r[t]));
  std::vector<double> dsum(mm, 0.0);
  for (int r = 0; r < w->nrp; ++r) {
    auto it = rp.find({-w->rp[3 * r], -w->rp[3 * r + 1], -w->rp[3 * r + 2]});
    if (it == rp.end()) return fail_create("R_p list is not closed under R -> -R");
    const int m = it->second;
    const double wr = w->wrp ? w->wrp[r] : 1.0, wm = w->wrp ? w->wrp[m] : 1.0;
    for (int a = 0; a < nbr; ++a)
      for (int b = 0; b < nbr; ++b) {
        if (std::fabs(wr * w->d_r[(size_t)r * mm + a * nbr + b] - wm * w->d_r[(size_t)m * mm + b * nbr + a]) >
            1e-8 * dmax)
          return fail_create("D(R) is not symmetric: D(-R) != D(R)^T");
        dsum[a * nbr + b] += wr * w->d_r[(size_t)r * mm + a * nbr + b];
      }
  }
  double msum = 0;
  for (int t = 0; t < w->natom; ++t) msum += w->mass[t];
  for (int al = 0; al < 3; ++al)
    for (int a = 0; a < nbr; ++a) {
      double acc = 0;
      for (int t = 0; t < w->natom; ++t) acc += dsum[a * nbr + 3 * t + al] * std::sqrt(w->mass[t] / msum);
      if (std::fabs(acc) > 1e-8 * dmax * std::sqrt((double)w->nrp)) return fail_create("acoustic sum rule violated");
    }
  return ELPH_OK;
}

extern "C" elph_status elph_create(const elph_wannier* w, const elph_params* p, void* hip_stream,
                                   elph_ctx* out) {
  if (!out) return fail_create("null output handle");
  *out = nullptr;
  elph_status st = validate(w, p);
  if (st != ELPH_OK) return st;
  elph_ctx ctx = new (std::nothrow) elph_ctx_s();
  if (!ctx) {
    g_create_err = "host allocation failed";
    return ELPH_ENOMEM;
  }
  ctx->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    g_create_err = "no HIP device";
    return ELPH_EHIP;
  }
  ctx->nb = w->nwann;
  ctx->na = w->natom;
  ctx->nbr = 3 * w->natom;
  ctx->nre = w->nre;
  ctx->nrp = w->nrp;
  for (int d = 0; d < 3; ++d) ctx->mesh[d] = p->mesh[d];
  ctx->nk = (int64_t)p->mesh[0] * p->mesh[1] * p->mesh[2];
  ctx->precision = p->precision;
  ctx->mu = p->mu_eV;
  ctx->window = p->window_eV;
  ctx->sigma = p->sigma_eV;
  ctx->omega_min = p->omega_min_eV > 0 ? p->omega_min_eV : 1.0e-4;
  if (ctx->precision == ELPH_FP16X3) {
    // powers of two that put each operand's largest possible magnitude at
    // 2^13 (FP16 holds up to 65504): |A_e| <= max|w_e|, |A_p| <= max|w_p|
    // (unit eigenvectors times phases), |gR| <= max|g|, and
    // |B2| <= N_Re nb max|w_e| max|g|
    auto maxabs = [](const double* v, size_t n, double dflt) {
      if (!v) return dflt;
      double m = 0.0;
      for (size_t k = 0; k < n; ++k) m = std::max(m, std::fabs(v[k]));
      return m;
    };
    const int nb_ = w->nwann, nbr_ = 3 * w->natom;
    const double we = maxabs(w->wre, (size_t)w->nre, 1.0), wp = maxabs(w->wrp, (size_t)w->nrp, 1.0);
    const double gm = maxabs(w->g_r, 2 * (size_t)w->nre * w->nrp * nbr_ * nb_ * nb_, 1.0);
    auto scale_for = [](double bound) { return bound > 0.0 ? std::ldexp(1.0, 13 - std::ilogb(bound) - 1) : 1.0; };
    ctx->sc_ae = scale_for(we);
    ctx->sc_ap = scale_for(wp);
    ctx->sc_g = scale_for(gm);
    ctx->sc_b2 = scale_for((double)w->nre * nb_ * we * gm);
  }
  std::memcpy(ctx->lat, w->lat, sizeof(ctx->lat));
  const double* L = w->lat;
  ctx->volume_A3 = std::fabs(L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                             L[2] * (L[3] * L[7] - L[4] * L[6]));
  ctx->mass.assign(w->mass, w->mass + w->natom);

  const int nb = ctx->nb, nbr = ctx->nbr;
  const size_t nn = (size_t)nb * nb, mm = (size_t)nbr * nbr;
  struct Up {
    void** dst;
    const void* src;
    size_t bytes;
  };
  std::vector<double> mass_x(nbr);
  for (int x = 0; x < nbr; ++x) mass_x[x] = w->mass[x / 3];
  std::vector<Up> ups = {
      {(void**)&ctx->d_re, w->re, (size_t)w->nre * 3 * sizeof(int32_t)},
      {(void**)&ctx->d_rp, w->rp, (size_t)w->nrp * 3 * sizeof(int32_t)},
      {(void**)&ctx->d_hr, w->h_r, (size_t)w->nre * nn * 2 * sizeof(double)},
      {(void**)&ctx->d_dr, w->d_r, (size_t)w->nrp * mm * sizeof(double)},
      {(void**)&ctx->d_gr, w->g_r, (size_t)w->nre * w->nrp * nbr * nn * 2 * sizeof(double)},
      {(void**)&ctx->d_mass_x, mass_x.data(), nbr * sizeof(double)},
      {(void**)&ctx->d_lat, w->lat, 9 * sizeof(double)},
  };
  if (w->wre) ups.push_back({(void**)&ctx->d_wre, w->wre, (size_t)w->nre * sizeof(double)});
  if (w->wrp) ups.push_back({(void**)&ctx->d_wrp, w->wrp, (size_t)w->nrp * sizeof(double)});
  for (auto& u : ups) {
    if (dev_alloc(ctx, u.dst, u.bytes) != hipSuccess) {
      (void)hipGetLastError();
      g_create_err = "device allocation of the inputs failed";
      elph_destroy(ctx);
      return ELPH_ENOMEM;
    }
    if (hipMemcpy(*u.dst, u.src, u.bytes, hipMemcpyHostToDevice) != hipSuccess) {
      g_create_err = "copy of the inputs to the device failed";
      elph_destroy(ctx);
      return ELPH_EHIP;
    }
  }
  st = make_axis_tables(ctx);
  if (st != ELPH_OK) {
    g_create_err = ctx->err;
    elph_destroy(ctx);
    return st;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    g_create_err = "stream synchronisation failed";
    elph_destroy(ctx);
    return ELPH_EHIP;
  }
  g_create_err.clear();
  *out = ctx;
  return ELPH_OK;
}

extern "C" elph_status elph_timing(elph_ctx ctx, int32_t enable, double* ms) {
  CHECK_CTX(ctx);
  if (enable && !ctx->ev[0]) {
    for (int e = 0; e < 12; ++e) HIPCHK(hipEventCreate(&ctx->ev[e]));
  }
  if (ms) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int t = 0; t < 4; ++t) {
      ms[t] = -1.0;
      if (ctx->ev_recorded[t]) {
        float v = 0.f;
        HIPCHK(hipEventElapsedTime(&v, ctx->ev[2 * t], ctx->ev[2 * t + 1]));
        ms[t] = v;
      }
    }
  }
  ctx->timing = enable != 0;
  return ELPH_OK;
}

extern "C" elph_status elph_save(elph_ctx ctx, const char* path) {
  CHECK_CTX(ctx);
  return enomem_guard(ctx, save_state(ctx, path));
}

extern "C" elph_status elph_load(elph_ctx ctx, const char* path) {
  CHECK_CTX(ctx);
  return enomem_guard(ctx, load_state(ctx, path));
}

extern "C" elph_status elph_set_memory_limit(elph_ctx ctx, int64_t bytes) {
  CHECK_CTX(ctx);
  if (bytes < 0) {
    ctx->err = "memory limit must be >= 0";
    return ELPH_EINVAL;
  }
  ctx->mem_limit = (size_t)bytes;
  if (ctx->mem_limit > 0) pool_trim(ctx);  // the budget starts from the live blocks
  return ELPH_OK;
}

extern "C" elph_status elph_set_gemm_chunk(elph_ctx ctx, int64_t bytes) {
  CHECK_CTX(ctx);
  if (bytes < ((int64_t)1 << 20)) {
    ctx->err = "GEMM output chunk must be at least 1 MiB";
    return ELPH_EINVAL;
  }
  ctx->gemm_chunk = (size_t)bytes;
  return ELPH_OK;
}

extern "C" elph_status elph_memory_held(elph_ctx ctx, int64_t* bytes) {
  CHECK_CTX(ctx);
  if (!bytes) {
    ctx->err = "null output";
    return ELPH_EINVAL;
  }
  *bytes = (int64_t)held_bytes(ctx);
  return ELPH_OK;
}

extern "C" elph_status elph_set_refine(elph_ctx ctx, double theta) {
  CHECK_CTX(ctx);
  if (!(theta >= 0.0) || !std::isfinite(theta)) {
    ctx->err = "refinement threshold must be finite and >= 0";
    return ELPH_EINVAL;
  }
  if (theta != ctx->refine_theta) {
    // the codes stay with the store; only the rates are reduced again
    ctx->refine_theta = theta;
    ctx->rates_valid = false;
  }
  return ELPH_OK;
}

extern "C" elph_status elph_refine_info(elph_ctx ctx, int64_t* stats, double* ms) {
  CHECK_CTX(ctx);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (stats)
    for (int k = 0; k < 8; ++k) stats[k] = ctx->ref_stats[k];
  if (ms) {
    *ms = -1.0;
    if (ctx->ev_recorded[5]) {
      float v = 0.f;
      HIPCHK(hipEventElapsedTime(&v, ctx->ev[10], ctx->ev[11]));
      *ms = v;
    }
  }
  return ELPH_OK;
}

__global__ void k_rho_decode(int64_t n, int nbr, int stride, const uint8_t* __restrict__ rho,
                             double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = rho_decode(rho[(t / nbr) * stride + t % nbr]);
}

extern "C" elph_status elph_refine_estimates(elph_ctx ctx, double* rel_err) {
  CHECK_CTX(ctx);
  if (!rel_err) {
    ctx->err = "null output";
    return ELPH_EINVAL;
  }
  if (!ctx->store_ready || !ctx->rho_valid) {
    ctx->err = "no error estimates: the vertex store of a GEMM form with the refinement on is needed";
    return ELPH_ESTATE;
  }
  const int64_t n = ctx->nstates * ctx->nstates * ctx->nbr;
  hipLaunchKernelGGL(k_rho_decode, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, n, ctx->nbr,
                     ctx->rho_stride, ctx->d_rho, rel_err);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ELPH_OK;
}

extern "C" elph_status elph_timing_extra(elph_ctx ctx, double* ms) {
  CHECK_CTX(ctx);
  if (!ms) return ELPH_EINVAL;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *ms = -1.0;
  if (ctx->ev_recorded[4]) {
    float v = 0.f;
    HIPCHK(hipEventElapsedTime(&v, ctx->ev[8], ctx->ev[9]));
    *ms = v;
  }
  return ELPH_OK;
}

extern "C" void elph_destroy(elph_ctx ctx) {
  if (!ctx) return;
  if (!ctx->hip_dead) (void)hipStreamSynchronize(ctx->stream);
  for (int e = 0; e < 12; ++e)
    if (ctx->ev[e]) (void)hipEventDestroy(ctx->ev[e]);
  for (auto& b : ctx->allocs) (void)hipFree(b.first);
  for (auto& b : ctx->pool) (void)hipFree(b.first);
  ctx->allocs.clear();
  ctx->pool.clear();
  if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
  delete ctx;
}

extern "C" const char* elph_last_error(elph_ctx ctx) {
  if (!ctx) return g_create_err.c_str();
  return ctx->err.c_str();
}

// Drop every derived table, operand and the vertex store (inputs stay).
static void drop_derived(elph_ctx ctx) {
  void** ptrs[] = {(void**)&ctx->d_eps_all, (void**)&ctx->d_kidx,      (void**)&ctx->d_kept,
                   (void**)&ctx->d_soff,    (void**)&ctx->d_state_k,   (void**)&ctx->d_state_kidx,
                   (void**)&ctx->d_state_m, (void**)&ctx->d_eps,       (void**)&ctx->d_vel,
                   (void**)&ctx->d_group,   (void**)&ctx->d_U,         (void**)&ctx->d_hw,
                   (void**)&ctx->d_Lq,      (void**)&ctx->d_vph,       (void**)&ctx->d_Ee,
                   (void**)&ctx->d_Ep,      (void**)&ctx->d_Ae,        (void**)&ctx->d_Ap,
                   (void**)&ctx->d_gR,      (void**)&ctx->d_B2,        (void**)&ctx->d_Bp,
                   (void**)&ctx->d_Bm,      (void**)&ctx->d_we_part,   (void**)&ctx->d_order,
                   (void**)&ctx->d_goff,    (void**)&ctx->d_we_cache,  (void**)&ctx->d_wph_cache,
                   (void**)&ctx->d_poff,    (void**)&ctx->d_plist,     (void**)&ctx->d_frohlich, (void**)&ctx->d_ppk,
                   (void**)&ctx->d_ustate,  (void**)&ctx->d_rho,       (void**)&ctx->d_b2n,
                   (void**)&ctx->d_i3_fold};
  for (void** p : ptrs) {
    dev_free(ctx, *p);
    *p = nullptr;
  }
  ctx->we_part_len = 0;
  ctx->tables_ready = ctx->operands_ready = ctx->store_ready = false;
  ctx->groups_ready = ctx->rates_valid = ctx->pairs_ready = ctx->pairs_failed = false;
  ctx->rho_valid = false;
  ctx->nkept = ctx->nstates = 0;
  ctx->ngroups = 0;
}

extern "C" elph_status elph_reset(elph_ctx ctx, int32_t what) {
  CHECK_CTX(ctx);
  if (what != ELPH_RESET_ALL && what != ELPH_RESET_STORE && what != ELPH_RESET_TRIM) {
    ctx->err = "unknown reset mode";
    return ELPH_EINVAL;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (what == ELPH_RESET_ALL) {
    drop_derived(ctx);
  } else if (what == ELPH_RESET_STORE) {
    ctx->store_ready = false;
    ctx->rates_valid = false;
  } else {
    drop_derived(ctx);
    // the FP64 vertex operand of the refinement depends on the inputs only
    // and survives the other resets
    dev_free(ctx, ctx->d_gR64);
    ctx->d_gR64 = nullptr;
    pool_trim(ctx);
  }
  return ELPH_OK;
}

static elph_status sizes_impl(elph_ctx ctx, elph_sizes_t* out) {
  CHECK_CTX(ctx);
  if (!out) {
    ctx->err = "null output";
    return ELPH_EINVAL;
  }
  elph_status st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  out->nk = ctx->nk;
  out->nkept = ctx->nkept;
  out->nstates = ctx->nstates;
  out->nwann = ctx->nb;
  out->nbr = ctx->nbr;
  out->nterms = ctx->nstates * ctx->nstates * ctx->nbr;
  out->hw_max_eV = ctx->hw_max;
  out->ngroups = ctx->ngroups;
  out->reserved = 0;
  return ELPH_OK;
}

extern "C" elph_status elph_sizes(elph_ctx ctx, elph_sizes_t* out) {
  return enomem_guard(ctx, sizes_impl(ctx, out));
}

static elph_status tables_impl(elph_ctx ctx, int32_t* state_k, int32_t* state_m, double* eps, double* vel,
                               double* hw, double* vph) {
  CHECK_CTX(ctx);
  elph_status st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, nm = ctx->nk * ctx->nbr;
  if (state_k) HIPCHK(hipMemcpyAsync(state_k, ctx->d_state_k, M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (state_m) HIPCHK(hipMemcpyAsync(state_m, ctx->d_state_m, M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  if (eps) HIPCHK(hipMemcpyAsync(eps, ctx->d_eps, M * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (vel) HIPCHK(hipMemcpyAsync(vel, ctx->d_vel, M * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (hw) HIPCHK(hipMemcpyAsync(hw, ctx->d_hw, nm * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (vph) HIPCHK(hipMemcpyAsync(vph, ctx->d_vph, nm * 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  return ELPH_OK;
}

extern "C" elph_status elph_tables(elph_ctx ctx, int32_t* state_k, int32_t* state_m, double* eps, double* vel,
                                   double* hw, double* vph) {
  return enomem_guard(ctx, tables_impl(ctx, state_k, state_m, eps, vel, hw, vph));
}

static elph_status interp_g_impl(elph_ctx ctx, int64_t npairs, const int32_t* kidx, const int32_t* qidx,
                                 double* g_out) {
  CHECK_CTX(ctx);
  if (npairs < 0 || (npairs > 0 && (!kidx || !qidx || !g_out))) {
    ctx->err = "invalid pair list or output";
    return ELPH_EINVAL;
  }
  return interp_g(ctx, npairs, kidx, qidx, g_out);
}

extern "C" elph_status elph_interp_g(elph_ctx ctx, int64_t npairs, const int32_t* kidx, const int32_t* qidx,
                                     double* g_out) {
  return enomem_guard(ctx, interp_g_impl(ctx, npairs, kidx, qidx, g_out));
}

extern "C" elph_status elph_interp_g_noalloc(elph_ctx ctx, int64_t npairs, const int32_t* kidx,
                                             const int32_t* qidx, double* g_out) {
  CHECK_CTX(ctx);
  if (npairs < 0 || (npairs > 0 && (!kidx || !qidx || !g_out))) {
    ctx->err = "invalid pair list or output";
    return ELPH_EINVAL;
  }
  return interp_g_noalloc(ctx, npairs, kidx, qidx, g_out);
}

static elph_status check_T(elph_ctx ctx, double T) {
  if (!(T > 0) || !std::isfinite(T)) {
    ctx->err = "temperature must be positive";
    return ELPH_EINVAL;
  }
  return ELPH_OK;
}

template <typename ST>
__global__ void k_x_inplace(int64_t M, int nbr, int n0, int n1, int n2, const int32_t* __restrict__ st_k,
                            const double* __restrict__ f, const double* __restrict__ omf,
                            const double* __restrict__ nocc, double* __restrict__ Xp, double* __restrict__ Xm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * M * nbr) return;
  const int s = (int)(t % nbr);
  const int64_t ij = t / nbr;
  const int64_t i = ij / M, j = ij % M;
  const int64_t kj = st_k[j], ki = st_k[i];
  int cj = (int)(kj % n2), ci = (int)(ki % n2);
  int64_t tj = kj / n2, ti = ki / n2;
  int bj = (int)(tj % n1), bi = (int)(ti % n1);
  int aj = (int)(tj / n1), ai = (int)(ti / n1);
  int a = aj - ai; if (a < 0) a += n0;
  int b = bj - bi; if (b < 0) b += n1;
  int c = cj - ci; if (c < 0) c += n2;
  const int64_t q = ((int64_t)a * n1 + b) * n2 + c;
  const double n = nocc[q * nbr + s];
  const double occ = f[i] * omf[j];
  Xp[t] *= occ * n;
  Xm[t] *= occ * (1.0 + n);
}

extern "C" elph_status elph_set_ifc3(elph_ctx ctx, int32_t n, const int32_t* rj, const int32_t* rk,
                                     const double* psi) {
  CHECK_CTX(ctx);
  return elph::phph_set_ifc3(ctx, n, rj, rk, psi);
}

static elph_status phph_vertex_impl(elph_ctx ctx, int64_t npairs, const int32_t* q, const int32_t* qp,
                                    double* V2) {
  CHECK_CTX(ctx);
  return elph::phph_vertex(ctx, npairs, q, qp, V2);
}

extern "C" elph_status elph_phph_vertex(elph_ctx ctx, int64_t npairs, const int32_t* q, const int32_t* qp,
                                        double* V2) {
  return enomem_guard(ctx, phph_vertex_impl(ctx, npairs, q, qp, V2));
}

static elph_status phph_rates_impl(elph_ctx ctx, double T_K, double sigma_eV, double* W_ph) {
  CHECK_CTX(ctx);
  elph_status st = check_T(ctx, T_K);
  if (st != ELPH_OK) return st;
  return elph::phph_rates(ctx, T_K, sigma_eV, W_ph);
}

extern "C" elph_status elph_phph_rates(elph_ctx ctx, double T_K, double sigma_eV, double* W_ph) {
  return enomem_guard(ctx, phph_rates_impl(ctx, T_K, sigma_eV, W_ph));
}

extern "C" elph_status elph_set_phph(elph_ctx ctx, double sigma_eV) {
  CHECK_CTX(ctx);
  if (!(sigma_eV >= 0.0) || !std::isfinite(sigma_eV)) {
    ctx->err = "elph_set_phph: sigma must be finite and non-negative";
    return ELPH_EINVAL;
  }
  ctx->phph_sigma = sigma_eV;
  return ELPH_OK;
}

static elph_status phph_inscatter_impl(elph_ctx ctx, double T_K, double sigma_eV, const double* F,
                                       double* S) {
  CHECK_CTX(ctx);
  elph_status st = check_T(ctx, T_K);
  if (st != ELPH_OK) return st;
  return elph::phph_inscatter(ctx, T_K, sigma_eV, F, S);
}

extern "C" elph_status elph_phph_inscatter(elph_ctx ctx, double T_K, double sigma_eV, const double* F,
                                           double* S) {
  return enomem_guard(ctx, phph_inscatter_impl(ctx, T_K, sigma_eV, F, S));
}

extern "C" elph_status elph_set_polar(elph_ctx ctx, const double* zstar, const double* eps_inf, const double* tau) {
  CHECK_CTX(ctx);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!zstar) {
    if (ctx->d_nac) dev_free(ctx, ctx->d_nac);
    ctx->d_nac = nullptr;
    ctx->frohlich = false;
    drop_derived(ctx);
    return ELPH_OK;
  }
  if (!eps_inf) {
    ctx->err = "eps_inf is required with zstar";
    return ELPH_EINVAL;
  }
  const int na = ctx->na;
  for (int k = 0; k < 9 * na; ++k)
    if (!std::isfinite(zstar[k])) {
      ctx->err = "zstar is not finite";
      return ELPH_EINVAL;
    }
  const double* e = eps_inf;
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(e[k])) {
      ctx->err = "eps_inf is not finite";
      return ELPH_EINVAL;
    }
  const double scale = std::fabs(e[0]) + std::fabs(e[4]) + std::fabs(e[8]);
  if (std::fabs(e[1] - e[3]) > 1e-12 * scale || std::fabs(e[2] - e[6]) > 1e-12 * scale ||
      std::fabs(e[5] - e[7]) > 1e-12 * scale) {
    ctx->err = "eps_inf must be symmetric";
    return ELPH_EINVAL;
  }
  const double m1 = e[0], m2 = e[0] * e[4] - e[1] * e[3];
  const double m3 = e[0] * (e[4] * e[8] - e[5] * e[7]) - e[1] * (e[3] * e[8] - e[5] * e[6]) +
                    e[2] * (e[3] * e[7] - e[4] * e[6]);
  if (!(m1 > 0.0 && m2 > 0.0 && m3 > 0.0)) {
    ctx->err = "eps_inf must be positive definite";
    return ELPH_EINVAL;
  }
  // reciprocal basis: rows b_i with a_i . b_j = delta_ij, times 2 pi
  const double* L = ctx->lat;
  const double det = L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                     L[2] * (L[3] * L[7] - L[4] * L[6]);
  if (tau)
    for (int k = 0; k < 3 * na; ++k)
      if (!std::isfinite(tau[k])) {
        ctx->err = "tau is not finite";
        return ELPH_EINVAL;
      }
  std::vector<double> h(9 * na + 18 + 3 * na, 0.0);
  if (tau) std::memcpy(h.data() + 9 * na + 18, tau, 3 * na * sizeof(double));
  std::memcpy(h.data(), zstar, 9 * na * sizeof(double));
  std::memcpy(h.data() + 9 * na, eps_inf, 9 * sizeof(double));
  double* B = h.data() + 9 * na + 9;
  for (int i = 0; i < 3; ++i) {
    const double* a1 = L + 3 * ((i + 1) % 3);
    const double* a2 = L + 3 * ((i + 2) % 3);
    B[3 * i + 0] = 2.0 * kPi * (a1[1] * a2[2] - a1[2] * a2[1]) / det;
    B[3 * i + 1] = 2.0 * kPi * (a1[2] * a2[0] - a1[0] * a2[2]) / det;
    B[3 * i + 2] = 2.0 * kPi * (a1[0] * a2[1] - a1[1] * a2[0]) / det;
  }
  drop_derived(ctx);
  if (ctx->d_nac) dev_free(ctx, ctx->d_nac);
  ctx->d_nac = nullptr;
  ALLOC(ctx->d_nac, h.size() * sizeof(double));
  HIPCHK(hipMemcpy(ctx->d_nac, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  ctx->nac_coef = kCharge / (kEps0 * ctx->volume_A3) * 1e10;
  ctx->frohlich = tau != nullptr;
  if (ctx->frohlich) {
    // G box of the Ewald sum of Eq. 7: every G with (q+G).eps.(q+G) / (4 alpha) <= 40
    // for any q of the cell has |q+G| <= sqrt(160 alpha / lambda_min(eps)), and
    // |n_i| <= (|q+G| + sum |2 pi b|) |a_i| / (2 pi) + 1
    // a positive lower bound of the smallest eigenvalue of eps_inf: the larger
    // of Gershgorin's and det / trace^2 (the other two eigenvalues are below the trace)
    double gersh = INFINITY;
    for (int r = 0; r < 3; ++r)
      gersh = std::min(gersh, e[4 * r] - std::fabs(e[3 * r + (r + 1) % 3]) - std::fabs(e[3 * r + (r + 2) % 3]));
    const double tr = e[0] + e[4] + e[8];
    const double lmin = std::max(gersh, m3 / (tr * tr));
    const double alpha = 1.0 / (0.529177210903 * 0.529177210903);
    const double gmax = std::sqrt(4.0 * alpha * 40.0 / lmin);
    double bsum = 0.0;
    for (int i = 0; i < 3; ++i) bsum += std::sqrt(B[3 * i] * B[3 * i] + B[3 * i + 1] * B[3 * i + 1] + B[3 * i + 2] * B[3 * i + 2]);
    for (int i = 0; i < 3; ++i) {
      const double al = std::sqrt(L[3 * i] * L[3 * i] + L[3 * i + 1] * L[3 * i + 1] + L[3 * i + 2] * L[3 * i + 2]);
      ctx->fr_box[i] = (int)std::ceil((gmax + bsum) * al / (2.0 * kPi)) + 1;
    }
  }
  return ELPH_OK;
}

extern "C" elph_status elph_set_delta(elph_ctx ctx, int32_t method) {
  CHECK_CTX(ctx);
  if (method != ELPH_DELTA_GAUSS && method != ELPH_DELTA_TETRA && method != ELPH_DELTA_TRIANGLE) {
    ctx->err = "unknown delta method";
    return ELPH_EINVAL;
  }
  if (method != ctx->delta) {
    ctx->delta = method;
    ctx->store_ready = false;
    ctx->rates_valid = false;
  }
  return ELPH_OK;
}

static elph_status transition_probs_impl(elph_ctx ctx, double T_K, double* Xp, double* Xm, int32_t store_B) {
  CHECK_CTX(ctx);
  elph_status st = check_T(ctx, T_K);
  if (st != ELPH_OK) return st;
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  Thermal th;
  st = make_thermal(ctx, T_K, &th);
  if (st != ELPH_OK) return st;
  if (store_B) {
    st = ensure_store(ctx);
    if (st == ELPH_OK && (Xp || Xm)) st = x_from_store(ctx, th, Xp, Xm);
  } else if (Xp || Xm) {
    const int64_t n = ctx->nstates * ctx->nstates * ctx->nbr;
    double* a = Xp;
    double* b = Xm;
    void* tmp = nullptr;
    if (!a || !b) {
      if (dev_alloc(ctx, &tmp, (size_t)n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        free_thermal(ctx, &th);
        ctx->err = "device allocation failed";
        return ELPH_ENOMEM;
      }
      if (!a) a = (double*)tmp;
      if (!b) b = (double*)tmp;
    }
    st = run_vertex(ctx, a, b, true, nullptr, nullptr, nullptr);
    if (st == ELPH_OK) {
      hipLaunchKernelGGL(k_x_inplace<double>, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, ctx->nstates,
                         ctx->nbr, ctx->mesh[0], ctx->mesh[1], ctx->mesh[2], ctx->d_state_k, th.f, th.omf, th.nocc,
                         a, b);
      HIPCHK(hipGetLastError());
    }
    if (tmp) {
      HIPCHK(hipStreamSynchronize(ctx->stream));
      dev_free(ctx, tmp);
    }
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  free_thermal(ctx, &th);
  return st;
}

extern "C" elph_status elph_transition_probs(elph_ctx ctx, double T_K, double* Xp, double* Xm, int32_t store_B) {
  return enomem_guard(ctx, transition_probs_impl(ctx, T_K, Xp, Xm, store_B));
}

static elph_status scatt_rates_impl(elph_ctx ctx, double T_K, double* W_e, double* W_ph) {
  CHECK_CTX(ctx);
  elph_status st = check_T(ctx, T_K);
  if (st != ELPH_OK) return st;
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  Thermal th;
  st = make_thermal(ctx, T_K, &th);
  if (st != ELPH_OK) return st;
  if (!ctx->store_ready) {
    // the vertices into the store; every rate is then reduced from the
    // store (one definition of each rate: a later evaluation from the same
    // store, or from a saved one, gives the same bits), after the FP64
    // refinement of the terms whose error estimate a rate cannot absorb in
    // the GEMM forms
    const bool f64 = ctx->precision == ELPH_FP64;
    const size_t n = (size_t)ctx->nstates * ctx->nstates * ctx->nbr;
    if (!ctx->d_Bp) {
      void *a = nullptr, *b = nullptr;
      if (dev_alloc(ctx, &a, n * (f64 ? 8 : 4)) != hipSuccess || dev_alloc(ctx, &b, n * (f64 ? 8 : 4)) != hipSuccess) {
        (void)hipGetLastError();
        dev_free(ctx, a);
        free_thermal(ctx, &th);
        ctx->err = "device allocation of the vertex store failed";
        return ELPH_ENOMEM;
      }
      ctx->d_Bp = a;
      ctx->d_Bm = b;
    }
    ctx->store_f32 = !f64;
    st = run_vertex(ctx, ctx->d_Bp, ctx->d_Bm, f64, nullptr, nullptr, nullptr);
    if (st == ELPH_OK) ctx->store_ready = true;
  }
  if (st == ELPH_OK) st = rates_from_store(ctx, th, W_e, W_ph);
  if (st == ELPH_OK && W_e && W_ph) {
    // keep the rates for an iteration at the same temperature
    const int64_t M = ctx->nstates, nm = ctx->nk * ctx->nbr;
    if (!ctx->d_we_cache) ALLOC(ctx->d_we_cache, M * sizeof(double));
    if (!ctx->d_wph_cache) ALLOC(ctx->d_wph_cache, nm * sizeof(double));
    HIPCHK(hipMemcpyAsync(ctx->d_we_cache, W_e, M * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->d_wph_cache, W_ph, nm * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    ctx->rates_T = T_K;
    ctx->rates_valid = true;
  } else {
    ctx->rates_valid = false;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  free_thermal(ctx, &th);
  return st;
}

extern "C" elph_status elph_scatt_rates(elph_ctx ctx, double T_K, double* W_e, double* W_ph) {
  return enomem_guard(ctx, scatt_rates_impl(ctx, T_K, W_e, W_ph));
}

static elph_status iterate_impl(elph_ctx ctx, double T_K, const double* W_ph_ext, int32_t level, double tol,
                                int32_t maxit, double* I, double* J, double* F, double* G, double* tensors,
                                int32_t* iters, double* ko_residual) {
  CHECK_CTX(ctx);
  elph_status st = check_T(ctx, T_K);
  if (st != ELPH_OK) return st;
  if (level < ELPH_LEVEL_RTA || level > ELPH_LEVEL_COUPLED || !(tol > 0) || maxit < 1) {
    ctx->err = "invalid level, tolerance or maxit";
    return ELPH_EINVAL;
  }
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  int it = 0;
  mark(ctx, 6);
  st = iterate(ctx, T_K, W_ph_ext, level, tol, maxit, I, J, F, G, tensors, &it, ko_residual);
  mark(ctx, 7);
  if (iters) *iters = it;
  return st;
}

extern "C" elph_status elph_iterate(elph_ctx ctx, double T_K, const double* W_ph_ext, int32_t level, double tol,
                                    int32_t maxit, double* I, double* J, double* F, double* G, double* tensors,
                                    int32_t* iters, double* ko_residual) {
  return enomem_guard(ctx, iterate_impl(ctx, T_K, W_ph_ext, level, tol, maxit, I, J, F, G, tensors, iters, ko_residual));
}

static elph_status ko_enforce_impl(elph_ctx ctx, double T_K, double* I, const double* J, const double* F,
                                   const double* G, double* tensors, double* lambda, double* ko_residual) {
  CHECK_CTX(ctx);
  elph_status st = check_T(ctx, T_K);
  if (st != ELPH_OK) return st;
  if (!I || !J || !F || !G) {
    ctx->err = "I, J, F and G are required";
    return ELPH_EINVAL;
  }
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  return ko_enforce(ctx, T_K, I, J, F, G, tensors, lambda, ko_residual);
}

extern "C" elph_status elph_ko_enforce(elph_ctx ctx, double T_K, double* I, const double* J, const double* F,
                                       const double* G, double* tensors, double* lambda, double* ko_residual) {
  return enomem_guard(ctx, ko_enforce_impl(ctx, T_K, I, J, F, G, tensors, lambda, ko_residual));
}

// ---------------------------------------------------------------------------
// batches

struct elph_batch_s {
  BatchImpl* impl = nullptr;
  std::string err;
};

static thread_local std::string g_batch_err;

extern "C" elph_status elph_batch_create(int32_t n, const elph_ctx* ctxs, elph_batch* out) {
  if (!out || n < 1 || !ctxs) {
    g_batch_err = "invalid arguments";
    return ELPH_EINVAL;
  }
  *out = nullptr;
  std::vector<elph_ctx> v(ctxs, ctxs + n);
  for (elph_ctx c : v) {
    if (!c) {
      g_batch_err = "null context";
      return ELPH_EINVAL;
    }
    if (c->delta != ELPH_DELTA_GAUSS) {
      g_batch_err = "batches support the Gaussian delta only";
      return ELPH_EINVAL;
    }
  }
  std::string err;
  BatchImpl* impl = batch_new(v, &err);
  if (!impl) {
    g_batch_err = err;
    return ELPH_EINVAL;
  }
  elph_batch b = new (std::nothrow) elph_batch_s();
  if (!b) {
    batch_free(impl);
    g_batch_err = "host allocation failed";
    return ELPH_ENOMEM;
  }
  b->impl = impl;
  *out = b;
  return ELPH_OK;
}

extern "C" void elph_batch_destroy(elph_batch b) {
  if (!b) return;
  batch_free(b->impl);
  delete b;
}

extern "C" const char* elph_batch_last_error(elph_batch b) {
  if (!b) return g_batch_err.c_str();
  return b->err.c_str();
}

extern "C" elph_status elph_batch_scatt_rates(elph_batch b, double T_K, double* const* W_e, double* const* W_ph,
                                              int32_t use_graph) {
  if (!b) return ELPH_EINVAL;
  b->err.clear();
  if (!(T_K > 0) || !std::isfinite(T_K)) {
    b->err = "temperature must be positive";
    return ELPH_EINVAL;
  }
  elph_status st = batch_rates(b->impl, T_K, W_e, W_ph, use_graph != 0);
  if (st != ELPH_OK) b->err = batch_error(b->impl);
  return st;
}

extern "C" elph_status elph_batch_tune(elph_batch b, double T_K, int32_t* choice, double* best_ms) {
  if (!b) return ELPH_EINVAL;
  b->err.clear();
  if (!(T_K > 0) || !std::isfinite(T_K)) {
    b->err = "temperature must be positive";
    return ELPH_EINVAL;
  }
  int ch[3] = {0, 0, 0};
  elph_status st = batch_tune(b->impl, T_K, ch, best_ms);
  if (st != ELPH_OK) b->err = batch_error(b->impl);
  if (choice) {
    choice[0] = ch[0];
    choice[1] = ch[1];
    choice[2] = ch[2];
  }
  return st;
}

extern "C" elph_status elph_batch_set_shape(elph_batch b, int32_t blocks_per_cu, int32_t cost_ordered,
                                            int32_t tile_rows) {
  if (!b) return ELPH_EINVAL;
  b->err.clear();
  if (tile_rows != 64 && tile_rows != 128) {
    b->err = "tile rows must be 64 or 128";
    return ELPH_EINVAL;
  }
  elph_status st = batch_set_shape(b->impl, blocks_per_cu, cost_ordered != 0, tile_rows / 32);
  if (st != ELPH_OK) b->err = batch_error(b->impl);
  return st;
}
