// Learned screen of negligible transition-probability terms.
//
// Samples: the exact vertex of Eq. 6 (interp_g) at chosen mesh pairs gives the
// target log10 |g|^2 of every (s, n, m) together with its feature row.
// Screen: every term (i initial state, j final state, branch s) of the window
// gets a predicted X from the network's |g|^2 and the exact Gaussian factors
// and occupations of Eq. 8; step-2 tiles whose predicted terms are all below
// tau times the largest predicted term of their initial state are skipped.
// The energy mode is the exact alternative: a term is kept when one of its
// Gaussian factors exceeds exp(-18).
#include "common.h"
#include "devutil.h"
#include "mlp.h"
#include "tables.h"
#include "vertex.h"

#include <cmath>
#include <cstring>

namespace elph {

__device__ inline unsigned short to_bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline void mesh_frac(int k, MeshDims md, float* out) {
  const int c = k % md.n2, t = k / md.n2;
  const int b = t % md.n1, a = t / md.n1;
  out[0] = (float)a / (float)md.n0;
  out[1] = (float)b / (float)md.n1;
  out[2] = (float)c / (float)md.n2;
}

__device__ inline int mesh_add(int k, int q, MeshDims md) {
  const int kc = k % md.n2, kt = k / md.n2, kb = kt % md.n1, ka = kt / md.n1;
  const int qc = q % md.n2, qt = q / md.n2, qb = qt % md.n1, qa = qt / md.n1;
  int c = kc + qc; if (c >= md.n2) c -= md.n2;
  int b = kb + qb; if (b >= md.n1) b -= md.n1;
  int a = ka + qa; if (a >= md.n0) a -= md.n0;
  return (a * md.n1 + b) * md.n2 + c;
}

// Feature row (length 9 + 2 nb + nbr) of the term (k, q, m, n, s); written
// through put(index, value)
template <typename Put>
__device__ inline void features(int k, int q, int m, int n, int s, double em, double en, double hw, double inv_hwmax,
                                int nb, int nbr, MeshDims md, Put put) {
  float f[3];
  mesh_frac(k, md, f);
  put(0, f[0]);
  put(1, f[1]);
  put(2, f[2]);
  mesh_frac(q, md, f);
  put(3, f[0]);
  put(4, f[1]);
  put(5, f[2]);
  put(6, (float)em);
  put(7, (float)en);
  put(8, (float)(hw * inv_hwmax));
  for (int b = 0; b < nb; ++b) put(9 + b, b == m ? 1.f : 0.f);
  for (int b = 0; b < nb; ++b) put(9 + nb + b, b == n ? 1.f : 0.f);
  for (int b = 0; b < nbr; ++b) put(9 + 2 * nb + b, b == s ? 1.f : 0.f);
}

// one thread per (pair, s, n, m), in the order of interp_g's output
__global__ void k_screen_samples(int64_t total, int nb, int nbr, int nin, MeshDims md,
                                 const int32_t* __restrict__ kidx, const int32_t* __restrict__ qidx,
                                 const double* __restrict__ eps_all, const double* __restrict__ hw, double inv_hwmax,
                                 double mu, const double* __restrict__ g, float* __restrict__ x,
                                 float* __restrict__ t) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int m = (int)(e % nb);
  const int n = (int)((e / nb) % nb);
  const int s = (int)((e / (nb * nb)) % nbr);
  const int64_t p = e / ((int64_t)nb * nb * nbr);
  const int k = kidx[p], q = qidx[p];
  const int kq = mesh_add(k, q, md);
  float* xr = x + e * nin;
  features(k, q, m, n, s, eps_all[(int64_t)k * nb + m] - mu, eps_all[(int64_t)kq * nb + n] - mu,
           hw[(int64_t)q * nbr + s], inv_hwmax, nb, nbr, md, [&](int c, float v) { xr[c] = v; });
  const double gr = g[2 * e], gi = g[2 * e + 1];
  t[e] = (float)log10(fmax(gr * gr + gi * gi, 1e-12));
}

// BF16 feature rows of the terms (i0 + r / (M nbr), j, s) into x [rows][in_pad]
__global__ void k_screen_rows(int64_t i0, int64_t rows, int64_t M, int nb, int nbr, int in_pad, MeshDims md,
                              const int32_t* __restrict__ st_k, const int32_t* __restrict__ st_m,
                              const double* __restrict__ eps, const double* __restrict__ hw, double inv_hwmax,
                              double mu, unsigned short* __restrict__ x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int s = (int)(r % nbr);
  const int64_t j = (r / nbr) % M;
  const int64_t i = i0 + r / ((int64_t)nbr * M);
  const int ki = st_k[i], kj = st_k[j];
  const int q = q_between(kj, ki, md.n0, md.n1, md.n2);
  unsigned short* xr = x + r * in_pad;
  for (int c = 9 + 2 * nb + nbr; c < in_pad; ++c) xr[c] = 0;
  features(ki, q, st_m[i], st_m[j], s, eps[i] - mu, eps[j] - mu, hw[(int64_t)q * nbr + s], inv_hwmax, nb, nbr, md,
           [&](int c, float v) { xr[c] = to_bf(v); });
}

// Predicted X (up to the common prefactor) of the chunk's terms and the row
// maxima of its initial states: one block per initial state.
__global__ void __launch_bounds__(256) k_screen_predict(int64_t i0, int64_t M, int nbr, MeshDims md, double inv2s2,
                                                        double omega_min, const int32_t* __restrict__ st_k,
                                                        const double* __restrict__ eps, const double* __restrict__ hw,
                                                        const double* __restrict__ f, const double* __restrict__ omf,
                                                        const double* __restrict__ nocc, const float* __restrict__ y,
                                                        float* __restrict__ xs, float* __restrict__ rowmax) {
  __shared__ float sh[256];
  const int64_t il = blockIdx.x, i = i0 + il;
  const int ki = st_k[i];
  const double ei = eps[i], fi = f[i];
  float mx = 0.f;
  for (int64_t t = threadIdx.x; t < M * nbr; t += 256) {
    const int64_t j = t / nbr;
    const int s = (int)(t - j * nbr);
    const int q = q_between(st_k[j], ki, md.n0, md.n1, md.n2);
    const double w = hw[(int64_t)q * nbr + s];
    float v = 0.f;
    if (w >= omega_min) {
      const double de = eps[j] - ei, n = nocc[(int64_t)q * nbr + s];
      const double gp = exp(-(de - w) * (de - w) * inv2s2), gm = exp(-(de + w) * (de + w) * inv2s2);
      v = (float)(exp10((double)y[il * M * nbr + t]) * fi * omf[j] * (gp * n + gm * (1.0 + n)));
    }
    xs[il * M * nbr + t] = v;
    mx = fmaxf(mx, v);
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) rowmax[il] = sh[0];
}

// keep[(j/32) nt + i/32] = 1 for every kept term (all writers store 1)
__global__ void k_screen_mark(int64_t i0, int64_t rows, int64_t M, int nbr, int64_t nt, double tau,
                              const float* __restrict__ xs, const float* __restrict__ rowmax,
                              uint8_t* __restrict__ keep) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t il = r / ((int64_t)nbr * M);
  const int64_t j = (r / nbr) % M;
  const float v = xs[r], mx = rowmax[il];
  if (v > 0.f && (double)v >= tau * (double)mx) keep[(j / 32) * nt + (i0 + il) / 32] = 1;
}

// energy screen: keep a term when exp(-(dE -/+ hw)^2 / 2 sigma^2) >= exp(-18)
__global__ void k_screen_energy(int64_t M, int nbr, MeshDims md, double inv2s2, double omega_min, int64_t nt,
                                const int32_t* __restrict__ st_k, const double* __restrict__ eps,
                                const double* __restrict__ hw, uint8_t* __restrict__ keep) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M * M * nbr) return;
  const int s = (int)(r % nbr);
  const int64_t ij = r / nbr;
  const int64_t i = ij / M, j = ij - i * M;
  const int q = q_between(st_k[j], st_k[i], md.n0, md.n1, md.n2);
  const double w = hw[(int64_t)q * nbr + s];
  if (w < omega_min) return;
  const double de = eps[j] - eps[i];
  const double a = fmin((de - w) * (de - w), (de + w) * (de + w)) * inv2s2;
  if (a <= 18.0) keep[(j / 32) * nt + i / 32] = 1;
}

}  // namespace elph

using namespace elph;

extern "C" int32_t elph_screen_nin(elph_ctx ctx) { return ctx ? 9 + 2 * ctx->nb + ctx->nbr : 0; }

extern "C" elph_status elph_screen_samples(elph_ctx ctx, int64_t npairs, const int32_t* kidx, const int32_t* qidx,
                                           float* x, float* t) {
  if (!ctx) return ELPH_EINVAL;
  if (ctx->hip_dead) {
    ctx->err = "context unusable after a HIP error";
    return ELPH_ESTATE;
  }
  ctx->err.clear();
  if (npairs < 0 || (npairs > 0 && (!kidx || !qidx || !x || !t))) {
    ctx->err = "bad sizes or null pointers";
    return ELPH_EINVAL;
  }
  if (npairs == 0) return ELPH_OK;
  elph_status st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  const int64_t total = npairs * ctx->nbr * ctx->nb * ctx->nb;
  double* g = nullptr;
  ALLOC(g, total * 2 * sizeof(double));
  st = interp_g(ctx, npairs, kidx, qidx, g);
  if (st != ELPH_OK) return st;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  const int nin = 9 + 2 * ctx->nb + ctx->nbr;
  hipLaunchKernelGGL(k_screen_samples, dim3(blocks_for(total, 256)), dim3(256), 0, ctx->stream, total, ctx->nb,
                     ctx->nbr, nin, md, kidx, qidx, ctx->d_eps_all, ctx->d_hw, 1.0 / ctx->hw_max, ctx->mu, g, x, t);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dev_free(ctx, g);
  return ELPH_OK;
}

extern "C" elph_status elph_scatt_rates_screened(elph_ctx ctx, elph_mlp m, int32_t mode, double tau, double T_K,
                                                 double* W_e, double* W_ph, double* stats) {
  if (!ctx) return ELPH_EINVAL;
  if (ctx->hip_dead) {
    ctx->err = "context unusable after a HIP error";
    return ELPH_ESTATE;
  }
  ctx->err.clear();
  if (mode < ELPH_SCREEN_NONE || mode > ELPH_SCREEN_MLP || !(T_K > 0) || !std::isfinite(T_K)) {
    ctx->err = "unknown screen mode or bad temperature";
    return ELPH_EINVAL;
  }
  if (ctx->delta != ELPH_DELTA_GAUSS) {
    ctx->err = "the screened rates support the Gaussian delta only";
    return ELPH_EINVAL;
  }
  if (mode == ELPH_SCREEN_MLP && (!m || !(tau > 0.0 && tau < 1.0) || m->hip_dead)) {
    ctx->err = "the MLP screen needs a live network and 0 < tau < 1";
    return ELPH_EINVAL;
  }
  elph_status st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  if (mode == ELPH_SCREEN_MLP && m->nin != 9 + 2 * ctx->nb + ctx->nbr) {
    ctx->err = "network input size differs from the context's screen features";
    return ELPH_EINVAL;
  }
  st = build_operands(ctx);  // fixes m_pad
  if (st != ELPH_OK) return st;
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, nbr = ctx->nbr, nt = ctx->m_pad / 32;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  const double inv2s2 = 1.0 / (2.0 * ctx->sigma * ctx->sigma);
  uint8_t* keep = nullptr;
  ALLOC(keep, nt * nt);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  int64_t evaluated = 0;
  if (mode == ELPH_SCREEN_NONE) {
    HIPCHK(hipMemsetAsync(keep, 1, nt * nt, s));
  } else {
    HIPCHK(hipMemsetAsync(keep, 0, nt * nt, s));
    evaluated = M * M * nbr;
    if (mode == ELPH_SCREEN_ENERGY) {
      hipLaunchKernelGGL(k_screen_energy, dim3(blocks_for(M * M * nbr, 256)), dim3(256), 0, s, M, (int)nbr, md,
                         inv2s2, ctx->omega_min, nt, ctx->d_state_k, ctx->d_eps, ctx->d_hw, keep);
    } else {
      Thermal th;
      st = make_thermal(ctx, T_K, &th);
      if (st != ELPH_OK) return st;
      const int64_t per_i = M * nbr;
      int64_t ci = ((int64_t)1 << 20) / per_i;
      if (ci < 1) ci = 1;
      if (ci > M) ci = M;
      float *xs = nullptr, *rowmax = nullptr, *y = nullptr;
      ALLOC(xs, ci * per_i * sizeof(float));
      ALLOC(rowmax, ci * sizeof(float));
      ALLOC(y, ci * per_i * sizeof(float));
      hipStream_t ms = m->stream;
      m->stream = s;  // network kernels on the context stream
      st = mlp_reserve(m, ci * per_i);
      if (st != ELPH_OK) ctx->err = "network: " + m->err;
      for (int64_t i0 = 0; st == ELPH_OK && i0 < M; i0 += ci) {
        const int64_t nrow_i = (M - i0 < ci) ? M - i0 : ci;
        const int64_t rows = nrow_i * per_i;
        hipLaunchKernelGGL(k_screen_rows, dim3(blocks_for(rows, 256)), dim3(256), 0, s, i0, rows, M, ctx->nb,
                           (int)nbr, m->in_pad, md, ctx->d_state_k, ctx->d_state_m, ctx->d_eps, ctx->d_hw,
                           1.0 / ctx->hw_max, ctx->mu, m->d_x);
        st = mlp_forward_rows(m, rows, false, y);
        if (st != ELPH_OK) {
          ctx->err = "network: " + m->err;
          break;
        }
        hipLaunchKernelGGL(k_screen_predict, dim3((unsigned)nrow_i), dim3(256), 0, s, i0, M, (int)nbr, md, inv2s2,
                           ctx->omega_min, ctx->d_state_k, ctx->d_eps, ctx->d_hw, th.f, th.omf, th.nocc, y, xs,
                           rowmax);
        hipLaunchKernelGGL(k_screen_mark, dim3(blocks_for(rows, 256)), dim3(256), 0, s, i0, rows, M, (int)nbr, nt,
                           tau, xs, rowmax, keep);
      }
      m->stream = ms;
      HIPCHK(hipStreamSynchronize(s));
      dev_free(ctx, xs);
      dev_free(ctx, rowmax);
      dev_free(ctx, y);
      free_thermal(ctx, &th);
      if (st != ELPH_OK) return st;
    }
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipGetLastError());
  // screened vertices and rates
  ctx->d_tile_keep = keep;
  ctx->store_ready = false;
  st = elph_scatt_rates(ctx, T_K, W_e, W_ph);
  ctx->d_tile_keep = nullptr;
  if (st != ELPH_OK) return st;
  std::vector<uint8_t> hk(nt * nt);
  HIPCHK(hipMemcpy(hk.data(), keep, nt * nt, hipMemcpyDeviceToHost));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int64_t tiles = 0, kept = 0;
  for (int64_t bx = 0; bx < nt; ++bx)
    for (int64_t by = 0; by < nt; ++by)
      if (bx * 32 < M && by * 32 < M) {
        ++tiles;
        kept += hk[bx * nt + by] ? 1 : 0;
      }
  dev_free(ctx, keep);
  if (stats) {
    stats[0] = (double)tiles;
    stats[1] = (double)kept;
    stats[2] = (double)evaluated;
    stats[3] = (double)ms;
  }
  return ELPH_OK;
}
