// Learned screen of negligible transition-probability terms.
//
// Samples: the exact vertex of Eq. 6 (interp_g) at chosen mesh pairs gives the
// target log10 |g|^2 of every (s, n, m) together with its feature row.
// Screen: the states of the window are ranked by energy and cut into tiles of
// 32 final x 32 initial consecutive ranks, so that whole tiles lie far from
// the energy shell of Eq. 8.  The energy stage (exact) keeps a tile when one
// of its terms has a Gaussian factor of at least gauss_min.  The network
// stage gives every term of those tiles a predicted X from the network's
// |g|^2 and the exact Gaussian factors and occupations of Eq. 8, and keeps a
// tile when one of them is at least tau times the largest predicted X of its
// initial state (the W_e sum of Eq. 21), or its predicted X+ at least tau
// times the largest of its phonon mode (the W_ph sum of Eq. 25).  Skipped
// tiles have zero vertex-store entries.
#include "common.h"
#include "devutil.h"
#include "mlp.h"
#include "tables.h"
#include "vertex.h"

#include <algorithm>
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

// Tiles of the screen: 32 x 32 consecutive positions in the energy order
// (perm[pos] = state at rank pos); a term (initial state at position pi,
// final state at position pj, branch s) belongs to tile pj / 32 (row block,
// bx) x pi / 32 (column block, by), stored at keep[bx nt + by].

// Gaussian exponent min over +/- of (dE -/+ hw)^2 / 2 sigma^2 of a term, or
// a negative value for a mode below omega_min
__device__ inline double screen_arg(int64_t i, int64_t j, int s, int nbr, MeshDims md, double inv2s2,
                                    double omega_min, const int32_t* __restrict__ st_k,
                                    const double* __restrict__ eps, const double* __restrict__ hw, int* qout) {
  const int q = q_between(st_k[j], st_k[i], md.n0, md.n1, md.n2);
  *qout = q;
  const double w = hw[(int64_t)q * nbr + s];
  if (w < omega_min) return -1.0;
  const double de = eps[j] - eps[i];
  return fmin((de - w) * (de - w), (de + w) * (de + w)) * inv2s2;
}

// energy stage: keep a tile when one of its terms has a Gaussian factor at
// least exp(-amax); one thread per (pi, pj, s)
__global__ void k_screen_energy(int64_t M, int nbr, MeshDims md, double inv2s2, double omega_min, double amax,
                                int64_t nt, const int32_t* __restrict__ perm, const int32_t* __restrict__ st_k,
                                const double* __restrict__ eps, const double* __restrict__ hw,
                                uint8_t* __restrict__ keep) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M * M * nbr) return;
  const int s = (int)(r % nbr);
  const int64_t pp = r / nbr;
  const int64_t pi = pp / M, pj = pp - pi * M;
  int q;
  const double a = screen_arg(perm[pi], perm[pj], s, nbr, md, inv2s2, omega_min, st_k, eps, hw, &q);
  if (a >= 0.0 && a <= amax) keep[(pj / 32) * nt + pi / 32] = 1;
}

// BF16 feature rows of the terms of listed tiles: row r = (tile t, ii, jj, s)
// with t = r / (1024 nbr), s fastest; rows of padding positions are zero
__global__ void k_screen_rows(int64_t rows, const int32_t* __restrict__ tiles, int64_t M, int nb, int nbr,
                              int in_pad, MeshDims md, const int32_t* __restrict__ perm,
                              const int32_t* __restrict__ st_k, const int32_t* __restrict__ st_m,
                              const double* __restrict__ eps, const double* __restrict__ hw, double inv_hwmax,
                              double mu, unsigned short* __restrict__ x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t per = 1024 * (int64_t)nbr;
  const int64_t t = r / per;
  const int e = (int)(r - t * per);
  const int s = e % nbr, jj = (e / nbr) % 32, ii = e / (nbr * 32);
  const int64_t pj = (int64_t)tiles[2 * t] * 32 + jj, pi = (int64_t)tiles[2 * t + 1] * 32 + ii;
  unsigned short* xr = x + r * in_pad;
  if (pi >= M || pj >= M) {
    for (int c = 0; c < in_pad; ++c) xr[c] = 0;
    return;
  }
  const int64_t i = perm[pi], j = perm[pj];
  const int ki = st_k[i];
  const int q = q_between(st_k[j], ki, md.n0, md.n1, md.n2);
  for (int c = 9 + 2 * nb + nbr; c < in_pad; ++c) xr[c] = 0;
  features(ki, q, st_m[i], st_m[j], s, eps[i] - mu, eps[j] - mu, hw[(int64_t)q * nbr + s], inv_hwmax, nb, nbr, md,
           [&](int c, float v) { xr[c] = to_bf(v); });
}

// Predicted X+ and X- (up to the common prefactor) of the rows above from
// the network's log10 |g|^2 and the exact Gaussian factors and occupations of
// Eq. 8; zero for padding, modes below omega_min and terms the energy stage
// drops.  Running maxima of X+ + X- per initial-state position (rowmax: W_e
// of Eq. 21 sums them over a row) and of X+ per phonon mode (colmax: W_ph of
// Eq. 25 sums X+ over a mode), as FP32 bits: the values are not negative, so
// their order is that of the integers.
__device__ inline void atomic_max_pos(unsigned* p, float v) {
  if (v > 0.f && v > __uint_as_float(*p)) atomicMax(p, __float_as_uint(v));
}

__global__ void k_screen_predict(int64_t rows, const int32_t* __restrict__ tiles, int64_t M, int nbr, MeshDims md,
                                 double inv2s2, double omega_min, double amax, const int32_t* __restrict__ perm,
                                 const int32_t* __restrict__ st_k, const double* __restrict__ eps,
                                 const double* __restrict__ hw, const double* __restrict__ f,
                                 const double* __restrict__ omf, const double* __restrict__ nocc,
                                 const float* __restrict__ y, float2* __restrict__ xs, unsigned* rowmax,
                                 unsigned* colmax) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = r < rows;
  const int64_t per = 1024 * (int64_t)nbr;
  const int64_t t = live ? r / per : 0;
  const int e = live ? (int)(r - t * per) : 0;
  const int s = e % nbr, jj = (e / nbr) % 32, ii = e / (nbr * 32);
  const int64_t pj = (int64_t)tiles[2 * t] * 32 + jj, pi = (int64_t)tiles[2 * t + 1] * 32 + ii;
  float xp = 0.f, xm = 0.f;
  int q = 0;
  if (live && pi < M && pj < M) {
    const int64_t i = perm[pi], j = perm[pj];
    const double a = screen_arg(i, j, s, nbr, md, inv2s2, omega_min, st_k, eps, hw, &q);
    if (a >= 0.0 && a <= amax) {
      const double w = hw[(int64_t)q * nbr + s], de = eps[j] - eps[i], n = nocc[(int64_t)q * nbr + s];
      const double c = exp10((double)y[r]) * f[i] * omf[j];
      xp = (float)(c * exp(-(de - w) * (de - w) * inv2s2) * n);
      xm = (float)(c * exp(-(de + w) * (de + w) * inv2s2) * (1.0 + n));
    }
  }
  if (live) xs[r] = make_float2(xp, xm);
  const float v = xp + xm;
  // one atomic per wavefront when all its rows share the initial state
  const int64_t p0 = __shfl(pi, 0, 64);
  if (__all(!live || pi == p0)) {
    float mx = v;
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0 && p0 < M) atomic_max_pos(rowmax + p0, mx);
  } else if (live && pi < M) {
    atomic_max_pos(rowmax + pi, v);
  }
  if (live) atomic_max_pos(colmax + (int64_t)q * nbr + s, xp);
}

// network stage: keep a tile when one of its terms has a predicted X+ + X-
// of at least tau times its initial state's largest, or a predicted X+ of at
// least tau times its phonon mode's largest (all writers store 1)
__global__ void k_screen_mark(int64_t rows, const int32_t* __restrict__ tiles, int64_t M, int nbr, int64_t nt,
                              MeshDims md, double tau, const int32_t* __restrict__ perm,
                              const int32_t* __restrict__ st_k, const float2* __restrict__ xs,
                              const unsigned* __restrict__ rowmax, const unsigned* __restrict__ colmax,
                              uint8_t* __restrict__ keep) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t per = 1024 * (int64_t)nbr;
  const int64_t t = r / per;
  const int e = (int)(r - t * per);
  const int s = e % nbr, jj = (e / nbr) % 32, ii = e / (nbr * 32);
  const int64_t pj = (int64_t)tiles[2 * t] * 32 + jj, pi = (int64_t)tiles[2 * t + 1] * 32 + ii;
  if (pi >= M || pj >= M) return;
  const float2 v = xs[r];
  if (v.x + v.y <= 0.f) return;
  const int q = q_between(st_k[perm[pj]], st_k[perm[pi]], md.n0, md.n1, md.n2);
  const bool row = (double)(v.x + v.y) >= tau * (double)__uint_as_float(rowmax[pi]);
  const bool col = v.x > 0.f && (double)v.x >= tau * (double)__uint_as_float(colmax[(int64_t)q * nbr + s]);
  if (row || col) keep[(int64_t)tiles[2 * t] * nt + tiles[2 * t + 1]] = 1;
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

extern "C" elph_status elph_scatt_rates_screened(elph_ctx ctx, elph_mlp m, int32_t mode, double tau,
                                                 double gauss_min, double T_K, double* W_e, double* W_ph,
                                                 double* stats) {
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
  if (mode != ELPH_SCREEN_NONE && !(gauss_min > 0.0 && gauss_min < 1.0)) {
    ctx->err = "the energy stage needs 0 < gauss_min < 1";
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
  const double amax = mode == ELPH_SCREEN_NONE ? 0.0 : -std::log(gauss_min);
  // tile positions: states ranked by energy (ties by index), padding in place
  std::vector<double> he(M);
  HIPCHK(hipMemcpy(he.data(), ctx->d_eps, M * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<int32_t> hp(ctx->m_pad);
  for (int64_t p = 0; p < ctx->m_pad; ++p) hp[p] = (int32_t)p;
  std::stable_sort(hp.begin(), hp.begin() + M, [&](int32_t a, int32_t b) { return he[a] < he[b]; });
  int32_t* perm = nullptr;
  uint8_t* keep = nullptr;
  ALLOC(perm, ctx->m_pad * sizeof(int32_t));
  ALLOC(keep, nt * nt);
  HIPCHK(hipMemcpy(perm, hp.data(), ctx->m_pad * sizeof(int32_t), hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  int64_t queried = 0, kept_energy = 0;
  auto count_tiles = [&](const std::vector<uint8_t>& hk, int64_t* tiles, int64_t* kept) {
    *tiles = *kept = 0;
    for (int64_t bx = 0; bx * 32 < M; ++bx)
      for (int64_t by = 0; by * 32 < M; ++by) {
        ++*tiles;
        *kept += hk[bx * nt + by] ? 1 : 0;
      }
  };
  std::vector<uint8_t> hk(nt * nt);
  int64_t tiles = 0;
  if (mode == ELPH_SCREEN_NONE) {
    HIPCHK(hipMemsetAsync(keep, 1, nt * nt, s));
  } else {
    HIPCHK(hipMemsetAsync(keep, 0, nt * nt, s));
    hipLaunchKernelGGL(k_screen_energy, dim3(blocks_for(M * M * nbr, 256)), dim3(256), 0, s, M, (int)nbr, md, inv2s2,
                       ctx->omega_min, amax, nt, perm, ctx->d_state_k, ctx->d_eps, ctx->d_hw, keep);
    HIPCHK(hipGetLastError());
    if (mode == ELPH_SCREEN_MLP) {
      // the network sees the terms of the tiles the energy stage keeps
      HIPCHK(hipMemcpyAsync(hk.data(), keep, nt * nt, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      count_tiles(hk, &tiles, &kept_energy);
      std::vector<int32_t> tl;
      for (int64_t bx = 0; bx * 32 < M; ++bx)
        for (int64_t by = 0; by * 32 < M; ++by)
          if (hk[bx * nt + by]) {
            tl.push_back((int32_t)bx);
            tl.push_back((int32_t)by);
          }
      const int64_t ntl = (int64_t)tl.size() / 2, per = 1024 * nbr;
      queried = ntl * per;
      Thermal th;
      st = make_thermal(ctx, T_K, &th);
      if (st != ELPH_OK) return st;
      int64_t tc = ((int64_t)1 << 20) / per;
      if (tc < 1) tc = 1;
      if (tc > ntl) tc = ntl;
      int32_t* dtl = nullptr;
      float2* xs = nullptr;
      float* y = nullptr;
      unsigned *rowmax = nullptr, *colmax = nullptr;
      const int64_t nmodes = ctx->nk * nbr;
      if (ntl > 0) {
        ALLOC(dtl, tl.size() * sizeof(int32_t));
        ALLOC(xs, queried * sizeof(float2));
        ALLOC(y, tc * per * sizeof(float));
        ALLOC(rowmax, ctx->m_pad * sizeof(unsigned));
        ALLOC(colmax, nmodes * sizeof(unsigned));
        HIPCHK(hipMemcpyAsync(dtl, tl.data(), tl.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(rowmax, 0, ctx->m_pad * sizeof(unsigned), s));
        HIPCHK(hipMemsetAsync(colmax, 0, nmodes * sizeof(unsigned), s));
        HIPCHK(hipMemsetAsync(keep, 0, nt * nt, s));
      }
      hipStream_t ms = m->stream;
      m->stream = s;  // network kernels on the context stream
      if (ntl > 0) {
        st = mlp_reserve(m, tc * per);
        if (st != ELPH_OK) ctx->err = "network: " + m->err;
      }
      for (int64_t t0 = 0; st == ELPH_OK && t0 < ntl; t0 += tc) {
        const int64_t rows = std::min(tc, ntl - t0) * per;
        hipLaunchKernelGGL(k_screen_rows, dim3(blocks_for(rows, 256)), dim3(256), 0, s, rows, dtl + 2 * t0, M,
                           ctx->nb, (int)nbr, m->in_pad, md, perm, ctx->d_state_k, ctx->d_state_m, ctx->d_eps,
                           ctx->d_hw, 1.0 / ctx->hw_max, ctx->mu, m->d_x);
        st = mlp_forward_rows(m, rows, false, y);
        if (st != ELPH_OK) {
          ctx->err = "network: " + m->err;
          break;
        }
        hipLaunchKernelGGL(k_screen_predict, dim3(blocks_for(rows, 256)), dim3(256), 0, s, rows, dtl + 2 * t0, M,
                           (int)nbr, md, inv2s2, ctx->omega_min, amax, perm, ctx->d_state_k, ctx->d_eps, ctx->d_hw,
                           th.f, th.omf, th.nocc, y, xs + t0 * per, rowmax, colmax);
      }
      if (st == ELPH_OK && ntl > 0)
        hipLaunchKernelGGL(k_screen_mark, dim3(blocks_for(queried, 256)), dim3(256), 0, s, queried, dtl, M,
                           (int)nbr, nt, md, tau, perm, ctx->d_state_k, xs, rowmax, colmax, keep);
      m->stream = ms;
      HIPCHK(hipStreamSynchronize(s));
      if (ntl > 0) {
        dev_free(ctx, dtl);
        dev_free(ctx, xs);
        dev_free(ctx, y);
        dev_free(ctx, rowmax);
        dev_free(ctx, colmax);
      }
      free_thermal(ctx, &th);
      if (st != ELPH_OK) return st;
    }
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hk.data(), keep, nt * nt, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t kept = 0;
  count_tiles(hk, &tiles, &kept);
  if (mode != ELPH_SCREEN_MLP) kept_energy = kept;
  // screened vertices and rates; the store is not kept as the exact one
  ctx->d_tile_keep = keep;
  ctx->d_tile_perm = perm;
  ctx->store_ready = false;
  st = elph_scatt_rates(ctx, T_K, W_e, W_ph);
  ctx->d_tile_keep = nullptr;
  ctx->d_tile_perm = nullptr;
  ctx->store_ready = false;
  if (st != ELPH_OK) return st;
  float msec = 0.f;
  HIPCHK(hipEventElapsedTime(&msec, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(ctx, keep);
  dev_free(ctx, perm);
  if (stats) {
    stats[0] = (double)tiles;
    stats[1] = (double)kept;
    stats[2] = (double)kept_energy;
    stats[3] = (double)queried;
    stats[4] = (double)msec;
  }
  return ELPH_OK;
}
