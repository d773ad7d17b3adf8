// Temperature-dependent parts of the path ("The elphbolt ab initio solver
// ...", section "Electrons, phonons, and interactions" and section "Coupled
// and decoupled BTEs"):
//  * Fermi-Dirac / Bose-Einstein tables, with 1 - f and log(1 - f) each from
//    its own stable expression,
//  * X^{+/-} of Eq. 8 from the temperature-independent term store,
//  * electron RTA rates (Eq. 21, e-ph part) and phonon ph-e rates (Eq. 25 with
//    Y of Eq. 12) from the store,
//  * the coupled BTEs (Eqs. 19-27) with the unified iteration, and the
//    transport tensors of Eqs. 28-30,
//  * the vertex of Eq. 6 at arbitrary mesh pairs (elph_interp_g).
#include "tables.h"
#include "vertex.h"
#include "devutil.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

namespace elph {


// ---------------------------------------------------------------------------
// thermal tables

__global__ void k_thermal_states(int64_t n, const double* __restrict__ eps, double mu, double kT,
                                 double* __restrict__ f, double* __restrict__ omf, double* __restrict__ lomf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = (eps[i] - mu) / kT;
  double fi, oi, li;
  if (x > 0) {
    const double e = exp(-x);
    fi = e / (1.0 + e);
    oi = 1.0 / (1.0 + e);
    li = -log1p(e);
  } else {
    const double e = exp(x);
    fi = 1.0 / (1.0 + e);
    oi = e / (1.0 + e);
    li = x - log1p(e);
  }
  f[i] = fi;
  omf[i] = oi;
  lomf[i] = li;
}

__global__ void k_bose(int64_t n, const double* __restrict__ hw, double kT, double omega_min,
                       double* __restrict__ nocc) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double w = hw[t];
  nocc[t] = (w >= omega_min) ? 1.0 / expm1(w / kT) : 0.0;
}

elph_status alloc_thermal(elph_ctx ctx, Thermal* th) {
  const int64_t M = ctx->nstates;
  const int64_t nm = ctx->nk * ctx->nbr;
  ALLOC(th->f, M * sizeof(double));
  ALLOC(th->omf, M * sizeof(double));
  ALLOC(th->lomf, M * sizeof(double));
  ALLOC(th->nocc, nm * sizeof(double));
  return ELPH_OK;
}

void fill_thermal(elph_ctx ctx, double T, const Thermal& th, hipStream_t s) {
  const int64_t M = ctx->nstates;
  const int64_t nm = ctx->nk * ctx->nbr;
  const double kT = kBoltzEVK * T;
  hipLaunchKernelGGL(k_thermal_states, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, ctx->d_eps, ctx->mu, kT, th.f,
                     th.omf, th.lomf);
  hipLaunchKernelGGL(k_bose, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, ctx->d_hw, kT, ctx->omega_min,
                     th.nocc);
}

elph_status make_thermal(elph_ctx ctx, double T, Thermal* th) {
  elph_status st = alloc_thermal(ctx, th);
  if (st != ELPH_OK) return st;
  fill_thermal(ctx, T, *th, ctx->stream);
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}

void free_thermal(elph_ctx ctx, Thermal* th) {
  dev_free(ctx, th->f);
  dev_free(ctx, th->omf);
  dev_free(ctx, th->lomf);
  dev_free(ctx, th->nocc);
  *th = Thermal();
}


// ---------------------------------------------------------------------------
// X from the store:  X+ = B+ f_i (1 - f_j) n,  X- = B- f_i (1 - f_j) (1 + n)

template <typename ST>
__global__ void k_x_from_store(int64_t M, int nbr, MeshDims md, const ST* __restrict__ Bp, const ST* __restrict__ Bm,
                               const int32_t* __restrict__ st_k, const double* __restrict__ f,
                               const double* __restrict__ omf, const double* __restrict__ nocc,
                               double* __restrict__ Xp, double* __restrict__ Xm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * M * nbr) return;
  const int s = (int)(t % nbr);
  const int64_t ij = t / nbr;
  const int64_t i = ij / M, j = ij % M;
  const int64_t q = q_between(st_k[j], st_k[i], md.n0, md.n1, md.n2);
  const double n = nocc[q * nbr + s];
  const double occ = f[i] * omf[j];
  if (Xp) Xp[t] = (double)Bp[t] * occ * n;
  if (Xm) Xm[t] = (double)Bm[t] * occ * (1.0 + n);
}

// W_e[i] = sum_{j,s} (B+ n + B- (1+n)) (1 - f_j)/(1 - f_i): Eq. 21 with X/(f(1-f))
// With error codes (er.rho) the row also sums each term's contribution times
// its relative error estimate and flags the row when that exceeds er.theta
// of the rate; er.idx restricts the launch to listed rows.
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_we_rows(int64_t M, MeshDims md, const ST* __restrict__ Bp,
                                                 const ST* __restrict__ Bm, const int32_t* __restrict__ st_k,
                                                 const double* __restrict__ lomf, const double* __restrict__ nocc,
                                                 double* __restrict__ we, RateErr er) {
  // The row goes in chunks of 256 final states: their q indices and
  // occupation ratios are formed once per j into LDS, then the threads take
  // the chunk's (j, s) terms in order, so the B+- rows (and the codes) are
  // read contiguously.
  __shared__ double sh[8];
  __shared__ double rtab[256];
  __shared__ int sq[256];
  __shared__ double sw[256];
  const int64_t i = er.idx ? er.idx[blockIdx.x] : blockIdx.x;
  const int ki = st_k[i];
  const double li = lomf[i];
  const uint8_t* __restrict__ rho = er.rho;
  if (rho) rtab[threadIdx.x] = rho_decode(threadIdx.x);  // read after the first chunk's barrier
  double acc[2] = {0.0, 0.0};
  const ST* __restrict__ bp = Bp + i * M * NX;
  const ST* __restrict__ bm = Bm + i * M * NX;
  constexpr int RS = RhoStride<NX>::value;
  const uint8_t* __restrict__ rrow = rho ? rho + i * M * RS : nullptr;
  for (int64_t j0 = 0; j0 < M; j0 += 256) {
    const int nj = (int)(M - j0 < 256 ? M - j0 : 256);
    __syncthreads();  // the previous chunk is consumed
    if ((int)threadIdx.x < nj) {
      const int64_t j = j0 + threadIdx.x;
      sq[threadIdx.x] = q_between(st_k[j], ki, md.n0, md.n1, md.n2);
      sw[threadIdx.x] = exp(lomf[j] - li);
    }
    __syncthreads();
    const ST* __restrict__ cp = bp + j0 * NX;
    const ST* __restrict__ cm = bm + j0 * NX;
    for (int t = threadIdx.x; t < nj * NX; t += 256) {
      const int jl = t / NX, s = t - jl * NX;
      const double n = nocc[(int64_t)sq[jl] * NX + s];
      const double b = (double)cp[t] * n + (double)cm[t] * (1.0 + n);
      if (b != 0.0) {  // a vanished term never meets the ratio (which may overflow far below mu)
        const double v = b * sw[jl];
        acc[0] += v;
        if (rho) acc[1] += v * rtab[rrow[(j0 + jl) * RS + s]];
      }
    }
  }
  if (rho) {
    block_sum<2>(acc, sh);
  } else {
    double a1[1] = {acc[0]};
    block_sum<1>(a1, sh);
    acc[0] = a1[0];
  }
  if (threadIdx.x == 0) {
    we[i] = acc[0];
    if (rho && er.cnt && acc[1] > er.theta * acc[0]) er.list[atomicAdd(er.cnt, 1)] = (int32_t)i;
  }
}

// Deterministic q-gather over the term store.  One wavefront per phonon
// wave vector q: its lanes walk the kept k (stride 64), find k' = k + q through
// the mesh -> kept map and accumulate, per branch s and NV weight columns,
//   acc[q][s][c] = sum_{i in k, j in k'} B+[i][j][s] f_i (1 - f_j) w_c(i, j),
// with w = 1 (NV = 1, the phonon rate of Eq. 25) or w = x_j - x_i (NV = 6,
// the drag term of Eq. 27).  Lane partials are combined in a fixed order.
template <typename ST, int NV, int NX>
__global__ void __launch_bounds__(256) k_q_gather(int64_t nq, int64_t M, int nbr, MeshDims md,
                                                  const ST* __restrict__ Bp, const int32_t* __restrict__ kept,
                                                  int64_t nkept, const int32_t* __restrict__ kidx,
                                                  const int32_t* __restrict__ soff, const double* __restrict__ f,
                                                  const double* __restrict__ omf, const double* __restrict__ x,
                                                  double* __restrict__ acc) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;  // whole wavefront exits together
  const int qc = (int)(q % md.n2);
  const int64_t qt = q / md.n2;
  const int qb = (int)(qt % md.n1), qa = (int)(qt / md.n1);
  double a[NX][NV];
#pragma unroll
  for (int s = 0; s < NX; ++s)
#pragma unroll
    for (int c = 0; c < NV; ++c) a[s][c] = 0.0;
  for (int64_t t = lane; t < nkept; t += 64) {
    const int64_t k = kept[t];
    const int kc = (int)(k % md.n2);
    const int64_t kt = k / md.n2;
    const int kb = (int)(kt % md.n1), ka = (int)(kt / md.n1);
    int c2 = kc + qc; if (c2 >= md.n2) c2 -= md.n2;
    int b2 = kb + qb; if (b2 >= md.n1) b2 -= md.n1;
    int a2 = ka + qa; if (a2 >= md.n0) a2 -= md.n0;
    const int32_t u = kidx[((int64_t)a2 * md.n1 + b2) * md.n2 + c2];
    if (u < 0) continue;
    for (int32_t i = soff[t]; i < soff[t + 1]; ++i) {
      for (int32_t j = soff[u]; j < soff[u + 1]; ++j) {
        const double occ = f[i] * omf[j];
        double w[NV];
        if (NV == 1) w[0] = 1.0;
        else
#pragma unroll
          for (int c = 0; c < NV; ++c) w[c] = x[(int64_t)j * NV + c] - x[(int64_t)i * NV + c];
        const ST* b = Bp + ((int64_t)i * M + j) * NX;
#pragma unroll
        for (int s = 0; s < NX; ++s) {
          const double v = (double)b[s] * occ;
#pragma unroll
          for (int c = 0; c < NV; ++c) a[s][c] += v * w[c];
        }
      }
    }
  }
  // fixed-order butterfly over the wavefront
#pragma unroll
  for (int s = 0; s < NX; ++s) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double v = a[s][c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) acc[(q * NX + s) * NV + c] = v;
    }
  }
}

// ---- pairs by q: for every q the kept k, by ascending kept index t, whose
// k + q is also kept.  Counted and placed with integer atomics, then each q's
// list is sorted, so the lists (and every sum over them) are deterministic.

__global__ void k_pair_count(int64_t nkept, const int32_t* __restrict__ kept, MeshDims md,
                             int32_t* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nkept * nkept) return;
  const int64_t t = p / nkept, u = p - t * nkept;
  atomicAdd(&cnt[q_between(kept[u], kept[t], md.n0, md.n1, md.n2)], 1);
}

__global__ void k_pair_fill(int64_t nkept, const int32_t* __restrict__ kept, MeshDims md,
                            const int32_t* __restrict__ off, int32_t* __restrict__ cur, uint64_t* __restrict__ tmp) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nkept * nkept) return;
  const int64_t t = p / nkept, u = p - t * nkept;
  const int q = q_between(kept[u], kept[t], md.n0, md.n1, md.n2);
  tmp[off[q] + atomicAdd(&cur[q], 1)] = (uint64_t)t | ((uint64_t)u << 32);
}

// A pair's two state ranges in one word: first state and count of k_t in the
// low half, of k_u = k_t + q in the high half (26 bits of first state, 6 of
// count - 1 each; states < 2^26 and at most 64 per k, which the callers check).
__device__ inline uint64_t pack_pair(int32_t ib, int32_t ni, int32_t jb, int32_t nj) {
  return (uint64_t)((uint32_t)ib | ((uint32_t)(ni - 1) << 26)) |
         ((uint64_t)((uint32_t)jb | ((uint32_t)(nj - 1) << 26)) << 32);
}
__device__ inline void unpack_pair(uint64_t w, int32_t& ib, int32_t& ni, int32_t& jb, int32_t& nj) {
  const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
  ib = (int32_t)(lo & 0x3ffffffu);
  ni = (int32_t)(lo >> 26) + 1;
  jb = (int32_t)(hi & 0x3ffffffu);
  nj = (int32_t)(hi >> 26) + 1;
}

// The entries of one q are distinct kept indices t < nkept, so each lands at
// its rank among them: one wavefront per q sets bit t of a bitmap in LDS,
// takes exclusive prefix sums of the words' popcounts, and places every
// entry at prefix + popcount of the lower bits of its word.  The block's
// four wavefronts pass the same barriers whatever their list lengths.
__global__ void __launch_bounds__(256) k_pair_place(int64_t nq, int nkept, const int32_t* __restrict__ off,
                                                    const uint64_t* __restrict__ tmp, const int32_t* __restrict__ soff,
                                                    int32_t* __restrict__ list, uint64_t* __restrict__ ppk) {
  extern __shared__ uint32_t sm[];  // per wavefront: bitmap [W], prefix [W]
  const int W = (nkept + 31) / 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + wave;
  uint32_t* bits = sm + (size_t)wave * 2 * W;
  uint32_t* pre = bits + W;
  int32_t b = 0, len = 0;
  if (q < nq) {
    b = off[q];
    len = off[q + 1] - b;
  }
  for (int w = lane; w < W; w += 64) bits[w] = 0u;
  __syncthreads();
  for (int e = lane; e < len; e += 64) {
    const int32_t v = (int32_t)(uint32_t)tmp[b + e];
    atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
  __syncthreads();
  // exclusive prefix of the popcounts: lane owns words [lane per, lane per + per)
  const int per = (W + 63) / 64;
  int own = 0;
  for (int k = 0; k < per; ++k) {
    const int w = lane * per + k;
    if (w < W) own += __popc(bits[w]);
  }
  int incl = own;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  int run = incl - own;
  for (int k = 0; k < per; ++k) {
    const int w = lane * per + k;
    if (w < W) {
      pre[w] = (uint32_t)run;
      run += __popc(bits[w]);
    }
  }
  __syncthreads();
  for (int e = lane; e < len; e += 64) {
    const uint64_t tu = tmp[b + e];
    const int32_t v = (int32_t)(uint32_t)tu, u = (int32_t)(tu >> 32);
    const uint32_t word = bits[v >> 5];
    const int32_t at = b + (int32_t)pre[v >> 5] + __popc(word & ((1u << (v & 31)) - 1u));
    list[at] = v;
    ppk[at] = pack_pair(soff[v], soff[v + 1] - soff[v], soff[u], soff[u + 1] - soff[u]);
  }
}

elph_status ensure_pairs(elph_ctx ctx) {
  if (ctx->pairs_ready) return ELPH_OK;
  if (ctx->nkept > kMaxPairKept) {
    ctx->err = "too many kept k for per-q pair lists (nkept^2 must stay below 2^31)";
    return ELPH_EINVAL;
  }
  hipStream_t s = ctx->stream;
  const int64_t nk = ctx->nk, nkept = ctx->nkept, npairs = nkept * nkept;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  if (ctx->nstates >= ((int64_t)1 << 26)) {
    ctx->err = "too many states for packed pair ranges (2^26)";
    return ELPH_EINVAL;
  }
  int32_t *cnt = nullptr, *scr = nullptr, *tot = nullptr;
  uint64_t* tmp = nullptr;
  if (!ctx->d_poff) ALLOC(ctx->d_poff, (nk + 1) * sizeof(int32_t));
  if (!ctx->d_plist) ALLOC(ctx->d_plist, npairs * sizeof(int32_t));
  if (!ctx->d_ppk) ALLOC(ctx->d_ppk, npairs * sizeof(uint64_t));
  ALLOC(cnt, nk * sizeof(int32_t));
  ALLOC(tmp, npairs * sizeof(uint64_t));
  ALLOC(scr, (4 * ((nk + 1023) / 1024) + 64) * sizeof(int32_t));
  HIPCHK(hipMemsetAsync(cnt, 0, nk * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_pair_count, dim3(blocks_for(npairs, 256)), dim3(256), 0, s, nkept, ctx->d_kept, md, cnt);
  tot = ctx->d_poff + nk;  // total lands in the last offset
  scan_exclusive(ctx, cnt, nk, ctx->d_poff, tot, scr, s);
  HIPCHK(hipMemsetAsync(cnt, 0, nk * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_pair_fill, dim3(blocks_for(npairs, 256)), dim3(256), 0, s, nkept, ctx->d_kept, md,
                     ctx->d_poff, cnt, tmp);
  const size_t place_lds = (size_t)4 * 2 * ((nkept + 31) / 32) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_pair_place, dim3((unsigned)((nk + 3) / 4)), dim3(256), place_lds, s, nk, (int)nkept,
                     ctx->d_poff, tmp, ctx->d_soff, ctx->d_plist, ctx->d_ppk);
  HIPCHK(hipGetLastError());
  dev_free(ctx, cnt);
  dev_free(ctx, tmp);
  dev_free(ctx, scr);
  ctx->pairs_ready = true;
  return ELPH_OK;
}

// acc[q][s][c] over the pair list of q: lanes take every 64th pair, then a
// fixed-order butterfly over the wavefront
// (NV = 1: optional error codes as in k_we_rows, per branch; er.idx
// restricts the launch to er.n listed wave vectors).  The phonon rates use
// it (NV = 1); the six drag columns go through k_q_gather_lds.
template <typename ST, int NV, int NX>
__global__ void __launch_bounds__(256) k_q_gather_csr(int64_t nq, int64_t M, const ST* __restrict__ Bp,
                                                      const int32_t* __restrict__ poff,
                                                      const uint64_t* __restrict__ ppk, const double* __restrict__ f,
                                                      const double* __restrict__ omf, const double* __restrict__ x,
                                                      double* __restrict__ acc, RateErr er) {
  const int lane = threadIdx.x & 63;
  __shared__ double rtab[NV == 1 ? 256 : 1];
  const uint8_t* __restrict__ rho = NV == 1 ? er.rho : nullptr;
  if constexpr (NV == 1) {
    if (rho) {
      rtab[threadIdx.x] = rho_decode(threadIdx.x);
      __syncthreads();
    }
  }
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= (er.idx ? er.n : nq)) return;  // whole wavefront exits together
  const int64_t q = er.idx ? er.idx[w] : w;
  double ev[NV == 1 ? NX : 1];
#pragma unroll
  for (int s = 0; s < (NV == 1 ? NX : 1); ++s) ev[s] = 0.0;
  double a[NX][NV];
#pragma unroll
  for (int s = 0; s < NX; ++s)
#pragma unroll
    for (int c = 0; c < NV; ++c) a[s][c] = 0.0;
  const int32_t pe = poff[q + 1];
  for (int32_t p = poff[q] + lane; p < pe; p += 64) {
    int32_t ib, ni, jb, nj;
    unpack_pair(ppk[p], ib, ni, jb, nj);
    for (int32_t i = ib; i < ib + ni; ++i) {
      const double fi = f[i];
      for (int32_t j = jb; j < jb + nj; ++j) {
        const double occ = fi * omf[j];
        double w[NV];
        if (NV == 1) w[0] = 1.0;
        else
#pragma unroll
          for (int c = 0; c < NV; ++c) w[c] = x[(int64_t)j * NV + c] - x[(int64_t)i * NV + c];
        const ST* b = Bp + ((int64_t)i * M + j) * NX;
        PairCodes<NX> pc;
        if constexpr (NV == 1) {
          if (rho) pc.load(rho + ((int64_t)i * M + j) * RhoStride<NX>::value);
        }
#pragma unroll
        for (int s = 0; s < NX; ++s) {
          const double v = (double)b[s] * occ;
#pragma unroll
          for (int c = 0; c < NV; ++c) a[s][c] += v * w[c];
          if constexpr (NV == 1) {
            if (rho) ev[s] += v * rtab[pc[s]];
          }
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < NX; ++s) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double v = a[s][c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) acc[(q * NX + s) * NV + c] = v;
      if constexpr (NV == 1) {
        if (rho) {
          double e = ev[s];
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
          if (lane == 0 && er.cnt && e > er.theta * v) er.list[atomicAdd(er.cnt, 1)] = (int32_t)(q * NX + s);
        }
      }
    }
  }
}

// The six-column gather with the pair terms staged in LDS.  A wavefront
// per q (the four of a block take neighbouring q, as in k_q_gather_csr)
// takes its list 64 pairs at a time; each lane stages its pair's terms
// v_s = B+_ijs f_i (1 - f_j) and w_c = (x_j - x_i)_c, one state pair per
// round (pairs of several bands take several rounds, lanes already done
// stage zeros).  Lane (s, g), g < G = 64 / NX, then adds v_s w_c of the
// staged pairs g, g + G, ... for the six c, and a last pass sums the G
// partial rows in g order.  A lane holds six accumulators instead of NX x 6,
// so the gather runs at a higher occupancy; the order of the sum is fixed.
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_q_gather_lds(int64_t nq, int64_t M, const ST* __restrict__ Bp,
                                                      const int32_t* __restrict__ poff,
                                                      const uint64_t* __restrict__ ppk, const double* __restrict__ f,
                                                      const double* __restrict__ omf, const double* __restrict__ x,
                                                      double* __restrict__ acc) {
  constexpr int G = 64 / NX, NO = NX * 6;
  static_assert(G * NO <= 64 * 6, "partial rows fit the staged w block");
  __shared__ double Ys[4][64][NX];
  __shared__ double Ws[4][64][6];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 4 + wave;
  if (q >= nq) return;  // whole wavefront; only wavefront barriers below
  const int ms = lane % NX, mg = lane / NX;  // lanes with mg >= G idle in the sum
  double a[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) a[c] = 0.0;
  double(*__restrict__ ys)[NX] = Ys[wave];
  double(*__restrict__ ws)[6] = Ws[wave];
  const int32_t pe = poff[q + 1];
  for (int32_t p0 = poff[q]; p0 < pe; p0 += 64) {
    const int32_t p = p0 + lane;
    int32_t ib = 0, ni = 0, jb = 0, nj = 0;
    if (p < pe) unpack_pair(ppk[p], ib, ni, jb, nj);
    int nr = ni * nj;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nr = max(nr, __shfl_xor(nr, o, 64));
    for (int r = 0; r < nr; ++r) {
      if (r < ni * nj) {
        const int64_t i = ib + r / nj, j = jb + r % nj;
        const double occ = f[i] * omf[j];
        const ST* b = Bp + (i * M + j) * NX;
#pragma unroll
        for (int s = 0; s < NX; ++s) ys[lane][s] = (double)b[s] * occ;
#pragma unroll
        for (int c = 0; c < 6; ++c) ws[lane][c] = x[j * 6 + c] - x[i * 6 + c];
      } else {
#pragma unroll
        for (int s = 0; s < NX; ++s) ys[lane][s] = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) ws[lane][c] = 0.0;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (mg < G) {
        for (int l = mg; l < 64; l += G) {
          const double v = ys[l][ms];
#pragma unroll
          for (int c = 0; c < 6; ++c) a[c] += v * ws[l][c];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // staged values consumed before the next round
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // partial rows into the w block, then outputs e = s * 6 + c summed over g
  double* red = &ws[0][0];
  if (mg < G) {
#pragma unroll
    for (int c = 0; c < 6; ++c) red[(mg * NX + ms) * 6 + c] = a[c];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int e = lane; e < NO; e += 64) {
    double v = 0.0;
    for (int g = 0; g < G; ++g) v += red[g * NO + e];
    acc[q * NO + e] = v;
  }
}

template <typename ST, int NV>
void launch_q_gather(elph_ctx ctx, const ST* Bp, const double* f, const double* omf, const double* x,
                     double* acc, const RateErr* err) {
  const RateErr er = err ? *err : RateErr();
  const dim3 grid(blocks_for(er.idx ? er.n : ctx->nk, 4)), blk(256);
  if (er.idx && er.n == 0) return;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  bool csr = ctx->pairs_ready;
  if (!csr && !ctx->pairs_failed && ctx->nkept <= kMaxPairKept) {
    const elph_status st = ensure_pairs(ctx);
    csr = st == ELPH_OK;
    if (!csr) ctx->pairs_failed = true;
    if (st == ELPH_ENOMEM) ctx->err.clear();  // the walk below needs no extra memory
  }
  if (csr) {
    if constexpr (NV == 6) {
      // the drag columns (no row list or codes come with them)
#define QL(NXV)                                                                                                 \
  hipLaunchKernelGGL((k_q_gather_lds<ST, NXV>), grid, blk, 0, ctx->stream, ctx->nk, ctx->nstates, Bp,            \
                     ctx->d_poff, ctx->d_ppk, f, omf, x, acc)
      switch (ctx->nbr) {
        case 3: QL(3); break;
        case 6: QL(6); break;
        case 9: QL(9); break;
        case 12: QL(12); break;
        default: QL(15); break;
      }
#undef QL
    } else {
#define QG(NXV)                                                                                                \
  hipLaunchKernelGGL((k_q_gather_csr<ST, NV, NXV>), grid, blk, 0, ctx->stream, ctx->nk, ctx->nstates, Bp,       \
                     ctx->d_poff, ctx->d_ppk, f, omf, x, acc, er)
      switch (ctx->nbr) {
        case 3: QG(3); break;
        case 6: QG(6); break;
        case 9: QG(9); break;
        case 12: QG(12); break;
        default: QG(15); break;
      }
#undef QG
    }
    return;
  }
  // pair lists beyond 2^31 entries (or not allocatable): walk every kept k per q
#define QG(NXV)                                                                                           \
  hipLaunchKernelGGL((k_q_gather<ST, NV, NXV>), grid, blk, 0, ctx->stream, ctx->nk, ctx->nstates, NXV, md, Bp, \
                     ctx->d_kept, ctx->nkept, ctx->d_kidx, ctx->d_soff, f, omf, x, acc)
  switch (ctx->nbr) {
    case 3: QG(3); break;
    case 6: QG(6); break;
    case 9: QG(9); break;
    case 12: QG(12); break;
    default: QG(15); break;
  }
#undef QG
}

// W_ph = d_s (N_k/N_q) acc / (1 + n)
__global__ void k_wph_finalize(int64_t n, const double* __restrict__ acc, const double* __restrict__ hw,
                               const double* __restrict__ nocc, double omega_min, double scale,
                               double* __restrict__ wph) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  wph[t] = (hw[t] >= omega_min) ? scale * acc[t] / (1.0 + nocc[t]) : 0.0;
}

static MeshDims mdims(elph_ctx ctx) { return MeshDims{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]}; }

template void launch_q_gather<float, 1>(elph_ctx, const float*, const double*, const double*, const double*,
                                       double*, const RateErr*);
template void launch_q_gather<double, 1>(elph_ctx, const double*, const double*, const double*, const double*,
                                        double*, const RateErr*);

elph_status ensure_store(elph_ctx ctx) {
  if (ctx->store_ready) return ELPH_OK;
  const bool f64 = ctx->precision == ELPH_FP64;
  const size_t n = (size_t)ctx->nstates * ctx->nstates * ctx->nbr;
  const size_t esz = f64 ? 8 : 4;
  if (!ctx->d_Bp) {
    ALLOC(ctx->d_Bp, n * esz);
    ALLOC(ctx->d_Bm, n * esz);
  }
  ctx->store_f32 = !f64;
  elph_status st = run_vertex(ctx, ctx->d_Bp, ctx->d_Bm, f64, nullptr, nullptr, nullptr);
  if (st != ELPH_OK) return st;
  ctx->store_ready = true;
  return ELPH_OK;
}

elph_status finalize_wph(elph_ctx ctx, const Thermal& th, double* acc, double* wph) {
  const int64_t nm = ctx->nk * ctx->nbr;
  hipLaunchKernelGGL(k_wph_finalize, dim3(blocks_for(nm, 256)), dim3(256), 0, ctx->stream, nm, acc, ctx->d_hw,
                     th.nocc, ctx->omega_min, kSpinDeg * 1.0 /* N_k / N_q = 1 */, wph);
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}

template <typename ST>
void launch_we_rows(elph_ctx ctx, const ST* Bp, const ST* Bm, const double* lomf, const double* nocc, double* we,
                    const RateErr* err) {
  const int64_t M = ctx->nstates;
  hipStream_t s = ctx->stream;
  const RateErr er = err ? *err : RateErr();
  const int64_t nrows = er.idx ? er.n : M;
  if (nrows == 0) return;
#define WR(NXV)                                                                                            \
  hipLaunchKernelGGL((k_we_rows<ST, NXV>), dim3((unsigned)nrows), dim3(256), 0, s, M, mdims(ctx), Bp, Bm,  \
                     ctx->d_state_k, lomf, nocc, we, er)
  switch (ctx->nbr) {
    case 3: WR(3); break;
    case 6: WR(6); break;
    case 9: WR(9); break;
    case 12: WR(12); break;
    default: WR(15); break;
  }
#undef WR
}
template void launch_we_rows<float>(elph_ctx, const float*, const float*, const double*, const double*, double*,
                                    const RateErr*);
template void launch_we_rows<double>(elph_ctx, const double*, const double*, const double*, const double*, double*,
                                     const RateErr*);

template <typename ST>
static elph_status rates_from_store_t(elph_ctx ctx, const Thermal& th, double* we, double* wph) {
  const int nbr = ctx->nbr;
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, nm = ctx->nk * nbr;
  // GEMM forms with error codes: the reductions flag rates whose estimated
  // relative error exceeds refine_theta; their dominant terms are then
  // recomputed in FP64 and the affected rates reduced again
  const bool refine = std::is_same<ST, float>::value && ctx->rho_valid && ctx->refine_theta > 0.0 &&
                      refine_applicable(ctx) && (we || wph);
  RateErr ee, ep;
  int32_t* cnt = nullptr;
  double* acc = nullptr;
  if (wph) ALLOC(acc, nm * sizeof(double));
  if (refine) {
    // the phonon side selects terms along the pair lists of q
    if (wph && !ctx->pairs_ready && !ctx->pairs_failed && ctx->nkept <= kMaxPairKept) {
      const elph_status st = ensure_pairs(ctx);
      if (st != ELPH_OK) ctx->pairs_failed = true;
      if (st == ELPH_ENOMEM) ctx->err.clear();
      else if (st != ELPH_OK) return st;
    }
    ALLOC(cnt, 16 * sizeof(int32_t));
    HIPCHK(hipMemsetAsync(cnt, 0, 16 * sizeof(int32_t), s));
    ee.rho = ctx->d_rho;
    if (ctx->pairs_ready) ep.rho = ctx->d_rho;
    ee.theta = ep.theta = ctx->refine_theta;
    ee.cnt = cnt;
    ep.cnt = cnt + 1;
    ALLOC(ee.list, M * sizeof(int32_t));
    ALLOC(ep.list, nm * sizeof(int32_t));
  }
  if (we) launch_we_rows<ST>(ctx, (const ST*)ctx->d_Bp, (const ST*)ctx->d_Bm, th.lomf, th.nocc, we,
                             refine ? &ee : nullptr);
  if (wph) launch_q_gather<ST, 1>(ctx, (const ST*)ctx->d_Bp, th.f, th.omf, nullptr, acc,
                                  refine && ep.rho ? &ep : nullptr);
  if (refine) {
    mark(ctx, 10);
    const elph_status st = refine_terms(ctx, th, we, wph ? acc : nullptr, ee, ep, cnt);
    mark(ctx, 11);
    if (st != ELPH_OK) return st;
  }
  if (wph) {
    elph_status st = finalize_wph(ctx, th, acc, wph);
    HIPCHK(hipStreamSynchronize(s));
    if (st != ELPH_OK) return st;
  }
  HIPCHK(hipStreamSynchronize(s));
  dev_free(ctx, acc);
  if (refine) {
    dev_free(ctx, cnt);
    dev_free(ctx, (void*)ee.list);
    dev_free(ctx, (void*)ep.list);
  }
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}

elph_status rates_from_store(elph_ctx ctx, const Thermal& th, double* we, double* wph) {
  return ctx->store_f32 ? rates_from_store_t<float>(ctx, th, we, wph) : rates_from_store_t<double>(ctx, th, we, wph);
}

elph_status x_from_store(elph_ctx ctx, const Thermal& th, double* Xp, double* Xm) {
  const int64_t M = ctx->nstates;
  const int64_t n = M * M * ctx->nbr;
  if (ctx->store_f32)
    hipLaunchKernelGGL(k_x_from_store<float>, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, M, ctx->nbr,
                       mdims(ctx), (const float*)ctx->d_Bp, (const float*)ctx->d_Bm, ctx->d_state_k, th.f, th.omf,
                       th.nocc, Xp, Xm);
  else
    hipLaunchKernelGGL(k_x_from_store<double>, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, M, ctx->nbr,
                       mdims(ctx), (const double*)ctx->d_Bp, (const double*)ctx->d_Bm, ctx->d_state_k, th.f, th.omf,
                       th.nocc, Xp, Xm);
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}

// ---------------------------------------------------------------------------
// elph_interp_g: Eq. 6 at arbitrary mesh pairs, all bands

__global__ void k_pair_points(int64_t np, const int32_t* __restrict__ kidx, const int32_t* __restrict__ qidx,
                              MeshDims md, int32_t* __restrict__ kq) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int64_t k = kidx[p], q = qidx[p];
  const int64_t mq = q_neg(q, md.n0, md.n1, md.n2);
  kq[p] = (int32_t)q_between(k, mq, md.n0, md.n1, md.n2);  // k - (-q) = k + q
}

__global__ void k_pair_phases(int64_t np, const int32_t* __restrict__ pts, MeshDims md, const double2* t0,
                              const double2* t1, const double2* t2, const int32_t* __restrict__ R,
                              const double* __restrict__ w, int nR, cd* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * nR) return;
  const int64_t p = e / nR;
  const int r = (int)(e % nR);
  const int64_t lin = pts[p];
  const int c = (int)(lin % md.n2);
  const int64_t t = lin / md.n2;
  const int b = (int)(t % md.n1), a = (int)(t / md.n1);
  int i0 = (int)(((int64_t)a * R[3 * r]) % md.n0); if (i0 < 0) i0 += md.n0;
  int i1 = (int)(((int64_t)b * R[3 * r + 1]) % md.n1); if (i1 < 0) i1 += md.n1;
  int i2 = (int)(((int64_t)c * R[3 * r + 2]) % md.n2); if (i2 < 0) i2 += md.n2;
  const double2 p0 = t0[i0], p1 = t1[i1], p2 = t2[i2];
  cd z = cmul(cmul(cmake(p0.x, p0.y), cmake(p1.x, p1.y)), cmake(p2.x, p2.y));
  out[e] = cscale(z, w ? w[r] : 1.0);
}

// G1[p][col] = sum_Re phe[p][Re] g[Re][col], col = (Rp, x, n', m'); up to 8 pairs per thread
__global__ void k_interp_stage1(int64_t np, int nre, int64_t ncol, const cd* __restrict__ phe,
                                const cd* __restrict__ g, cd* __restrict__ G1) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.y * 8;
  if (col >= ncol) return;
  cd acc[8];
  for (int t = 0; t < 8; ++t) acc[t] = cmake(0, 0);
  for (int r = 0; r < nre; ++r) {
    const cd gv = g[(int64_t)r * ncol + col];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (p0 + t < np) acc[t] = cadd(acc[t], cmul(phe[(p0 + t) * nre + r], gv));
  }
  for (int t = 0; t < 8; ++t)
    if (p0 + t < np) G1[(p0 + t) * ncol + col] = acc[t];
}

// gW[p][x][n'][m'] = sum_Rp php[p][Rp] G1[p][Rp][x][n'][m']
__global__ void k_interp_stage2(int64_t np, int nrp, int64_t inner, const cd* __restrict__ php,
                                const cd* __restrict__ G1, cd* __restrict__ gW) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * inner) return;
  const int64_t p = e / inner, x = e % inner;
  cd acc = cmake(0, 0);
  for (int r = 0; r < nrp; ++r) acc = cadd(acc, cmul(php[p * nrp + r], G1[(p * nrp + r) * inner + x]));
  gW[e] = acc;
}

// g[p][s][n][m] = sum_x Lq[x][s] sum_{n',m'} conj(Ukq[n'][n]) gW[x][n'][m'] Uk[m'][m]
__global__ void k_interp_stage3(int64_t np, int nb, int nbr, const cd* __restrict__ gW, const cd* __restrict__ Uk,
                                const cd* __restrict__ Ukq, const cd* __restrict__ Lq, const cd* __restrict__ Fr,
                                cd* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nbr * nb * nb;
  if (e >= np * per) return;
  const int64_t p = e / per;
  int t = (int)(e % per);
  const int m = t % nb;
  t /= nb;
  const int n = t % nb;
  const int s = t / nb;
  const int64_t nn = (int64_t)nb * nb;
  cd acc = cmake(0, 0);
  for (int x = 0; x < nbr; ++x) {
    const cd l = Lq[(p * nbr + x) * nbr + s];
    if (l.x == 0.0 && l.y == 0.0) continue;
    cd rot = cmake(0, 0);
    for (int a = 0; a < nb; ++a) {
      cd row = cmake(0, 0);
      for (int b = 0; b < nb; ++b) row = cadd(row, cmul(gW[((p * nbr + x) * nb + a) * nb + b], Uk[p * nn + b * nb + m]));
      rot = cadd(rot, cmul(cconj(Ukq[p * nn + a * nb + n]), row));
    }
    acc = cadd(acc, cmul(l, rot));
  }
  if (Fr) {
    // Eq. 7: F_s(q) times the overlap sum_w conj(Ukq[w][n]) Uk[w][m]
    cd ov = cmake(0, 0);
    for (int w = 0; w < nb; ++w) ov = cadd(ov, cmul(cconj(Ukq[p * nn + w * nb + n]), Uk[p * nn + w * nb + m]));
    acc = cadd(acc, cmul(Fr[p * nbr + s], ov));
  }
  out[e] = acc;
}

__global__ void k_lq_only(int64_t nq, int nbr, const double* __restrict__ lam, const cd* __restrict__ u,
                          const double* __restrict__ mass_x, double omega_min, cd* __restrict__ Lq) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * nbr * nbr) return;
  const int64_t q = e / ((int64_t)nbr * nbr);
  const int t = (int)(e % ((int64_t)nbr * nbr));
  const int x = t / nbr, s = t % nbr;
  const double l = lam[q * nbr + s];
  const double w = sqrt(kPhononC * (l > 0.0 ? l : 0.0));
  Lq[e] = (w >= omega_min) ? cscale(u[e], sqrt(kPhononC / (2.0 * mass_x[x] * w))) : cmake(0, 0);
}

// Work buffers of Eq. 6 at arbitrary pairs, for a chunk of pairs, carved
// from one block (each region 256-byte aligned).  Every kernel of a chunk
// writes what it later reads, so nothing needs to start at zero.
struct InterpScratch {
  int32_t* kq = nullptr;
  cd *H = nullptr, *Uk = nullptr, *Ukq = nullptr, *u = nullptr, *Lq = nullptr, *Fr = nullptr;
  cd *phe = nullptr, *php = nullptr, *G1 = nullptr, *gW = nullptr;
  double* lam = nullptr;
};

// bytes of the work buffers for `chunk` pairs (carve = true: also point S
// into base)
static size_t interp_scratch(elph_ctx ctx, int64_t chunk, void* base, InterpScratch* S) {
  const int nb = ctx->nb, nbr = ctx->nbr;
  const int64_t nn = (int64_t)nb * nb, mm = (int64_t)nbr * nbr;
  const int64_t ncol = (int64_t)ctx->nrp * nbr * nn, inner = (int64_t)nbr * nn;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)((char*)base + off) : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  InterpScratch T;
  T.kq = (int32_t*)take(chunk * sizeof(int32_t));
  T.H = (cd*)take(chunk * std::max(nn, mm) * sizeof(cd));
  T.Uk = (cd*)take(chunk * nn * sizeof(cd));
  T.Ukq = (cd*)take(chunk * nn * sizeof(cd));
  T.u = (cd*)take(chunk * mm * sizeof(cd));
  T.Lq = (cd*)take(chunk * mm * sizeof(cd));
  T.Fr = ctx->frohlich ? (cd*)take(chunk * nbr * sizeof(cd)) : nullptr;
  T.lam = (double*)take(chunk * nbr * sizeof(double));
  T.phe = (cd*)take(chunk * ctx->nre * sizeof(cd));
  T.php = (cd*)take(chunk * ctx->nrp * sizeof(cd));
  T.G1 = (cd*)take(chunk * ncol * sizeof(cd));
  T.gW = (cd*)take(chunk * inner * sizeof(cd));
  if (S) *S = T;
  return off;
}

// Eq. 6 for np pairs in chunks through the work buffers S (queued on the
// context stream, no synchronisation)
static elph_status interp_run(elph_ctx ctx, int64_t np, const int32_t* kidx, const int32_t* qidx, double* g_out,
                              const InterpScratch& S, int64_t chunk) {
  hipStream_t s = ctx->stream;
  const int nb = ctx->nb, nbr = ctx->nbr;
  const int64_t nn = (int64_t)nb * nb, mm = (int64_t)nbr * nbr;
  const int64_t ncol = (int64_t)ctx->nrp * nbr * nn;  // per Re row of g
  const int64_t inner = (int64_t)nbr * nn;
  const MeshDims md = mdims(ctx);
  for (int64_t p0 = 0; p0 < np; p0 += chunk) {
    const int64_t cnt = std::min(chunk, np - p0);
    const int32_t* kp = kidx + p0;
    const int32_t* qp = qidx + p0;
    hipLaunchKernelGGL(k_pair_points, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, cnt, kp, qp, md, S.kq);
    elph_status st = fourier_points(ctx, false, kp, cnt, S.H);
    if (st != ELPH_OK) return st;
    launch_jacobi(S.H, cnt, nb, nullptr, S.Uk, s);
    st = fourier_points(ctx, false, S.kq, cnt, S.H);
    if (st != ELPH_OK) return st;
    launch_jacobi(S.H, cnt, nb, nullptr, S.Ukq, s);
    st = fourier_points(ctx, true, qp, cnt, S.H);
    if (st != ELPH_OK) return st;
    launch_jacobi(S.H, cnt, nbr, S.lam, S.u, s);
    hipLaunchKernelGGL(k_lq_only, dim3(blocks_for(cnt * mm, 256)), dim3(256), 0, s, cnt, nbr, S.lam, S.u,
                       ctx->d_mass_x, ctx->omega_min, S.Lq);
    hipLaunchKernelGGL(k_pair_phases, dim3(blocks_for(cnt * ctx->nre, 256)), dim3(256), 0, s, cnt, kp, md,
                       ctx->d_tab[0], ctx->d_tab[1], ctx->d_tab[2], ctx->d_re, ctx->d_wre, ctx->nre, S.phe);
    hipLaunchKernelGGL(k_pair_phases, dim3(blocks_for(cnt * ctx->nrp, 256)), dim3(256), 0, s, cnt, qp, md,
                       ctx->d_tab[0], ctx->d_tab[1], ctx->d_tab[2], ctx->d_rp, ctx->d_wrp, ctx->nrp, S.php);
    hipLaunchKernelGGL(k_interp_stage1, dim3(blocks_for(ncol, 256), (unsigned)((cnt + 7) / 8)), dim3(256), 0, s,
                       cnt, ctx->nre, ncol, S.phe, (const cd*)ctx->d_gr, S.G1);
    hipLaunchKernelGGL(k_interp_stage2, dim3(blocks_for(cnt * inner, 256)), dim3(256), 0, s, cnt, ctx->nrp, inner,
                       S.php, S.G1, S.gW);
    if (S.Fr) launch_frohlich(ctx, qp, cnt, S.Lq, S.Fr, s);
    hipLaunchKernelGGL(k_interp_stage3, dim3(blocks_for(cnt * inner, 256)), dim3(256), 0, s, cnt, nb, nbr, S.gW,
                       S.Uk, S.Ukq, S.Lq, (const cd*)S.Fr, (cd*)g_out + p0 * inner);
    HIPCHK(hipGetLastError());
  }
  return ELPH_OK;
}

elph_status interp_g(elph_ctx ctx, int64_t np, const int32_t* kidx, const int32_t* qidx, double* g_out) {
  if (np <= 0) return ELPH_OK;
  const int64_t ncol = (int64_t)ctx->nrp * ctx->nbr * ctx->nb * ctx->nb;
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(np, (int64_t)(512ll << 20) / (ncol * 16)));
  void* base = nullptr;
  ALLOC(base, interp_scratch(ctx, chunk, nullptr, nullptr));
  InterpScratch S;
  interp_scratch(ctx, chunk, base, &S);
  elph_status st = interp_run(ctx, np, kidx, qidx, g_out, S, chunk);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dev_free(ctx, base);
  return st;
}

// ---------------------------------------------------------------------------
// Eq. 6 at arbitrary pairs without allocation: the work buffers live in a
// static device array (each GPU the library runs on holds its own copy until
// the process ends); host code reaches it only through the address
// hipGetSymbolAddress returns on that device.

static __device__ __align__(256) unsigned char scratch[kInterpScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;  // device -> address of its copy of the array

static elph_status scratch_address(elph_ctx ctx, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(ctx->device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return ELPH_OK;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
    ctx->err = "the context's device must be current for its first allocation-free call";
    return ELPH_ESTATE;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    ctx->err = std::string("hipGetSymbolAddress of the static work array failed: ") + hipGetErrorString(e);
    (void)hipGetLastError();
    return ELPH_EHIP;
  }
  g_scratch_ptr[ctx->device] = p;
  *out = p;
  return ELPH_OK;
}

elph_status interp_g_noalloc(elph_ctx ctx, int64_t np, const int32_t* kidx, const int32_t* qidx, double* g_out) {
  const size_t per_pair = interp_scratch(ctx, 1, nullptr, nullptr);
  if (per_pair > kInterpScratchBytes) {
    ctx->err = "one pair needs " + std::to_string(per_pair) + " bytes of work space, more than the " +
               std::to_string((size_t)kInterpScratchBytes) + " bytes of the static array";
    return ELPH_EINVAL;
  }
  void* base = nullptr;
  elph_status st = scratch_address(ctx, &base);
  if (st != ELPH_OK) return st;
  if (np <= 0) return ELPH_OK;
  // largest chunk whose buffers fit the array
  int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(np, (int64_t)(kInterpScratchBytes / per_pair)));
  while (chunk > 1 && interp_scratch(ctx, chunk, nullptr, nullptr) > kInterpScratchBytes) --chunk;
  InterpScratch S;
  interp_scratch(ctx, chunk, base, &S);
  return interp_run(ctx, np, kidx, qidx, g_out, S, chunk);
}

// ---------------------------------------------------------------------------
// coupled BTEs (Eqs. 19-27)

// energy groups: bitonic sort of (eps, index) then split at wide gaps
__global__ void k_sort_init(int64_t n, int64_t npow, const double* __restrict__ eps, double* __restrict__ key,
                            int32_t* __restrict__ idx) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npow) return;
  key[t] = t < n ? eps[t] : INFINITY;
  idx[t] = (int32_t)t;
}

__global__ void k_bitonic(int64_t npow, int64_t kk, int64_t jj, double* __restrict__ key, int32_t* __restrict__ idx) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npow) return;
  int64_t p = t ^ jj;
  if (p <= t) return;
  const bool up = (t & kk) == 0;
  const double a = key[t], b = key[p];
  const int32_t ia = idx[t], ib = idx[p];
  const bool greater = (a > b) || (a == b && ia > ib);
  if (greater == up) {
    key[t] = b;
    key[p] = a;
    idx[t] = ib;
    idx[p] = ia;
  }
}

// The same sort in one block through LDS when npow <= kSortLds (one launch
// instead of one per stage); the order (key, then index) is total, so the
// result is the same.
constexpr int kSortLds = 4096;

__global__ void __launch_bounds__(1024) k_bitonic_lds(int npow, double* __restrict__ key, int32_t* __restrict__ idx) {
  __shared__ double sk[kSortLds];
  __shared__ int32_t si[kSortLds];
  for (int t = threadIdx.x; t < npow; t += 1024) {
    sk[t] = key[t];
    si[t] = idx[t];
  }
  __syncthreads();
  for (int kk = 2; kk <= npow; kk <<= 1)
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int t = threadIdx.x; t < npow; t += 1024) {
        const int p = t ^ jj;
        if (p > t) {
          const bool up = (t & kk) == 0;
          const double a = sk[t], b = sk[p];
          const int32_t ia = si[t], ib = si[p];
          const bool greater = (a > b) || (a == b && ia > ib);
          if (greater == up) {
            sk[t] = b;
            sk[p] = a;
            si[t] = ib;
            si[p] = ia;
          }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < npow; t += 1024) {
    key[t] = sk[t];
    idx[t] = si[t];
  }
}

__global__ void k_group_flags(int64_t n, const double* __restrict__ key, double gap, int32_t* __restrict__ flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  flag[t] = (t > 0 && key[t] - key[t - 1] > gap) ? 1 : 0;
}

__global__ void k_group_bounds(int64_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ lab,
                               int32_t* __restrict__ off, const int32_t* __restrict__ order,
                               int32_t* __restrict__ group) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t g = lab[t] + flag[t];  // inclusive label
  if (t == 0 || flag[t]) off[g] = (int32_t)t;
  group[order[t]] = g;
}

// The electron drag of the current phonon iterate P (Eq. 22's Delta I^D
// and its J counterpart):
//   De[i][c] = sum_{j,s} r_ij / W_i (-n_qs P[q][s][c] B+ + (1 + n_qs) P[-q][s][c] B-),
// q = k_j - k_i, r_ij = (1 - f_j) / (1 - f_i), c = 0..5.  The two phonon
// factors depend on (q, s) only and are tabulated first, side by side:
// uv[q][s][0..5] = -n_qs P[q][s], uv[q][s][6..11] = (1 + n_qs) P[-q][s]
// (n at -q equals n at q), so a term reads one contiguous row.  The table
// stays FP64 in every form: an FP32 table puts a rounding floor near 1e-7
// into the phonon map, which stalls the coupled iteration above 1e-8.
// Rows of the electron drag resident per CU.  Each row sweeps its own
// window of the (q, s) table; with more than three rows per CU at once their
// windows crowd each other out of the L2, and the gathers slow down (six
// rows: 0.58 ms for 3318 states and 6 branches, three: 0.54; for 9581
// states and 15 branches 13.7 and 11.4 ms).
constexpr int kDragRowsPerCU = 3;
constexpr int kDragOwnLds = 256 * 4 + 256 * 8 + 24 * 8;  // sq, sr, sh of k_drag_e

__global__ void k_drag_uv(int64_t nm, int nbr, MeshDims md, const double* __restrict__ nocc,
                          const double* __restrict__ phon, double* __restrict__ uv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nm * 12) return;
  const int64_t m = t / 12;
  const int c = (int)(t - m * 12);
  const double n = nocc[m];
  if (c < 6) {
    uv[t] = -n * phon[m * 6 + c];
  } else {
    const int q = (int)(m / nbr), s = (int)(m - (int64_t)q * nbr);
    const int mq = q_neg(q, md.n0, md.n1, md.n2);
    uv[t] = (1.0 + n) * phon[((int64_t)mq * nbr + s) * 6 + c - 6];
  }
}

// One block per initial state i.  The j range goes in chunks of 256: the
// chunk's q indices and occupation ratios are formed once per j into LDS,
// then the block's threads take the chunk's (j, s) terms in order, reading
// B+- along the row and the (q, s) row of uv.  Blocks are numbered so that
// each XCD (blocks b, b + 8, ... dispatched to one) takes a contiguous range
// of `rows`, a list of the states in Z order of their k: rows run together
// on one XCD then sit at nearby k, so the uv rows they visit overlap in that
// XCD's L2.  Each row is one block's fixed-order sum, whatever the list.
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_drag_e(int64_t M, int64_t per_xcd, MeshDims md, const ST* __restrict__ Bp,
                                                const ST* __restrict__ Bm, const int32_t* __restrict__ rows,
                                                const int32_t* __restrict__ st_k,
                                                const double* __restrict__ lomf, const double* __restrict__ we,
                                                const double* __restrict__ uv, double* __restrict__ De) {
  __shared__ int sq[256];
  __shared__ double sr[256];
  __shared__ double sh[6 * 4];
  const int64_t pos = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (pos >= M) return;  // whole block
  const int64_t i = rows[pos];
  const int ki = st_k[i];
  const double li = lomf[i];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const ST* __restrict__ bp = Bp + i * M * NX;
  const ST* __restrict__ bm = Bm + i * M * NX;
  for (int64_t j0 = 0; j0 < M; j0 += 256) {
    const int nj = (int)(M - j0 < 256 ? M - j0 : 256);
    __syncthreads();  // the previous chunk is consumed
    if ((int)threadIdx.x < nj) {
      const int64_t j = j0 + threadIdx.x;
      sq[threadIdx.x] = q_between(st_k[j], ki, md.n0, md.n1, md.n2);
      sr[threadIdx.x] = exp(lomf[j] - li);
    }
    __syncthreads();
    const ST* __restrict__ cp = bp + j0 * NX;
    const ST* __restrict__ cm = bm + j0 * NX;
    for (int t = threadIdx.x; t < nj * NX; t += 256) {
      const double vp = (double)cp[t], vm = (double)cm[t];
      if (vp == 0.0 && vm == 0.0) continue;
      const int jl = t / NX, s = t - jl * NX;
      const double r = sr[jl];
      const double* __restrict__ u = uv + ((int64_t)sq[jl] * NX + s) * 12;
      const double a = r * vp, b = r * vm;
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] += a * u[c] + b * u[6 + c];
    }
  }
  block_sum<6>(acc, sh);
  double v = acc[0];
#pragma unroll
  for (int c = 1; c < 6; ++c)
    if ((int)threadIdx.x == c) v = acc[c];
  if (threadIdx.x < 6) {
    const double w = we[i];
    De[i * 6 + threadIdx.x] = (w > 0.0) ? v / w : 0.0;
  }
}

// six-column scalars for the vector kernels
struct Col6 {
  double v[6];
};

// y = a + sa * b + sc * c   (column-wise scalars; b or c may be null)
__global__ void k_lin6(int64_t n, const double* __restrict__ a, Col6 sa, const double* __restrict__ b, Col6 sc,
                       const double* __restrict__ c, double* __restrict__ y) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * 6) return;
  const int col = (int)(t % 6);
  double v = a ? a[t] : 0.0;
  if (b) v += sa.v[col] * b[t];
  if (c) v += sc.v[col] * c[t];
  y[t] = v;
}

// remove the weighted mean of every energy group (no change of carrier number)
__global__ void __launch_bounds__(256) k_project(const int32_t* __restrict__ order, const int32_t* __restrict__ off,
                                                 const double* __restrict__ w, double* __restrict__ x) {
  __shared__ double sh[7 * 4];
  const int g = blockIdx.x;
  const int32_t b = off[g], e = off[g + 1];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int32_t t = b + threadIdx.x; t < e; t += 256) {
    const int32_t i = order[t];
    const double wi = w[i];
    acc[6] += wi;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += wi * x[(int64_t)i * 6 + c];
  }
  block_sum<7>(acc, sh);
  if (!(acc[6] > 0.0)) return;
  for (int32_t t = b + threadIdx.x; t < e; t += 256) {
    const int32_t i = order[t];
#pragma unroll
    for (int c = 0; c < 6; ++c) x[(int64_t)i * 6 + c] -= acc[c] / acc[6];
  }
}

// phon[p][c] = phon0[p][c] + d_s (N_k/N_q) acc[p][c] / ((1 + n_p) W_p)
__global__ void k_ph_drag_finalize(int64_t nm, const double* __restrict__ acc, const double* __restrict__ phon0,
                                   const double* __restrict__ hw, const double* __restrict__ nocc,
                                   const double* __restrict__ wp, double omega_min, double* __restrict__ phon) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nm) return;
  const bool on = hw[p] >= omega_min && wp[p] > 0.0;
  const double sc = on ? kSpinDeg / ((1.0 + nocc[p]) * wp[p]) : 0.0;
  for (int c = 0; c < 6; ++c) phon[p * 6 + c] = phon0[p * 6 + c] + sc * acc[p * 6 + c];
}

// RTA drives (Eqs. 20, 24) into x0 [M][6] and phon0 [nm][6]
__global__ void k_rta_e(int64_t M, const double* __restrict__ eps, const double* __restrict__ vel, double mu,
                        double T, const double* __restrict__ we, double* __restrict__ x0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double inv = we[i] > 0.0 ? 1.0 / we[i] : 0.0;
  const double a = (eps[i] - mu) / T * inv;
  for (int c = 0; c < 3; ++c) {
    x0[i * 6 + c] = a * vel[i * 3 + c];
    x0[i * 6 + 3 + c] = inv * vel[i * 3 + c];
  }
}

__global__ void k_rta_ph(int64_t nm, const double* __restrict__ hw, const double* __restrict__ vph, double T,
                         double omega_min, const double* __restrict__ wp, double* __restrict__ phon0) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nm) return;
  const bool on = hw[p] >= omega_min && wp[p] > 0.0;
  const double a = on ? hw[p] / T / wp[p] : 0.0;
  for (int c = 0; c < 3; ++c) {
    phon0[p * 6 + c] = a * vph[p * 3 + c];
    phon0[p * 6 + 3 + c] = 0.0;
  }
}

// W^RTA of the phonons: ph-e + external (or the model rate when neither an
// external rate nor three-phonon rates are given) + three-phonon (wpp)
__global__ void k_wp_total(int64_t nm, const double* __restrict__ wphe, const double* __restrict__ wext,
                           const double* __restrict__ wpp, const double* __restrict__ hw, double hw_max, double T,
                           double omega_min, double* __restrict__ wp) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nm) return;
  double e = 0.0;
  if (wext) e = wext[p];
  else if (!wpp) {
    const double r = hw[p] / hw_max;
    e = 1.0e12 * r * r * (T / 300.0);
  }
  if (wpp) e += wpp[p];
  wp[p] = (hw[p] >= omega_min) ? wphe[p] + e : 0.0;
}

// t3[p][c] = phon[p][3h + c]
__global__ void k_cols_get(int64_t nm, const double* __restrict__ phon, int h, double* __restrict__ t3) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nm * 3) return;
  const int64_t p = e / 3;
  t3[e] = phon[p * 6 + 3 * h + (e - p * 3)];
}

// phon[p][3h + c] += s3[p][c] / W^RTA_p (Delta F^S of Eq. 26), modes that take part only
__global__ void k_cols_add_self(int64_t nm, const double* __restrict__ s3, const double* __restrict__ wp,
                                const double* __restrict__ hw, double omega_min, int h, double* __restrict__ phon) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nm * 3) return;
  const int64_t p = e / 3;
  if (hw[p] >= omega_min && wp[p] > 0.0) phon[p * 6 + 3 * h + (e - p * 3)] += s3[e] / wp[p];
}

// sums of (a - b)^2 and a^2 over column groups [0,3) and [3,6) of [n][6] arrays
__global__ void __launch_bounds__(256) k_diff_norms(int64_t n, const double* __restrict__ a,
                                                    const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[4 * 4];
  double acc[4] = {0, 0, 0, 0};
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n * 6; t += (int64_t)gridDim.x * 256) {
    const int c = (int)(t % 6);
    const double d = a[t] - b[t];
    const int h = c < 3 ? 0 : 1;
    acc[2 * h] += d * d;
    acc[2 * h + 1] += a[t] * a[t];
  }
  block_sum<4>(acc, sh);
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = acc[threadIdx.x];
}

// ---- Anderson acceleration of the outer (phonon) fixed point
constexpr int kAA = 6;  // history length
struct Ptr8 {
  const double* p[8];
};
struct Gam8 {
  double g[8][6];
};

// part[block][v][c] = sum over the block's elements of column c of vs[v] . a
// (one pass over a; 192 threads and a stride that is a multiple of 6, so each
// thread keeps one column; two strides per iteration keep twice the loads in
// flight; the 32 threads of a column are summed in order)
constexpr int kDotsBlocks = 1024;

__global__ void __launch_bounds__(192) k_dots_multi(int64_t n6, int nv, Ptr8 vs, const double* __restrict__ a,
                                                    double* __restrict__ part) {
  __shared__ double sh[8][192];
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * 192;
  int64_t t = (int64_t)blockIdx.x * 192 + threadIdx.x;
  for (; t + stride < n6; t += 2 * stride) {
    const double a0 = a[t], a1 = a[t + stride];
#pragma unroll
    for (int v = 0; v < 8; ++v)
      if (v < nv) s[v] += vs.p[v][t] * a0 + vs.p[v][t + stride] * a1;
  }
  if (t < n6) {
    const double a0 = a[t];
#pragma unroll
    for (int v = 0; v < 8; ++v)
      if (v < nv) s[v] += vs.p[v][t] * a0;
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) sh[v][threadIdx.x] = s[v];
  __syncthreads();
  if (threadIdx.x < 48) {
    const int v = threadIdx.x / 6, c = threadIdx.x % 6;
    double sum = 0.0;
    for (int k = c; k < 192; k += 6) sum += sh[v][k];
    part[((int64_t)blockIdx.x * 8 + v) * 6 + c] = sum;
  }
}

// y = a - b
__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = a[t] - b[t];
}

// x += f - sum_l gamma_l (dX_l + dF_l)   (column-wise gamma)
__global__ void k_aa_update(int64_t n6, int nh, Ptr8 dX, Ptr8 dF, Gam8 gm, const double* __restrict__ f,
                            double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n6) return;
  const int c = (int)(t % 6);
  double v = x[t] + f[t];
  for (int l = 0; l < nh; ++l) v -= gm.g[l][c] * (dX.p[l][t] + dF.p[l][t]);
  x[t] = v;
}

// transport tensors: 6 tensors of 9 = 54 partial sums per block
__global__ void __launch_bounds__(256) k_tensor_e(int64_t M, const double* __restrict__ eps, double mu,
                                                  const double* __restrict__ f, const double* __restrict__ omf,
                                                  const double* __restrict__ vel, const double* __restrict__ x,
                                                  double* __restrict__ part) {
  __shared__ double sh[36 * 4];
  double acc[36];
  for (int c = 0; c < 36; ++c) acc[c] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256) {
    const double ff = f[i] * omf[i];
    const double de = eps[i] - mu;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double vJ = ff * vel[i * 3 + a] * x[i * 6 + 3 + b];
        const double vI = ff * vel[i * 3 + a] * x[i * 6 + b];
        acc[a * 3 + b] += vJ;            // sigma
        acc[9 + a * 3 + b] -= vI;        // sigma S
        acc[18 + a * 3 + b] += de * vJ;  // alpha_el (sign applied on host)
        acc[27 + a * 3 + b] -= de * vI;  // kappa0_el (sign applied on host)
      }
  }
  block_sum<36>(acc, sh);
  if (threadIdx.x < 36) part[blockIdx.x * 36 + threadIdx.x] = acc[threadIdx.x];
}

__global__ void __launch_bounds__(256) k_tensor_ph(int64_t nm, const double* __restrict__ hw,
                                                   const double* __restrict__ nocc, double omega_min,
                                                   const double* __restrict__ vph, const double* __restrict__ phon,
                                                   double* __restrict__ part) {
  __shared__ double sh[18 * 4];
  double acc[18];
  for (int c = 0; c < 18; ++c) acc[c] = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nm; p += (int64_t)gridDim.x * 256) {
    if (hw[p] < omega_min) continue;
    const double n = nocc[p];
    const double wgt = hw[p] * n * (1.0 + n);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        acc[a * 3 + b] -= wgt * vph[p * 3 + a] * phon[p * 6 + 3 + b];  // alpha_ph: -G
        acc[9 + a * 3 + b] += wgt * vph[p * 3 + a] * phon[p * 6 + b];  // kappa_ph: F
      }
  }
  block_sum<18>(acc, sh);
  if (threadIdx.x < 18) part[blockIdx.x * 18 + threadIdx.x] = acc[threadIdx.x];
}

__global__ void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) c[t] = a[t] * b[t];
}

__global__ void k_split_out(int64_t n, const double* __restrict__ x, double* __restrict__ A, double* __restrict__ B) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int c = 0; c < 3; ++c) {
    if (A) A[t * 3 + c] = x[t * 6 + c];
    if (B) B[t * 3 + c] = x[t * 6 + 3 + c];
  }
}

__global__ void k_join(int64_t n, const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ x) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int c = 0; c < 3; ++c) {
    x[t * 6 + c] = A[t * 3 + c];
    x[t * 6 + 3 + c] = B[t * 3 + c];
  }
}

// I <- I_diff + lambda (I - I_diff), I_diff = (eps - mu)/T J (Eqs. 33-35),
// in x [M][6] and in I [M][3]
__global__ void k_ko_apply(int64_t M, const double* __restrict__ eps, double mu, double T, double lambda,
                           double* __restrict__ x, double* __restrict__ I) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double d = (eps[i] - mu) / T;
  for (int c = 0; c < 3; ++c) {
    const double idiff = d * x[i * 6 + 3 + c];
    const double v = idiff + lambda * (x[i * 6 + c] - idiff);
    x[i * 6 + c] = v;
    I[i * 3 + c] = v;
  }
}

static elph_status build_groups(elph_ctx ctx, int32_t** order_out, int32_t** off_out) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates;
  int64_t npow = 1;
  while (npow < M) npow <<= 1;
  double* key = nullptr;
  int32_t *idx = nullptr, *flag = nullptr, *lab = nullptr, *scr = nullptr, *tot = nullptr, *off = nullptr;
  ALLOC(key, npow * sizeof(double));
  ALLOC(idx, npow * sizeof(int32_t));
  ALLOC(flag, M * sizeof(int32_t));
  ALLOC(lab, M * sizeof(int32_t));
  ALLOC(scr, (4 * ((M + 1023) / 1024) + 64) * sizeof(int32_t));
  ALLOC(tot, sizeof(int32_t));
  hipLaunchKernelGGL(k_sort_init, dim3(blocks_for(npow, 256)), dim3(256), 0, s, M, npow, ctx->d_eps, key, idx);
  if (npow <= kSortLds) {
    hipLaunchKernelGGL(k_bitonic_lds, dim3(1), dim3(1024), 0, s, (int)npow, key, idx);
  } else {
    for (int64_t kk = 2; kk <= npow; kk <<= 1)
      for (int64_t jj = kk >> 1; jj > 0; jj >>= 1)
        hipLaunchKernelGGL(k_bitonic, dim3(blocks_for(npow, 256)), dim3(256), 0, s, npow, kk, jj, key, idx);
  }
  const double gap = ctx->hw_max + 12.0 * ctx->sigma;
  hipLaunchKernelGGL(k_group_flags, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, key, gap, flag);
  scan_exclusive(ctx, flag, M, lab, tot, scr, s);
  int32_t nflag = 0;
  HIPCHK(hipMemcpyAsync(&nflag, tot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->ngroups = nflag + 1;
  ALLOC(off, (ctx->ngroups + 1) * sizeof(int32_t));
  if (!ctx->d_group) ALLOC(ctx->d_group, M * sizeof(int32_t));
  hipLaunchKernelGGL(k_group_bounds, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, flag, lab, off, idx,
                     ctx->d_group);
  int32_t Mi = (int32_t)M;
  HIPCHK(hipMemcpyAsync(off + ctx->ngroups, &Mi, sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  dev_free(ctx, key);
  dev_free(ctx, flag);
  dev_free(ctx, lab);
  dev_free(ctx, scr);
  dev_free(ctx, tot);
  *order_out = idx;
  *off_out = off;
  return ELPH_OK;
}

struct Norms {
  double dI, nI, dJ, nJ;
};

static elph_status diff_norms(elph_ctx ctx, int64_t n, const double* a, const double* b, double* part,
                              std::vector<double>& hpart, Norms* out) {
  const int blocks = 256;
  hipLaunchKernelGGL(k_diff_norms, dim3(blocks), dim3(256), 0, ctx->stream, n, a, b, part);
  HIPCHK(hipMemcpyAsync(hpart.data(), part, blocks * 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  Norms r{0, 0, 0, 0};
  for (int b = 0; b < blocks; ++b) {
    r.dI += hpart[b * 4 + 0];
    r.nI += hpart[b * 4 + 1];
    r.dJ += hpart[b * 4 + 2];
    r.nJ += hpart[b * 4 + 3];
  }
  *out = r;
  return ELPH_OK;
}

static double rel(double d2, double n2) { return std::sqrt(d2) / std::max(std::sqrt(n2), 1e-300); }

// out[v][c] = column-c dot of vs[v] and a, v < nv (block partials summed in order)
static elph_status dots_multi(elph_ctx ctx, int64_t n6, int nv, const Ptr8& vs, const double* a, double* part,
                              std::vector<double>& hpart, double (*out)[6]) {
  const int blocks = kDotsBlocks;
  hipLaunchKernelGGL(k_dots_multi, dim3(blocks), dim3(192), 0, ctx->stream, n6, nv, vs, a, part);
  HIPCHK(hipMemcpyAsync(hpart.data(), part, blocks * 8 * 6 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int v = 0; v < nv; ++v)
    for (int c = 0; c < 6; ++c) {
      double s = 0.0;
      for (int b = 0; b < blocks; ++b) s += hpart[((size_t)b * 8 + v) * 6 + c];
      out[v][c] = s;
    }
  return ELPH_OK;
}

// Solve (G + lambda I) g = r for an n x n symmetric system (n <= 8) by
// Gaussian elimination with partial pivoting; false when singular.
static bool small_solve(int n, double (*G)[8], const double* r, double* g) {
  double A[8][9];
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(G[i][i]));
  if (!(dmax > 0.0)) return false;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) A[i][j] = G[i][j] + (i == j ? 1e-12 * dmax : 0.0);
    A[i][n] = r[i];
  }
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i][k]) > std::fabs(A[p][k])) p = i;
    if (!(std::fabs(A[p][k]) > 1e-300)) return false;
    if (p != k)
      for (int j = 0; j <= n; ++j) std::swap(A[k][j], A[p][j]);
    for (int i = k + 1; i < n; ++i) {
      const double m = A[i][k] / A[k][k];
      for (int j = k; j <= n; ++j) A[i][j] -= m * A[k][j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = A[i][n];
    for (int j = i + 1; j < n; ++j) s -= A[i][j] * g[j];
    g[i] = s / A[i][i];
  }
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(g[i])) return false;
  return true;
}

// The 54 transport-tensor values of Eqs. 28-30 (SI units) from the electron
// responses x [M][6] (I, J) and the phonon responses phon [nm][6] (F, G);
// part holds 64 x 54 block partials, summed on the host in block order.
static elph_status transport_tensors(elph_ctx ctx, double T, const Thermal& th, const double* x, const double* phon,
                                     double* part, double out[54]) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, nm = ctx->nk * ctx->nbr;
  const int blocks = 64;
  std::vector<double> hpart(blocks * 54);
  hipLaunchKernelGGL(k_tensor_e, dim3(blocks), dim3(256), 0, s, M, ctx->d_eps, ctx->mu, th.f, th.omf, ctx->d_vel, x,
                     part);
  hipLaunchKernelGGL(k_tensor_ph, dim3(blocks), dim3(256), 0, s, nm, ctx->d_hw, th.nocc, ctx->omega_min, ctx->d_vph,
                     phon, part + blocks * 36);
  HIPCHK(hipMemcpyAsync(hpart.data(), part, blocks * 54 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double te[36] = {0}, tp[18] = {0};
  for (int b = 0; b < blocks; ++b) {
    for (int c = 0; c < 36; ++c) te[c] += hpart[b * 36 + c];
    for (int c = 0; c < 18; ++c) tp[c] += hpart[blocks * 36 + b * 18 + c];
  }
  const double V = ctx->volume_A3 * 1e-30;
  const double kT = kBoltzEVK * T * kCharge;
  const double ce = kSpinDeg / (V * kT * (double)ctx->nk);
  const double cp = 1.0 / (V * kT * (double)ctx->nk);
  const double e = kCharge;
  for (int c = 0; c < 9; ++c) {
    out[c] = ce * e * te[c] * e;                  // sigma: J in C m
    out[9 + c] = ce * e * te[9 + c] * e;          // sigma S: I in J m / K
    out[18 + c] = -ce * te[18 + c] * e * e;       // alpha_el: (eps - mu) in J, J in C m
    out[27 + c] = -ce * te[27 + c] * e * e;       // kappa0_el
    out[36 + c] = cp * tp[c] * e * e;             // alpha_ph: hw in J, G in C m
    out[45 + c] = cp * tp[9 + c] * e * e;         // kappa_ph
  }
  return ELPH_OK;
}

// Eq. 31: |sigma S - (alpha_el + alpha_ph)/T| / |sigma S| (Frobenius)
static double ko_residual_of(const double out[54], double T) {
  double dn = 0, sn = 0;
  for (int c = 0; c < 9; ++c) {
    const double d = out[9 + c] - (out[18 + c] + out[36 + c]) / T;
    dn += d * d;
    sn += out[9 + c] * out[9 + c];
  }
  return std::sqrt(dn) / std::max(std::sqrt(sn), 1e-300);
}

template <typename ST>
static elph_status iterate_t(elph_ctx ctx, double T, const double* wext, int level, double tol, int maxit,
                             double* I, double* J, double* F, double* G, double* tensors, int* iters, double* ko) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates;
  const int nbr = ctx->nbr;
  const int64_t nm = ctx->nk * nbr;
  const MeshDims md = mdims(ctx);
  const ST* Bp = (const ST*)ctx->d_Bp;
  const ST* Bm = (const ST*)ctx->d_Bm;
  Thermal th;
  elph_status st = make_thermal(ctx, T, &th);
  if (st != ELPH_OK) return st;

  double *we = nullptr, *wphe = nullptr, *wp = nullptr, *x0 = nullptr, *x = nullptr, *De = nullptr;
  double *phon0 = nullptr, *phon = nullptr, *phonn = nullptr, *acc = nullptr, *part = nullptr, *wff = nullptr;
  double *xprev = nullptr, *sbase = nullptr;
  double* uvt = nullptr;
  int32_t* drow = nullptr;
  ALLOC(we, M * sizeof(double));
  ALLOC(uvt, nm * 12 * sizeof(double));
  ALLOC(drow, M * sizeof(int32_t));
  ALLOC(wphe, nm * sizeof(double));
  ALLOC(wp, nm * sizeof(double));
  ALLOC(x0, M * 6 * sizeof(double));
  ALLOC(x, M * 6 * sizeof(double));
  ALLOC(De, M * 6 * sizeof(double));
  ALLOC(phon0, nm * 6 * sizeof(double));
  ALLOC(phon, nm * 6 * sizeof(double));
  ALLOC(phonn, nm * 6 * sizeof(double));
  ALLOC(acc, nm * 6 * sizeof(double));
  ALLOC(part, std::max(256 * 64, kDotsBlocks * 8 * 6) * sizeof(double));
  ALLOC(wff, M * sizeof(double));
  ALLOC(xprev, M * 6 * sizeof(double));
  std::vector<double> hpart(256 * 64);
  {
    // rows of the electron drag in Z order of their k (bit-interleaved
    // mesh coordinates), so that the rows an XCD runs together have nearby
    // k and the uv rows they visit overlap in that XCD's L2
    std::vector<int32_t> hk(M), ord(M);
    std::vector<uint64_t> key(M);
    HIPCHK(hipMemcpyAsync(hk.data(), ctx->d_state_k, M * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t i = 0; i < M; ++i) {
      const int k = hk[i];
      const uint32_t c = (uint32_t)(k % md.n2), b = (uint32_t)((k / md.n2) % md.n1), a = (uint32_t)(k / md.n2 / md.n1);
      uint64_t z = 0;
      for (int bit = 0; bit < 21; ++bit)
        z |= (uint64_t)((a >> bit) & 1) << (3 * bit + 2) | (uint64_t)((b >> bit) & 1) << (3 * bit + 1) |
             (uint64_t)((c >> bit) & 1) << (3 * bit);
      key[i] = z;
      ord[i] = (int32_t)i;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t u, int32_t v) { return key[u] < key[v]; });
    HIPCHK(hipMemcpyAsync(drow, ord.data(), M * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }

  if (ctx->rates_valid && ctx->rates_T == T) {
    // rates of the preceding elph_scatt_rates at this temperature
    HIPCHK(hipMemcpyAsync(we, ctx->d_we_cache, M * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(wphe, ctx->d_wph_cache, nm * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    st = rates_from_store(ctx, th, we, wphe);
    if (st != ELPH_OK) return st;
  }
  // three-phonon processes (Eq. 26): their RTA rate joins W^RTA, and Delta
  // F^S = S[phon] / W^RTA joins every phonon update (add_self)
  const bool phph = ctx->phph_sigma > 0.0;
  double *wpp = nullptr, *t3 = nullptr, *s3 = nullptr;
  if (phph) {
    if (!ctx->d_i3_psi) {
      ctx->err = "three-phonon processes enabled without force constants (elph_set_ifc3)";
      return ELPH_ESTATE;
    }
    ALLOC(wpp, nm * sizeof(double));
    ALLOC(t3, nm * 3 * sizeof(double));
    ALLOC(s3, nm * 3 * sizeof(double));
    st = phph_rates(ctx, T, ctx->phph_sigma, wpp);
    if (st != ELPH_OK) return st;
  }
  auto add_self = [&](const double* src, double* dst, int halves) -> elph_status {
    for (int h = 0; h < halves; ++h) {
      hipLaunchKernelGGL(k_cols_get, dim3(blocks_for(nm * 3, 256)), dim3(256), 0, s, nm, src, h, t3);
      elph_status e2 = phph_inscatter(ctx, T, ctx->phph_sigma, t3, s3);
      if (e2 != ELPH_OK) return e2;
      hipLaunchKernelGGL(k_cols_add_self, dim3(blocks_for(nm * 3, 256)), dim3(256), 0, s, nm, s3, wp, ctx->d_hw,
                         ctx->omega_min, h, dst);
      HIPCHK(hipGetLastError());
    }
    return ELPH_OK;
  };
  hipLaunchKernelGGL(k_wp_total, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, wphe, wext, wpp, ctx->d_hw,
                     ctx->hw_max, T, ctx->omega_min, wp);
  hipLaunchKernelGGL(k_rta_e, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, ctx->d_eps, ctx->d_vel, ctx->mu, T, we,
                     x0);
  hipLaunchKernelGGL(k_rta_ph, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, ctx->d_hw, ctx->d_vph, T,
                     ctx->omega_min, wp, phon0);
  HIPCHK(hipMemcpyAsync(x, x0, M * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(phon, phon0, nm * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());

  int used = 0;
  bool converged = true;
  if (level != ELPH_LEVEL_RTA) {
    if (!ctx->groups_ready) {
      st = build_groups(ctx, &ctx->d_order, &ctx->d_goff);
      if (st != ELPH_OK) return st;
      ctx->groups_ready = true;
    }
    const int32_t* order = ctx->d_order;
    const int32_t* goff = ctx->d_goff;
    const unsigned ng = (unsigned)ctx->ngroups;
    // f(1-f) weights of the projection
    hipLaunchKernelGGL(k_mul, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, th.f, th.omf, wff);
    SelfSolver sv;
    // the self operator is kept in the store's precision (FP32 in the forms)
    const bool kt_f32 = sizeof(ST) == 4;
    ALLOC(sbase, self_solver_doubles(M, kt_f32) * sizeof(double));
    self_solver_carve(M, kt_f32, sbase, &sv);
    st = build_self_operator<ST>(ctx, Bp, Bm, th.lomf, th.nocc, we, order, goff, wff, sv);
    if (st != ELPH_OK) return st;

    int last_inner = 0;
    const bool verbose = std::getenv("ELPH_VERBOSE") != nullptr;
    Col6 one6, zero6;
    for (int c = 0; c < 6; ++c) {
      one6.v[c] = 1.0;
      zero6.v[c] = 0.0;
    }
    // Inner tolerance: tol/10 when one phonon step is taken; tol/100 when the
    // phonon iterates are driven to tol, since the error an inner solve
    // leaves, amplified by the operator's conditioning, becomes noise in the
    // outer differences that stalls the accelerated iteration above tol.
    const double inner_thr = (level == ELPH_LEVEL_COUPLED ? 0.01 : 0.1) * tol;
    auto solve_e = [&](bool drag, bool* ok) -> elph_status {
      // drive b = P(x0 (+ electron drag from the current phonons)); the
      // fixed point x = P(b + K x) solves L x = b with L = 1 - P K on the
      // range of P, started from the previous solution
      if (drag) {
        hipLaunchKernelGGL(k_drag_uv, dim3(blocks_for(nm * 12, 256)), dim3(256), 0, s, nm, (int)nbr, md, th.nocc,
                           phon, uvt);
        const int64_t per_xcd = (M + 7) / 8;
        const size_t dpad = lds_pad_for(kDragRowsPerCU, kDragOwnLds);
#define DE(NXV)                                                                                                 \
  hipLaunchKernelGGL((k_drag_e<ST, NXV>), dim3((unsigned)(8 * per_xcd)), dim3(256), dpad, s, M, per_xcd, md, Bp, Bm, \
                     drow, ctx->d_state_k, th.lomf, we, uvt, De)
        switch (nbr) {
          case 3: DE(3); break;
          case 6: DE(6); break;
          case 9: DE(9); break;
          case 12: DE(12); break;
          default: DE(15); break;
        }
#undef DE
      }
      hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, x0, one6,
                         drag ? De : nullptr, zero6, (const double*)nullptr, sv.b);
      hipLaunchKernelGGL(k_project, dim3(ng), dim3(256), 0, s, order, goff, wff, sv.b);
      hipLaunchKernelGGL(k_project, dim3(ng), dim3(256), 0, s, order, goff, wff, x);
      elph_status e2 = self_solve(ctx, sv, x, inner_thr, maxit, ok, &last_inner);
      if (e2 != ELPH_OK) return e2;
      // remove what rounding left along the group directions
      hipLaunchKernelGGL(k_project, dim3(ng), dim3(256), 0, s, order, goff, wff, x);
      HIPCHK(hipGetLastError());
      return ELPH_OK;
    };

    if (level == ELPH_LEVEL_DRAGLESS) {
      bool ok = false;
      st = solve_e(false, &ok);
      if (st != ELPH_OK) return st;
      converged = ok;
      used = 1;
      if (phph) {
        // the phonons' own BTE F = F0 + Delta F^S[F] (G stays zero)
        bool okp = false;
        for (int it = 1; it <= maxit && !okp; ++it) {
          HIPCHK(hipMemcpyAsync(phonn, phon0, nm * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
          st = add_self(phon, phonn, 1);
          if (st != ELPH_OK) return st;
          Norms np_;
          st = diff_norms(ctx, nm, phonn, phon, part, hpart, &np_);
          if (st != ELPH_OK) return st;
          std::swap(phon, phonn);
          used = std::max(used, it);
          okp = rel(np_.dI, np_.nI) < tol;
        }
        converged = converged && okp;
      }
    } else {
      converged = false;
      // Anderson acceleration of the phonon fixed point phon -> Phi(phon)
      // (the unified scheme's outer map); the electrons are always solved
      // for the current phonon iterate, so a converged pair is the scheme's
      // fixed point.  PARTIAL stops after the first map evaluation.
      const int64_t n6 = nm * 6;
      double *fcur = nullptr, *fprev = nullptr, *pprev = nullptr, *aabuf = nullptr;
      const bool accel = level == ELPH_LEVEL_COUPLED;
      if (accel) {
        ALLOC(fcur, n6 * sizeof(double));
        ALLOC(fprev, n6 * sizeof(double));
        ALLOC(pprev, n6 * sizeof(double));
        ALLOC(aabuf, 2 * kAA * n6 * sizeof(double));
      }
      Ptr8 dX{}, dF{};
      for (int l = 0; l < kAA; ++l) {
        dX.p[l] = accel ? aabuf + (size_t)l * n6 : nullptr;
        dF.p[l] = accel ? aabuf + (size_t)(kAA + l) * n6 : nullptr;
      }
      double Gm[6][8][8];
      int nh = 0, head = 0;
      std::vector<double> hp2(kDotsBlocks * 8 * 6);
      for (int it = 1; it <= maxit; ++it) {
        bool ok = false;
        HIPCHK(hipMemcpyAsync(xprev, x, M * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = solve_e(true, &ok);
        if (st != ELPH_OK) return st;
        Norms ne;
        st = diff_norms(ctx, M, x, xprev, part, hpart, &ne);
        if (st != ELPH_OK) return st;
        // phonon drag from the new electrons: phonn = Phi(phon)
        launch_q_gather<ST, 6>(ctx, Bp, th.f, th.omf, x, acc);
        hipLaunchKernelGGL(k_ph_drag_finalize, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, acc, phon0,
                           ctx->d_hw, th.nocc, wp, ctx->omega_min, phonn);
        if (phph) {
          st = add_self(phon, phonn, 2);
          if (st != ELPH_OK) return st;
        }
        Norms np_;
        st = diff_norms(ctx, nm, phonn, phon, part, hpart, &np_);
        if (st != ELPH_OK) return st;
        used = it;
        const double r = std::max(std::max(rel(ne.dI, ne.nI), rel(ne.dJ, ne.nJ)),
                                  std::max(rel(np_.dI, np_.nI), rel(np_.dJ, np_.nJ)));
        if (verbose)
          std::fprintf(stderr, "elph_iterate: outer %d inner %d res I %.3e J %.3e F %.3e G %.3e\n", it, last_inner,
                       rel(ne.dI, ne.nI), rel(ne.dJ, ne.nJ), rel(np_.dI, np_.nI), rel(np_.dJ, np_.nJ));
        if (level == ELPH_LEVEL_PARTIAL) {
          std::swap(phon, phonn);
          converged = ok;
          break;
        }
        if (ok && r < tol) {
          std::swap(phon, phonn);
          converged = true;
          break;
        }
        // f = Phi(phon) - phon; history of differences of f and of phon
        hipLaunchKernelGGL(k_sub, dim3(blocks_for(n6, 256)), dim3(256), 0, s, n6, phonn, phon, fcur);
        if (it > 1) {
          double* dXh = const_cast<double*>(dX.p[head]);
          double* dFh = const_cast<double*>(dF.p[head]);
          hipLaunchKernelGGL(k_sub, dim3(blocks_for(n6, 256)), dim3(256), 0, s, n6, fcur, fprev, dFh);
          hipLaunchKernelGGL(k_sub, dim3(blocks_for(n6, 256)), dim3(256), 0, s, n6, phon, pprev, dXh);
          nh = std::min(nh + 1, kAA);
          double row[8][6];
          st = dots_multi(ctx, n6, nh, dF, dFh, part, hp2, row);
          if (st != ELPH_OK) return st;
          for (int c = 0; c < 6; ++c)
            for (int l = 0; l < nh; ++l) Gm[c][head][l] = Gm[c][l][head] = row[l][c];
          head = (head + 1) % kAA;
        }
        HIPCHK(hipMemcpyAsync(fprev, fcur, n6 * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(pprev, phon, n6 * sizeof(double), hipMemcpyDeviceToDevice, s));
        Gam8 gm{};
        if (nh > 0) {
          double rhs[8][6];
          st = dots_multi(ctx, n6, nh, dF, fcur, part, hp2, rhs);
          if (st != ELPH_OK) return st;
          for (int c = 0; c < 6; ++c) {
            double Gc[8][8], rc[8], gc[8];
            for (int a = 0; a < nh; ++a) {
              rc[a] = rhs[a][c];
              for (int b = 0; b < nh; ++b) Gc[a][b] = Gm[c][a][b];
            }
            if (small_solve(nh, Gc, rc, gc))
              for (int a = 0; a < nh; ++a) gm.g[a][c] = gc[a];
          }
        }
        // phon <- phon + f - sum_l gamma_l (dX_l + dF_l)
        hipLaunchKernelGGL(k_aa_update, dim3(blocks_for(n6, 256)), dim3(256), 0, s, n6, nh, dX, dF, gm, fcur, phon);
        HIPCHK(hipGetLastError());
      }
      if (!converged && level == ELPH_LEVEL_COUPLED) {
        // return the last map value with the electrons it came from
        std::swap(phon, phonn);
      }
      for (double* pbuf : {fcur, fprev, pprev, aabuf}) dev_free(ctx, pbuf);
    }
  }

  // outputs
  hipLaunchKernelGGL(k_split_out, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, x, I, J);
  hipLaunchKernelGGL(k_split_out, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, phon, F, G);
  HIPCHK(hipGetLastError());
  if (tensors || ko) {
    double out[54];
    st = transport_tensors(ctx, T, th, x, phon, part, out);
    if (st != ELPH_OK) return st;
    if (tensors)
      for (int c = 0; c < 54; ++c) tensors[c] = out[c];
    if (ko) *ko = ko_residual_of(out, T);
  }
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = used;
  for (void* p : {(void*)we, (void*)wphe, (void*)wp, (void*)x0, (void*)x, (void*)De, (void*)phon0, (void*)phon,
                  (void*)phonn, (void*)acc, (void*)part, (void*)wff, (void*)xprev, (void*)sbase, (void*)wpp,
                  (void*)t3, (void*)s3, (void*)uvt, (void*)drow})
    dev_free(ctx, p);
  free_thermal(ctx, &th);
  if (!converged) {
    ctx->err = "iteration did not reach the tolerance within maxit";
    return ELPH_ENOCONV;
  }
  return ELPH_OK;
}

// Kelvin-Onsager enforcement (Eqs. 32-35) on responses I, J, F, G: with
// I_diff = (eps - mu)/T J, sigma S_diff[I_diff] = alpha_el/T holds exactly,
// so sigma S_drag[I_drag] = sigma S - alpha_el/T; lambda minimises
// |lambda sigma S_drag - alpha_ph/T| (Frobenius), the root of the scalar
// condition the bisection of the method solves, written in closed form.
elph_status ko_enforce(elph_ctx ctx, double T, double* I, const double* J, const double* F, const double* G,
                       double* tensors, double* lambda, double* ko) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, nm = ctx->nk * ctx->nbr;
  Thermal th;
  elph_status st = make_thermal(ctx, T, &th);
  if (st != ELPH_OK) return st;
  double *x = nullptr, *phon = nullptr, *part = nullptr;
  ALLOC(x, M * 6 * sizeof(double));
  ALLOC(phon, nm * 6 * sizeof(double));
  ALLOC(part, 64 * 54 * sizeof(double));
  hipLaunchKernelGGL(k_join, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, (const double*)I, J, x);
  hipLaunchKernelGGL(k_join, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, F, G, phon);
  HIPCHK(hipGetLastError());
  double out[54];
  st = transport_tensors(ctx, T, th, x, phon, part, out);
  double lam = 0.0;
  if (st == ELPH_OK) {
    double sa = 0.0, ss = 0.0;
    for (int c = 0; c < 9; ++c) {
      const double sd = out[9 + c] - out[18 + c] / T;  // sigma S_drag[I_drag]
      sa += sd * (out[36 + c] / T);
      ss += sd * sd;
    }
    if (!(ss > 0.0)) {
      ctx->err = "sigma S has no drag part to rescale (I = (eps - mu)/T J)";
      st = ELPH_EINVAL;
    } else {
      lam = sa / ss;
      hipLaunchKernelGGL(k_ko_apply, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, ctx->d_eps, ctx->mu, T, lam, x,
                         I);
      HIPCHK(hipGetLastError());
      st = transport_tensors(ctx, T, th, x, phon, part, out);
    }
  }
  if (st == ELPH_OK) {
    if (tensors)
      for (int c = 0; c < 54; ++c) tensors[c] = out[c];
    if (lambda) *lambda = lam;
    if (ko) *ko = ko_residual_of(out, T);
  }
  HIPCHK(hipStreamSynchronize(s));
  dev_free(ctx, x);
  dev_free(ctx, phon);
  dev_free(ctx, part);
  free_thermal(ctx, &th);
  return st;
}

elph_status iterate(elph_ctx ctx, double T, const double* wext, int level, double tol, int maxit, double* I,
                    double* J, double* F, double* G, double* tensors, int* iters, double* ko) {
  elph_status st = ensure_store(ctx);
  if (st != ELPH_OK) return st;
  if (ctx->store_f32) return iterate_t<float>(ctx, T, wext, level, tol, maxit, I, J, F, G, tensors, iters, ko);
  return iterate_t<double>(ctx, T, wext, level, tol, maxit, I, J, F, G, tensors, iters, ko);
}

}  // namespace elph
