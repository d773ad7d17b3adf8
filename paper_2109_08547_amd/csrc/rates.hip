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

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace elph {

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
// helpers

__device__ inline int64_t q_between(int64_t kj, int64_t ki, int n0, int n1, int n2) {
  int cj = (int)(kj % n2), ci = (int)(ki % n2);
  int64_t tj = kj / n2, ti = ki / n2;
  int bj = (int)(tj % n1), bi = (int)(ti % n1);
  int aj = (int)(tj / n1), ai = (int)(ti / n1);
  int a = aj - ai; if (a < 0) a += n0;
  int b = bj - bi; if (b < 0) b += n1;
  int c = cj - ci; if (c < 0) c += n2;
  return ((int64_t)a * n1 + b) * n2 + c;
}

__device__ inline int64_t q_neg(int64_t q, int n0, int n1, int n2) {
  int c = (int)(q % n2);
  int64_t t = q / n2;
  int b = (int)(t % n1);
  int a = (int)(t / n1);
  a = a ? n0 - a : 0;
  b = b ? n1 - b : 0;
  c = c ? n2 - c : 0;
  return ((int64_t)a * n1 + b) * n2 + c;
}

// Sum of NV values over a 256-thread block (fixed order): wave butterflies,
// then the four wave results in LDS.  sh holds at least NV * 4 doubles.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* sh) {
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[c] = x;
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < NV; ++c) sh[c * 4 + wave] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = (sh[c * 4 + 0] + sh[c * 4 + 1]) + (sh[c * 4 + 2] + sh[c * 4 + 3]);
  __syncthreads();
}

struct MeshDims {
  int n0, n1, n2;
};

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
template <typename ST>
__global__ void __launch_bounds__(256) k_we_rows(int64_t M, int nbr, MeshDims md, const ST* __restrict__ Bp,
                                                 const ST* __restrict__ Bm, const int32_t* __restrict__ st_k,
                                                 const double* __restrict__ lomf, const double* __restrict__ nocc,
                                                 double* __restrict__ we) {
  __shared__ double sh[4];
  const int64_t i = blockIdx.x;
  const int64_t ki = st_k[i];
  const double li = lomf[i];
  double acc[1] = {0.0};
  const int64_t row = M * nbr;
  for (int64_t t = threadIdx.x; t < row; t += 256) {
    const int64_t j = t / nbr;
    const int s = (int)(t % nbr);
    const int64_t q = q_between(st_k[j], ki, md.n0, md.n1, md.n2);
    const double n = nocc[q * nbr + s];
    const double b = (double)Bp[i * row + t] * n + (double)Bm[i * row + t] * (1.0 + n);
    if (b != 0.0) acc[0] += b * exp(lomf[j] - li);
  }
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) we[i] = acc[0];
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

template <typename ST, int NV>
void launch_q_gather(elph_ctx ctx, const ST* Bp, const double* f, const double* omf, const double* x,
                     double* acc) {
  const dim3 grid(blocks_for(ctx->nk, 4)), blk(256);
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
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
                                       double*);
template void launch_q_gather<double, 1>(elph_ctx, const double*, const double*, const double*, const double*,
                                        double*);

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
static elph_status rates_from_store_t(elph_ctx ctx, const Thermal& th, double* we, double* wph) {
  const int64_t M = ctx->nstates;
  const int nbr = ctx->nbr;
  hipStream_t s = ctx->stream;
  if (we) {
    hipLaunchKernelGGL(k_we_rows<ST>, dim3((unsigned)M), dim3(256), 0, s, M, nbr, mdims(ctx), (const ST*)ctx->d_Bp,
                       (const ST*)ctx->d_Bm, ctx->d_state_k, th.lomf, th.nocc, we);
  }
  if (wph) {
    const int64_t nm = ctx->nk * nbr;
    double* acc = nullptr;
    ALLOC(acc, nm * sizeof(double));
    launch_q_gather<ST, 1>(ctx, (const ST*)ctx->d_Bp, th.f, th.omf, nullptr, acc);
    elph_status st = finalize_wph(ctx, th, acc, wph);
    HIPCHK(hipStreamSynchronize(s));
    dev_free(ctx, acc);
    if (st != ELPH_OK) return st;
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
                                const cd* __restrict__ Ukq, const cd* __restrict__ Lq, cd* __restrict__ out) {
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

elph_status interp_g(elph_ctx ctx, int64_t np, const int32_t* kidx, const int32_t* qidx, double* g_out) {
  if (np <= 0) return ELPH_OK;
  hipStream_t s = ctx->stream;
  const int nb = ctx->nb, nbr = ctx->nbr;
  const int64_t nn = (int64_t)nb * nb, mm = (int64_t)nbr * nbr;
  const int64_t ncol = (int64_t)ctx->nrp * nbr * nn;  // per Re row of g
  const int64_t inner = (int64_t)nbr * nn;
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(np, (int64_t)(512ll << 20) / (ncol * 16)));
  int32_t* kq = nullptr;
  cd *H = nullptr, *Uk = nullptr, *Ukq = nullptr, *u = nullptr, *Lq = nullptr, *phe = nullptr, *php = nullptr,
     *G1 = nullptr, *gW = nullptr;
  double* lam = nullptr;
  ALLOC(kq, chunk * sizeof(int32_t));
  ALLOC(H, chunk * std::max(nn, mm) * sizeof(cd));
  ALLOC(Uk, chunk * nn * sizeof(cd));
  ALLOC(Ukq, chunk * nn * sizeof(cd));
  ALLOC(u, chunk * mm * sizeof(cd));
  ALLOC(Lq, chunk * mm * sizeof(cd));
  ALLOC(lam, chunk * nbr * sizeof(double));
  ALLOC(phe, chunk * ctx->nre * sizeof(cd));
  ALLOC(php, chunk * ctx->nrp * sizeof(cd));
  ALLOC(G1, chunk * ncol * sizeof(cd));
  ALLOC(gW, chunk * inner * sizeof(cd));
  const MeshDims md = mdims(ctx);
  for (int64_t p0 = 0; p0 < np; p0 += chunk) {
    const int64_t cnt = std::min(chunk, np - p0);
    const int32_t* kp = kidx + p0;
    const int32_t* qp = qidx + p0;
    hipLaunchKernelGGL(k_pair_points, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, cnt, kp, qp, md, kq);
    elph_status st = fourier_points(ctx, false, kp, cnt, H);
    if (st != ELPH_OK) return st;
    launch_jacobi(H, cnt, nb, nullptr, Uk, s);
    st = fourier_points(ctx, false, kq, cnt, H);
    if (st != ELPH_OK) return st;
    launch_jacobi(H, cnt, nb, nullptr, Ukq, s);
    st = fourier_points(ctx, true, qp, cnt, H);
    if (st != ELPH_OK) return st;
    launch_jacobi(H, cnt, nbr, lam, u, s);
    hipLaunchKernelGGL(k_lq_only, dim3(blocks_for(cnt * mm, 256)), dim3(256), 0, s, cnt, nbr, lam, u,
                       ctx->d_mass_x, ctx->omega_min, Lq);
    hipLaunchKernelGGL(k_pair_phases, dim3(blocks_for(cnt * ctx->nre, 256)), dim3(256), 0, s, cnt, kp, md,
                       ctx->d_tab[0], ctx->d_tab[1], ctx->d_tab[2], ctx->d_re, ctx->d_wre, ctx->nre, phe);
    hipLaunchKernelGGL(k_pair_phases, dim3(blocks_for(cnt * ctx->nrp, 256)), dim3(256), 0, s, cnt, qp, md,
                       ctx->d_tab[0], ctx->d_tab[1], ctx->d_tab[2], ctx->d_rp, ctx->d_wrp, ctx->nrp, php);
    hipLaunchKernelGGL(k_interp_stage1, dim3(blocks_for(ncol, 256), (unsigned)((cnt + 7) / 8)), dim3(256), 0, s,
                       cnt, ctx->nre, ncol, phe, (const cd*)ctx->d_gr, G1);
    hipLaunchKernelGGL(k_interp_stage2, dim3(blocks_for(cnt * inner, 256)), dim3(256), 0, s, cnt, ctx->nrp, inner,
                       php, G1, gW);
    hipLaunchKernelGGL(k_interp_stage3, dim3(blocks_for(cnt * inner, 256)), dim3(256), 0, s, cnt, nb, nbr, gW, Uk,
                       Ukq, Lq, (cd*)g_out + p0 * inner);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(s));
  dev_free(ctx, kq);
  dev_free(ctx, H);
  dev_free(ctx, Uk);
  dev_free(ctx, Ukq);
  dev_free(ctx, u);
  dev_free(ctx, Lq);
  dev_free(ctx, lam);
  dev_free(ctx, phe);
  dev_free(ctx, php);
  dev_free(ctx, G1);
  dev_free(ctx, gW);
  return ELPH_OK;
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

template <typename ST>
__global__ void __launch_bounds__(256) k_build_kself(int64_t M, int nbr, MeshDims md, const ST* __restrict__ Bp,
                                                     const ST* __restrict__ Bm, const int32_t* __restrict__ st_k,
                                                     const double* __restrict__ lomf,
                                                     const double* __restrict__ nocc, const double* __restrict__ we,
                                                     double* __restrict__ K) {
  int64_t ij = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ij >= M * M) return;
  const int64_t i = ij / M, j = ij % M;
  const int64_t q = q_between(st_k[j], st_k[i], md.n0, md.n1, md.n2);
  double acc = 0.0;
  for (int s = 0; s < nbr; ++s) {
    const double n = nocc[q * nbr + s];
    acc += (double)Bp[ij * nbr + s] * n + (double)Bm[ij * nbr + s] * (1.0 + n);
  }
  const double w = we[i];
  K[ij] = (w > 0.0 && acc != 0.0) ? acc * exp(lomf[j] - lomf[i]) / w : 0.0;
}

// De[i][c] = sum_{j,s} r_ij / W_i (-P[q][s][c] B+ n + P[-q][s][c] B- (1+n)), c = 0..5
template <typename ST>
__global__ void __launch_bounds__(256) k_drag_e(int64_t M, int nbr, MeshDims md, const ST* __restrict__ Bp,
                                                const ST* __restrict__ Bm, const int32_t* __restrict__ st_k,
                                                const double* __restrict__ lomf, const double* __restrict__ nocc,
                                                const double* __restrict__ we, const double* __restrict__ phon,
                                                double* __restrict__ De) {
  __shared__ double sh[6 * 4];
  const int64_t i = blockIdx.x;
  const int64_t ki = st_k[i];
  const double li = lomf[i];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t row = M * nbr;
  for (int64_t t = threadIdx.x; t < row; t += 256) {
    const int64_t j = t / nbr;
    const int s = (int)(t % nbr);
    const double bp = (double)Bp[i * row + t], bm = (double)Bm[i * row + t];
    if (bp == 0.0 && bm == 0.0) continue;
    const int64_t q = q_between(st_k[j], ki, md.n0, md.n1, md.n2);
    const int64_t mq = q_neg(q, md.n0, md.n1, md.n2);
    const double n = nocc[q * nbr + s];
    const double r = exp(lomf[j] - li);
    const double a = -bp * n * r, b = bm * (1.0 + n) * r;
    const double* pq = phon + (q * nbr + s) * 6;
    const double* pm = phon + (mq * nbr + s) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += a * pq[c] + b * pm[c];
  }
  block_sum<6>(acc, sh);
  if (threadIdx.x < 6) {
    const double w = we[i];
    De[i * 6 + threadIdx.x] = (w > 0.0) ? acc[threadIdx.x] / w : 0.0;
  }
}

// xn[i][c] = x0[i][c] + De[i][c] + sgn * sum_j K[i][j] x[j][c].  A block owns
// 4 rows (one wavefront each); chunks of 256 rows of x are staged in LDS and
// shared by the 4 rows; each wavefront reduces with butterflies (fixed order).
__global__ void __launch_bounds__(256) k_self_sweep(int64_t M, const double* __restrict__ K,
                                                    const double* __restrict__ x, const double* __restrict__ x0,
                                                    const double* __restrict__ De, double sgn,
                                                    double* __restrict__ xn) {
  __shared__ double xs[256 * 6];
  const int r = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + r;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t j0 = 0; j0 < M; j0 += 256) {
    const int64_t nj = (M - j0 < 256) ? M - j0 : 256;
    for (int t = threadIdx.x; t < nj * 6; t += 256) xs[t] = x[j0 * 6 + t];
    __syncthreads();
    if (i < M) {
      const double* Ki = K + i * M + j0;
      for (int jj = l; jj < nj; jj += 64) {
        const double k = Ki[jj];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += k * xs[jj * 6 + c];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
  if (i < M && l < 6) {
    double v = acc[0];
#pragma unroll
    for (int c = 1; c < 6; ++c)
      if (c == l) v = acc[c];
    xn[i * 6 + l] = x0[i * 6 + l] + (De ? De[i * 6 + l] : 0.0) + sgn * v;
  }
}

// ---- BiCGSTAB on the projected electron operator: six independent columns
// (I and J, three Cartesian components each) share every sweep.
struct Col6 {
  double v[6];
};

// per-column dot products of up to three pairs of [n][6] arrays; part[block][18]
__global__ void __launch_bounds__(256) k_dots6(int64_t n, const double* __restrict__ a0,
                                               const double* __restrict__ b0, const double* __restrict__ a1,
                                               const double* __restrict__ b1, const double* __restrict__ a2,
                                               const double* __restrict__ b2, double* __restrict__ part) {
  __shared__ double sh[18 * 4];
  double acc[18];
#pragma unroll
  for (int c = 0; c < 18; ++c) acc[c] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n * 6; t += (int64_t)gridDim.x * 256) {
    const int c = (int)(t % 6);
    const double p0 = a0[t] * b0[t];
    const double p1 = a1 ? a1[t] * b1[t] : 0.0;
    const double p2 = a2 ? a2[t] * b2[t] : 0.0;
#pragma unroll
    for (int cc = 0; cc < 6; ++cc)
      if (cc == c) {
        acc[cc] += p0;
        acc[6 + cc] += p1;
        acc[12 + cc] += p2;
      }
  }
  block_sum<18>(acc, sh);
  if (threadIdx.x < 18) part[blockIdx.x * 18 + threadIdx.x] = acc[threadIdx.x];
}

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

__global__ void k_wp_total(int64_t nm, const double* __restrict__ wphe, const double* __restrict__ wext,
                           const double* __restrict__ hw, double hw_max, double T, double omega_min,
                           double* __restrict__ wp) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nm) return;
  double e;
  if (wext) e = wext[p];
  else {
    const double r = hw[p] / hw_max;
    e = 1.0e12 * r * r * (T / 300.0);
  }
  wp[p] = (hw[p] >= omega_min) ? wphe[p] + e : 0.0;
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
  for (int64_t kk = 2; kk <= npow; kk <<= 1)
    for (int64_t jj = kk >> 1; jj > 0; jj >>= 1)
      hipLaunchKernelGGL(k_bitonic, dim3(blocks_for(npow, 256)), dim3(256), 0, s, npow, kk, jj, key, idx);
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

  double *we = nullptr, *wphe = nullptr, *wp = nullptr, *x0 = nullptr, *x = nullptr, *xn = nullptr, *De = nullptr;
  double *phon0 = nullptr, *phon = nullptr, *phonn = nullptr, *acc = nullptr, *K = nullptr, *part = nullptr,
         *wff = nullptr;
  ALLOC(we, M * sizeof(double));
  ALLOC(wphe, nm * sizeof(double));
  ALLOC(wp, nm * sizeof(double));
  ALLOC(x0, M * 6 * sizeof(double));
  ALLOC(x, M * 6 * sizeof(double));
  ALLOC(xn, M * 6 * sizeof(double));
  ALLOC(De, M * 6 * sizeof(double));
  ALLOC(phon0, nm * 6 * sizeof(double));
  ALLOC(phon, nm * 6 * sizeof(double));
  ALLOC(phonn, nm * 6 * sizeof(double));
  ALLOC(acc, nm * 6 * sizeof(double));
  ALLOC(K, M * M * sizeof(double));
  ALLOC(part, 256 * 64 * sizeof(double));
  ALLOC(wff, M * sizeof(double));
  double* xprev = nullptr;
  ALLOC(xprev, M * 6 * sizeof(double));
  std::vector<double> hpart(256 * 64);

  st = rates_from_store(ctx, th, we, wphe);
  if (st != ELPH_OK) return st;
  hipLaunchKernelGGL(k_wp_total, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, wphe, wext, ctx->d_hw, ctx->hw_max,
                     T, ctx->omega_min, wp);
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
    int32_t *order = nullptr, *goff = nullptr;
    st = build_groups(ctx, &order, &goff);
    if (st != ELPH_OK) return st;
    // f(1-f) weights of the projection
    hipLaunchKernelGGL(k_mul, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, th.f, th.omf, wff);
    hipLaunchKernelGGL(k_build_kself<ST>, dim3(blocks_for(M * M, 256)), dim3(256), 0, s, M, nbr, md, Bp, Bm,
                       ctx->d_state_k, th.lomf, th.nocc, we, K);
    HIPCHK(hipGetLastError());

    int last_inner = 0;
    const bool verbose = std::getenv("ELPH_VERBOSE") != nullptr;
    Col6 one6, zero6, mone6;
    for (int c = 0; c < 6; ++c) {
      one6.v[c] = 1.0;
      zero6.v[c] = 0.0;
      mone6.v[c] = -1.0;
    }
    double *kr = nullptr, *krh = nullptr, *kp = nullptr, *kv = nullptr, *ks = nullptr, *kt = nullptr;
    ALLOC(kr, M * 6 * sizeof(double));
    ALLOC(krh, M * 6 * sizeof(double));
    ALLOC(kp, M * 6 * sizeof(double));
    ALLOC(kv, M * 6 * sizeof(double));
    ALLOC(ks, M * 6 * sizeof(double));
    ALLOC(kt, M * 6 * sizeof(double));
    auto solve_e = [&](bool drag, bool* ok) -> elph_status {
      // drive: x0 (+ electron drag from the current phonons)
      if (drag) {
        hipLaunchKernelGGL(k_drag_e<ST>, dim3((unsigned)M), dim3(256), 0, s, M, nbr, md, Bp, Bm, ctx->d_state_k,
                           th.lomf, th.nocc, we, phon, De);
      }
      // Self-consistency of the electrons for this drive: the fixed point of
      // x = P(b + K x) (P removes the group means), reached with BiCGSTAB on
      // L x = P(x - K x) = P b for the six columns at once.
      *ok = false;
      double* b = xn;  // drive b = x0 (+ drag), projected
      hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, x0, one6,
                         drag ? De : nullptr, zero6, (const double*)nullptr, b);
      if (!drag) hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, x0, zero6,
                                    (const double*)nullptr, zero6, (const double*)nullptr, b);
      hipLaunchKernelGGL(k_project, dim3((unsigned)ctx->ngroups), dim3(256), 0, s, order, goff, wff, b);
      auto applyL = [&](const double* in, double* out) {
        hipLaunchKernelGGL(k_self_sweep, dim3(blocks_for(M, 4)), dim3(256), 0, s, M, K, in, in,
                           (const double*)nullptr, -1.0, out);
        hipLaunchKernelGGL(k_project, dim3((unsigned)ctx->ngroups), dim3(256), 0, s, order, goff, wff, out);
      };
      auto dots = [&](const double* a0, const double* b0, const double* a1, const double* b1, const double* a2,
                      const double* b2, double (&out)[18]) -> elph_status {
        const int blocks = 128;
        hipLaunchKernelGGL(k_dots6, dim3(blocks), dim3(256), 0, s, M, a0, b0, a1, b1, a2, b2, part);
        HIPCHK(hipMemcpyAsync(hpart.data(), part, blocks * 18 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < 18; ++c) out[c] = 0.0;
        for (int bl = 0; bl < blocks; ++bl)
          for (int c = 0; c < 18; ++c) out[c] += hpart[bl * 18 + c];
        return ELPH_OK;
      };
      // x starts from the previous solution, projected
      hipLaunchKernelGGL(k_project, dim3((unsigned)ctx->ngroups), dim3(256), 0, s, order, goff, wff, x);
      applyL(x, kv);
      hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, b, mone6, kv, zero6,
                         (const double*)nullptr, kr);  // r = b - L x
      HIPCHK(hipMemcpyAsync(krh, kr, M * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemsetAsync(kp, 0, M * 6 * sizeof(double), s));
      HIPCHK(hipMemsetAsync(kv, 0, M * 6 * sizeof(double), s));
      double rho_old[6], alpha[6], omega[6], d[18];
      bool done[6];
      for (int c = 0; c < 6; ++c) {
        rho_old[c] = alpha[c] = omega[c] = 1.0;
        done[c] = false;
      }
      elph_status e2 = dots(b, b, x, x, kr, kr, d);
      if (e2 != ELPH_OK) return e2;
      double bnorm[6];
      for (int c = 0; c < 6; ++c) {
        bnorm[c] = std::sqrt(d[c]);
        done[c] = std::sqrt(d[12 + c]) <= 0.1 * tol * std::max(bnorm[c], 1e-300);
      }
      for (int it = 0; it < maxit && !std::all_of(done, done + 6, [](bool v) { return v; }); ++it) {
        last_inner = it + 1;
        e2 = dots(krh, kr, nullptr, nullptr, nullptr, nullptr, d);
        if (e2 != ELPH_OK) return e2;
        Col6 beta, mbo;
        for (int c = 0; c < 6; ++c) {
          const double rho = d[c];
          if (done[c] || rho == 0.0 || omega[c] == 0.0) {
            beta.v[c] = 0.0;
            mbo.v[c] = 0.0;
            rho_old[c] = rho;
            continue;
          }
          beta.v[c] = (rho / rho_old[c]) * (alpha[c] / omega[c]);
          mbo.v[c] = -beta.v[c] * omega[c];
          rho_old[c] = rho;
        }
        // p = r + beta p - beta omega v
        hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, kr, beta, kp, mbo, kv, kp);
        applyL(kp, kv);
        e2 = dots(krh, kv, nullptr, nullptr, nullptr, nullptr, d);
        if (e2 != ELPH_OK) return e2;
        Col6 ma;
        for (int c = 0; c < 6; ++c) {
          alpha[c] = (!done[c] && d[c] != 0.0) ? rho_old[c] / d[c] : 0.0;
          ma.v[c] = -alpha[c];
        }
        // s = r - alpha v  (into ks)
        hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, kr, ma, kv, zero6,
                           (const double*)nullptr, ks);
        applyL(ks, kt);
        e2 = dots(kt, ks, kt, kt, nullptr, nullptr, d);
        if (e2 != ELPH_OK) return e2;
        Col6 al, om, mom;
        for (int c = 0; c < 6; ++c) {
          omega[c] = (!done[c] && d[6 + c] > 0.0) ? d[c] / d[6 + c] : 0.0;
          al.v[c] = done[c] ? 0.0 : alpha[c];
          om.v[c] = done[c] ? 0.0 : omega[c];
          mom.v[c] = -om.v[c];
        }
        // x = x + alpha p + omega s ; r = s - omega t
        hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, x, al, kp, om, ks, x);
        hipLaunchKernelGGL(k_lin6, dim3(blocks_for(M * 6, 256)), dim3(256), 0, s, M, ks, mom, kt, zero6,
                           (const double*)nullptr, kr);
        e2 = dots(kr, kr, nullptr, nullptr, nullptr, nullptr, d);
        if (e2 != ELPH_OK) return e2;
        for (int c = 0; c < 6; ++c)
          if (!done[c] && std::sqrt(d[c]) <= 0.1 * tol * std::max(bnorm[c], 1e-300)) done[c] = true;
      }
      *ok = std::all_of(done, done + 6, [](bool v) { return v; });
      return ELPH_OK;
    };

    if (level == ELPH_LEVEL_DRAGLESS) {
      bool ok = false;
      st = solve_e(false, &ok);
      if (st != ELPH_OK) return st;
      converged = ok;
      used = 1;
    } else {
      converged = false;
      for (int it = 1; it <= maxit; ++it) {
        bool ok = false;
        HIPCHK(hipMemcpyAsync(xprev, x, M * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = solve_e(true, &ok);
        if (st != ELPH_OK) return st;
        Norms ne;
        st = diff_norms(ctx, M, x, xprev, part, hpart, &ne);
        if (st != ELPH_OK) return st;
        // phonon drag from the new electrons
        launch_q_gather<ST, 6>(ctx, Bp, th.f, th.omf, x, acc);
        hipLaunchKernelGGL(k_ph_drag_finalize, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, acc, phon0,
                           ctx->d_hw, th.nocc, wp, ctx->omega_min, phonn);
        Norms np_;
        st = diff_norms(ctx, nm, phonn, phon, part, hpart, &np_);
        if (st != ELPH_OK) return st;
        std::swap(phon, phonn);
        used = it;
        const double r = std::max(std::max(rel(ne.dI, ne.nI), rel(ne.dJ, ne.nJ)),
                                  std::max(rel(np_.dI, np_.nI), rel(np_.dJ, np_.nJ)));
        if (verbose)
          std::fprintf(stderr, "elph_iterate: outer %d inner %d res I %.3e J %.3e F %.3e G %.3e\n", it, last_inner,
                       rel(ne.dI, ne.nI), rel(ne.dJ, ne.nJ), rel(np_.dI, np_.nI), rel(np_.dJ, np_.nJ));
        if (level == ELPH_LEVEL_PARTIAL) {
          converged = ok;
          break;
        }
        if (ok && r < tol) {
          converged = true;
          break;
        }
      }
    }
    dev_free(ctx, order);
    dev_free(ctx, goff);
    for (double* pbuf : {kr, krh, kp, kv, ks, kt}) dev_free(ctx, pbuf);
  }

  // outputs
  hipLaunchKernelGGL(k_split_out, dim3(blocks_for(M, 256)), dim3(256), 0, s, M, x, I, J);
  hipLaunchKernelGGL(k_split_out, dim3(blocks_for(nm, 256)), dim3(256), 0, s, nm, phon, F, G);
  HIPCHK(hipGetLastError());
  if (tensors || ko) {
    const int blocks = 64;
    hipLaunchKernelGGL(k_tensor_e, dim3(blocks), dim3(256), 0, s, M, ctx->d_eps, ctx->mu, th.f, th.omf, ctx->d_vel,
                       x, part);
    hipLaunchKernelGGL(k_tensor_ph, dim3(blocks), dim3(256), 0, s, nm, ctx->d_hw, th.nocc, ctx->omega_min,
                       ctx->d_vph, phon, part + blocks * 36);
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
    double out[54];
    for (int c = 0; c < 9; ++c) {
      out[c] = ce * e * te[c] * e;                  // sigma: J in C m
      out[9 + c] = ce * e * te[9 + c] * e;          // sigma S: I in J m / K
      out[18 + c] = -ce * te[18 + c] * e * e;       // alpha_el: (eps - mu) in J, J in C m
      out[27 + c] = -ce * te[27 + c] * e * e;       // kappa0_el
      out[36 + c] = cp * tp[c] * e * e;             // alpha_ph: hw in J, G in C m
      out[45 + c] = cp * tp[9 + c] * e * e;         // kappa_ph
    }
    if (tensors)
      for (int c = 0; c < 54; ++c) tensors[c] = out[c];
    if (ko) {
      double dn = 0, sn = 0;
      for (int c = 0; c < 9; ++c) {
        const double d = out[9 + c] - (out[18 + c] + out[36 + c]) / T;
        dn += d * d;
        sn += out[9 + c] * out[9 + c];
      }
      *ko = std::sqrt(dn) / std::max(std::sqrt(sn), 1e-300);
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = used;
  for (void* p : {(void*)we, (void*)wphe, (void*)wp, (void*)x0, (void*)x, (void*)xn, (void*)De, (void*)phon0,
                  (void*)phon, (void*)phonn, (void*)acc, (void*)K, (void*)part, (void*)wff, (void*)xprev})
    dev_free(ctx, p);
  free_thermal(ctx, &th);
  if (!converged) {
    ctx->err = "iteration did not reach the tolerance within maxit";
    return ELPH_ENOCONV;
  }
  return ELPH_OK;
}

elph_status iterate(elph_ctx ctx, double T, const double* wext, int level, double tol, int maxit, double* I,
                    double* J, double* F, double* G, double* tensors, int* iters, double* ko) {
  elph_status st = ensure_store(ctx);
  if (st != ELPH_OK) return st;
  if (ctx->store_f32) return iterate_t<float>(ctx, T, wext, level, tol, maxit, I, J, F, G, tensors, iters, ko);
  return iterate_t<double>(ctx, T, wext, level, tol, maxit, I, J, F, G, tensors, iters, ko);
}

}  // namespace elph
