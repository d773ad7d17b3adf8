// Electron self-consistency inside the unified iteration scheme (Sec. 2.3,
// Eqs. 22-23): for a fixed drive b (RTA term plus the drag of the current
// phonons) the electron response solves x = P(b + K x), where K is the
// self-scattering operator of the e-ph part of Eq. 22 and P removes, per
// energy group, the f(1-f)-weighted mean (carrier-number conservation).
//
// K is kept transposed (K^T[j][i]) so that a matrix-vector product reads it
// in coalesced rows while each wavefront owns 64 output states, and it is
// projected once per call (K' = P K), so the operator applied by the solver
// is L x = x - K' x on the range of P.  The six driving columns (I and J,
// three Cartesian components each) run through one BiCGSTAB whose scalars
// live on the device: the host enqueues whole iterations and reads the
// convergence flags every few iterations.
#include "common.h"
#include "devutil.h"
#include "vertex.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace elph {

// K^T[j][i] = K[i][j] = sum_s (B+_ijs n_qs + B-_ijs (1 + n_qs)) e^{lomf_j - lomf_i} / W_i,
// q = k_j - k_i.  64 x 64 tiles through LDS: the store is read along j and
// K^T written along i.
template <typename ST, typename KS>
__global__ void __launch_bounds__(256) k_build_kT(int64_t M, int nbr, MeshDims md, const ST* __restrict__ Bp,
                                                  const ST* __restrict__ Bm, const int32_t* __restrict__ st_k,
                                                  const double* __restrict__ lomf, const double* __restrict__ nocc,
                                                  const double* __restrict__ we, KS* __restrict__ KT) {
  __shared__ double tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  {
    const int jl = threadIdx.x & 63;
    const int64_t j = j0 + jl;
    for (int il = threadIdx.x >> 6; il < 64; il += 4) {
      const int64_t i = i0 + il;
      double v = 0.0;
      if (i < M && j < M) {
        const int64_t q = q_between(st_k[j], st_k[i], md.n0, md.n1, md.n2);
        const int64_t base = (i * M + j) * nbr;
        double acc = 0.0;
        for (int s = 0; s < nbr; ++s) {
          const double n = nocc[q * nbr + s];
          acc += (double)Bp[base + s] * n + (double)Bm[base + s] * (1.0 + n);
        }
        const double w = we[i];
        v = (w > 0.0 && acc != 0.0) ? acc * exp(lomf[j] - lomf[i]) / w : 0.0;
      }
      tile[il][jl] = v;
    }
  }
  __syncthreads();
  const int il = threadIdx.x & 63;
  const int64_t i = i0 + il;
  for (int jl = threadIdx.x >> 6; jl < 64; jl += 4) {
    const int64_t j = j0 + jl;
    if (i < M && j < M) KT[j * M + i] = (KS)tile[il][jl];
  }
}

// K' = P K on the transposed storage: in row j of K^T, subtract from every
// member i of group g the weighted mean sum_{i' in g} w_i' K^T[j][i'] / sum w.
// One block per row; groups in order, each reduced in a fixed order.
template <typename KS>
__global__ void __launch_bounds__(256) k_kT_project(int64_t M, int ngroups, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ goff, const double* __restrict__ w,
                                                    KS* __restrict__ KT) {
  __shared__ double sh[2 * 4];
  KS* row = KT + (int64_t)blockIdx.x * M;
  for (int g = 0; g < ngroups; ++g) {
    const int32_t b = goff[g], e = goff[g + 1];
    double acc[2] = {0.0, 0.0};
    for (int32_t t = b + (int32_t)threadIdx.x; t < e; t += 256) {
      const int32_t i = order[t];
      acc[0] += w[i] * (double)row[i];
      acc[1] += w[i];
    }
    block_sum<2>(acc, sh);
    if (!(acc[1] > 0.0)) continue;
    const double mean = acc[0] / acc[1];
    for (int32_t t = b + (int32_t)threadIdx.x; t < e; t += 256) {
      const int32_t i = order[t];
      row[i] = (KS)((double)row[i] - mean);
    }
  }
}

// part[split][i][c] = sum_{j in split} K^T[j][i] in[j][c].  Block = 64
// states (one per lane) x one j split; the four wavefronts take every fourth
// j (eight rows of K^T loaded before they are used, to keep enough bytes in
// flight) and are summed in wave order.
template <typename KS>
__global__ void __launch_bounds__(256) k_kmv(int64_t M, int64_t jlen, const KS* __restrict__ KT,
                                             const double* __restrict__ in, double* __restrict__ part) {
  __shared__ double red[3][6][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t ic = i < M ? i : M - 1;
  const int64_t jb = (int64_t)blockIdx.y * jlen;
  const int64_t je = jb + jlen < M ? jb + jlen : M;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t j = jb + wave;
  for (; j + 28 < je; j += 32) {
    double kk[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) kk[u] = (double)KT[(j + 4 * u) * M + ic];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* xj = in + (j + 4 * u) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] += kk[u] * xj[c];
    }
  }
  for (; j < je; j += 4) {
    const double k = (double)KT[j * M + ic];
    const double* xj = in + j * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += k * xj[c];
  }
  if (wave > 0)
#pragma unroll
    for (int c = 0; c < 6; ++c) red[wave - 1][c][lane] = acc[c];
  __syncthreads();
  if (wave == 0 && i < M) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] += red[w][c][lane];
#pragma unroll
    for (int c = 0; c < 6; ++c) part[((int64_t)blockIdx.y * M + i) * 6 + c] = acc[c];
  }
}

// Vector kernels with dot products run blocks of kVB threads over a
// grid-stride loop; kVB and the stride are multiples of 6, so every thread
// stays on one column of the [n][6] arrays.  dpart[block][12] holds two
// six-column sums, each reduced in thread order.
constexpr int kVB = 192;

__device__ inline void dots_out(double d0, double d1, double* sh, double* dpart) {
  sh[threadIdx.x] = d0;
  sh[kVB + threadIdx.x] = d1;
  __syncthreads();
  if (threadIdx.x < 12) {
    const int c = threadIdx.x % 6, h = threadIdx.x / 6;
    double sum = 0.0;
    for (int k = c; k < kVB; k += 6) sum += sh[h * kVB + k];
    dpart[blockIdx.x * 12 + threadIdx.x] = sum;
  }
}

// out = in - sum_split part (splits in order); optional dots a0.out and out.out
__global__ void __launch_bounds__(kVB) k_kmv_fin(int64_t n6, int S, const double* __restrict__ in,
                                                 const double* __restrict__ part, double* __restrict__ out,
                                                 const double* __restrict__ a0, int sq, double* __restrict__ dpart) {
  __shared__ double sh[2 * kVB];
  double d0 = 0.0, d1 = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kVB + threadIdx.x; t < n6; t += (int64_t)gridDim.x * kVB) {
    double v = 0.0;
#pragma unroll 8
    for (int s = 0; s < S; ++s) v += part[(int64_t)s * n6 + t];
    v = in[t] - v;
    out[t] = v;
    if (a0) d0 += a0[t] * v;
    if (sq) d1 += v * v;
  }
  if (dpart) dots_out(d0, d1, sh, dpart);
}

// Device-resident BiCGSTAB scalars, six columns each.
enum {
  SC_RHO = 0,
  SC_ALPHA = 6,
  SC_OMEGA = 12,
  SC_BETA = 18,
  SC_BNORM = 24,
  SC_RNORM = 30,
  SC_DONE = 36,
  SC_ALL = 42,
  SC_N = 48
};
enum { BI_INIT = 0, BI_ALPHA = 1, BI_OMEGA = 2, BI_RHO = 3 };

// r = b - Lx, rh = r, p = v = 0 (v may alias lx); dots r.r, b.b
__global__ void __launch_bounds__(kVB) k_bi_init(int64_t n6, const double* __restrict__ b, const double* lx,
                                                 double* __restrict__ r, double* __restrict__ rh,
                                                 double* __restrict__ p, double* v, double* __restrict__ dpart) {
  __shared__ double sh[2 * kVB];
  double d0 = 0.0, d1 = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kVB + threadIdx.x; t < n6; t += (int64_t)gridDim.x * kVB) {
    const double bt = b[t];
    const double rv = bt - lx[t];
    r[t] = rv;
    rh[t] = rv;
    p[t] = 0.0;
    v[t] = 0.0;
    d0 += rv * rv;
    d1 += bt * bt;
  }
  dots_out(d0, d1, sh, dpart);
}

// p = r + beta (p - omega v)
__global__ void k_bi_p(int64_t n6, const double* __restrict__ r, const double* __restrict__ v,
                       const double* __restrict__ sc, double* __restrict__ p) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n6) return;
  const int c = (int)(t % 6);
  p[t] = r[t] + sc[SC_BETA + c] * (p[t] - sc[SC_OMEGA + c] * v[t]);
}

// s = r - alpha v
__global__ void k_bi_s(int64_t n6, const double* __restrict__ r, const double* __restrict__ v,
                       const double* __restrict__ sc, double* __restrict__ s) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n6) return;
  const int c = (int)(t % 6);
  s[t] = r[t] - sc[SC_ALPHA + c] * v[t];
}

// x += alpha p + omega s; r = s - omega t; dots rh.r, r.r
__global__ void __launch_bounds__(kVB) k_bi_xr(int64_t n6, const double* __restrict__ p,
                                               const double* __restrict__ s, const double* __restrict__ tv,
                                               const double* __restrict__ rh, const double* __restrict__ sc,
                                               double* __restrict__ x, double* __restrict__ r,
                                               double* __restrict__ dpart) {
  __shared__ double sh[2 * kVB];
  const int c = (int)(((int64_t)blockIdx.x * kVB + threadIdx.x) % 6);
  const double al = sc[SC_ALPHA + c], om = sc[SC_OMEGA + c];
  double d0 = 0.0, d1 = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kVB + threadIdx.x; t < n6; t += (int64_t)gridDim.x * kVB) {
    x[t] += al * p[t] + om * s[t];
    const double rv = s[t] - om * tv[t];
    r[t] = rv;
    d0 += rh[t] * rv;
    d1 += rv * rv;
  }
  dots_out(d0, d1, sh, dpart);
}

// Reduce the dot partials (blocks in order) and advance the scalars.
// thr = relative residual at which a column is frozen (its updates become 0).
__global__ void __launch_bounds__(192) k_bi_scal(int mode, int nblk, const double* __restrict__ dpart,
                                                double* __restrict__ sc, double thr) {
  __shared__ double d[12];
  __shared__ int dn[6];
  // 16 lanes per value: lane l sums blocks l, l + 16, ... then a fixed
  // butterfly over the 16 lanes
  {
    const int v = threadIdx.x >> 4, l = threadIdx.x & 15;
    double sum = 0.0;
#pragma unroll 8
    for (int b = l; b < nblk; b += 16) sum += dpart[b * 12 + v];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 16);
    if (l == 0) d[v] = sum;
  }
  const int c = threadIdx.x;
  __syncthreads();
  if (c < 6) {
    bool done = sc[SC_DONE + c] != 0.0;
    if (mode == BI_INIT) {
      const double bn = sqrt(d[6 + c]), rn = sqrt(d[c]);
      sc[SC_BNORM + c] = bn;
      sc[SC_RNORM + c] = rn;
      sc[SC_RHO + c] = d[c];
      sc[SC_ALPHA + c] = 1.0;
      sc[SC_OMEGA + c] = 1.0;
      sc[SC_BETA + c] = 0.0;
      done = rn <= thr * fmax(bn, 1e-300);
    } else if (mode == BI_ALPHA) {
      sc[SC_ALPHA + c] = (!done && d[c] != 0.0) ? sc[SC_RHO + c] / d[c] : 0.0;
    } else if (mode == BI_OMEGA) {
      sc[SC_OMEGA + c] = (!done && d[6 + c] > 0.0) ? d[c] / d[6 + c] : 0.0;
    } else {
      const double rn = sqrt(d[6 + c]);
      sc[SC_RNORM + c] = rn;
      if (!done && rn <= thr * fmax(sc[SC_BNORM + c], 1e-300)) done = true;
      const double rho_old = sc[SC_RHO + c], om = sc[SC_OMEGA + c];
      sc[SC_BETA + c] = (done || rho_old == 0.0 || om == 0.0) ? 0.0 : (d[c] / rho_old) * (sc[SC_ALPHA + c] / om);
      sc[SC_RHO + c] = d[c];
    }
    sc[SC_DONE + c] = done ? 1.0 : 0.0;
    dn[c] = done ? 1 : 0;
  }
  __syncthreads();
  if (c == 0) sc[SC_ALL] = (dn[0] && dn[1] && dn[2] && dn[3] && dn[4] && dn[5]) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// host side

template <typename ST>
elph_status build_self_operator(elph_ctx ctx, const ST* Bp, const ST* Bm, const double* lomf, const double* nocc,
                                const double* we, const int32_t* order, const int32_t* goff, const double* wff,
                                const SelfSolver& sv) {
  const int64_t M = ctx->nstates;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  const unsigned nt = blocks_for(M, 64);
  if (sv.kt_f32) {
    hipLaunchKernelGGL((k_build_kT<ST, float>), dim3(nt, nt), dim3(256), 0, ctx->stream, M, ctx->nbr, md, Bp, Bm,
                       ctx->d_state_k, lomf, nocc, we, (float*)sv.KT);
    hipLaunchKernelGGL(k_kT_project<float>, dim3((unsigned)M), dim3(256), 0, ctx->stream, M, ctx->ngroups, order,
                       goff, wff, (float*)sv.KT);
  } else {
    hipLaunchKernelGGL((k_build_kT<ST, double>), dim3(nt, nt), dim3(256), 0, ctx->stream, M, ctx->nbr, md, Bp, Bm,
                       ctx->d_state_k, lomf, nocc, we, (double*)sv.KT);
    hipLaunchKernelGGL(k_kT_project<double>, dim3((unsigned)M), dim3(256), 0, ctx->stream, M, ctx->ngroups, order,
                       goff, wff, (double*)sv.KT);
  }
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}
template elph_status build_self_operator<double>(elph_ctx, const double*, const double*, const double*,
                                                 const double*, const double*, const int32_t*, const int32_t*,
                                                 const double*, const SelfSolver&);
template elph_status build_self_operator<float>(elph_ctx, const float*, const float*, const double*, const double*,
                                                const double*, const int32_t*, const int32_t*, const double*,
                                                const SelfSolver&);

void self_solver_layout(int64_t M, SelfSolver* sv) {
  const int64_t rows = M > 0 ? (M + 63) / 64 : 1;
  int64_t S = (1024 + rows - 1) / rows;
  if (S < 1) S = 1;
  if (S > 32) S = 32;
  if (S > M) S = M > 0 ? M : 1;
  sv->jlen = M > 0 ? (M + S - 1) / S : 1;
  sv->S = M > 0 ? (int)((M + sv->jlen - 1) / sv->jlen) : 1;
  const int64_t need = (6 * M + kVB - 1) / kVB;
  sv->nblk = (int)(need < 1 ? 1 : need < 256 ? need : 256);
}

static size_t kt_doubles(int64_t M, bool f32) { return f32 ? ((size_t)M * M + 1) / 2 : (size_t)M * M; }

size_t self_solver_doubles(int64_t M, bool kt_f32) {
  SelfSolver sv;
  self_solver_layout(M, &sv);
  return kt_doubles(M, kt_f32) + 7 * (size_t)M * 6 + (size_t)sv.S * M * 6 + (size_t)sv.nblk * 12 + SC_N;
}

void self_solver_carve(int64_t M, bool kt_f32, double* base, SelfSolver* sv) {
  self_solver_layout(M, sv);
  double* p = base;
  sv->KT = p;
  sv->kt_f32 = kt_f32;
  p += kt_doubles(M, kt_f32);
  double** vecs[] = {&sv->b, &sv->r, &sv->rh, &sv->p, &sv->v, &sv->s, &sv->t};
  for (double** v : vecs) {
    *v = p;
    p += (size_t)M * 6;
  }
  sv->part = p;
  p += (size_t)sv->S * M * 6;
  sv->dpart = p;
  p += (size_t)sv->nblk * 12;
  sv->sc = p;
}

// out = in - K' in (with dots as for k_kmv_fin)
static void apply_L(elph_ctx ctx, const SelfSolver& sv, const double* in, double* out, const double* a0, int sq,
                    double* dpart) {
  const int64_t M = ctx->nstates;
  if (sv.kt_f32)
    hipLaunchKernelGGL(k_kmv<float>, dim3(blocks_for(M, 64), (unsigned)sv.S), dim3(256), 0, ctx->stream, M, sv.jlen,
                       (const float*)sv.KT, in, sv.part);
  else
    hipLaunchKernelGGL(k_kmv<double>, dim3(blocks_for(M, 64), (unsigned)sv.S), dim3(256), 0, ctx->stream, M,
                       sv.jlen, (const double*)sv.KT, in, sv.part);
  hipLaunchKernelGGL(k_kmv_fin, dim3((unsigned)sv.nblk), dim3(kVB), 0, ctx->stream, 6 * M, sv.S, in, sv.part, out,
                     a0, sq, dpart);
}

elph_status self_solve(elph_ctx ctx, const SelfSolver& sv, double* x, double thr, int maxit, bool* ok,
                       int* iters) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, n6 = 6 * M;
  const unsigned ev = blocks_for(n6, 256);
  if (!ctx->h_pin) HIPCHK(hipHostMalloc((void**)&ctx->h_pin, SC_N * sizeof(double), hipHostMallocDefault));
  // r0 = b - L x0 (v holds L x0 until the init kernel clears it)
  apply_L(ctx, sv, x, sv.v, nullptr, 0, nullptr);
  hipLaunchKernelGGL(k_bi_init, dim3((unsigned)sv.nblk), dim3(kVB), 0, s, n6, sv.b, sv.v, sv.r, sv.rh, sv.p, sv.v,
                     sv.dpart);
  hipLaunchKernelGGL(k_bi_scal, dim3(1), dim3(192), 0, s, (int)BI_INIT, sv.nblk, sv.dpart, sv.sc, thr);
  HIPCHK(hipGetLastError());
  const int kCheck = 4;  // iterations between reads of the convergence flags
  int it = 0;
  bool all = false;
  for (;;) {
    if (it % kCheck == 0 || it >= maxit) {
      HIPCHK(hipMemcpyAsync(ctx->h_pin, sv.sc, SC_N * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      all = ctx->h_pin[SC_ALL] != 0.0;
      if (all || it >= maxit) break;
    }
    ++it;
    hipLaunchKernelGGL(k_bi_p, dim3(ev), dim3(256), 0, s, n6, sv.r, sv.v, sv.sc, sv.p);
    apply_L(ctx, sv, sv.p, sv.v, sv.rh, 0, sv.dpart);  // v = L p; rh.v
    hipLaunchKernelGGL(k_bi_scal, dim3(1), dim3(192), 0, s, (int)BI_ALPHA, sv.nblk, sv.dpart, sv.sc, thr);
    hipLaunchKernelGGL(k_bi_s, dim3(ev), dim3(256), 0, s, n6, sv.r, sv.v, sv.sc, sv.s);
    apply_L(ctx, sv, sv.s, sv.t, sv.s, 1, sv.dpart);  // t = L s; s.t, t.t
    hipLaunchKernelGGL(k_bi_scal, dim3(1), dim3(192), 0, s, (int)BI_OMEGA, sv.nblk, sv.dpart, sv.sc, thr);
    hipLaunchKernelGGL(k_bi_xr, dim3((unsigned)sv.nblk), dim3(kVB), 0, s, n6, sv.p, sv.s, sv.t, sv.rh, sv.sc, x,
                       sv.r, sv.dpart);
    hipLaunchKernelGGL(k_bi_scal, dim3(1), dim3(192), 0, s, (int)BI_RHO, sv.nblk, sv.dpart, sv.sc, thr);
    HIPCHK(hipGetLastError());
  }
  *ok = all;
  *iters = it;
  return ELPH_OK;
}

}  // namespace elph
