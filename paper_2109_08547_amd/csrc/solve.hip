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

// States per row tile of the matrix-vector product (two per lane); rows of
// K^T are padded to a multiple of it, with zeros past M, so every row
// starts 512-byte aligned and a lane reads two adjacent entries at once.
constexpr int kKmvRows = 128;
constexpr int kKmvChunk = 128;  // j rows per LDS chunk of the in vector (a multiple of 32)
inline int64_t kt_ld(int64_t M) { return (M + kKmvRows - 1) / kKmvRows * kKmvRows; }

// K^T[j][i] = K[i][j] = sum_s (B+_ijs n_qs + B-_ijs (1 + n_qs)) e^{lomf_j - lomf_i} / W_i,
// q = k_j - k_i.  64 x 64 tiles through LDS: the store is read along j and
// K^T written along i (row stride ldk; the tiles in i cover the padding).
template <typename ST, typename KS>
__global__ void __launch_bounds__(256) k_build_kT(int64_t M, int64_t ldk, int nbr, MeshDims md, const ST* __restrict__ Bp,
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
    if (j < M) KT[j * ldk + i] = (KS)tile[il][jl];
  }
}

// K' = P K on the transposed storage: in row j of K^T, subtract from every
// member i of group g the weighted mean sum_{i' in g} w_i' K^T[j][i'] / sum w.
// One block per row; groups in order, each reduced in a fixed order.
template <typename KS>
__global__ void __launch_bounds__(256) k_kT_project(int64_t ldk, int ngroups, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ goff, const double* __restrict__ w,
                                                    KS* __restrict__ KT) {
  __shared__ double sh[2 * 4];
  KS* row = KT + (int64_t)blockIdx.x * ldk;
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

// Vector kernels with dot products run blocks of kVB threads; kVB and every
// stride are multiples of 6, so a thread stays on one column of the [n][6]
// arrays.  dpart[block][12] holds two six-column sums, each reduced in
// thread order.
constexpr int kVB = 192;

__device__ inline void dots_out(double d0, double d1, double* sh, double* dpart) {
  if (threadIdx.x < kVB) {
    sh[threadIdx.x] = d0;
    sh[kVB + threadIdx.x] = d1;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    const int c = threadIdx.x % 6, h = threadIdx.x / 6;
    double sum = 0.0;
    for (int k = c; k < kVB; k += 6) sum += sh[h * kVB + k];
    dpart[blockIdx.x * 12 + threadIdx.x] = sum;
  }
}

// Device-resident BiCGSTAB scalars, six columns each, and the count of
// iterations that ran.
enum {
  SC_RHO = 0,
  SC_ALPHA = 6,
  SC_OMEGA = 12,
  SC_BETA = 18,
  SC_BNORM = 24,
  SC_RNORM = 30,
  SC_DONE = 36,
  SC_ALL = 42,
  SC_IT = 43,
  SC_N = 48
};
enum { BI_INIT = 0, BI_RHO = 1 };

// d[12] = the dot partials of nblk blocks summed over blocks in order, by
// the first kVB threads of a block (16 lanes per value: lane l sums blocks
// l, l + 16, ... then a fixed butterfly over the 16 lanes).  Every block
// that calls it on the same partials gets the same sums.
__device__ inline void dots_reduce(int nblk, const double* dpart, double* d) {
  if (threadIdx.x < kVB) {
    const int v = threadIdx.x >> 4, l = threadIdx.x & 15;
    double sum = 0.0;
#pragma unroll 8
    for (int b = l; b < nblk; b += 16) sum += dpart[b * 12 + v];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 16);
    if (l == 0) d[v] = sum;
  }
  __syncthreads();
}

// One block: reduce the dots and advance the scalars.  INIT: norms of b and
// r0, rho = r0.r0.  RHO (after an x, r update): residual norms, convergence
// flags, beta and rho.  thr = relative residual at which a column is frozen
// (from then on its alpha, omega and beta are 0).  Nothing to do once every
// column is done.
__global__ void __launch_bounds__(kVB) k_bi_scal(int mode, int nblk, const double* __restrict__ dpart,
                                                double* __restrict__ sc, double thr) {
  __shared__ double d[12];
  __shared__ int dn[6];
  if (mode != BI_INIT && sc[SC_ALL] != 0.0) return;
  dots_reduce(nblk, dpart, d);
  const int c = threadIdx.x;
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
  if (c == 0) {
    sc[SC_ALL] = (dn[0] && dn[1] && dn[2] && dn[3] && dn[4] && dn[5]) ? 1.0 : 0.0;
    sc[SC_IT] = mode == BI_INIT ? 0.0 : sc[SC_IT] + 1.0;
  }
}

// The vector a product is taken of, formed where it is read: PLAIN the
// given vector a; P the new search direction p' = r + beta (p - omega v)
// (a = p, b = v of the previous iteration); S the intermediate residual
// s = r - alpha v (a = v = L p'), alpha from the dots rh.v of the previous
// launch, reduced by every block alike and stored by the first.
enum { KMV_PLAIN = 0, KMV_P = 1, KMV_S = 2 };

// part[split][i][c] = sum_{j in split} K^T[j][i] in[j][c] for the in of MODE.
// Grid = (row tiles of kKmvRows states) x (S splits of the j range).  A block
// takes two adjacent states per lane; its four wavefronts take every fourth
// j (eight rows of K^T loaded before they are used, to keep bytes in
// flight; the in vector read from an LDS chunk) and are summed in wave
// order.  P and S store their in vector (p' or s) from the first row tile,
// and return at once when every column is done.
// P with sco != null also takes the rho / beta / convergence step of the
// previous iteration's x, r update (its dots dxr of nxr blocks): every block
// reduces them alike from the scalars sco of the previous iteration, and
// the first block stores the new scalars into sc, a different slot, so no
// block reads a scalar another one writes during the launch.
template <typename KS, int MODE>
__global__ void __launch_bounds__(256) k_kmv(int64_t M, int64_t ldk, int64_t jlen, const KS* __restrict__ KT,
                                             const double* __restrict__ r, const double* __restrict__ a,
                                             const double* __restrict__ b, const double* __restrict__ dpart,
                                             int nblk, double* sc, double* __restrict__ wv,
                                             double* __restrict__ part, const double* __restrict__ sco,
                                             const double* __restrict__ dxr, int nxr, double thr) {
  __shared__ double red[3][2][6][64];
  __shared__ double xs[kKmvChunk * 6];
  __shared__ double d[12];
  __shared__ double s0[6], s1[6];
  __shared__ int dn[6];
  typedef typename Two<KS>::type K2;
  const bool first = blockIdx.x == 0 && blockIdx.y == 0;
  if (MODE == KMV_P && sco) {
    if (sco[SC_ALL] != 0.0) {  // converged earlier: carry the scalars over and stop
      if (first && threadIdx.x < SC_N) sc[threadIdx.x] = sco[threadIdx.x];
      return;
    }
    dots_reduce(nxr, dxr, d);
    if (threadIdx.x < 6) {
      const int c = threadIdx.x;
      const double rn = sqrt(d[6 + c]);
      bool done = sco[SC_DONE + c] != 0.0;
      if (!done && rn <= thr * fmax(sco[SC_BNORM + c], 1e-300)) done = true;
      const double rho_old = sco[SC_RHO + c], om = sco[SC_OMEGA + c], al = sco[SC_ALPHA + c];
      const double beta = (done || rho_old == 0.0 || om == 0.0) ? 0.0 : (d[c] / rho_old) * (al / om);
      s0[c] = beta;
      s1[c] = om;
      dn[c] = done ? 1 : 0;
      if (first) {
        sc[SC_RHO + c] = d[c];
        sc[SC_ALPHA + c] = al;
        sc[SC_OMEGA + c] = om;
        sc[SC_BETA + c] = beta;
        sc[SC_BNORM + c] = sco[SC_BNORM + c];
        sc[SC_RNORM + c] = rn;
        sc[SC_DONE + c] = done ? 1.0 : 0.0;
      }
    }
    __syncthreads();
    const bool all = dn[0] && dn[1] && dn[2] && dn[3] && dn[4] && dn[5];
    if (first && threadIdx.x == 0) {
      sc[SC_ALL] = all ? 1.0 : 0.0;
      sc[SC_IT] = sco[SC_IT] + 1.0;
    }
    if (all) return;  // the whole grid returns
  } else if (MODE != KMV_PLAIN && sc[SC_ALL] != 0.0) {
    return;  // the whole grid returns
  }
  if (MODE == KMV_S) {
    dots_reduce(nblk, dpart, d);
    if (threadIdx.x < 6) {
      const int c = threadIdx.x;
      const double al = (sc[SC_DONE + c] == 0.0 && d[c] != 0.0) ? sc[SC_RHO + c] / d[c] : 0.0;
      s0[c] = al;
      if (blockIdx.x == 0 && blockIdx.y == 0) sc[SC_ALPHA + c] = al;
    }
  } else if (MODE == KMV_P && !sco) {
    if (threadIdx.x < 6) {
      s0[threadIdx.x] = sc[SC_BETA + threadIdx.x];
      s1[threadIdx.x] = sc[SC_OMEGA + threadIdx.x];
    }
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t il = (int64_t)blockIdx.x * kKmvRows + 2 * lane;  // il, il + 1 < ldk
  const int64_t jb = (int64_t)blockIdx.y * jlen;
  const int64_t je = jb + jlen < M ? jb + jlen : M;
  double acc[2][6];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[h][c] = 0.0;
  // the j range in chunks: the chunk's in vector is formed once into LDS
  // (and stored by the first row tile), then every wavefront reads it there
  for (int64_t cb = jb; cb < je; cb += kKmvChunk) {
    const int64_t ce = cb + kKmvChunk < je ? cb + kKmvChunk : je;
    __syncthreads();  // the previous chunk is consumed (and s0, s1 are set)
    for (int t = threadIdx.x; t < (int)(ce - cb) * 6; t += 256) {
      const int64_t e = cb * 6 + t;
      const int c = t % 6;
      double val;
      if (MODE == KMV_P) val = r[e] + s0[c] * (a[e] - s1[c] * b[e]);
      else if (MODE == KMV_S) val = r[e] - s0[c] * a[e];
      else val = a[e];
      xs[t] = val;
      if (MODE != KMV_PLAIN && blockIdx.x == 0) wv[e] = val;
    }
    __syncthreads();
    int64_t j = cb + wave;
    for (; j + 28 < ce; j += 32) {
      K2 kk[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) kk[u] = *reinterpret_cast<const K2*>(KT + (j + 4 * u) * ldk + il);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double* xj = xs + (j + 4 * u - cb) * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          acc[0][c] += (double)kk[u].x * xj[c];
          acc[1][c] += (double)kk[u].y * xj[c];
        }
      }
    }
    for (; j < ce; j += 4) {
      const K2 k = *reinterpret_cast<const K2*>(KT + j * ldk + il);
      const double* xj = xs + (j - cb) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        acc[0][c] += (double)k.x * xj[c];
        acc[1][c] += (double)k.y * xj[c];
      }
    }
  }
  if (wave > 0)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 6; ++c) red[wave - 1][h][c][lane] = acc[h][c];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[h][c] += red[w][h][c][lane];
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (il + h < M)
#pragma unroll
        for (int c = 0; c < 6; ++c) part[((int64_t)blockIdx.y * M + il + h) * 6 + c] = acc[h][c];
  }
}

// out = in - sum_split part (splits in order); optional dots a0.out and
// out.out; returns at once when every column is done (sc given)
__global__ void __launch_bounds__(kVB) k_kmv_fin(int64_t n6, int S, const double* __restrict__ in,
                                                 const double* __restrict__ part, double* __restrict__ out,
                                                 const double* __restrict__ a0, int sq, const double* sc,
                                                 double* __restrict__ dpart) {
  __shared__ double sh[2 * kVB];
  if (sc && sc[SC_ALL] != 0.0) return;
  double d0 = 0.0, d1 = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kVB + threadIdx.x; t < n6; t += (int64_t)gridDim.x * kVB) {
    // every split's partial is requested before the first is added (S <= 32)
    double ps[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) ps[s] = s < S ? part[(int64_t)s * n6 + t] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < 32; ++s)
      if (s < S) v += ps[s];
    v = in[t] - v;
    out[t] = v;
    if (a0) d0 += a0[t] * v;
    if (sq) d1 += v * v;
  }
  if (dpart) dots_out(d0, d1, sh, dpart);
}

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

// omega from the dots s.t, t.t of the previous launch (reduced by every
// block alike, stored by the first); x += alpha p + omega s; r = s - omega t;
// dots rh.r, r.r into dxr
__global__ void __launch_bounds__(kVB) k_bi_xr(int64_t n6, const double* __restrict__ p,
                                               const double* __restrict__ s, const double* __restrict__ tv,
                                               const double* __restrict__ rh, const double* __restrict__ dpart,
                                               int nblk, double* sc, double* __restrict__ x,
                                               double* __restrict__ r, double* __restrict__ dxr) {
  __shared__ double sh[2 * kVB];
  __shared__ double d[12];
  __shared__ double om6[6];
  if (sc[SC_ALL] != 0.0) return;  // the whole grid returns
  dots_reduce(nblk, dpart, d);
  if (threadIdx.x < 6) {
    const int c = threadIdx.x;
    const double om = (sc[SC_DONE + c] == 0.0 && d[6 + c] > 0.0) ? d[c] / d[6 + c] : 0.0;
    om6[c] = om;
    if (blockIdx.x == 0) sc[SC_OMEGA + c] = om;
  }
  __syncthreads();
  const int c = (int)(((int64_t)blockIdx.x * kVB + threadIdx.x) % 6);
  const double al = sc[SC_ALPHA + c], om = om6[c];
  double d0 = 0.0, d1 = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kVB + threadIdx.x; t < n6; t += (int64_t)gridDim.x * kVB) {
    x[t] += al * p[t] + om * s[t];
    const double rv = s[t] - om * tv[t];
    r[t] = rv;
    d0 += rh[t] * rv;
    d1 += rv * rv;
  }
  dots_out(d0, d1, sh, dxr);
}

// ---------------------------------------------------------------------------
// host side

template <typename ST>
elph_status build_self_operator(elph_ctx ctx, const ST* Bp, const ST* Bm, const double* lomf, const double* nocc,
                                const double* we, const int32_t* order, const int32_t* goff, const double* wff,
                                const SelfSolver& sv) {
  const int64_t M = ctx->nstates;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  const dim3 grid(blocks_for(M, 64), (unsigned)(sv.ldk / 64));
  if (sv.kt_f32) {
    hipLaunchKernelGGL((k_build_kT<ST, float>), grid, dim3(256), 0, ctx->stream, M, sv.ldk, ctx->nbr, md, Bp, Bm,
                       ctx->d_state_k, lomf, nocc, we, (float*)sv.KT);
    hipLaunchKernelGGL(k_kT_project<float>, dim3((unsigned)M), dim3(256), 0, ctx->stream, sv.ldk, ctx->ngroups,
                       order, goff, wff, (float*)sv.KT);
  } else {
    hipLaunchKernelGGL((k_build_kT<ST, double>), grid, dim3(256), 0, ctx->stream, M, sv.ldk, ctx->nbr, md, Bp, Bm,
                       ctx->d_state_k, lomf, nocc, we, (double*)sv.KT);
    hipLaunchKernelGGL(k_kT_project<double>, dim3((unsigned)M), dim3(256), 0, ctx->stream, sv.ldk, ctx->ngroups,
                       order, goff, wff, (double*)sv.KT);
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

// blocks aimed at per matrix-vector product (row tiles x j splits)
constexpr int64_t kKmvBlocks = 640;

void self_solver_layout(int64_t M, SelfSolver* sv) {
  sv->ldk = M > 0 ? kt_ld(M) : kKmvRows;
  sv->nt = (int)(sv->ldk / kKmvRows);
  int64_t S = (kKmvBlocks + sv->nt - 1) / sv->nt;
  if (S < 1) S = 1;
  if (S > 32) S = 32;
  if (S > M) S = M > 0 ? M : 1;
  sv->jlen = M > 0 ? (M + S - 1) / S : 1;
  sv->S = M > 0 ? (int)((M + sv->jlen - 1) / sv->jlen) : 1;
  const int64_t need = (6 * M + kVB - 1) / kVB;
  sv->nblk = (int)(need < 1 ? 1 : need < 256 ? need : 256);
}

static size_t kt_doubles(int64_t M, int64_t ldk, bool f32) {
  return f32 ? ((size_t)M * ldk + 1) / 2 : (size_t)M * ldk;
}

size_t self_solver_doubles(int64_t M, bool kt_f32) {
  SelfSolver sv;
  self_solver_layout(M, &sv);
  return kt_doubles(M, sv.ldk, kt_f32) + 9 * (size_t)M * 6 + (size_t)sv.S * M * 6 + 2 * (size_t)sv.nblk * 12 +
         2 * SC_N;
}

void self_solver_carve(int64_t M, bool kt_f32, double* base, SelfSolver* sv) {
  self_solver_layout(M, sv);
  double* p = base;
  sv->KT = p;
  sv->kt_f32 = kt_f32;
  p += kt_doubles(M, sv->ldk, kt_f32);
  double** vecs[] = {&sv->b, &sv->r, &sv->rh, &sv->p, &sv->p2, &sv->v, &sv->v2, &sv->s, &sv->t};
  for (double** v : vecs) {
    *v = p;
    p += (size_t)M * 6;
  }
  sv->part = p;
  p += (size_t)sv->S * M * 6;
  sv->dpart = p;
  p += (size_t)sv->nblk * 12;
  sv->dxr = p;
  p += (size_t)sv->nblk * 12;
  sv->sc = p;
}

// split partial products K' in of the in vector of MODE (see k_kmv)
template <int MODE>
static void kmv(elph_ctx ctx, const SelfSolver& sv, double* sc, const double* a, const double* b, double* wv,
                const double* sco = nullptr, double thr = 0.0) {
  const int64_t M = ctx->nstates;
  const dim3 grid((unsigned)sv.nt, (unsigned)sv.S);
  if (sv.kt_f32)
    hipLaunchKernelGGL((k_kmv<float, MODE>), grid, dim3(256), 0, ctx->stream, M, sv.ldk, sv.jlen,
                       (const float*)sv.KT, sv.r, a, b, sv.dpart, sv.nblk, sc, wv, sv.part, sco, sv.dxr, sv.nblk,
                       thr);
  else
    hipLaunchKernelGGL((k_kmv<double, MODE>), grid, dim3(256), 0, ctx->stream, M, sv.ldk, sv.jlen,
                       (const double*)sv.KT, sv.r, a, b, sv.dpart, sv.nblk, sc, wv, sv.part, sco, sv.dxr, sv.nblk,
                       thr);
}

static void kmv_fin(elph_ctx ctx, const SelfSolver& sv, const double* in, double* out, const double* a0, int sq,
                    const double* sc, double* dpart) {
  hipLaunchKernelGGL(k_kmv_fin, dim3((unsigned)sv.nblk), dim3(kVB), 0, ctx->stream, 6 * ctx->nstates, sv.S, in,
                     sv.part, out, a0, sq, sc, dpart);
}

// BiCGSTAB with every scalar on the device.  An iteration is five launches:
// the rho / beta / convergence step of the previous iteration's dots with p'
// and the products of v' = L p'; v' with rh.v'; alpha (in every block) with
// s and the products of t = L s; t with s.t, t.t; omega (in every block)
// with the x, r update and rh.r, r.r.  The scalars alternate between two
// slots, since the first launch reads the previous iteration's while its
// first block writes the new ones.  Before a read of the convergence flags
// the pending rho step runs on its own (k_bi_scal, in place).  p and v
// alternate between two buffers, since the first launch reads the old pair
// while it writes the new p'.
elph_status self_solve(elph_ctx ctx, const SelfSolver& sv, double* x, double thr, int maxit, bool* ok,
                       int* iters) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, n6 = 6 * M;
  if (!ctx->h_pin) HIPCHK(hipHostMalloc((void**)&ctx->h_pin, SC_N * sizeof(double), hipHostMallocDefault));
  if (M == 0) {
    *ok = true;
    *iters = 0;
    return ELPH_OK;
  }
  double* slot[2] = {sv.sc, sv.sc + SC_N};
  int cur = 0;
  // r0 = b - L x0 (v holds L x0 until the init kernel clears it)
  kmv<KMV_PLAIN>(ctx, sv, slot[cur], x, nullptr, nullptr);
  kmv_fin(ctx, sv, x, sv.v, nullptr, 0, nullptr, nullptr);
  hipLaunchKernelGGL(k_bi_init, dim3((unsigned)sv.nblk), dim3(kVB), 0, s, n6, sv.b, sv.v, sv.r, sv.rh, sv.p, sv.v,
                     sv.dpart);
  hipLaunchKernelGGL(k_bi_scal, dim3(1), dim3(kVB), 0, s, (int)BI_INIT, sv.nblk, sv.dpart, slot[cur], thr);
  HIPCHK(hipGetLastError());
  // iterations between reads of the convergence flags; once every column is
  // done the launches of the iterations in between return at once
  const int kCheck = 8;
  double* pv[2] = {sv.p, sv.p2};
  double* vv[2] = {sv.v, sv.v2};
  int it = 0;
  bool all = false, pending = false;  // pending: x, r updated, rho step not yet run
  for (;;) {
    if (it % kCheck == 0 || it >= maxit) {
      if (pending)
        hipLaunchKernelGGL(k_bi_scal, dim3(1), dim3(kVB), 0, s, (int)BI_RHO, sv.nblk, sv.dxr, slot[cur], thr);
      pending = false;
      HIPCHK(hipMemcpyAsync(ctx->h_pin, slot[cur], SC_N * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      all = ctx->h_pin[SC_ALL] != 0.0;
      if (all || it >= maxit) break;
    }
    const int o = it & 1, n = o ^ 1;
    ++it;
    if (pending) {
      kmv<KMV_P>(ctx, sv, slot[cur ^ 1], pv[o], vv[o], pv[n], slot[cur], thr);  // rho step, p', products of L p'
      cur ^= 1;
    } else {
      kmv<KMV_P>(ctx, sv, slot[cur], pv[o], vv[o], pv[n]);                      // p', products of L p'
    }
    double* sc = slot[cur];
    kmv_fin(ctx, sv, pv[n], vv[n], sv.rh, 0, sc, sv.dpart);     // v' = L p'; rh.v'
    kmv<KMV_S>(ctx, sv, sc, vv[n], nullptr, sv.s);             // alpha, s, products of L s
    kmv_fin(ctx, sv, sv.s, sv.t, sv.s, 1, sc, sv.dpart);        // t = L s; s.t, t.t
    hipLaunchKernelGGL(k_bi_xr, dim3((unsigned)sv.nblk), dim3(kVB), 0, s, n6, pv[n], sv.s, sv.t, sv.rh, sv.dpart,
                       sv.nblk, sc, x, sv.r, sv.dxr);           // omega, x, r; rh.r, r.r
    pending = true;
    HIPCHK(hipGetLastError());
  }
  *ok = all;
  *iters = (int)ctx->h_pin[SC_IT];
  return ELPH_OK;
}

}  // namespace elph
