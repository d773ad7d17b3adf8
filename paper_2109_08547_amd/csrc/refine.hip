// FP64 refinement of ill-conditioned vertices in the GEMM forms (FP32 and
// the BF16 / FP16 splits).
//
// A vertex component of Eq. 6 is a sum of a few thousand products; the GEMM
// forms accumulate it with an error of about cu times the root-sum-square of
// those products (cu: the form's contraction error unit: FP32 rounding of
// the MFMA partial sums and of the operands).  Where the component, or its
// projection g_s = sum_x l u gh_x on a branch, is much smaller than that
// scale (a near-cancellation, which happens for a few terms in every large
// material), |g|^2 carries a relative error far above 1e-5, and a rate
// that such a term dominates inherits it; the phonon rates of Eq. 25, which
// the Gaussian of Eq. 8 often reduces to one or two pairs, are the usual
// victims.
//
// The epilogue stores, per term, a log-coded estimate of the relative error
// of |g|^2.  At a temperature the rate reductions add up each term's
// contribution times its estimate and flag the rates whose estimated
// relative error exceeds refine_theta.  Here the terms that carry a
// sizeable part of a flagged rate's error are recomputed in FP64 (the
// step-1 rows of their initial states by the FP64 MFMA kernel, then the
// step-2 sum and the epilogue per pair), written back to the store with
// code 0 (exact), and the rates of the affected rows and wave vectors are
// reduced again.
#include "common.h"
#include "devutil.h"
#include "vertex.h"

#include <algorithm>
#include <vector>

namespace elph {

bool refine_applicable(elph_ctx ctx) {
  return ctx->precision != ELPH_FP64 && ctx->refine_theta > 0.0 && ctx->delta == ELPH_DELTA_GAUSS &&
         !ctx->d_tile_keep;
}

// Contraction error units per form.  The error of a vertex component has a
// part that scales with the root-sum-square of its products (operand
// rounding: FP32 and the three-part BF16 split keep 24 bits, the two-part
// FP16 split 22, the two-part BF16 split 16; MFMA partial sums in FP32) and
// a part that scales with the component itself (FP32 partial sums that grow
// with it when the products add up coherently, and the FP32 output of the
// GEMM).  The units are set at about 1.5 times the observed median, so that
// an estimate is of the order of one standard deviation of the error.
double refine_unit(elph_ctx ctx, bool coherent) {
  switch (ctx->precision) {
    case ELPH_FP32: return coherent ? 1.0e-7 : 1.2e-7;
    case ELPH_FP16X3: return coherent ? 1.0e-7 : 1.2e-7;
    case ELPH_BF16X6: return coherent ? 1.0e-7 : 1.2e-7;
    case ELPH_BF16X3: return coherent ? 2.0e-6 : 6.0e-6;
    default: return 0.0;
  }
}

elph_status refine_prepare(elph_ctx ctx) {
  const int64_t M = ctx->nstates;
  ctx->rho_stride = ctx->nbr <= 8 ? 8 : 16;
  if (!ctx->d_rho) ALLOC(ctx->d_rho, (size_t)M * M * ctx->rho_stride);
  if (!ctx->d_b2n) ALLOC(ctx->d_b2n, (size_t)M * ctx->nbr * sizeof(float));
  return ELPH_OK;
}

// b2n[i][x] = (1/nb) sum_(Rp,n') w_p(Rp)^2 |C1[i][(x, Rp, n')]|^2 / s^2, C1
// the step-1 GEMM rows (operand scale s): with unit eigenvectors,
// sum_n' |U_j[n', n]|^2 = 1, so this is the expected root-sum-square^2 of the
// products behind any step-2 component of row (i, x).  One wavefront per
// (i, x) over the contiguous (Rp, n') block.
__global__ void __launch_bounds__(256) k_b2_norms(int64_t i0, int64_t ni, int nbr, int nrp, int nb,
                                                  const float* __restrict__ C1, const double* __restrict__ wrp,
                                                  double scale, float* __restrict__ b2n) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= ni * nbr) return;
  const int64_t il = w / nbr;
  const int x = (int)(w - il * nbr);
  const int64_t len = (int64_t)nrp * nb;
  const float* __restrict__ row = C1 + 2 * (il * nbr + x) * len;
  double a = 0.0;
  for (int64_t k = lane; k < len; k += 64) {
    const float2 v = *reinterpret_cast<const float2*>(row + 2 * k);
    const double wr = wrp ? wrp[k / nb] : 1.0;
    a += wr * wr * ((double)v.x * v.x + (double)v.y * v.y);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if (lane == 0) b2n[(i0 + il) * nbr + x] = (float)(a * scale);
}

void refine_b2_norms(elph_ctx ctx, int64_t i0, int64_t ni, const float* C1) {
  const int64_t n = ni * ctx->nbr;
  const double s = ctx->sc_ae * ctx->sc_g;
  hipLaunchKernelGGL(k_b2_norms, dim3(blocks_for(n, 4)), dim3(256), 0, ctx->stream, i0, ni, ctx->nbr, ctx->nrp,
                     ctx->nb, C1, ctx->d_wrp, 1.0 / (s * s * ctx->nb), ctx->d_b2n);
}

// ---------------------------------------------------------------------------
// term selection

// Counters (cnt): 0 flagged rows, 1 flagged modes (written by the rate
// reductions), 2 selected pairs, 3 states with selected pairs, 4 wave vectors
// with selected pairs, 5 pairs beyond the list's capacity, 6 rows and 7 modes
// still above the threshold after the refinement.
struct Sel {
  int32_t* cnt;
  uint32_t* pbits;    // [ceil(M*M/32)] pair (i, j) selected
  int32_t* pi;        // [cap]
  int32_t* pj;        // [cap]
  int64_t cap;
  int32_t* slot;      // [M] index of state i in the state list, -1 if none
  int32_t* states;    // [M]
  int32_t* qflag;     // [nk]
  int32_t* qlist;     // [nk]
  const int32_t* st_k;
  int64_t M;
  MeshDims md;
};

__device__ inline void select_pair(const Sel& S, int32_t i, int32_t j) {
  const int64_t b = (int64_t)i * S.M + j;
  const uint32_t bit = 1u << (b & 31);
  if (atomicOr(&S.pbits[b >> 5], bit) & bit) return;
  const int32_t p = atomicAdd(&S.cnt[2], 1);
  if (p >= S.cap) {
    atomicAdd(&S.cnt[5], 1);
    return;
  }
  S.pi[p] = i;
  S.pj[p] = j;
  if (atomicCAS(&S.slot[i], -1, -2) == -1) {
    const int32_t t = atomicAdd(&S.cnt[3], 1);
    S.states[t] = i;
    atomicExch(&S.slot[i], t);
  }
  const int q = q_between(S.st_k[j], S.st_k[i], S.md.n0, S.md.n1, S.md.n2);
  if (atomicCAS(&S.qflag[q], 0, 1) == 0) S.qlist[atomicAdd(&S.cnt[4], 1)] = q;
}

// One block per flagged row i: select every (i, j) with a term whose
// contribution times its error estimate reaches frac * theta * W_e[i].
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_sel_rows(Sel S, const int32_t* __restrict__ rows, const ST* __restrict__ Bp,
                                                  const ST* __restrict__ Bm, const uint8_t* __restrict__ rho,
                                                  const double* __restrict__ lomf, const double* __restrict__ nocc,
                                                  const double* __restrict__ we, double thr) {
  const int32_t i = rows[blockIdx.x];
  const int64_t M = S.M;
  const int ki = S.st_k[i];
  const double li = lomf[i];
  const double lim = thr * we[i];
  for (int64_t j = threadIdx.x; j < M; j += 256) {
    const int q = q_between(S.st_k[j], ki, S.md.n0, S.md.n1, S.md.n2);
    const double w = exp(lomf[j] - li);
    const int64_t tb = ((int64_t)i * M + j) * NX;
    const uint8_t* __restrict__ rc = rho + ((int64_t)i * M + j) * RhoStride<NX>::value;
    bool take = false;
#pragma unroll
    for (int s = 0; s < NX; ++s) {
      const double n = nocc[(int64_t)q * NX + s];
      const double t = ((double)Bp[tb + s] * n + (double)Bm[tb + s] * (1.0 + n)) * w;
      take |= t * rho_decode(rc[s]) >= lim && t > 0.0;
    }
    if (take) select_pair(S, i, (int32_t)j);
  }
}

// One wavefront per flagged mode (q, s): select every pair of q's list whose
// term carries at least frac * theta of the accumulated rate acc[q][s].
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_sel_modes(Sel S, const int32_t* __restrict__ modes, int32_t nmodes,
                                                   const int32_t* __restrict__ kept,
                                                   const int32_t* __restrict__ kidx,
                                                   const int32_t* __restrict__ soff,
                                                   const int32_t* __restrict__ poff,
                                                   const int32_t* __restrict__ plist, const ST* __restrict__ Bp,
                                                   const uint8_t* __restrict__ rho, const double* __restrict__ f,
                                                   const double* __restrict__ omf, const double* __restrict__ acc,
                                                   double thr) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nmodes) return;
  const int32_t mode = modes[w];
  const int q = mode / NX, s = mode % NX;
  const double lim = thr * acc[mode];
  const MeshDims md = S.md;
  const int qc = q % md.n2, qt = q / md.n2;
  const int qb = qt % md.n1, qa = qt / md.n1;
  const int32_t pe = poff[q + 1];
  for (int32_t p = poff[q] + lane; p < pe; p += 64) {
    const int32_t t = plist[p];
    const int k = kept[t];
    const int kc = k % md.n2, kt = k / md.n2;
    const int kb = kt % md.n1, ka = kt / md.n1;
    int c2 = kc + qc; if (c2 >= md.n2) c2 -= md.n2;
    int b2 = kb + qb; if (b2 >= md.n1) b2 -= md.n1;
    int a2 = ka + qa; if (a2 >= md.n0) a2 -= md.n0;
    const int32_t u = kidx[(a2 * md.n1 + b2) * md.n2 + c2];
    for (int32_t i = soff[t]; i < soff[t + 1]; ++i)
      for (int32_t j = soff[u]; j < soff[u + 1]; ++j) {
        const int64_t pr = (int64_t)i * S.M + j;
        const double v = (double)Bp[pr * NX + s] * f[i] * omf[j];
        if (v > 0.0 && v * rho_decode(rho[pr * RhoStride<NX>::value + s]) >= lim) select_pair(S, i, j);
      }
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

__global__ void k_state_rows(int32_t ns, const int32_t* __restrict__ states, const int32_t* __restrict__ st_kidx,
                             const int32_t* __restrict__ st_m, int32_t* __restrict__ kid, int32_t* __restrict__ mm) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  kid[t] = st_kidx[states[t]];
  mm[t] = st_m[states[t]];
}

// ---------------------------------------------------------------------------
// FP64 recomputation of selected pairs

struct RefPairs {
  int64_t M;
  int nb, nrp;
  int64_t kp64;
  MeshDims md;
  const int32_t* pi;
  const int32_t* pj;
  const int32_t* slot;
  const double* B2;       // [slots][nbr][kp64] complex FP64 step-1 rows
  const cd* Ep;           // [nkept][nrp]
  const double* wrp;      // [nrp] or null
  const cd* ust;          // [nstates][nb]
  const int32_t* st_k;
  const int32_t* st_kidx;
  const double* eps;
  const double* hw;       // [nk][nbr]
  const cd* Lq;           // [nk][nbr][nbr]
  const cd* fr;           // Froehlich factors or null
  double pref, inv2s2, omega_min;
};

// One wavefront per selected pair (i, j): gh_x = sum_(Rp,n') A_p[j] B2[(i,x)]
// with A_p[j][(Rp,n')] = w_p e^{2 pi i k_j.Rp} conj(U_j[n']), then the
// epilogue of Eq. 6 / Eq. 8 as in the GEMM path, in FP64; the store entries
// of the pair are overwritten and their codes set to 0 (exact).
template <int NX>
__global__ void __launch_bounds__(256) k_ref_pairs(RefPairs R, int32_t npairs, float* __restrict__ Bp,
                                                   float* __restrict__ Bm, uint8_t* __restrict__ rho) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= npairs) return;
  const int32_t i = R.pi[w], j = R.pj[w];
  const int64_t si = R.slot[i];
  const int kj = R.st_kidx[j];
  const int nb = R.nb;
  const int64_t K = (int64_t)R.nrp * nb;
  double ar[NX], ai[NX];
#pragma unroll
  for (int x = 0; x < NX; ++x) ar[x] = ai[x] = 0.0;
  const double* __restrict__ brow = R.B2 + 2 * si * NX * R.kp64;
  for (int64_t k = lane; k < K; k += 64) {
    const int r = (int)(k / nb), n = (int)(k - (int64_t)r * nb);
    cd a = cmulc(R.Ep[(int64_t)kj * R.nrp + r], R.ust[(int64_t)j * nb + n]);   // e^{i k_j.Rp} conj(U_j[n'])
    if (R.wrp) a = cscale(a, R.wrp[r]);
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      const double2 b = *reinterpret_cast<const double2*>(brow + 2 * (x * R.kp64 + k));
      ar[x] += a.x * b.x - a.y * b.y;
      ai[x] += a.x * b.y + a.y * b.x;
    }
  }
#pragma unroll
  for (int x = 0; x < NX; ++x)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ar[x] += __shfl_xor(ar[x], o, 64);
      ai[x] += __shfl_xor(ai[x], o, 64);
    }
  if (lane >= NX) return;
  const int s = lane;
  const int q = q_between(R.st_k[j], R.st_k[i], R.md.n0, R.md.n1, R.md.n2);
  const cd* __restrict__ L = R.Lq + (int64_t)q * NX * NX;
  double gr = 0.0, gi = 0.0;
#pragma unroll
  for (int x = 0; x < NX; ++x) {
    const cd l = L[x * NX + s];
    gr += l.x * ar[x] - l.y * ai[x];
    gi += l.x * ai[x] + l.y * ar[x];
  }
  if (R.fr) {  // Eq. 7: F_s(q) times the overlap of the two states
    double orr = 0.0, oi = 0.0;
    for (int n = 0; n < nb; ++n) {
      const cd uj = R.ust[(int64_t)j * nb + n], ui = R.ust[(int64_t)i * nb + n];
      orr += uj.x * ui.x + uj.y * ui.y;
      oi += uj.x * ui.y - uj.y * ui.x;
    }
    const cd f = R.fr[(int64_t)q * NX + s];
    gr += f.x * orr - f.y * oi;
    gi += f.x * oi + f.y * orr;
  }
  const double g2 = gr * gr + gi * gi;
  const double hw = R.hw[(int64_t)q * NX + s];
  double bp = 0.0, bm = 0.0;
  if (hw >= R.omega_min) {
    const double de = R.eps[j] - R.eps[i];
    const double dp = de - hw, dm = de + hw;
    bp = R.pref * g2 * exp(-dp * dp * R.inv2s2);
    bm = R.pref * g2 * exp(-dm * dm * R.inv2s2);
  }
  const int64_t pr = (int64_t)i * R.M + j;
  Bp[pr * NX + s] = (float)bp;
  Bm[pr * NX + s] = (float)bm;
  rho[pr * RhoStride<NX>::value + s] = 0;
}

template <int NX>
static void launch_sel(elph_ctx ctx, const Sel& S, const Thermal& th, const double* we, const double* acc,
                       const RateErr& ee, const RateErr& ep, int32_t nrows, int32_t nmodes, double thr) {
  hipStream_t s = ctx->stream;
  const float* Bp = (const float*)ctx->d_Bp;
  const float* Bm = (const float*)ctx->d_Bm;
  if (nrows > 0)
    hipLaunchKernelGGL((k_sel_rows<float, NX>), dim3((unsigned)nrows), dim3(256), 0, s, S, ee.list, Bp, Bm,
                       ctx->d_rho, th.lomf, th.nocc, we, thr);
  if (nmodes > 0)
    hipLaunchKernelGGL((k_sel_modes<float, NX>), dim3((unsigned)((nmodes + 3) / 4)), dim3(256), 0, s, S, ep.list,
                       nmodes, ctx->d_kept, ctx->d_kidx, ctx->d_soff, ctx->d_poff, ctx->d_plist, Bp, ctx->d_rho,
                       th.f, th.omf, acc, thr);
}

template <int NX>
static void launch_ref_pairs(elph_ctx ctx, const RefPairs& R, int32_t npairs) {
  hipLaunchKernelGGL((k_ref_pairs<NX>), dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, ctx->stream, R, npairs,
                     (float*)ctx->d_Bp, (float*)ctx->d_Bm, ctx->d_rho);
}

// Fraction of theta that one term's estimated error must reach to be
// recomputed in a flagged rate.
constexpr double kSelFrac = 1.0 / 8.0;
// Largest number of pairs recomputed per call.
constexpr int64_t kMaxRefinePairs = (int64_t)1 << 22;

elph_status refine_terms(elph_ctx ctx, const Thermal& th, double* we, double* acc, const RateErr& ee,
                         const RateErr& ep, int32_t* cnt) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates, nk = ctx->nk;
  const int nbr = ctx->nbr;
  for (int k = 0; k < 8; ++k) ctx->ref_stats[k] = 0;
  int32_t h[8];
  HIPCHK(hipMemcpyAsync(h, cnt, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int32_t nrows = we ? h[0] : 0, nmodes = acc ? h[1] : 0;
  ctx->ref_stats[0] = nrows;
  ctx->ref_stats[1] = nmodes;
  if (nrows == 0 && nmodes == 0) return ELPH_OK;

  Sel S;
  S.cnt = cnt;
  S.M = M;
  S.md = MeshDims{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  S.st_k = ctx->d_state_k;
  S.cap = std::min<int64_t>(kMaxRefinePairs, M * M);
  const int64_t nwords = (M * M + 31) / 32;
  ALLOC(S.pbits, nwords * sizeof(uint32_t));
  ALLOC(S.pi, S.cap * sizeof(int32_t));
  ALLOC(S.pj, S.cap * sizeof(int32_t));
  ALLOC(S.slot, M * sizeof(int32_t));
  ALLOC(S.states, M * sizeof(int32_t));
  ALLOC(S.qflag, nk * sizeof(int32_t));
  ALLOC(S.qlist, nk * sizeof(int32_t));
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nwords, 256)), dim3(256), 0, s, (int32_t*)S.pbits, nwords, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(M, 256)), dim3(256), 0, s, S.slot, M, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nk, 256)), dim3(256), 0, s, S.qflag, nk, 0);
  const double thr = kSelFrac * ctx->refine_theta;
#define SEL(NXV) launch_sel<NXV>(ctx, S, th, we, acc, ee, ep, nrows, nmodes, thr)
  switch (nbr) {
    case 3: SEL(3); break;
    case 6: SEL(6); break;
    case 9: SEL(9); break;
    case 12: SEL(12); break;
    default: SEL(15); break;
  }
#undef SEL
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h, cnt, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int32_t npairs = (int32_t)std::min<int64_t>(h[2], S.cap), ns = h[3], nq = h[4];
  ctx->ref_stats[2] = npairs;
  ctx->ref_stats[3] = ns;
  ctx->ref_stats[4] = nq;
  ctx->ref_stats[5] = h[5];
  elph_status st = ELPH_OK;
  if (npairs > 0) {
    st = ensure_gR64(ctx);
    if (st != ELPH_OK) return st;
    const int64_t ns_pad = ((int64_t)ns + 63) / 64 * 64;
    int32_t *kid = nullptr, *mm = nullptr;
    double *Ae64 = nullptr, *B2_64 = nullptr;
    ALLOC(kid, ns * sizeof(int32_t));
    ALLOC(mm, ns * sizeof(int32_t));
    ALLOC(Ae64, (size_t)ns_pad * ctx->ke64 * 16);
    ALLOC(B2_64, (size_t)ns_pad * nbr * ctx->kp64 * 16);
    hipLaunchKernelGGL(k_state_rows, dim3(blocks_for(ns, 256)), dim3(256), 0, s, ns, S.states, ctx->d_state_kidx,
                       ctx->d_state_m, kid, mm);
    st = step1_fp64_rows(ctx, ns, kid, mm, Ae64, B2_64);
    if (st != ELPH_OK) return st;
    RefPairs R;
    R.M = M;
    R.nb = ctx->nb;
    R.nrp = ctx->nrp;
    R.kp64 = ctx->kp64;
    R.md = S.md;
    R.pi = S.pi;
    R.pj = S.pj;
    R.slot = S.slot;
    R.B2 = B2_64;
    R.Ep = (const cd*)ctx->d_Ep;
    R.wrp = ctx->d_wrp;
    R.ust = (const cd*)ctx->d_ustate;
    R.st_k = ctx->d_state_k;
    R.st_kidx = ctx->d_state_kidx;
    R.eps = ctx->d_eps;
    R.hw = ctx->d_hw;
    R.Lq = (const cd*)ctx->d_Lq;
    R.fr = ctx->frohlich ? (const cd*)ctx->d_frohlich : nullptr;
    R.pref = 2.0 * kPi / (kHbarEVs * (double)ctx->nk) / (sqrt(2.0 * kPi) * ctx->sigma);
    R.inv2s2 = 1.0 / (2.0 * ctx->sigma * ctx->sigma);
    R.omega_min = ctx->omega_min;
    switch (nbr) {
      case 3: launch_ref_pairs<3>(ctx, R, npairs); break;
      case 6: launch_ref_pairs<6>(ctx, R, npairs); break;
      case 9: launch_ref_pairs<9>(ctx, R, npairs); break;
      case 12: launch_ref_pairs<12>(ctx, R, npairs); break;
      default: launch_ref_pairs<15>(ctx, R, npairs); break;
    }
    HIPCHK(hipGetLastError());
    // the rates of every row and wave vector with a recomputed term, reduced
    // again in the same order (counting those still above the threshold)
    RateErr re = ee, rp = ep;
    re.cnt = cnt + 6;
    rp.cnt = cnt + 7;
    re.idx = S.states;
    re.n = ns;
    rp.idx = S.qlist;
    rp.n = nq;
    if (we) launch_we_rows<float>(ctx, (const float*)ctx->d_Bp, (const float*)ctx->d_Bm, th.lomf, th.nocc, we, &re);
    if (acc && ep.rho)
      launch_q_gather<float, 1>(ctx, (const float*)ctx->d_Bp, th.f, th.omf, nullptr, acc, &rp);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h, cnt, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->ref_stats[6] = h[6];
    ctx->ref_stats[7] = h[7];
    dev_free(ctx, kid);
    dev_free(ctx, mm);
    dev_free(ctx, Ae64);
    dev_free(ctx, B2_64);
  } else {
    HIPCHK(hipStreamSynchronize(s));
  }
  dev_free(ctx, S.pbits);
  dev_free(ctx, S.pi);
  dev_free(ctx, S.pj);
  dev_free(ctx, S.slot);
  dev_free(ctx, S.states);
  dev_free(ctx, S.qflag);
  dev_free(ctx, S.qlist);
  return st;
}

}  // namespace elph
