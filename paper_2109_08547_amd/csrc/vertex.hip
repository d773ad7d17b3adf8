// The e-ph vertex of Eq. 6 ("The elphbolt ab initio solver ...") over all
// pairs of active states, as two complex contractions on MFMA:
//
//   step 1 (per initial state i = (k, m)):
//     Z[i][(x, Rp, n')] = sum_{(Re, m')} Ae[i][(Re, m')] g[Re][Rp][x][n'][m'],
//     Ae[i][(Re, m')]   = w_e e^{2 pi i k.Re} U_k[m'][m]
//     B2[(i, x)][(Rp, n')] = e^{-2 pi i k.Rp} Z[i][(x, Rp, n')]
//   step 2 (all final states j = (k', n) against all initial states i):
//     gh[j][(i, x)] = sum_{(Rp, n')} Ap[j][(Rp, n')] B2[(i, x)][(Rp, n')],
//     Ap[j][(Rp, n')] = w_p e^{2 pi i k'.Rp} conj(U_k'[n'][n])
//
// so that gh is the Bloch-rotated vertex conj(U_k')^T gW(k, q) U_k of the
// paper's Eq. 6 with q = k' - k (e^{2 pi i q.Rp} = e^{2 pi i k'.Rp}
// e^{-2 pi i k.Rp}).  The epilogue of step 2 projects on the phonon
// eigenvectors with the length prefactor (g_s = sum_x l_{x,s} u_q[x][s] gh_x),
// forms |g_s|^2 and the Gaussian energy-conserving delta of Eq. 8, stores the
// temperature-independent terms B^{+/-} = (2 pi / hbar N_k) |g|^2 delta(...)
// and accumulates the electron rate of Eq. 21 and the phonon rate of Eq. 25.
//
// Complex products use four real MFMAs (re*re - im*im, re*im + im*re).
// MFMA 16x16x4 operand layout (f64 and f32): lane l supplies A[row l%16][k l/16]
// and B[k l/16][col l%16]; accumulator r of lane l holds column l%16 and row
// l/16 + 4r (f64) or 4(l/16) + r (f32).
#include "devutil.h"
#include "vertex.h"
#include "tables.h"

#include <algorithm>
#include <map>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

namespace elph {

// ---------------------------------------------------------------------------
// precision policies

template <typename T>
struct Mfma;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <>
struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int r) { return lk + 4 * r; }
  static constexpr bool kFold = false;
};

template <>
struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int r) { return 4 * lk + r; }
  static constexpr bool kFold = true;
};

// BF16 split forms: every operand value a = a_1 + a_2 (+ a_3), each a_s a
// BF16 number (a_1 = bf16(a), a_2 = bf16(a - a_1), ...).  Storage per row:
// groups of 8 consecutive k, each group holding the planes re_1, im_1, re_2,
// im_2 (, re_3, im_3) of 8 BF16 values (16 bytes), so that a lane reads its
// 8-k MFMA fragment of every plane with 16-byte loads.
template <int NS>
struct Bf16S {};

// FP16 split form: the same layout with FP16 parts (a_1 = f16(a),
// a_2 = f16(a - a_1): 22 significant bits with NS = 2).  FP16's exponent
// range is narrow, so every operand carries a power-of-two scale that puts
// its largest possible magnitude at 2^12-2^13; the second part of any value
// within 2^-16 of that bound is then a normal FP16 number.  The epilogues
// undo the scales exactly.
template <int NS>
struct F16S {};

template <typename T>
struct Store {
  typedef T type;
  static constexpr int per_c = 2;      // storage elements per complex value
  static constexpr int kalign = sizeof(T) == 4 ? 32 : 16;  // padding of the contraction length (GEMM stages: 32)
};
template <int NS>
struct Store<Bf16S<NS>> {
  typedef unsigned short type;
  static constexpr int per_c = 2 * NS;
  static constexpr int kalign = 32;
};
template <int NS>
struct Store<F16S<NS>> : Store<Bf16S<NS>> {};

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef unsigned short us8v __attribute__((ext_vector_type(8)));

template <int NS>
struct Mfma<Bf16S<NS>> {
  typedef f4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mma(us8v a, us8v b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0,
                                                  0, 0);
  }
  __device__ static inline int row(int lk, int r) { return 4 * lk + r; }
  static constexpr bool kFold = true;
};

template <int NS>
struct Mfma<F16S<NS>> : Mfma<Bf16S<NS>> {
  typedef f4 acc_t;
  __device__ static inline acc_t mma(us8v a, us8v b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0,
                                                 0);
  }
};

// FP16 nearest of a double (through its float value) and back
__device__ inline unsigned short f16_of(double v) { return __builtin_bit_cast(unsigned short, (_Float16)(float)v); }
__device__ inline double f16_val(unsigned short h) { return (double)(float)__builtin_bit_cast(_Float16, h); }

// BF16 nearest (ties to even) of a double, through its float value
__device__ inline unsigned short bf16_of(double v) {
  unsigned u = __float_as_uint((float)v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline double bf16_val(unsigned short h) { return (double)__uint_as_float(((unsigned)h) << 16); }

// write the complex value (re, im) at (row, k) of an operand of padded length K
template <typename T>
__device__ inline void put_c(typename Store<T>::type* base, int64_t row, int64_t K, int64_t k, double re, double im) {
  base[2 * (row * K + k)] = (T)re;
  base[2 * (row * K + k) + 1] = (T)im;
}

template <int NS, bool F16 = false>
__device__ inline void put_split(unsigned short* base, int64_t row, int64_t K, int64_t k, double re, double im) {
  unsigned short* g = base + row * K * 2 * NS + (k >> 3) * (16 * NS) + (k & 7);
  double r = re, i = im;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const unsigned short hr = F16 ? f16_of(r) : bf16_of(r), hi = F16 ? f16_of(i) : bf16_of(i);
    g[(2 * s) * 8] = hr;
    g[(2 * s + 1) * 8] = hi;
    r -= F16 ? f16_val(hr) : bf16_val(hr);
    i -= F16 ? f16_val(hi) : bf16_val(hi);
  }
}

template <typename T>
struct PutC {
  __device__ static inline void put(typename Store<T>::type* base, int64_t row, int64_t K, int64_t k, double re,
                                    double im) {
    put_c<T>(base, row, K, k, re, im);
  }
};
template <int NS>
struct PutC<Bf16S<NS>> {
  __device__ static inline void put(unsigned short* base, int64_t row, int64_t K, int64_t k, double re, double im) {
    put_split<NS>(base, row, K, k, re, im);
  }
};
template <int NS>
struct PutC<F16S<NS>> {
  __device__ static inline void put(unsigned short* base, int64_t row, int64_t K, int64_t k, double re, double im) {
    put_split<NS, true>(base, row, K, k, re, im);
  }
};

// Products of a split complex fragment pair, smallest terms first:
// cr += Re(a) Re(b) - Im(a) Im(b), ci += Re(a) Im(b) + Im(a) Re(b), keeping
// the split pairs (s_a, s_b) with s_a + s_b <= 1 (NS = 2: three products)
// or <= 2 (NS = 3: six products).
template <class SP, int NS>
__device__ inline void split_cmma(const us8v (&a)[2 * NS], const us8v (&na_im)[NS], const us8v (&b)[2 * NS], f4& cr,
                                  f4& ci) {
  typedef Mfma<SP> MM;
  constexpr int np = NS == 2 ? 3 : 6;
#pragma unroll
  for (int t = 0; t < np; ++t) {
    int sa, sb;
    if (NS == 2) {  // (0,1), (1,0), (0,0)
      sa = t == 1 ? 1 : 0;
      sb = t == 0 ? 1 : 0;
    } else {        // (1,1), (0,2), (2,0), (0,1), (1,0), (0,0)
      sa = t == 0 ? 1 : t == 2 ? 2 : t == 4 ? 1 : 0;
      sb = t == 0 ? 1 : t == 1 ? 2 : t == 3 ? 1 : 0;
    }
    cr = MM::mma(a[2 * sa], b[2 * sb], cr);
    cr = MM::mma(na_im[sa], b[2 * sb + 1], cr);
    ci = MM::mma(a[2 * sa], b[2 * sb + 1], ci);
    ci = MM::mma(a[2 * sa + 1], b[2 * sb], ci);
  }
}

template <int NS>
__device__ inline void load_split(const unsigned short* p, us8v (&v)[2 * NS]) {
#pragma unroll
  for (int s = 0; s < 2 * NS; ++s) v[s] = *reinterpret_cast<const us8v*>(p + 8 * s);
}

template <int NS>
__device__ inline void neg_im(const us8v (&a)[2 * NS], us8v (&na)[NS]) {
  const us8v sign = {0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000, 0x8000};
#pragma unroll
  for (int s = 0; s < NS; ++s) na[s] = a[2 * s + 1] ^ sign;
}

template <typename T>
struct Cplx {
  T x, y;
};

template <typename T>
__device__ inline Cplx<T> ldc(const T* p) {
  if constexpr (sizeof(T) == 8) {
    double2 v = *reinterpret_cast<const double2*>(p);
    return Cplx<T>{(T)v.x, (T)v.y};
  } else {
    float2 v = *reinterpret_cast<const float2*>(p);
    return Cplx<T>{(T)v.x, (T)v.y};
  }
}

// ---------------------------------------------------------------------------
// operand builders (write the precision T of the contraction)

template <typename T>
__global__ void k_build_Ae(int64_t nstates, int nb, int nre, int64_t ke, const int32_t* __restrict__ st_kidx,
                           const int32_t* __restrict__ st_m, const cd* __restrict__ Ee, const cd* __restrict__ U,
                           double scale, typename Store<T>::type* __restrict__ Ae) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cols = (int64_t)nre * nb;
  if (e >= nstates * cols) return;
  int64_t i = e / cols;
  int64_t col = e % cols;
  int r = (int)(col / nb), mp = (int)(col % nb);
  int t = st_kidx[i], m = st_m[i];
  cd z = cmul(Ee[(int64_t)t * nre + r], U[((int64_t)t * nb + mp) * nb + m]);
  PutC<T>::put(Ae, i, ke, col, z.x * scale, z.y * scale);
}

template <typename T>
__global__ void k_build_Ap(int64_t nstates, int nb, int nrp, int64_t kp, const int32_t* __restrict__ st_kidx,
                           const int32_t* __restrict__ st_m, const cd* __restrict__ Ep,
                           const double* __restrict__ wrp, const cd* __restrict__ U, double scale,
                           typename Store<T>::type* __restrict__ Ap) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cols = (int64_t)nrp * nb;
  if (e >= nstates * cols) return;
  int64_t j = e / cols;
  int64_t col = e % cols;
  int r = (int)(col / nb), np = (int)(col % nb);
  int t = st_kidx[j], n = st_m[j];
  cd z = cmul(Ep[(int64_t)t * nrp + r], cconj(U[((int64_t)t * nb + np) * nb + n]));
  if (wrp) z = cscale(z, wrp[r]);
  PutC<T>::put(Ap, j, kp, col, z.x * scale, z.y * scale);
}

// gR[(x, Rp, n')][(Re, m')] = g[Re][Rp][x][n'][m']
template <typename T>
__global__ void k_permute_g(int nre, int nrp, int nbr, int nb, int64_t ke, const double* __restrict__ g,
                            double scale, typename Store<T>::type* __restrict__ gR) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nre * nrp * nbr * nb * nb;
  if (e >= total) return;
  int mp = (int)(e % nb);
  int64_t t = e / nb;
  int np = (int)(t % nb);
  t /= nb;
  int x = (int)(t % nbr);
  t /= nbr;
  int rp = (int)(t % nrp);
  int re = (int)(t / nrp);
  int64_t row = ((int64_t)x * nrp + rp) * nb + np;
  int64_t col = (int64_t)re * nb + mp;
  PutC<T>::put(gR, row, ke, col, g[2 * e] * scale, g[2 * e + 1] * scale);
}

// ---------------------------------------------------------------------------
// step 1: C[i][col] = sum_k Ae[i][k] gR[col][k]; epilogue writes B2 with the
// e^{-2 pi i k_i . Rp} factor.  Block 2x2 waves, wave tile 32 x 32.

// Step-1 contraction of one material (operands and sizes).
template <typename T>
struct S1Desc {
  int64_t m_pad, ncol, ke, kp, nstates;
  const typename Store<T>::type* Ae;
  const typename Store<T>::type* gR;
  typename Store<T>::type* B2;
  int nrp, nb, nbr;
  const int32_t* st_kidx;
  const cd* Ep;
};

template <typename T>
struct IsSplit {
  static constexpr bool value = false;
  static constexpr int ns = 0;
};
template <int NS>
struct IsSplit<Bf16S<NS>> {
  static constexpr bool value = true;
  static constexpr int ns = NS;
};
template <int NS>
struct IsSplit<F16S<NS>> {
  static constexpr bool value = true;
  static constexpr int ns = NS;
};

// One 64 x 64 output tile (block column bx, block row by) of step 1.
template <typename T>
__device__ __forceinline__ void step1_tile(const S1Desc<T>& d, int64_t bx, int64_t by) {
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  typedef typename Store<T>::type SE;
  const int64_t ncol = d.ncol, ke = d.ke, kp = d.kp, nstates = d.nstates;
  const SE* __restrict__ Ae = d.Ae;
  const SE* __restrict__ gR = d.gR;
  SE* __restrict__ B2 = d.B2;
  const int nrp = d.nrp, nb = d.nb, nbr = d.nbr;
  const int32_t* __restrict__ st_kidx = d.st_kidx;
  const cd* __restrict__ Ep = d.Ep;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t m0 = by * 64 + (wave >> 1) * 32;
  const int64_t n0 = bx * 64 + (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  acc_t cr[2][2], ci[2][2];
  // FP64 running sums: the FP32 and BF16 forms fold their MFMA accumulators
  // in every 16 (32) k so that rounding is relative to a short partial sum
  double fr[2][2][4], fi[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = MM::zero();
      ci[a][b] = MM::zero();
#pragma unroll
      for (int r = 0; r < 4; ++r) fr[a][b][r] = fi[a][b][r] = 0.0;
    }
  if constexpr (IsSplit<T>::value) {
    constexpr int NS = IsSplit<T>::ns;
    const SE* pa[2];
    const SE* pb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      pa[t] = Ae + (m0 + 16 * t + lr) * ke * 2 * NS + lk * 16 * NS;
      int64_t nrow = n0 + 16 * t + lr;
      if (nrow >= ncol) nrow = ncol - 1;
      pb[t] = gR + nrow * ke * 2 * NS + lk * 16 * NS;
    }
    for (int64_t k0 = 0; k0 < ke; k0 += 32) {
      const int64_t go = (k0 >> 3) * 16 * NS;
      us8v fa[2][2 * NS], fb[2][2 * NS], na[2][NS];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        load_split<NS>(pa[t] + go, fa[t]);
        load_split<NS>(pb[t] + go, fb[t]);
        neg_im<NS>(fa[t], na[t]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) split_cmma<T, NS>(fa[a], na[a], fb[b], cr[a][b], ci[a][b]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            fr[a][b][r] += (double)cr[a][b][r];
            fi[a][b][r] += (double)ci[a][b][r];
          }
          cr[a][b] = MM::zero();
          ci[a][b] = MM::zero();
        }
    }
  } else {
    const T* pa[2];
    const T* pb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      pa[t] = Ae + 2 * ((m0 + 16 * t + lr) * ke + lk);
      int64_t nrow = n0 + 16 * t + lr;
      if (nrow >= ncol) nrow = ncol - 1;
      pb[t] = gR + 2 * (nrow * ke + lk);
    }
    for (int64_t k0 = 0; k0 < ke; k0 += 16) {
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int64_t k = k0 + kk;
        Cplx<T> fa[2], fb[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          fa[t] = ldc(pa[t] + 2 * k);
          fb[t] = ldc(pb[t] + 2 * k);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            cr[a][b] = MM::mma(fa[a].x, fb[b].x, cr[a][b]);
            cr[a][b] = MM::mma(-fa[a].y, fb[b].y, cr[a][b]);
            ci[a][b] = MM::mma(fa[a].x, fb[b].y, ci[a][b]);
            ci[a][b] = MM::mma(fa[a].y, fb[b].x, ci[a][b]);
          }
      }
      if constexpr (MM::kFold) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              fr[a][b][r] += (double)cr[a][b][r];
              fi[a][b][r] += (double)ci[a][b][r];
            }
            cr[a][b] = MM::zero();
            ci[a][b] = MM::zero();
          }
      }
    }
    if constexpr (!MM::kFold) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            fr[a][b][r] = (double)cr[a][b][r];
            fi[a][b][r] = (double)ci[a][b][r];
          }
    }
  }
  // epilogue
  const int64_t per_x = (int64_t)nrp * nb;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = m0 + 16 * a + MM::row(lk, r);
        const int64_t col = n0 + 16 * b + lr;
        if (i >= nstates || col >= ncol) continue;
        const int x = (int)(col / per_x);
        const int64_t rem = col % per_x;
        const int rp = (int)(rem / nb);
        const cd ph = Ep[(int64_t)st_kidx[i] * nrp + rp];
        const cd z = cmulc(cmake(fr[a][b][r], fi[a][b][r]), ph);  // * conj(ph)
        PutC<T>::put(B2, i * nbr + x, kp, rem, z.x, z.y);
      }
}

template <typename T>
__global__ void __launch_bounds__(256) k_step1(S1Desc<T> d) {
  step1_tile<T>(d, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// step 2 fused with the epilogue.  Block 2x2 waves: 32 final states j x 32
// initial states i; a wave owns 16 j x 16 i x NX branches-of-x tiles.

struct EpiParams {
  int64_t nstates;
  int nbr;
  int n0, n1, n2;            // mesh
  double pref;               // 2 pi / (hbar N_k) / (sqrt(2 pi) sigma)
  double inv2s2;             // 1 / (2 sigma^2)
  double omega_min;
  const int32_t* st_k;       // mesh index of each state
  const double* eps;         // [nstates]
  const double* hw;          // [nk][nbr]
  const cd* Lq;              // [nk][nbr][nbr]
  // temperature dependent (may be null when rates are not wanted)
  const double* lomf;        // [nstates] log(1 - f)
  const double* fstate;      // [nstates] f
  const double* omf;         // [nstates] 1 - f
  const double* nocc;        // [nk][nbr] Bose occupation
  double* we_part;           // [gridDim.x][m_pad]
  double* wph_acc;           // [nk][nbr]
  int64_t m_pad;
  const uint8_t* tile_keep;  // [m_pad/32][m_pad/32] computed tiles (null = all)
  const int32_t* perm;       // [m_pad] state at each tile position (null = identity; the padding maps to itself)
  double cscale;             // undoes the operand scales of the step-2 contraction (1 but in the FP16 form)
  int tetra;                 // 1: store pref |g|^2 without the delta (tetrahedron weights follow)
  const cd* fr;              // [nk][nbr] Froehlich factors F_s(q) of Eq. 7 (null: not polar)
  const cd* ust;             // [nstates][nb] eigenvector of each active state
  int nb;
  // error estimates of the GEMM forms (null: none): per stored term the
  // log-coded relative error of |g|^2 from the contraction's error units:
  // cu times the root-sum-square of its products (b2n: its expected square,
  // per initial state and branch row x) and cv times the magnitude of the
  // component itself (rounding of partial sums that grow with it when the
  // products add coherently, as at q near Gamma)
  uint8_t* rho;              // [nstates][nstates][RhoStride<nbr>]
  const float* b2n;          // [nstates][nbr]
  double cu, cv;
};

// overlap sum_w conj(U_j[w]) U_i[w] of two active states' eigenvectors (the
// [U_k' U_k^+]_{nm} of Eq. 7)
__device__ inline cd state_overlap(const cd* __restrict__ ust, int nb, int64_t i, int64_t j) {
  double orr = 0.0, oi = 0.0;
  for (int w = 0; w < nb; ++w) {
    const cd a = ust[i * nb + w], b = ust[j * nb + w];
    orr += b.x * a.x + b.y * a.y;
    oi += b.x * a.y - b.y * a.x;
  }
  return cmake(orr, oi);
}

__device__ inline int q_of(int kj, int ki, int n0, int n1, int n2) {
  const unsigned uj = (unsigned)kj, ui = (unsigned)ki;
  const unsigned u2 = (unsigned)n2, u1 = (unsigned)n1;
  const unsigned tj = uj / u2, ti = ui / u2;
  int c = (int)(uj - tj * u2) - (int)(ui - ti * u2);
  const unsigned aj = tj / u1, ai = ti / u1;
  int b = (int)(tj - aj * u1) - (int)(ti - ai * u1);
  int a = (int)aj - (int)ai;
  if (a < 0) a += n0;
  if (b < 0) b += n1;
  if (c < 0) c += n2;
  return (a * n1 + b) * n2 + c;
}

// Step-2 contraction of one material with its epilogue parameters.
template <typename T>
struct S2Desc {
  int64_t kp;
  const typename Store<T>::type* Ap;
  const typename Store<T>::type* B2;
  void* Bp;
  void* Bm;
  EpiParams ep;
};

// One 32 x 32 (j, i) tile (block row bx over j, block column by over i).
template <typename T, typename ST, int NX>
__device__ __forceinline__ void step2_tile(const S2Desc<T>& d, int64_t bx, int64_t by, double (*red)[16]) {
  typedef Mfma<T> MM;
  typedef typename MM::acc_t acc_t;
  const int64_t kp = d.kp;
  typedef typename Store<T>::type SE;
  const SE* __restrict__ Ap = d.Ap;
  const SE* __restrict__ B2 = d.B2;
  ST* __restrict__ Bp = (ST*)d.Bp;
  ST* __restrict__ Bm = (ST*)d.Bm;
  const EpiParams& ep = d.ep;
  // tile positions are state indices, or ranks in ep.perm's order
  auto state_at = [&](int64_t pos) -> int64_t { return ep.perm ? (int64_t)ep.perm[pos] : pos; };
  if (ep.tile_keep && !ep.tile_keep[bx * (ep.m_pad / 32) + by]) {
    // screened out: zero vertex-store entries and W_e partials of the tile
    for (int e = threadIdx.x; e < 32 * 32 * NX; e += 256) {
      const int s = e % NX, jj = (e / NX) % 32, ii = e / (NX * 32);
      const int64_t pi = by * 32 + ii, pj = bx * 32 + jj;
      if (pi < ep.nstates && pj < ep.nstates) {
        const int64_t tb = (state_at(pi) * ep.nstates + state_at(pj)) * NX + s;
        Bp[tb] = (ST)0;
        Bm[tb] = (ST)0;
      }
    }
    if (ep.we_part && threadIdx.x < 32 && by * 32 + threadIdx.x < ep.nstates)
      ep.we_part[bx * ep.m_pad + state_at(by * 32 + threadIdx.x)] = 0.0;
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t j0 = bx * 32 + (wave >> 1) * 16;
  const int64_t i0 = by * 32 + (wave & 1) * 16;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t jrow = state_at(j0 + lr), irow = state_at(i0 + lr);  // operand rows of this lane

  acc_t cr[NX], ci[NX];
  double fr[MM::kFold ? NX : 1][4], fi[MM::kFold ? NX : 1][4];
#pragma unroll
  for (int x = 0; x < NX; ++x) {
    cr[x] = MM::zero();
    ci[x] = MM::zero();
  }
  if constexpr (MM::kFold) {
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) fr[x][r] = fi[x][r] = 0.0;
  }
  if constexpr (IsSplit<T>::value) {
    constexpr int NS = IsSplit<T>::ns;
    const SE* pa = Ap + jrow * kp * 2 * NS + lk * 16 * NS;
    const SE* pb = B2 + (irow * NX) * kp * 2 * NS + lk * 16 * NS;
    for (int64_t k0 = 0; k0 < kp; k0 += 32) {
      const int64_t go = (k0 >> 3) * 16 * NS;
      us8v fa[2 * NS], na[NS];
      load_split<NS>(pa + go, fa);
      neg_im<NS>(fa, na);
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        us8v fb[2 * NS];
        load_split<NS>(pb + x * kp * 2 * NS + go, fb);
        split_cmma<T, NS>(fa, na, fb, cr[x], ci[x]);
      }
#pragma unroll
      for (int x = 0; x < NX; ++x) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          fr[x][r] += (double)cr[x][r];
          fi[x][r] += (double)ci[x][r];
        }
        cr[x] = MM::zero();
        ci[x] = MM::zero();
      }
    }
  } else {
    const T* pa = Ap + 2 * (jrow * kp + lk);
    const T* pb = B2 + 2 * ((irow * NX) * kp + lk);
    auto kstep = [&](int64_t k) {
      const Cplx<T> fa = ldc(pa + 2 * k);
      const T nai = -fa.y;
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        const Cplx<T> fb = ldc(pb + 2 * (x * kp + k));
        cr[x] = MM::mma(fa.x, fb.x, cr[x]);
        cr[x] = MM::mma(nai, fb.y, cr[x]);
        ci[x] = MM::mma(fa.x, fb.y, ci[x]);
        ci[x] = MM::mma(fa.y, fb.x, ci[x]);
      }
    };
    if constexpr (!MM::kFold) {
      for (int64_t k = 0; k < kp; k += 4) kstep(k);
    }
    for (int64_t k0 = 0; MM::kFold && k0 < kp; k0 += 16) {
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) kstep(k0 + kk);
      if constexpr (MM::kFold) {
#pragma unroll
        for (int x = 0; x < NX; ++x) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            fr[x][r] += (double)cr[x][r];
            fi[x][r] += (double)ci[x][r];
          }
          cr[x] = MM::zero();
          ci[x] = MM::zero();
        }
      }
    }
  }
  // epilogue: lane owns rows j at positions j0 + MM::row(lk, r), column i at
  // position i0 + lr
  const int64_t i = irow;
  const bool want_rates = ep.we_part != nullptr;
  double we = 0.0;
  if (i0 + lr < ep.nstates) {
    const int64_t ki = ep.st_k[i];
    const double ei = ep.eps[i];
    const double lomf_i = want_rates ? ep.lomf[i] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t pj = j0 + MM::row(lk, r);
      if (pj >= ep.nstates) continue;
      const int64_t j = state_at(pj);
      const int64_t q = q_of(ep.st_k[j], ki, ep.n0, ep.n1, ep.n2);
      const double de = ep.eps[j] - ei;
      const cd* L = ep.Lq + q * NX * NX;
      const double* hwq = ep.hw + q * NX;
      const double rij = want_rates ? exp(ep.lomf[j] - lomf_i) : 0.0;
      const int64_t tb = (i * ep.nstates + j) * NX;
      const cd ov = ep.fr ? state_overlap(ep.ust, ep.nb, i, j) : cmake(0.0, 0.0);
#pragma unroll
      for (int s = 0; s < NX; ++s) {
        double gr = 0.0, gi = 0.0;
#pragma unroll
        for (int x = 0; x < NX; ++x) {
          const cd l = L[x * NX + s];
          double ar, ai;
          if constexpr (MM::kFold) {
            ar = fr[x][r] * ep.cscale;
            ai = fi[x][r] * ep.cscale;
          } else {
            ar = (double)cr[x][r] * ep.cscale;
            ai = (double)ci[x][r] * ep.cscale;
          }
          gr += l.x * ar - l.y * ai;
          gi += l.x * ai + l.y * ar;
        }
        if (ep.fr) {  // Eq. 7: F_s(q) times the overlap
          const cd f = ep.fr[q * NX + s];
          gr += f.x * ov.x - f.y * ov.y;
          gi += f.x * ov.y + f.y * ov.x;
        }
        const double g2 = gr * gr + gi * gi;
        const double w = hwq[s];
        double bp = 0.0, bm = 0.0;
        if (w >= ep.omega_min) {
          if (ep.tetra) {
            bp = bm = ep.pref * g2;
          } else {
            const double dp = de - w, dm = de + w;
            bp = ep.pref * g2 * exp(-dp * dp * ep.inv2s2);
            bm = ep.pref * g2 * exp(-dm * dm * ep.inv2s2);
          }
        }
        Bp[tb + s] = (ST)bp;
        Bm[tb + s] = (ST)bm;
        if (want_rates && w >= ep.omega_min) {
          const double n = ep.nocc[q * NX + s];
          we += (bp * n + bm * (1.0 + n)) * rij;
        }
      }
    }
  }
  if (want_rates) {
    // sum over the 4 lanes sharing column i, then the two waves of this block
    we += __shfl_xor(we, 16, 64);
    we += __shfl_xor(we, 32, 64);
    if (lk == 0) red[wave][lr] = we;
    __syncthreads();
    if (wave < 2 && lk == 0) {
      const double tot = red[wave][lr] + red[wave + 2][lr];
      if (i0 + lr < ep.nstates) ep.we_part[bx * ep.m_pad + i] = tot;
    }
  }
}

template <typename T, typename ST, int NX>
__global__ void __launch_bounds__(256) k_step2(S2Desc<T> d) {
  __shared__ double red[4][16];
  step2_tile<T, ST, NX>(d, blockIdx.x, blockIdx.y, red);
}

// W_e[i] = sum over j-tiles of the partials, in tile order
__global__ void k_reduce_we(const double* __restrict__ part, int64_t ntiles, int64_t m_pad, int64_t nstates,
                            double* __restrict__ we) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nstates) return;
  double s = 0.0;
  for (int64_t t = 0; t < ntiles; ++t) s += part[t * m_pad + i];
  we[i] = s;
}

// ---------------------------------------------------------------------------
// The contractions of the BF16 and FP32 forms as plain complex GEMMs plus
// separate epilogues:
//   C[c][j] = sum_k A[c][k] B[j][k]
// (step 2: A = B2 with c = i*NX + x, B = A_p; step 1: A = A_e, B = gR).  All
// 32 x 32 MFMAs used here share one accumulator layout: register r of lane l
// holds row 8(r/4) + 4(l/32) + r%4, column l%32.  A block computes 32*WR
// rows c x 64 columns j (WR x 2 wavefronts of 32 x 32); each 32-k stage of
// both operands is staged in LDS (rows padded by 16 bytes so the fragment
// reads do not collide in banks).  C is FP32 complex.

typedef float f16v __attribute__((ext_vector_type(16)));
// plain vector type for the staged 16-byte chunks (not the HIP struct), so
// the copies stay in registers
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool F16>
__device__ inline f16v mma32(us8v a, us8v b, f16v c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0, 0,
                                                  0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0,
                                                   0);
}

// One 16-k slice of the complex product on a 32 x 32 tile: the real part's
// two terms go to separate accumulators (cr += a_re b_re, cn += a_im b_im,
// subtracted when folded), so no operand needs negating.
template <int NS, bool F16>
__device__ inline void split_cmma32(const us8v (&a)[2 * NS], const us8v (&b)[2 * NS], f16v& cr, f16v& cn,
                                    f16v& ci) {
  constexpr int np = NS == 2 ? 3 : 6;
#pragma unroll
  for (int t = 0; t < np; ++t) {
    int sa, sb;
    if (NS == 2) {
      sa = t == 1 ? 1 : 0;
      sb = t == 0 ? 1 : 0;
    } else {
      sa = t == 0 ? 1 : t == 2 ? 2 : t == 4 ? 1 : 0;
      sb = t == 0 ? 1 : t == 1 ? 2 : t == 3 ? 1 : 0;
    }
    cr = mma32<F16>(a[2 * sa], b[2 * sb], cr);
    cn = mma32<F16>(a[2 * sa + 1], b[2 * sb + 1], cn);
    ci = mma32<F16>(a[2 * sa], b[2 * sb + 1], ci);
    ci = mma32<F16>(a[2 * sa + 1], b[2 * sb], ci);
  }
}

// Operand formats, in 16-bit words per 32-k stage of a row (kRowU).
// OpSplit<NS, F16>: BF16 (or FP16) planes (groups of 8 k, each holding re/im
// of the NS parts), 32x32x16 BF16 (FP16) MFMA; lanes 0-31 take the first 8 k
// of each 16, lanes 32-63 the next 8.
template <int NS, bool F16 = false>
struct OpSplit {
  static constexpr int kRowU = 64 * NS;
  __device__ static inline void mac(const unsigned short* arow, const unsigned short* brow, int lh, f16v& cr,
                                    f16v& cn, f16v& ci) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      const int gofs = (2 * kh + lh) * 16 * NS;  // group 2kh + lh of the stage
      us8v a[2 * NS], b[2 * NS];
#pragma unroll
      for (int p = 0; p < 2 * NS; ++p) {
        a[p] = *reinterpret_cast<const us8v*>(arow + gofs + 8 * p);
        b[p] = *reinterpret_cast<const us8v*>(brow + gofs + 8 * p);
      }
      split_cmma32<NS, F16>(a, b, cr, cn, ci);
    }
  }
};

// OpF32: complex FP32 interleaved (re, im per k), 32x32x2 FP32 MFMA.  The
// stage's 32 k are split as k = 16 (l/32) + s over the MFMA's two k slots
// and its 16 steps s, so each lane reads 16 consecutive complex values of
// its row with 16-byte loads.
struct OpF32 {
  static constexpr int kRowU = 128;
  __device__ static inline void mac(const unsigned short* arow, const unsigned short* brow, int lh, f16v& cr,
                                    f16v& cn, f16v& ci) {
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const int off = lh * 64 + s2 * 8;  // two k of the lane's 16
      const float4 a = *reinterpret_cast<const float4*>(arow + off);
      const float4 b = *reinterpret_cast<const float4*>(brow + off);
      cr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, cr, 0, 0, 0);
      cn = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, cn, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, cr, 0, 0, 0);
      cn = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, cn, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.w, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.z, ci, 0, 0, 0);
    }
  }
};

// Block order: the 8 XCDs take workgroups round-robin (id % 8) and each runs
// 32 blocks at a time (one per CU), so blocks 8s + x with s in [32u, 32u+32)
// run together on XCD x.  Each such set of 32 is one group of kGY x kGX
// neighbouring blocks (4 row tiles x 8 column tiles, 512 x 512 outputs), so a
// staged slice of a row or column tile is fetched into that XCD's L2 once and
// read by 8 or 4 blocks.  Groups are numbered column-fastest over the block
// grid and dealt to the XCDs in turn.
constexpr int kGY = 4, kGX = 8;

struct GemmGrid {
  int32_t ny, nx;    // row and column tiles
  int32_t ngx, ng;   // groups per group row, groups
  int64_t blocks;    // workgroups launched (whole groups on every XCD)
};

inline GemmGrid gemm_grid(int64_t rows, int64_t cols, int rows_per_block) {
  GemmGrid g;
  g.ny = (int32_t)((rows + rows_per_block - 1) / rows_per_block);
  g.nx = (int32_t)((cols + 63) / 64);
  g.ngx = (g.nx + kGX - 1) / kGX;
  g.ng = ((g.ny + kGY - 1) / kGY) * g.ngx;
  g.blocks = (int64_t)((g.ng + 7) / 8) * 8 * (kGY * kGX);
  return g;
}

// One GEMM: rows c in [c0, c0 + nc) (c0 a multiple of nx) of A, all j < nj;
// C is stored as [(c - c0) / nx][j][(c - c0) % nx] with j stride nx
// (ldc >= nj).  K is a multiple of 32.
struct GemmArgs {
  int64_t c0, nc, nj, K;
  int nx;
  const unsigned short* A;
  const unsigned short* B;
  float* C;
  int64_t ldc;
};

template <class OP, int WR>
struct GemmLds {
  static constexpr int kLdsRow = OP::kRowU + 8;  // padded LDS row
  static constexpr int LA = 32 * WR * kLdsRow, LB = 64 * kLdsRow;
  unsigned short As[2 * LA];
  unsigned short Bs[2 * LB];
};

// Block (ty, tx) of one GEMM with 128*WR threads.  Two LDS buffers: stage
// s + 1 is loaded into registers while stage s is multiplied from one
// buffer, then stored into the other, with one barrier per stage; the FP32
// accumulators fold into FP64 after every stage.
template <class OP, int WR>
__device__ __forceinline__ void cgemm_block(const GemmArgs& g, int64_t ty, int64_t tx, GemmLds<OP, WR>& L) {
  constexpr int NT = 128 * WR, RA = 32 * WR;
  constexpr int kLdsRow = GemmLds<OP, WR>::kLdsRow, LA = GemmLds<OP, WR>::LA, LB = GemmLds<OP, WR>::LB;
  constexpr int kChunks = OP::kRowU / 8;              // 16-byte chunks per row and stage
  unsigned short* As = L.As;
  unsigned short* Bs = L.Bs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t cb = g.c0 + ty * RA;                  // first row c of the block
  const int64_t jb = tx * 64;                         // first column j
  const int64_t rowlen = g.K / 32 * OP::kRowU;        // 16-bit words per operand row
  const int nst = (int)(g.K / 32);
  constexpr int PA = RA * kChunks / NT;               // 16-byte chunks per thread, A tile
  constexpr int PB = 64 * kChunks / NT;               // and B tile
  static_assert(PA * NT == RA * kChunks && PB * NT == 64 * kChunks, "tile split");
  u32x4 ra[PA], rb[PB];
  // Loads are unconditional: rows past the end and stages past the last are
  // clamped to valid ones.  A clamped row only feeds outputs (c, j) outside
  // the result, which are never stored, and a clamped stage is never used.
  const int64_t clast = g.c0 + g.nc - 1, jlast = g.nj - 1;
  const unsigned short* __restrict__ Am = g.A;
  const unsigned short* __restrict__ Bm = g.B;
  auto fetch = [&](int s) {
    const int64_t so = (int64_t)(s < nst ? s : nst - 1) * OP::kRowU;
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int e = tid + NT * u;
      const int row = e / kChunks, w = e - row * kChunks;
      const int64_t ca = cb + row < clast ? cb + row : clast;
      ra[u] = *reinterpret_cast<const u32x4*>(Am + ca * rowlen + so + w * 8);
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + NT * u;
      const int row = e / kChunks, w = e - row * kChunks;
      const int64_t jr = jb + row < jlast ? jb + row : jlast;
      rb[u] = *reinterpret_cast<const u32x4*>(Bm + jr * rowlen + so + w * 8);
    }
  };
  auto stash = [&](unsigned short* as, unsigned short* bs) {
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int e = tid + NT * u;
      const int row = e / kChunks, w = e - row * kChunks;
      *reinterpret_cast<u32x4*>(as + row * kLdsRow + w * 8) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + NT * u;
      const int row = e / kChunks, w = e - row * kChunks;
      *reinterpret_cast<u32x4*>(bs + row * kLdsRow + w * 8) = rb[u];
    }
  };
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 31, lh = lane >> 5;
  f16v cr, cn, ci;
  double fr[16], fi[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    cr[r] = cn[r] = ci[r] = 0.f;
    fr[r] = fi[r] = 0.0;
  }
  auto compute = [&](const unsigned short* as, const unsigned short* bs) {
    OP::mac(as + (wm + lr) * kLdsRow, bs + (wn + lr) * kLdsRow, lh, cr, cn, ci);
  };
  // FP32 partial sums of one stage (32 k) into FP64
  auto fold = [&]() {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      fr[r] += (double)(cr[r] - cn[r]);
      fi[r] += (double)ci[r];
      cr[r] = cn[r] = ci[r] = 0.f;
    }
  };
  fetch(0);
  stash(As, Bs);
  __syncthreads();
  for (int s = 0; s < nst; s += 2) {
    // even stage s from buffer 0; stage s + 1 into buffer 1 (the scheduling
    // barriers keep the loads issued ahead of the multiplies they overlap)
    fetch(s + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(As, Bs);
    fold();
    stash(As + LA, Bs + LB);   // past the last stage: unused
    __syncthreads();
    if (s + 1 >= nst) break;
    // odd stage s + 1 from buffer 1; stage s + 2 into buffer 0
    fetch(s + 2);
    __builtin_amdgcn_sched_barrier(0);
    compute(As + LA, Bs + LB);
    fold();
    stash(As, Bs);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t c = cb + wm + 8 * (r >> 2) + 4 * lh + (r & 3);
    const int64_t j = jb + wn + lr;
    if (c <= clast && j <= jlast) {
      const int64_t il = (c - g.c0) / g.nx, x = (c - g.c0) - il * g.nx;
      *reinterpret_cast<float2*>(g.C + 2 * ((il * g.ldc + j) * g.nx + x)) =
          make_float2((float)fr[r], (float)fi[r]);
    }
  }
}

// One GEMM over the XCD-grouped block order.  STEP (1 or 2) only names the
// instance, so profiles tell the two steps apart.
template <class OP, int STEP, int WR>
__global__ void __launch_bounds__(128 * WR) k_cgemm(GemmArgs g, GemmGrid gg) {
  __shared__ __attribute__((aligned(16))) GemmLds<OP, WR> L;
  // block -> (row tile, column tile), uniform over the block
  const int32_t bid = (int32_t)blockIdx.x, slot = bid >> 3;
  const int32_t grp = (slot / (kGY * kGX)) * 8 + (bid & 7), pos = slot % (kGY * kGX);
  if (grp >= gg.ng) return;
  const int32_t ty = (grp / gg.ngx) * kGY + pos / kGX, tx = (grp % gg.ngx) * kGX + pos % kGX;
  if (ty >= gg.ny || tx >= gg.nx) return;
  cgemm_block<OP, WR>(g, ty, tx, L);
}

// Many GEMMs (one per material) in one persistent launch over a queue of
// (GEMM, row tile, column tile) items; every block ends when the queue is
// empty.  Each output block is computed exactly as by k_cgemm.
__device__ inline GemmArgs promoted(const GemmArgs& in);

template <class OP, int STEP, int WR>
__global__ void __launch_bounds__(128 * WR) k_cgemm_persist(const GemmArgs* __restrict__ args,
                                                            const int4* __restrict__ items, int nitems,
                                                            int* counter) {
  __shared__ __attribute__((aligned(16))) GemmLds<OP, WR> L;
  __shared__ int item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    if (it >= nitems) break;  // uniform over the block; every block reaches it
    const int4 w = items[it];
    cgemm_block<OP, WR>(promoted(args[w.x]), w.y, w.z, L);
    __syncthreads();          // the LDS buffers are reused by the next item
  }
}

// rows per block of the GEMMs (WR = 4: 128 rows)
constexpr int kGemmWR = 4;

template <class OP, int STEP>
static void launch_cgemm(hipStream_t s, int64_t c0, int64_t nc, int64_t nj, int64_t K, int nx, const void* A,
                         const void* B, float* C, int64_t ldc) {
  if (nc <= 0 || nj <= 0) return;
  const GemmGrid gg = gemm_grid(nc, nj, 32 * kGemmWR);
  GemmArgs g{c0, nc, nj, K, nx, (const unsigned short*)A, (const unsigned short*)B, C, ldc};
  hipLaunchKernelGGL((k_cgemm<OP, STEP, kGemmWR>), dim3((unsigned)gg.blocks), dim3(128 * kGemmWR), 0, s, g, gg);
}

// operand format of a form
template <typename T>
struct GemmOp;
template <int NS>
struct GemmOp<Bf16S<NS>> {
  typedef OpSplit<NS> type;
};
template <int NS>
struct GemmOp<F16S<NS>> {
  typedef OpSplit<NS, true> type;
};
template <>
struct GemmOp<float> {
  typedef OpF32 type;
};

// Epilogue of the split path, one wavefront per q: the phonon factors of q
// (l u, hbar omega) are wavefront-uniform; lanes take the kept pairs
// (k_t, k_t + q) of q's list with t in [t0, t1) (the chunk's initial
// states) and write g_s = sum_x l u gh_x, |g|^2 and the Gaussians into the
// store B+/-.
// One pair (i, j) of the GEMM forms' step-2 epilogue: cg is the pair's C
// row (NX complex FP32 values), L and hwq the q's l.u matrix and phonon
// energies; writes the pair's rows of B+ and B- (and its error codes).
template <typename ST, int NX>
__device__ __forceinline__ void epi_pair(int64_t i, int64_t j, int64_t q, double ei, const EpiParams& ep,
                                         const cd* __restrict__ L, const double* __restrict__ hwq,
                                         const float* __restrict__ cg, ST* __restrict__ Bp,
                                         ST* __restrict__ Bm) {
  const double de = ep.eps[j] - ei;
  const int64_t tb = ((int64_t)i * ep.nstates + j) * NX;
  const cd ov = ep.fr ? state_overlap(ep.ust, ep.nb, i, j) : cmake(0.0, 0.0);
  // g_s = sum_x l_xs gh_x with x outermost: one component of the C
  // row and one row of the q's l.u matrix live at a time (the sums
  // over x still run in x order), so the branch count does not
  // multiply the live registers; with error codes the weighted
  // squares d2_s = sum_x |l_xs|^2 e2_x go along
  double gr[NX], gi[NX];
  float d2[NX];
#pragma unroll
  for (int s = 0; s < NX; ++s) {
    gr[s] = gi[s] = 0.0;
    d2[s] = 0.f;
  }
  const float* __restrict__ bn = ep.rho ? ep.b2n + (int64_t)i * NX : nullptr;
  const float cu2 = (float)(ep.cu * ep.cu), cv2 = (float)(ep.cv * ep.cv);
#pragma unroll 1
  for (int x = 0; x < NX; ++x) {
    const float2 v = *reinterpret_cast<const float2*>(cg + 2 * x);
    const double ar = (double)v.x * ep.cscale, ai = (double)v.y * ep.cscale;
    const cd* __restrict__ Lx = L + x * NX;
#pragma unroll
    for (int s = 0; s < NX; ++s) {
      const cd l = Lx[s];
      gr[s] += l.x * ar - l.y * ai;
      gi[s] += l.x * ai + l.y * ar;
    }
    if (bn) {
      // b2n[i][x]: the expected square root-sum-square of the products
      // behind gh_x; a vertex component carries an error of about
      // cu rss[x] + cv |gh_x|, the projection sum_x l u gh_x the
      // root-sum-square of those weighted by |l u|
      const float e2 = cu2 * bn[x] + cv2 * (float)(ar * ar + ai * ai);
#pragma unroll
      for (int s = 0; s < NX; ++s) d2[s] += (float)cabs2(Lx[s]) * e2;
    }
  }
  double bpv[NX], bmv[NX];
  constexpr int RS = RhoStride<NX>::value;
  uint32_t w[RS / 4];
#pragma unroll
  for (int t = 0; t < RS / 4; ++t) w[t] = 0u;
#pragma unroll
  for (int s = 0; s < NX; ++s) {
    double g_r = gr[s], g_i = gi[s];
    if (ep.fr) {  // Eq. 7: F_s(q) times the overlap
      const cd f = ep.fr[q * NX + s];
      g_r += f.x * ov.x - f.y * ov.y;
      g_i += f.x * ov.y + f.y * ov.x;
    }
    const double g2 = g_r * g_r + g_i * g_i;
    const double wq = hwq[s];
    double bp = 0.0, bm = 0.0;
    if (wq >= ep.omega_min) {
      if (ep.tetra) {
        bp = bm = ep.pref * g2;
      } else {
        const double dp = de - wq, dm = de + wq;
        bp = ep.pref * g2 * exp(-dp * dp * ep.inv2s2);
        bm = ep.pref * g2 * exp(-dm * dm * ep.inv2s2);
      }
    }
    bpv[s] = bp;
    bmv[s] = bm;
    if (bn) w[s >> 2] |= rho_encode(d2[s], (float)g2) << (8 * (s & 3));
  }
  store_row<ST, NX>(Bp + tb, bpv);
  store_row<ST, NX>(Bm + tb, bmv);
  if (bn) {
    uint8_t* __restrict__ rp = ep.rho + ((int64_t)i * ep.nstates + j) * RS;
    if constexpr (RS == 8) {
      *reinterpret_cast<uint2*>(rp) = make_uint2(w[0], w[1]);
    } else {
      *reinterpret_cast<uint4*>(rp) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
}

template <typename ST, int NX>
__device__ __forceinline__ void epi_q_wave(int64_t q, const EpiParams& ep, const int32_t* __restrict__ poff,
                                           const uint64_t* __restrict__ ppk, const float* __restrict__ C,
                                           int64_t ldc, ST* __restrict__ Bp, ST* __restrict__ Bm) {
  const int lane = threadIdx.x & 63;
  const cd* __restrict__ L = ep.Lq + q * NX * NX;
  const double* __restrict__ hwq = ep.hw + q * NX;
  const int32_t pe = poff[q + 1];
  for (int32_t p = poff[q] + lane; p < pe; p += 64) {
    // the pair's state ranges: first state and count of k and of k + q
    const uint64_t w = ppk[p];
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    const int32_t ib = (int32_t)(lo & 0x3ffffffu), ie = ib + (int32_t)(lo >> 26) + 1;
    const int32_t jb = (int32_t)(hi & 0x3ffffffu), je = jb + (int32_t)(hi >> 26) + 1;
    for (int32_t i = ib; i < ie; ++i) {
      const double ei = ep.eps[i];
      for (int32_t j = jb; j < je; ++j) {
        epi_pair<ST, NX>(i, j, q, ei, ep, L, hwq, C + 2 * (((int64_t)i * ldc + j) * NX), Bp, Bm);
      }
    }
  }
}

// The same epilogue row by row: one block per initial state i of the chunk
// [i0, i0 + ni), its threads over final states j (256 at a time, their q
// indices formed once into LDS), so that the C row, the B+- rows and the
// error codes are read and written along j; each pair gathers its q's l.u
// matrix instead.  Blocks are numbered so that each XCD takes a contiguous
// range of states (neighbouring k: overlapping q, shared in its L2).
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_epi_rows(int64_t i0, int64_t ni, int64_t per_xcd, EpiParams ep,
                                                  const float* __restrict__ C, int64_t ldc, ST* __restrict__ Bp,
                                                  ST* __restrict__ Bm) {
  __shared__ int sq[256];
  const int64_t il = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (il >= ni) return;  // whole block
  const int64_t i = i0 + il, M = ep.nstates;
  const int ki = ep.st_k[i];
  const double ei = ep.eps[i];
  for (int64_t j0 = 0; j0 < M; j0 += 256) {
    const int nj = (int)(M - j0 < 256 ? M - j0 : 256);
    __syncthreads();  // the previous chunk is consumed
    if ((int)threadIdx.x < nj) sq[threadIdx.x] = q_of(ep.st_k[j0 + threadIdx.x], ki, ep.n0, ep.n1, ep.n2);
    __syncthreads();
    if ((int)threadIdx.x < nj) {
      const int64_t j = j0 + threadIdx.x, q = sq[threadIdx.x];
      epi_pair<ST, NX>(i, j, q, ei, ep, ep.Lq + q * NX * NX, ep.hw + q * NX, C + 2 * ((il * ldc + j) * NX), Bp,
                       Bm);
    }
  }
}

// Step-1 epilogue of the GEMM path: B2[(i, x)][(Rp, n')] = C1[i][col] e^{-2 pi i k_i.Rp}
// written in the form's operand format; col = (x, Rp, n'), rows [i0, i0 + ni).
template <typename T>
__device__ __forceinline__ void step1_epi_elem(int64_t e, int64_t i0, int64_t ncol, int nrp, int nb, int nbr,
                                               int64_t kp, const float* __restrict__ C1,
                                               const int32_t* __restrict__ st_kidx, const cd* __restrict__ Ep,
                                               double scale, typename Store<T>::type* __restrict__ B2) {
  const int64_t il = e / ncol, col = e - il * ncol;
  const int64_t i = i0 + il;
  const int64_t per_x = (int64_t)nrp * nb;
  const int x = (int)(col / per_x);
  const int64_t rem = col - x * per_x;
  const int rp = (int)(rem / nb);
  const float2 v = *reinterpret_cast<const float2*>(C1 + 2 * e);
  const cd z = cmulc(cmake(v.x, v.y), Ep[(int64_t)st_kidx[i] * nrp + rp]);  // * conj(phase)
  PutC<T>::put(B2, i * nbr + x, kp, rem, z.x * scale, z.y * scale);
}

template <typename T>
__global__ void k_step1_epi(int64_t i0, int64_t ni, int64_t ncol, int nrp, int nb, int nbr, int64_t kp,
                            const float* __restrict__ C1, const int32_t* __restrict__ st_kidx,
                            const cd* __restrict__ Ep, double scale, typename Store<T>::type* __restrict__ B2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ni * ncol) return;
  step1_epi_elem<T>(e, i0, ncol, nrp, nb, nbr, kp, C1, st_kidx, Ep, scale, B2);
}

// ---------------------------------------------------------------------------
// persistent launches over a work queue of (material, tile) items

__global__ void k_zero_ints(int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Descriptors are read from memory here, so the compiler cannot see that
// their pointers address global memory and would access through them with
// flat instructions; re-deriving each pointer from a global-address-space
// pointer lets every access compile to global loads and stores, as in the
// single-material kernels whose descriptors are kernel arguments.
template <typename P>
__device__ inline P* as_global(P* p) {
  typedef __attribute__((address_space(1))) P GP;
  return (P*)(GP*)(uintptr_t)p;
}

__device__ inline void promote(EpiParams& e) {
  e.st_k = as_global(e.st_k);
  e.eps = as_global(e.eps);
  e.hw = as_global(e.hw);
  e.Lq = as_global(e.Lq);
  e.lomf = as_global(e.lomf);
  e.fstate = as_global(e.fstate);
  e.omf = as_global(e.omf);
  e.nocc = as_global(e.nocc);
  e.we_part = as_global(e.we_part);
  e.wph_acc = as_global(e.wph_acc);
  e.tile_keep = as_global(e.tile_keep);
  e.perm = as_global(e.perm);
}

template <typename T>
__device__ inline S1Desc<T> promoted(const S1Desc<T>& in) {
  S1Desc<T> d = in;
  d.Ae = as_global(d.Ae);
  d.gR = as_global(d.gR);
  d.B2 = as_global(d.B2);
  d.st_kidx = as_global(d.st_kidx);
  d.Ep = as_global(d.Ep);
  return d;
}

__device__ inline GemmArgs promoted(const GemmArgs& in) {
  GemmArgs g = in;
  g.A = as_global(g.A);
  g.B = as_global(g.B);
  g.C = as_global(g.C);
  return g;
}

template <typename T>
__device__ inline S2Desc<T> promoted(const S2Desc<T>& in) {
  S2Desc<T> d = in;
  d.Ap = as_global(d.Ap);
  d.B2 = as_global(d.B2);
  d.Bp = as_global(d.Bp);
  d.Bm = as_global(d.Bm);
  promote(d.ep);
  return d;
}

template <typename T>
__global__ void __launch_bounds__(256) k_step1_persist(const S1Desc<T>* __restrict__ descs,
                                                       const int4* __restrict__ items, int nitems, int* counter) {
  __shared__ int item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    if (it >= nitems) break;  // uniform over the block; every block reaches it
    const int4 w = items[it];
    step1_tile<T>(promoted(descs[w.x]), w.y, w.z);
  }
}

template <typename T, typename ST, int NX>
__global__ void __launch_bounds__(256) k_step2_persist(const S2Desc<T>* __restrict__ descs,
                                                       const int4* __restrict__ items, int nitems, int* counter) {
  __shared__ double red[4][16];
  __shared__ int item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    if (it >= nitems) break;
    const int4 w = items[it];
    step2_tile<T, ST, NX>(promoted(descs[w.x]), w.y, w.z, red);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host side

template <typename T>
static elph_status build_operands_t(elph_ctx ctx) {
  hipStream_t s = ctx->stream;
  const int64_t M = ctx->nstates;
  const int nb = ctx->nb, nbr = ctx->nbr;
  typedef typename Store<T>::type SE;
  constexpr int64_t al = Store<T>::kalign;
  ctx->m_pad = (M + 63) / 64 * 64;
  ctx->ke = ((int64_t)ctx->nre * nb + al - 1) / al * al;
  ctx->kp = ((int64_t)ctx->nrp * nb + al - 1) / al * al;
  const int64_t ncol = (int64_t)nbr * ctx->nrp * nb;
  const size_t esz = Store<T>::per_c * sizeof(SE);
  size_t bytes_ae = (size_t)ctx->m_pad * ctx->ke * esz;
  size_t bytes_ap = (size_t)ctx->m_pad * ctx->kp * esz;
  size_t bytes_gr = (size_t)ncol * ctx->ke * esz;
  size_t bytes_b2 = (size_t)ctx->m_pad * nbr * ctx->kp * esz;
  void *ae, *ap, *gr, *b2;
  if (dev_alloc(ctx, &ae, bytes_ae) != hipSuccess || dev_alloc(ctx, &ap, bytes_ap) != hipSuccess ||
      dev_alloc(ctx, &gr, bytes_gr) != hipSuccess || dev_alloc(ctx, &b2, bytes_b2) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "device allocation of the contraction operands failed";
    return ELPH_ENOMEM;
  }
  ctx->d_Ae = ae;
  ctx->d_Ap = ap;
  ctx->d_gR = gr;
  ctx->d_B2 = b2;
  if (hipMemsetAsync(ae, 0, bytes_ae, s) != hipSuccess || hipMemsetAsync(ap, 0, bytes_ap, s) != hipSuccess ||
      hipMemsetAsync(gr, 0, bytes_gr, s) != hipSuccess || hipMemsetAsync(b2, 0, bytes_b2, s) != hipSuccess) {
    ctx->err = "hipMemsetAsync failed";
    ctx->hip_dead = true;
    return ELPH_EHIP;
  }
  hipLaunchKernelGGL(k_build_Ae<T>, dim3(blocks_for(M * ctx->nre * nb, 256)), dim3(256), 0, s, M, nb, ctx->nre,
                     ctx->ke, ctx->d_state_kidx, ctx->d_state_m, (const cd*)ctx->d_Ee, (const cd*)ctx->d_U,
                     ctx->sc_ae, (SE*)ae);
  hipLaunchKernelGGL(k_build_Ap<T>, dim3(blocks_for(M * ctx->nrp * nb, 256)), dim3(256), 0, s, M, nb, ctx->nrp,
                     ctx->kp, ctx->d_state_kidx, ctx->d_state_m, (const cd*)ctx->d_Ep, ctx->d_wrp,
                     (const cd*)ctx->d_U, ctx->sc_ap, (SE*)ap);
  const int64_t gtotal = (int64_t)ctx->nre * ctx->nrp * nbr * nb * nb;
  hipLaunchKernelGGL(k_permute_g<T>, dim3(blocks_for(gtotal, 256)), dim3(256), 0, s, ctx->nre, ctx->nrp, nbr, nb,
                     ctx->ke, ctx->d_gr, ctx->sc_g, (SE*)gr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = std::string("kernel launch failed: ") + hipGetErrorString(e);
    ctx->hip_dead = true;
    return ELPH_EHIP;
  }
  ctx->operands_ready = true;
  return ELPH_OK;
}

elph_status build_operands(elph_ctx ctx) {
  if (ctx->operands_ready) return ELPH_OK;
  if (ctx->precision == ELPH_FP64) return build_operands_t<double>(ctx);
  if (ctx->precision == ELPH_FP32) return build_operands_t<float>(ctx);
  if (ctx->precision == ELPH_BF16X3) return build_operands_t<Bf16S<2>>(ctx);
  if (ctx->precision == ELPH_BF16X6) return build_operands_t<Bf16S<3>>(ctx);
  if (ctx->precision == ELPH_FP16X3) return build_operands_t<F16S<2>>(ctx);
  ctx->err = "precision form not available";
  return ELPH_EINVAL;
}

template <typename T>
S1Desc<T> step1_desc(elph_ctx ctx) {
  S1Desc<T> d;
  d.m_pad = ctx->m_pad;
  d.ncol = (int64_t)ctx->nbr * ctx->nrp * ctx->nb;
  d.ke = ctx->ke;
  d.kp = ctx->kp;
  d.nstates = ctx->nstates;
  d.Ae = (const typename Store<T>::type*)ctx->d_Ae;
  d.gR = (const typename Store<T>::type*)ctx->d_gR;
  d.B2 = (typename Store<T>::type*)ctx->d_B2;
  d.nrp = ctx->nrp;
  d.nb = ctx->nb;
  d.nbr = ctx->nbr;
  d.st_kidx = ctx->d_state_kidx;
  d.Ep = (const cd*)ctx->d_Ep;
  return d;
}

// forms whose contractions run as GEMMs plus separate epilogues
template <typename T>
struct UsesGemm {
  static constexpr bool value = IsSplit<T>::value || std::is_same<T, float>::value;
};

template <typename T>
static elph_status launch_step1_t(elph_ctx ctx, bool norms = false) {
  const S1Desc<T> d = step1_desc<T>(ctx);
  if constexpr (UsesGemm<T>::value) {
    // GEMM into FP32 rows (chunks of at most gemm_chunk bytes, 2 GiB by
    // default), then the phase epilogue that writes B2 in the form's operand
    // format
    typedef typename GemmOp<T>::type OP;
    const int64_t M = ctx->nstates, ncol = d.ncol;
    int64_t ci = (int64_t)ctx->gemm_chunk / (ncol * 8);
    if (ci < 1) ci = 1;
    if (ci > M) ci = M;
    void* p = nullptr;
    if (dev_alloc(ctx, &p, (size_t)ci * ncol * 8) != hipSuccess) {
      (void)hipGetLastError();
      ctx->err = "device allocation of the step-1 buffer failed";
      return ELPH_ENOMEM;
    }
    for (int64_t i0 = 0; i0 < M; i0 += ci) {
      const int64_t ni = (M - i0 < ci) ? M - i0 : ci;
      launch_cgemm<OP, 1>(ctx->stream, i0, ni, ncol, ctx->ke, 1, ctx->d_Ae, ctx->d_gR, (float*)p, ncol);
      if (norms) refine_b2_norms(ctx, i0, ni, (const float*)p);
      hipLaunchKernelGGL(k_step1_epi<T>, dim3(blocks_for(ni * ncol, 256)), dim3(256), 0, ctx->stream, i0, ni, ncol,
                         ctx->nrp, ctx->nb, ctx->nbr, ctx->kp, (const float*)p, ctx->d_state_kidx,
                         (const cd*)ctx->d_Ep, ctx->sc_b2 / (ctx->sc_ae * ctx->sc_g),
                         (typename Store<T>::type*)ctx->d_B2);
    }
    dev_free(ctx, p);
    return ELPH_OK;
  }
  dim3 grid((unsigned)((d.ncol + 63) / 64), (unsigned)(ctx->m_pad / 64));
  hipLaunchKernelGGL(k_step1<T>, grid, dim3(256), 0, ctx->stream, d);
  return ELPH_OK;
}

template <typename T, typename ST, int NX>
static void launch_step2_nx(elph_ctx ctx, const EpiParams& ep, void* Bp, void* Bm) {
  S2Desc<T> d;
  d.kp = ctx->kp;
  d.Ap = (const typename Store<T>::type*)ctx->d_Ap;
  d.B2 = (const typename Store<T>::type*)ctx->d_B2;
  d.Bp = Bp;
  d.Bm = Bm;
  d.ep = ep;
  dim3 grid((unsigned)(ctx->m_pad / 32), (unsigned)(ctx->m_pad / 32));
  hipLaunchKernelGGL((k_step2<T, ST, NX>), grid, dim3(256), 0, ctx->stream, d);
}

// GEMM forms without a tile mask: GEMM into an FP32 buffer [i][j][x], then
// the per-q epilogue over the kept pairs, in chunks of initial states (whole
// kept k) so that the buffer stays within gemm_chunk bytes (2 GiB by
// default; at least 16 states); W_e from the finished store.
template <typename T, typename ST, int NX>
static elph_status launch_gemm_nx(elph_ctx ctx, const EpiParams& ep, void* Bp, void* Bm, int64_t* we_tiles) {
  typedef typename GemmOp<T>::type OP;
  const int64_t M = ctx->nstates, ldc = ctx->m_pad;
  elph_status st = ensure_pairs(ctx);
  if (st != ELPH_OK) return st;
  int64_t cap = (int64_t)ctx->gemm_chunk / ((int64_t)NX * ldc * 8);
  if (cap < kMaxBands) cap = kMaxBands;
  std::vector<int32_t> soff(ctx->nkept + 1);
  if (hipMemcpyAsync(soff.data(), ctx->d_soff, (ctx->nkept + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                     ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->err = "copy of the state offsets failed";
    ctx->hip_dead = true;
    return ELPH_EHIP;
  }
  void* p = nullptr;
  if (dev_alloc(ctx, &p, (size_t)std::min<int64_t>(cap, M) * NX * ldc * 8) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "device allocation of the step-2 buffer failed";
    return ELPH_ENOMEM;
  }
  float* C = (float*)p;
  // at most three epilogue rows per CU: their l.u gathers share the L2
  // better than four (1.40 ms against 1.45 for 3318 states, 6 branches)
  const size_t epad = lds_pad_for(3, 256 * 4);
  mark(ctx, 4);  // the step-2 window starts at the contraction (pair lists are built above)
  for (int32_t t0 = 0; t0 < ctx->nkept;) {
    // whole kept k per chunk
    int32_t t1 = t0 + 1;
    while (t1 < ctx->nkept && soff[t1 + 1] - soff[t0] <= cap) ++t1;
    const int64_t i0 = soff[t0], ni = soff[t1] - soff[t0];
    const int64_t c0 = i0 * NX, nc = ni * NX;
    launch_cgemm<OP, 2>(ctx->stream, c0, nc, M, ctx->kp, NX, ctx->d_B2, ctx->d_Ap, C, ldc);
    if (t1 == ctx->nkept) mark(ctx, 5);  // step-2 window: the contraction (and earlier chunks' epilogues)
    const int64_t per_xcd = (ni + 7) / 8;
    hipLaunchKernelGGL((k_epi_rows<ST, NX>), dim3((unsigned)(8 * per_xcd)), dim3(256), epad, ctx->stream, i0, ni,
                       per_xcd, ep, (const float*)C, ldc, (ST*)Bp, (ST*)Bm);
    t0 = t1;
  }
  dev_free(ctx, C);
  if (ep.we_part) {
    // W_e into the first partial row; the caller's reduction copies it out
    launch_we_rows<ST>(ctx, (const ST*)Bp, (const ST*)Bm, ep.lomf, ep.nocc, ep.we_part);
    *we_tiles = 1;
  }
  return ELPH_OK;
}

template <typename T, typename ST>
static elph_status launch_step2_t(elph_ctx ctx, const EpiParams& ep, void* Bp, void* Bm, int64_t* we_tiles) {
  *we_tiles = ctx->m_pad / 32;
  if constexpr (UsesGemm<T>::value) {
    if (!ep.tile_keep) {
      switch (ctx->nbr) {
        case 3: return launch_gemm_nx<T, ST, 3>(ctx, ep, Bp, Bm, we_tiles);
        case 6: return launch_gemm_nx<T, ST, 6>(ctx, ep, Bp, Bm, we_tiles);
        case 9: return launch_gemm_nx<T, ST, 9>(ctx, ep, Bp, Bm, we_tiles);
        case 12: return launch_gemm_nx<T, ST, 12>(ctx, ep, Bp, Bm, we_tiles);
        case 15: return launch_gemm_nx<T, ST, 15>(ctx, ep, Bp, Bm, we_tiles);
        default: ctx->err = "unsupported branch count"; return ELPH_EINVAL;
      }
    }
  }
  switch (ctx->nbr) {
    case 3: launch_step2_nx<T, ST, 3>(ctx, ep, Bp, Bm); break;
    case 6: launch_step2_nx<T, ST, 6>(ctx, ep, Bp, Bm); break;
    case 9: launch_step2_nx<T, ST, 9>(ctx, ep, Bp, Bm); break;
    case 12: launch_step2_nx<T, ST, 12>(ctx, ep, Bp, Bm); break;
    case 15: launch_step2_nx<T, ST, 15>(ctx, ep, Bp, Bm); break;
    default: ctx->err = "unsupported branch count"; return ELPH_EINVAL;
  }
  return ELPH_OK;
}

static EpiParams epi_params(elph_ctx ctx) {
  EpiParams ep;
  ep.nstates = ctx->nstates;
  ep.nbr = ctx->nbr;
  ep.n0 = ctx->mesh[0];
  ep.n1 = ctx->mesh[1];
  ep.n2 = ctx->mesh[2];
  ep.tetra = (ctx->delta == ELPH_DELTA_TETRA || ctx->delta == ELPH_DELTA_TRIANGLE) ? 1 : 0;
  ep.fr = ctx->frohlich ? (const cd*)ctx->d_frohlich : nullptr;
  ep.ust = (const cd*)ctx->d_ustate;
  ep.nb = ctx->nb;
  // with the tetrahedron delta the store first holds 2 pi / (hbar N_k) |g|^2
  ep.pref = ep.tetra ? 2.0 * kPi / (kHbarEVs * (double)ctx->nk)
                     : 2.0 * kPi / (kHbarEVs * (double)ctx->nk) / (sqrt(2.0 * kPi) * ctx->sigma);
  ep.inv2s2 = 1.0 / (2.0 * ctx->sigma * ctx->sigma);
  ep.omega_min = ctx->omega_min;
  ep.st_k = ctx->d_state_k;
  ep.eps = ctx->d_eps;
  ep.hw = ctx->d_hw;
  ep.Lq = (const cd*)ctx->d_Lq;
  ep.m_pad = ctx->m_pad;
  ep.lomf = ep.fstate = ep.omf = ep.nocc = nullptr;
  ep.we_part = nullptr;
  ep.wph_acc = nullptr;
  ep.tile_keep = ctx->d_tile_keep;
  ep.perm = ctx->d_tile_perm;
  ep.cscale = 1.0 / (ctx->sc_b2 * ctx->sc_ap);
  ep.rho = nullptr;
  ep.b2n = nullptr;
  ep.cu = ep.cv = 0.0;
  return ep;
}

static elph_status ensure_we_part(elph_ctx ctx) {
  const int64_t ntiles = ctx->m_pad / 32;
  if (ctx->we_part_len >= ntiles * ctx->m_pad) return ELPH_OK;
  void* p;
  if (dev_alloc(ctx, &p, (size_t)ntiles * ctx->m_pad * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "device allocation of rate partials failed";
    return ELPH_ENOMEM;
  }
  if (ctx->d_we_part) dev_free(ctx, ctx->d_we_part);
  ctx->d_we_part = (double*)p;
  ctx->we_part_len = ntiles * ctx->m_pad;
  return ELPH_OK;
}

// ---------------------------------------------------------------------------
// Analytic tetrahedron delta (the alternative to smearing the method offers
// beside the triangle method): the mesh cells are split into six
// tetrahedra along their main diagonal, E(k'') = eps_n(k'') -+ hw_s(k'' - k)
// - eps_m(k) is linear in each, and the delta at the final k' is replaced by
// the sum over the 24 tetrahedra with corner k' of the integral of
// delta(E) times the barycentric coordinate of k' (mesh units).

// integral over a tetrahedron of volume 1/6 of delta(E) lambda_c for linear
// E with corner energies e (coarea: each triangle of the section E = 0
// contributes its area times the mean of lambda_c over its corners, over
// |grad E|; the value depends only on the corner energies, so the sorted
// corners sit at 0, x, y, z; a triangular section has the closed form of
// the tetrahedron method's density of states)
__device__ inline double tetra_delta_corner(double e0, double e1, double e2, double e3, int c) {
  const int nneg = (e0 < 0.0) + (e1 < 0.0) + (e2 < 0.0) + (e3 < 0.0);
  if (nneg == 0 || nneg == 4) return 0.0;  // the level misses the tetrahedron
  // sort (insertion order: equal energies keep corner order), carrying the
  // mark of corner c along
  double s0 = e0, s1 = e1, s2 = e2, s3 = e3;
  bool m0 = c == 0, m1 = c == 1, m2 = c == 2, m3 = c == 3;
  auto cs = [](double& a, double& b, bool& ma, bool& mb) {
    if (b < a) {
      const double t = a;
      a = b;
      b = t;
      const bool u = ma;
      ma = mb;
      mb = u;
    }
  };
  cs(s2, s3, m2, m3);
  cs(s1, s2, m1, m2);
  cs(s2, s3, m2, m3);
  cs(s0, s1, m0, m1);
  cs(s1, s2, m1, m2);
  cs(s2, s3, m2, m3);
  const int pc = m1 ? 1 : m2 ? 2 : m3 ? 3 : 0;
  if (nneg == 1) {
    // triangle on the edges from corner 0: the section's measure over |grad E|
    // is s0^2 / (2 (s1-s0)(s2-s0)(s3-s0)); the crossing on edge (0, k) has
    // lambda_0 = s_k / (s_k - s0) and lambda_k = -s0 / (s_k - s0)
    const double d1 = s1 - s0, d2 = s2 - s0, d3 = s3 - s0;
    const double tot = 0.5 * s0 * s0 / (d1 * d2 * d3);
    const double l = pc == 0 ? s1 / d1 + s2 / d2 + s3 / d3 : -s0 / (pc == 1 ? d1 : pc == 2 ? d2 : d3);
    return tot * l / 3.0;
  }
  if (nneg == 3) {
    // triangle on the edges to corner 3, the mirror case
    const double d0 = s3 - s0, d1 = s3 - s1, d2 = s3 - s2;
    const double tot = 0.5 * s3 * s3 / (d0 * d1 * d2);
    const double l = pc == 3 ? -s0 / d0 - s1 / d1 - s2 / d2 : s3 / (pc == 0 ? d0 : pc == 1 ? d1 : d2);
    return tot * l / 3.0;
  }
  // quadrilateral section (two corners on each side): its two triangles'
  // areas in the tetrahedron with the sorted corners at 0, x, y, z
  const double s[4] = {s0, s1, s2, s3};
  const double g0 = s1 - s0, g1 = s2 - s0, g2 = s3 - s0;
  const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
  struct Pt {
    double x, y, z, l;
  };
  auto cross = [&](int a, int b) {
    const double t = s[a] / (s[a] - s[b]);
    const double pa[3] = {a == 1 ? 1.0 : 0.0, a == 2 ? 1.0 : 0.0, a == 3 ? 1.0 : 0.0};
    const double pb[3] = {b == 1 ? 1.0 : 0.0, b == 2 ? 1.0 : 0.0, b == 3 ? 1.0 : 0.0};
    Pt p;
    p.x = pa[0] + t * (pb[0] - pa[0]);
    p.y = pa[1] + t * (pb[1] - pa[1]);
    p.z = pa[2] + t * (pb[2] - pa[2]);
    p.l = (pc == a) ? 1.0 - t : (pc == b) ? t : 0.0;
    return p;
  };
  auto tri = [&](const Pt& A, const Pt& B, const Pt& C) {
    const double ux = B.x - A.x, uy = B.y - A.y, uz = B.z - A.z;
    const double vx = C.x - A.x, vy = C.y - A.y, vz = C.z - A.z;
    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    return 0.5 * sqrt(cx * cx + cy * cy + cz * cz) * (A.l + B.l + C.l) / 3.0;
  };
  const Pt q02 = cross(0, 2), q03 = cross(0, 3), q13 = cross(1, 3), q12 = cross(1, 2);
  return (tri(q02, q03, q13) + tri(q02, q13, q12)) / gn;  // the section's corners in cyclic order
}

// The 24 tetrahedra with a given mesh point as corner: the point's 3x3x3
// neighbourhood is numbered (dx+1)*9 + (dy+1)*3 + (dz+1) (centre 13); each
// of the 8 cells with the centre as a corner is cut along the paths
// 0 -> e_a -> e_a + e_b -> (1,1,1) over the 6 axis orders, and a path
// tetrahedron is kept when it passes through the centre.
struct TetraTab {
  unsigned char c[24][4];  // corners (neighbourhood numbers) along the path
  unsigned char ctr[24];   // which of them is the centre
};

constexpr TetraTab make_tetra_tab() {
  TetraTab t{};
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int n = 0;
  for (int o = 0; o < 8; ++o)
    for (int p = 0; p < 6; ++p) {
      int v[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
      int ids[4] = {0, 0, 0, 0};
      int ctr = -1;
      for (int k = 0; k < 4; ++k) {
        if (k > 0) v[perms[p][k - 1]] += 1;
        ids[k] = v[0] * 9 + v[1] * 3 + v[2];
        if (ids[k] == 13) ctr = k;
      }
      if (ctr >= 0) {
        for (int k = 0; k < 4; ++k) t.c[n][k] = (unsigned char)ids[k];
        t.ctr[n] = (unsigned char)ctr;
        ++n;
      }
    }
  return t;
}
constexpr TetraTab kTetra = make_tetra_tab();

// one tetrahedron's corner weight of the centre for both signs; the corner
// numbers are compile-time constants, so the neighbourhood arrays stay in
// registers
template <int K>
__device__ __attribute__((always_inline)) inline void tetra_one(const double (&ej)[27], const double (&w)[27], double ei, double& dp, double& dm) {
  constexpr int c0 = kTetra.c[K][0], c1 = kTetra.c[K][1], c2 = kTetra.c[K][2], c3 = kTetra.c[K][3];
  constexpr int ck = kTetra.ctr[K];
  dp += tetra_delta_corner(ej[c0] - w[c0] - ei, ej[c1] - w[c1] - ei, ej[c2] - w[c2] - ei, ej[c3] - w[c3] - ei, ck);
  dm += tetra_delta_corner(ej[c0] + w[c0] - ei, ej[c1] + w[c1] - ei, ej[c2] + w[c2] - ei, ej[c3] + w[c3] - ei, ck);
}

template <int... K>
__device__ __attribute__((always_inline)) inline void tetra_all(const double (&ej)[27], const double (&w)[27], double ei, double& dp, double& dm,
                                 std::integer_sequence<int, K...>) {
  (tetra_one<K>(ej, w, ei, dp, dm), ...);
}

// B+-[i][j][s] *= tetrahedron delta at k_j for E = eps_n(k'') -+ hw_s(k'' - k_i) - eps_i;
// one thread per pair (i, j)
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_tetra_scale(int64_t M, int nb, MeshDims md, const int32_t* __restrict__ st_k,
                                                     const int32_t* __restrict__ st_m,
                                                     const double* __restrict__ eps,
                                                     const double* __restrict__ eps_all,
                                                     const double* __restrict__ hw, ST* __restrict__ Bp,
                                                     ST* __restrict__ Bm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int64_t i = e / M, j = e - i * M;
  const int ki = st_k[i], kj = st_k[j], n = st_m[j];
  const int ic = ki % md.n2, it = ki / md.n2, ib = it % md.n1, ia = it / md.n1;
  const int jc = kj % md.n2, jt = kj / md.n2, jb = jt % md.n1, ja = jt / md.n1;
  const double ei = eps[i];
  double ej[27];
  int qi[27];
#pragma unroll
  for (int p = 0; p < 27; ++p) {
    int a = ja + p / 9 - 1, b = jb + (p / 3) % 3 - 1, c = jc + p % 3 - 1;
    a += (a < 0) ? md.n0 : (a >= md.n0 ? -md.n0 : 0);
    b += (b < 0) ? md.n1 : (b >= md.n1 ? -md.n1 : 0);
    c += (c < 0) ? md.n2 : (c >= md.n2 ? -md.n2 : 0);
    ej[p] = eps_all[(int64_t)((a * md.n1 + b) * md.n2 + c) * nb + n];
    int qa = a - ia, qb = b - ib, qc = c - ic;
    qa += qa < 0 ? md.n0 : 0;
    qb += qb < 0 ? md.n1 : 0;
    qc += qc < 0 ? md.n2 : 0;
    qi[p] = (qa * md.n1 + qb) * md.n2 + qc;
  }
  for (int s = 0; s < NX; ++s) {
    const int64_t t = e * NX + s;
    const double bp = (double)Bp[t], bm = (double)Bm[t];
    if (bp == 0.0 && bm == 0.0) continue;
    double w[27];
#pragma unroll
    for (int p = 0; p < 27; ++p) w[p] = hw[(int64_t)qi[p] * NX + s];
    double dp = 0.0, dm = 0.0;
    tetra_all(ej, w, ei, dp, dm, std::make_integer_sequence<int, 24>{});
    Bp[t] = (ST)(bp * dp);
    Bm[t] = (ST)(bm * dm);
  }
}

// Triangle delta: the corner weight of corner c (energies at level 0) for a
// triangle of area 1/2 (half a mesh cell of a plane) over which E is linear:
// the level-0 segment's length over |grad E| (the linear triangle DOS
// -s0 / ((s1-s0)(s2-s0)) below the middle corner, s2 / ((s2-s0)(s2-s1))
// above it) times the mean of the barycentric coordinate of c at the
// segment's two ends.
__device__ inline double triangle_delta_corner(double e0, double e1, double e2, int c) {
  const int nneg = (e0 < 0.0) + (e1 < 0.0) + (e2 < 0.0);
  if (nneg == 0 || nneg == 3) return 0.0;  // the level misses the triangle
  double s0 = e0, s1 = e1, s2 = e2;
  bool m0 = c == 0, m1 = c == 1, m2 = c == 2;
  auto cs = [](double& a, double& b, bool& ma, bool& mb) {
    if (b < a) {
      const double t = a;
      a = b;
      b = t;
      const bool u = ma;
      ma = mb;
      mb = u;
    }
  };
  cs(s1, s2, m1, m2);
  cs(s0, s1, m0, m1);
  cs(s1, s2, m1, m2);
  const int pc = m1 ? 1 : m2 ? 2 : 0;
  if (nneg == 1) {
    // ends on the edges (0, 1) and (0, 2)
    const double d1 = s1 - s0, d2 = s2 - s0;
    const double tot = -s0 / (d1 * d2);
    const double l = pc == 0 ? s1 / d1 + s2 / d2 : -s0 / (pc == 1 ? d1 : d2);
    return 0.5 * tot * l;
  }
  // ends on the edges (0, 2) and (1, 2)
  const double d0 = s2 - s0, d1 = s2 - s1;
  const double tot = s2 / (d0 * d1);
  const double l = pc == 2 ? -s0 / d0 - s1 / d1 : s2 / (pc == 0 ? d0 : d1);
  return 0.5 * tot * l;
}

// The 6 triangles of a mesh plane (normal to the third mesh axis) with a
// given point as corner: the 3x3 in-plane neighbourhood numbered
// (dx+1)*3 + (dy+1) (centre 4); each of the 4 cells with the centre as a
// corner is cut along the paths 0 -> e_a -> e_a + e_b over the 2 axis
// orders, and a path triangle is kept when it passes through the centre.
struct TriTab {
  unsigned char c[6][3];
  unsigned char ctr[6];
};

constexpr TriTab make_tri_tab() {
  TriTab t{};
  const int perms[2][2] = {{0, 1}, {1, 0}};
  int n = 0;
  for (int o = 0; o < 4; ++o)
    for (int p = 0; p < 2; ++p) {
      int v[2] = {(o >> 1) & 1, o & 1};
      int ids[3] = {0, 0, 0};
      int ctr = -1;
      for (int k = 0; k < 3; ++k) {
        if (k > 0) v[perms[p][k - 1]] += 1;
        ids[k] = v[0] * 3 + v[1];
        if (ids[k] == 4) ctr = k;
      }
      if (ctr >= 0) {
        for (int k = 0; k < 3; ++k) t.c[n][k] = (unsigned char)ids[k];
        t.ctr[n] = (unsigned char)ctr;
        ++n;
      }
    }
  return t;
}
constexpr TriTab kTri = make_tri_tab();

template <int K>
__device__ __attribute__((always_inline)) inline void tri_one(const double (&ej)[9], const double (&w)[9], double ei,
                                                              double& dp, double& dm) {
  constexpr int c0 = kTri.c[K][0], c1 = kTri.c[K][1], c2 = kTri.c[K][2];
  constexpr int ck = kTri.ctr[K];
  dp += triangle_delta_corner(ej[c0] - w[c0] - ei, ej[c1] - w[c1] - ei, ej[c2] - w[c2] - ei, ck);
  dm += triangle_delta_corner(ej[c0] + w[c0] - ei, ej[c1] + w[c1] - ei, ej[c2] + w[c2] - ei, ck);
}

template <int... K>
__device__ __attribute__((always_inline)) inline void tri_all(const double (&ej)[9], const double (&w)[9], double ei,
                                                              double& dp, double& dm, std::integer_sequence<int, K...>) {
  (tri_one<K>(ej, w, ei, dp, dm), ...);
}

// B+-[i][j][s] *= triangle delta at k_j for E = eps_n(k'') -+ hw_s(k'' - k_i) - eps_i
// over k_j's mesh plane; one thread per pair (i, j)
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_tri_scale(int64_t M, int nb, MeshDims md, const int32_t* __restrict__ st_k,
                                                   const int32_t* __restrict__ st_m, const double* __restrict__ eps,
                                                   const double* __restrict__ eps_all, const double* __restrict__ hw,
                                                   ST* __restrict__ Bp, ST* __restrict__ Bm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int64_t i = e / M, j = e - i * M;
  const int ki = st_k[i], kj = st_k[j], n = st_m[j];
  const int ic = ki % md.n2, it = ki / md.n2, ib = it % md.n1, ia = it / md.n1;
  const int jc = kj % md.n2, jt = kj / md.n2, jb = jt % md.n1, ja = jt / md.n1;
  const double ei = eps[i];
  double ej[9];
  int qi[9];
  int qc = jc - ic;
  qc += qc < 0 ? md.n2 : 0;
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    int a = ja + p / 3 - 1, b = jb + p % 3 - 1;
    a += (a < 0) ? md.n0 : (a >= md.n0 ? -md.n0 : 0);
    b += (b < 0) ? md.n1 : (b >= md.n1 ? -md.n1 : 0);
    ej[p] = eps_all[(int64_t)((a * md.n1 + b) * md.n2 + jc) * nb + n];
    int qa = a - ia, qb = b - ib;
    qa += qa < 0 ? md.n0 : 0;
    qb += qb < 0 ? md.n1 : 0;
    qi[p] = (qa * md.n1 + qb) * md.n2 + qc;
  }
  for (int s = 0; s < NX; ++s) {
    const int64_t t = e * NX + s;
    const double bp = (double)Bp[t], bm = (double)Bm[t];
    if (bp == 0.0 && bm == 0.0) continue;
    double w[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) w[p] = hw[(int64_t)qi[p] * NX + s];
    double dp = 0.0, dm = 0.0;
    tri_all(ej, w, ei, dp, dm, std::make_integer_sequence<int, 6>{});
    Bp[t] = (ST)(bp * dp);
    Bm[t] = (ST)(bm * dm);
  }
}

static void launch_tetra_scale(elph_ctx ctx, void* Bp, void* Bm, bool store_f64) {
  const int64_t M = ctx->nstates;
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  const dim3 grid(blocks_for(M * M, 256)), blk(256);
#define TS(STT, NXV)                                                                                            \
  if (ctx->delta == ELPH_DELTA_TRIANGLE)                                                                        \
    hipLaunchKernelGGL((k_tri_scale<STT, NXV>), grid, blk, 0, ctx->stream, M, ctx->nb, md, ctx->d_state_k,      \
                       ctx->d_state_m, ctx->d_eps, ctx->d_eps_all, ctx->d_hw, (STT*)Bp, (STT*)Bm);              \
  else                                                                                                          \
    hipLaunchKernelGGL((k_tetra_scale<STT, NXV>), grid, blk, 0, ctx->stream, M, ctx->nb, md, ctx->d_state_k,    \
                       ctx->d_state_m, ctx->d_eps, ctx->d_eps_all, ctx->d_hw, (STT*)Bp, (STT*)Bm)
#define TSN(STT)              \
  switch (ctx->nbr) {         \
    case 3: TS(STT, 3); break;   \
    case 6: TS(STT, 6); break;   \
    case 9: TS(STT, 9); break;   \
    case 12: TS(STT, 12); break; \
    default: TS(STT, 15); break; \
  }
  if (store_f64) {
    TSN(double)
  } else {
    TSN(float)
  }
#undef TSN
#undef TS
}

// Run both contractions and the epilogue.  Bp/Bm receive the term store
// (double when store_f64, else float).  If th != nullptr the rates at that
// temperature are accumulated into we_out [nstates] and wph_acc [nk][nbr]
// (wph_acc must be zeroed by the caller).
elph_status run_vertex(elph_ctx ctx, void* Bp, void* Bm, bool store_f64, const Thermal* th, double* we_out,
                       double* wph_acc) {
  elph_status st = build_operands(ctx);
  if (st != ELPH_OK) return st;
  EpiParams ep = epi_params(ctx);
  // GEMM forms writing the context's store keep an error estimate per term
  if (Bp == ctx->d_Bp) ctx->rho_valid = false;
  const bool want_rho = !store_f64 && Bp == ctx->d_Bp && refine_applicable(ctx);
  if (want_rho) {
    st = refine_prepare(ctx);
    if (st != ELPH_OK) return st;
    ep.rho = ctx->d_rho;
    ep.b2n = ctx->d_b2n;
    ep.cu = refine_unit(ctx, false);
    ep.cv = refine_unit(ctx, true);
  }
  int64_t we_tiles = ctx->m_pad / 32;
  if (th) {
    st = ensure_we_part(ctx);
    if (st != ELPH_OK) return st;
    ep.lomf = th->lomf;
    ep.fstate = th->f;
    ep.omf = th->omf;
    ep.nocc = th->nocc;
    // with the tetrahedron delta W_e comes from the store rows once the
    // weights are applied
    ep.we_part = ep.tetra ? nullptr : ctx->d_we_part;
    ep.wph_acc = wph_acc;
  }
  if (ctx->precision == ELPH_FP64) {
    mark(ctx, 2);
    st = launch_step1_t<double>(ctx);
    if (st != ELPH_OK) return st;
    mark(ctx, 3);
    mark(ctx, 4);
    st = store_f64 ? launch_step2_t<double, double>(ctx, ep, Bp, Bm, &we_tiles) : launch_step2_t<double, float>(ctx, ep, Bp, Bm, &we_tiles);
    mark(ctx, 5);
  } else if (ctx->precision == ELPH_FP32) {
    mark(ctx, 2);
    st = launch_step1_t<float>(ctx, want_rho);
    if (st != ELPH_OK) return st;
    mark(ctx, 3);
    mark(ctx, 4);
    st = store_f64 ? launch_step2_t<float, double>(ctx, ep, Bp, Bm, &we_tiles) : launch_step2_t<float, float>(ctx, ep, Bp, Bm, &we_tiles);
    if (ep.tile_keep) mark(ctx, 5);  // the GEMM path marks its own window (the contraction)
  } else if (ctx->precision == ELPH_FP16X3) {
    mark(ctx, 2);
    st = launch_step1_t<F16S<2>>(ctx, want_rho);
    if (st != ELPH_OK) return st;
    mark(ctx, 3);
    mark(ctx, 4);
    st = store_f64 ? launch_step2_t<F16S<2>, double>(ctx, ep, Bp, Bm, &we_tiles)
                   : launch_step2_t<F16S<2>, float>(ctx, ep, Bp, Bm, &we_tiles);
    if (ep.tile_keep) mark(ctx, 5);
  } else if (ctx->precision == ELPH_BF16X3) {
    mark(ctx, 2);
    st = launch_step1_t<Bf16S<2>>(ctx, want_rho);
    if (st != ELPH_OK) return st;
    mark(ctx, 3);
    mark(ctx, 4);
    st = store_f64 ? launch_step2_t<Bf16S<2>, double>(ctx, ep, Bp, Bm, &we_tiles)
                   : launch_step2_t<Bf16S<2>, float>(ctx, ep, Bp, Bm, &we_tiles);
    if (ep.tile_keep) mark(ctx, 5);
  } else {
    mark(ctx, 2);
    st = launch_step1_t<Bf16S<3>>(ctx, want_rho);
    if (st != ELPH_OK) return st;
    mark(ctx, 3);
    mark(ctx, 4);
    st = store_f64 ? launch_step2_t<Bf16S<3>, double>(ctx, ep, Bp, Bm, &we_tiles)
                   : launch_step2_t<Bf16S<3>, float>(ctx, ep, Bp, Bm, &we_tiles);
    if (ep.tile_keep) mark(ctx, 5);
  }
  if (st != ELPH_OK) return st;
  if (ep.tetra) {
    mark(ctx, 8);
    launch_tetra_scale(ctx, Bp, Bm, store_f64);
    mark(ctx, 9);
    if (th) {
      if (store_f64) launch_we_rows<double>(ctx, (const double*)Bp, (const double*)Bm, th->lomf, th->nocc,
                                            ctx->d_we_part);
      else launch_we_rows<float>(ctx, (const float*)Bp, (const float*)Bm, th->lomf, th->nocc, ctx->d_we_part);
      we_tiles = 1;
    }
  }
  if (th && we_out) {
    hipLaunchKernelGGL(k_reduce_we, dim3(blocks_for(ctx->nstates, 256)), dim3(256), 0, ctx->stream,
                       ctx->d_we_part, we_tiles, ctx->m_pad, ctx->nstates, we_out);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = std::string("kernel launch failed: ") + hipGetErrorString(e);
    ctx->hip_dead = true;
    return ELPH_EHIP;
  }
  if (want_rho) ctx->rho_valid = true;
  return ELPH_OK;
}

// FP64 vertex operand of the refinement, gR[(x, Rp, n')][(Re, m')]
elph_status ensure_gR64(elph_ctx ctx) {
  if (ctx->d_gR64) return ELPH_OK;
  const int nb = ctx->nb, nbr = ctx->nbr;
  ctx->ke64 = ((int64_t)ctx->nre * nb + 15) / 16 * 16;
  ctx->kp64 = ((int64_t)ctx->nrp * nb + 15) / 16 * 16;
  const int64_t ncol = (int64_t)nbr * ctx->nrp * nb;
  const size_t bytes = (size_t)ncol * ctx->ke64 * 16;
  ALLOC(ctx->d_gR64, bytes);
  HIPCHK(hipMemsetAsync(ctx->d_gR64, 0, bytes, ctx->stream));
  const int64_t gtotal = (int64_t)ctx->nre * ctx->nrp * nbr * nb * nb;
  hipLaunchKernelGGL(k_permute_g<double>, dim3(blocks_for(gtotal, 256)), dim3(256), 0, ctx->stream, ctx->nre,
                     ctx->nrp, nbr, nb, ctx->ke64, ctx->d_gr, 1.0, ctx->d_gR64);
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}

// FP64 step-1 rows B2[(s, x)][(Rp, n')] (row stride kp64) of ns listed
// states, given their kept index and band; Ae64 holds ceil(ns/64)*64 rows of
// ke64 complex values, B2_64 that many times nbr rows of kp64
elph_status step1_fp64_rows(elph_ctx ctx, int64_t ns, const int32_t* st_kidx, const int32_t* st_m, double* Ae64,
                            double* B2_64) {
  const int nb = ctx->nb;
  const int64_t ns_pad = (ns + 63) / 64 * 64;
  HIPCHK(hipMemsetAsync(Ae64, 0, (size_t)ns_pad * ctx->ke64 * 16, ctx->stream));
  hipLaunchKernelGGL(k_build_Ae<double>, dim3(blocks_for(ns * ctx->nre * nb, 256)), dim3(256), 0, ctx->stream, ns,
                     nb, ctx->nre, ctx->ke64, st_kidx, st_m, (const cd*)ctx->d_Ee, (const cd*)ctx->d_U, 1.0, Ae64);
  S1Desc<double> d;
  d.m_pad = ns_pad;
  d.ncol = (int64_t)ctx->nbr * ctx->nrp * nb;
  d.ke = ctx->ke64;
  d.kp = ctx->kp64;
  d.nstates = ns;
  d.Ae = Ae64;
  d.gR = ctx->d_gR64;
  d.B2 = B2_64;
  d.nrp = ctx->nrp;
  d.nb = nb;
  d.nbr = ctx->nbr;
  d.st_kidx = st_kidx;
  d.Ep = (const cd*)ctx->d_Ep;
  dim3 grid((unsigned)((d.ncol + 63) / 64), (unsigned)(ns_pad / 64));
  hipLaunchKernelGGL(k_step1<double>, grid, dim3(256), 0, ctx->stream, d);
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}


// ---------------------------------------------------------------------------
// Batches of materials: one persistent step-1 launch over every material's
// tiles and one persistent step-2 launch per branch count, items ordered
// longest contraction first; the whole per-temperature sequence can be
// captured in a HIP graph and replayed.

// Per-material descriptors of the batched epilogues.
template <typename ST>
struct EpiDesc {
  EpiParams ep;
  const int32_t* poff;
  const uint64_t* ppk;
  const float* C;
  int64_t ldc, nq;
  int32_t nkept;
  ST* Bp;
  ST* Bm;
};

template <typename T>
struct S1EpiDesc {
  int64_t M, ncol, kp;
  int nrp, nb, nbr;
  const float* C1;
  const int32_t* st_kidx;
  const cd* Ep;
  double scale;
  typename Store<T>::type* B2;
};

// The per-q epilogue of every material of one branch count in one launch:
// items (slot, q / 4), taken grid-stride; a block's four wavefronts take
// four q, each walking its pair list (packed state ranges) with the pair
// body of k_epi_rows.
template <typename ST, int NX>
__global__ void __launch_bounds__(256) k_epi_q_persist(const EpiDesc<ST>* __restrict__ d,
                                                       const int2* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    EpiDesc<ST> e = d[w.x];
    promote(e.ep);
    const int64_t q = (int64_t)w.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (q < e.nq)
      epi_q_wave<ST, NX>(q, e.ep, as_global(e.poff), as_global(e.ppk), as_global(e.C), e.ldc, as_global(e.Bp),
                         as_global(e.Bm));
  }
}

// The step-1 epilogue of every material in one launch: 256-element blocks
// numbered across the materials (boff), taken grid-stride.
template <typename T>
__global__ void __launch_bounds__(256) k_step1_epi_persist(const S1EpiDesc<T>* __restrict__ d,
                                                           const int32_t* __restrict__ boff, int n, int nblocks) {
  for (int g = blockIdx.x; g < nblocks; g += gridDim.x) {
    int lo = 0, hi = n - 1;  // material m with boff[m] <= g < boff[m + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (boff[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const S1EpiDesc<T> e = d[lo];
    const int64_t el = (int64_t)(g - boff[lo]) * 256 + threadIdx.x;
    if (el < e.M * e.ncol)
      step1_epi_elem<T>(el, 0, e.ncol, e.nrp, e.nb, e.nbr, e.kp, as_global(e.C1), as_global(e.st_kidx),
                        as_global(e.Ep), e.scale, as_global(e.B2));
  }
}

struct BatchImpl {
  struct Cls {
    int nx = 0;
    std::vector<int> mats;          // material of each descriptor slot
    void* d_desc = nullptr;         // S2Desc<T>[mats.size()]
    int4* d_items = nullptr;
    std::vector<int4> sorted, natural;
  };
  std::vector<elph_ctx> ctx;
  std::vector<hipStream_t> saved_streams;
  hipStream_t stream = nullptr;
  int precision = ELPH_FP32;
  bool prepared = false;
  std::vector<Thermal> th;
  std::vector<double*> acc, we_tmp;
  void* d_s1desc = nullptr;
  int4* d_s1items = nullptr;
  std::vector<int4> s1_sorted, s1_natural;
  std::vector<Cls> cls;
  int* d_counters = nullptr;
  int bpc = 2;
  bool sorted = true;
  bool tuned = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double gT = -1.0;
  std::vector<double*> gptrs;
  std::vector<void*> allocs;
  std::string err;
  int ncu = 256;
  // GEMM forms: persistent GEMMs over every material's block tiles, then
  // each material's epilogues
  bool gemm = false;
  GemmArgs* d_g1 = nullptr;
  GemmArgs* d_g2 = nullptr;
  int4* d_g1items = nullptr;
  int4* d_g2items = nullptr;
  // item lists per GEMM tile height (index 0: 64 rows, 1: 128 rows)
  std::vector<int4> g1_natural[2], g1_sorted[2], g2_natural[2], g2_sorted[2];
  int wr = kGemmWR;                // rows per GEMM tile / 32 (2 or 4)
  std::vector<float*> c1, c2;
  // persistent epilogues: the step-1 epilogue over every material, the
  // per-q epilogue over the materials of each branch count
  void* d_s1epi = nullptr;         // S1EpiDesc<T>[n]
  int32_t* d_s1boff = nullptr;     // [n + 1] first 256-element block of each material
  int s1blocks = 0;
  std::vector<void*> d_epi;        // per class: EpiDesc<ST>[mats]
  std::vector<int2*> d_epi_items;  // per class: (slot, q / 4)
  std::vector<int> epi_items;
};

// tuned launch shape of a batch: blocks per CU, cost order, GEMM tile rows / 32
struct BatchShape {
  int bpc;
  bool sorted;
  int wr;
};

static std::map<std::string, BatchShape>& tune_cache() {
  static std::map<std::string, BatchShape> c;
  return c;
}

#define BCHK(x)                                                          \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      b->err = std::string("HIP error ") + hipGetErrorString(e_) + " at " + __FILE__ + ":" + std::to_string(__LINE__); \
      return ELPH_EHIP;                                                  \
    }                                                                    \
  } while (0)

static hipError_t balloc(BatchImpl* b, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 1);
  if (e == hipSuccess) b->allocs.push_back(*p);
  return e;
}

struct StreamSwap {  // run the contexts' launches on the batch stream
  BatchImpl* b;
  explicit StreamSwap(BatchImpl* bb) : b(bb) {
    for (size_t m = 0; m < b->ctx.size(); ++m) b->ctx[m]->stream = b->stream;
  }
  ~StreamSwap() {
    for (size_t m = 0; m < b->ctx.size(); ++m) b->ctx[m]->stream = b->saved_streams[m];
  }
};

static std::string batch_signature(BatchImpl* b) {
  std::string sig = std::to_string(b->precision);
  for (elph_ctx c : b->ctx)
    sig += ":" + std::to_string(c->nstates) + "," + std::to_string(c->nbr) + "," + std::to_string(c->ke) + "," +
           std::to_string(c->kp);
  return sig;
}

template <typename T>
static elph_status batch_prepare_t(BatchImpl* b) {
  const int n = (int)b->ctx.size();
  StreamSwap sw(b);
  std::vector<S1Desc<T>> s1(n);
  std::map<int, int> cls_of_nx;
  for (int m = 0; m < n; ++m) {
    elph_ctx c = b->ctx[m];
    elph_status st = build_tables(c);
    if (st == ELPH_OK) st = build_operands(c);
    if (st == ELPH_OK) st = ensure_we_part(c);
    // pair lists now, so that no allocation happens under graph capture
    if (st == ELPH_OK && !c->pairs_ready && !c->pairs_failed && c->nkept <= kMaxPairKept) {
      if (ensure_pairs(c) != ELPH_OK) {
        c->pairs_failed = true;
        c->err.clear();
      }
    }
    if (st != ELPH_OK) {
      b->err = "material " + std::to_string(m) + ": " + c->err;
      return st;
    }
    const size_t nt = (size_t)c->nstates * c->nstates * c->nbr;
    const size_t esz = sizeof(T);
    if (!c->d_Bp) {
      if (dev_alloc(c, &c->d_Bp, nt * esz) != hipSuccess || dev_alloc(c, &c->d_Bm, nt * esz) != hipSuccess) {
        (void)hipGetLastError();
        b->err = "material " + std::to_string(m) + ": vertex store allocation failed";
        return ELPH_ENOMEM;
      }
    }
    c->store_f32 = sizeof(T) == 4;
    c->rho_valid = false;  // batched launches keep the plain form: no error estimates
    Thermal t;
    st = alloc_thermal(c, &t);
    if (st != ELPH_OK) {
      b->err = c->err;
      return st;
    }
    b->th.push_back(t);
    void *a = nullptr, *w = nullptr;
    if (dev_alloc(c, &a, (size_t)c->nk * c->nbr * sizeof(double)) != hipSuccess ||
        dev_alloc(c, &w, (size_t)c->nstates * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      b->err = "scratch allocation failed";
      return ELPH_ENOMEM;
    }
    b->acc.push_back((double*)a);
    b->we_tmp.push_back((double*)w);
    s1[m] = step1_desc<T>(c);
    if (!cls_of_nx.count(c->nbr)) {
      cls_of_nx[c->nbr] = (int)b->cls.size();
      b->cls.push_back(BatchImpl::Cls());
      b->cls.back().nx = c->nbr;
    }
    b->cls[cls_of_nx[c->nbr]].mats.push_back(m);
    for (int64_t by = 0; by < c->m_pad / 64; ++by)
      for (int64_t bx = 0; bx < (s1[m].ncol + 63) / 64; ++bx) b->s1_natural.push_back(make_int4(m, (int)bx, (int)by, 0));
  }
  if constexpr (UsesGemm<T>::value) {
    // GEMM path: full-size FP32 result buffers per material (no chunks)
    b->gemm = true;
    std::vector<GemmArgs> g1(n), g2(n);
    for (int m = 0; m < n; ++m) {
      elph_ctx c = b->ctx[m];
      if (!c->pairs_ready) {
        b->err = "material " + std::to_string(m) + ": per-q pair lists are unavailable";
        return ELPH_EINVAL;
      }
      const int64_t M = c->nstates, ncol = s1[m].ncol;
      void *p1 = nullptr, *p2 = nullptr;
      if (balloc(b, &p1, (size_t)M * ncol * 8) != hipSuccess ||
          balloc(b, &p2, (size_t)M * c->nbr * c->m_pad * 8) != hipSuccess) {
        b->err = "batch allocation of the GEMM buffers failed";
        return ELPH_ENOMEM;
      }
      b->c1.push_back((float*)p1);
      b->c2.push_back((float*)p2);
      g1[m] = GemmArgs{0, M, ncol, c->ke, 1, (const unsigned short*)c->d_Ae, (const unsigned short*)c->d_gR,
                       (float*)p1, ncol};
      g2[m] = GemmArgs{0, M * c->nbr, M, c->kp, c->nbr, (const unsigned short*)c->d_B2,
                       (const unsigned short*)c->d_Ap, (float*)p2, c->m_pad};
      for (int h = 0; h < 2; ++h)
        for (const auto& pr : {std::make_pair(&g1[m], &b->g1_natural[h]), std::make_pair(&g2[m], &b->g2_natural[h])}) {
          const GemmGrid gg = gemm_grid(pr.first->nc, pr.first->nj, 32 * (2 + 2 * h));
          for (int ty = 0; ty < gg.ny; ++ty)
            for (int tx = 0; tx < gg.nx; ++tx) pr.second->push_back(make_int4(m, ty, tx, 0));
        }
    }
    for (int h = 0; h < 2; ++h) {
      b->g1_sorted[h] = b->g1_natural[h];
      std::stable_sort(b->g1_sorted[h].begin(), b->g1_sorted[h].end(),
                       [&](const int4& a, const int4& c2) { return g1[a.x].K > g1[c2.x].K; });
      b->g2_sorted[h] = b->g2_natural[h];
      std::stable_sort(b->g2_sorted[h].begin(), b->g2_sorted[h].end(),
                       [&](const int4& a, const int4& c2) { return g2[a.x].K > g2[c2.x].K; });
    }
    // epilogue descriptors (the thermal buffers and results stay in place)
    std::vector<S1EpiDesc<T>> e1(n);
    std::vector<int32_t> boff(n + 1, 0);
    for (int m = 0; m < n; ++m) {
      elph_ctx c = b->ctx[m];
      S1EpiDesc<T>& e = e1[m];
      e.M = c->nstates;
      e.ncol = (int64_t)c->nbr * c->nrp * c->nb;
      e.kp = c->kp;
      e.nrp = c->nrp;
      e.nb = c->nb;
      e.nbr = c->nbr;
      e.C1 = b->c1[m];
      e.st_kidx = c->d_state_kidx;
      e.Ep = (const cd*)c->d_Ep;
      e.scale = c->sc_b2 / (c->sc_ae * c->sc_g);
      e.B2 = (typename Store<T>::type*)c->d_B2;
      boff[m + 1] = boff[m] + (int32_t)((e.M * e.ncol + 255) / 256);
    }
    b->s1blocks = boff[n];
    if (balloc(b, (void**)&b->d_g1, n * sizeof(GemmArgs)) != hipSuccess ||
        balloc(b, (void**)&b->d_g2, n * sizeof(GemmArgs)) != hipSuccess ||
        balloc(b, (void**)&b->d_g1items, b->g1_natural[0].size() * sizeof(int4)) != hipSuccess ||
        balloc(b, (void**)&b->d_g2items, b->g2_natural[0].size() * sizeof(int4)) != hipSuccess ||
        balloc(b, (void**)&b->d_counters, 64 * sizeof(int)) != hipSuccess ||
        balloc(b, &b->d_s1epi, n * sizeof(S1EpiDesc<T>)) != hipSuccess ||
        balloc(b, (void**)&b->d_s1boff, (n + 1) * sizeof(int32_t)) != hipSuccess) {
      b->err = "batch allocation failed";
      return ELPH_ENOMEM;
    }
    BCHK(hipMemcpy(b->d_g1, g1.data(), n * sizeof(GemmArgs), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(b->d_g2, g2.data(), n * sizeof(GemmArgs), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(b->d_s1epi, e1.data(), n * sizeof(S1EpiDesc<T>), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(b->d_s1boff, boff.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    for (auto& cl : b->cls) {
      std::vector<EpiDesc<T>> d(cl.mats.size());
      std::vector<int2> items;
      for (size_t slot = 0; slot < cl.mats.size(); ++slot) {
        const int m = cl.mats[slot];
        elph_ctx c = b->ctx[m];
        EpiDesc<T>& e = d[slot];
        e.ep = epi_params(c);
        e.ep.lomf = b->th[m].lomf;
        e.ep.fstate = b->th[m].f;
        e.ep.omf = b->th[m].omf;
        e.ep.nocc = b->th[m].nocc;
        e.ep.we_part = c->d_we_part;
        e.poff = c->d_poff;
        e.ppk = c->d_ppk;
        e.C = b->c2[m];
        e.ldc = c->m_pad;
        e.nq = c->nk;
        e.nkept = (int32_t)c->nkept;
        e.Bp = (T*)c->d_Bp;
        e.Bm = (T*)c->d_Bm;
        for (int64_t qb = 0; qb < (c->nk + 3) / 4; ++qb) items.push_back(make_int2((int)slot, (int)qb));
      }
      void *dd = nullptr, *di = nullptr;
      if (balloc(b, &dd, d.size() * sizeof(EpiDesc<T>)) != hipSuccess ||
          balloc(b, &di, items.size() * sizeof(int2)) != hipSuccess) {
        b->err = "batch allocation failed";
        return ELPH_ENOMEM;
      }
      BCHK(hipMemcpy(dd, d.data(), d.size() * sizeof(EpiDesc<T>), hipMemcpyHostToDevice));
      BCHK(hipMemcpy(di, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
      b->d_epi.push_back(dd);
      b->d_epi_items.push_back((int2*)di);
      b->epi_items.push_back((int)items.size());
    }
    b->prepared = true;
    return ELPH_OK;
  }
  auto cost1 = [&](const int4& w) { return b->ctx[w.x]->ke; };
  b->s1_sorted = b->s1_natural;
  std::stable_sort(b->s1_sorted.begin(), b->s1_sorted.end(),
                   [&](const int4& a, const int4& c) { return cost1(a) > cost1(c); });
  if (balloc(b, &b->d_s1desc, n * sizeof(S1Desc<T>)) != hipSuccess ||
      balloc(b, (void**)&b->d_s1items, b->s1_natural.size() * sizeof(int4)) != hipSuccess ||
      balloc(b, (void**)&b->d_counters, 64 * sizeof(int)) != hipSuccess) {
    b->err = "batch allocation failed";
    return ELPH_ENOMEM;
  }
  BCHK(hipMemcpy(b->d_s1desc, s1.data(), n * sizeof(S1Desc<T>), hipMemcpyHostToDevice));
  for (auto& cl : b->cls) {
    std::vector<S2Desc<T>> d(cl.mats.size());
    for (size_t slot = 0; slot < cl.mats.size(); ++slot) {
      const int m = cl.mats[slot];
      elph_ctx c = b->ctx[m];
      S2Desc<T>& e = d[slot];
      e.kp = c->kp;
      e.Ap = (const T*)c->d_Ap;
      e.B2 = (const T*)c->d_B2;
      e.Bp = c->d_Bp;
      e.Bm = c->d_Bm;
      e.ep = epi_params(c);
      e.ep.lomf = b->th[m].lomf;
      e.ep.fstate = b->th[m].f;
      e.ep.omf = b->th[m].omf;
      e.ep.nocc = b->th[m].nocc;
      e.ep.we_part = c->d_we_part;
      for (int64_t by = 0; by < c->m_pad / 32; ++by)
        for (int64_t bx = 0; bx < c->m_pad / 32; ++bx) cl.natural.push_back(make_int4((int)slot, (int)bx, (int)by, 0));
    }
    cl.sorted = cl.natural;
    std::stable_sort(cl.sorted.begin(), cl.sorted.end(), [&](const int4& a, const int4& c2) {
      return b->ctx[cl.mats[a.x]]->kp > b->ctx[cl.mats[c2.x]]->kp;
    });
    if (balloc(b, &cl.d_desc, d.size() * sizeof(S2Desc<T>)) != hipSuccess ||
        balloc(b, (void**)&cl.d_items, cl.natural.size() * sizeof(int4)) != hipSuccess) {
      b->err = "batch allocation failed";
      return ELPH_ENOMEM;
    }
    BCHK(hipMemcpy(cl.d_desc, d.data(), d.size() * sizeof(S2Desc<T>), hipMemcpyHostToDevice));
  }
  b->prepared = true;
  return ELPH_OK;
}

static elph_status batch_upload_order(BatchImpl* b) {
  if (b->gemm) {
    const int h = b->wr == 2 ? 0 : 1;
    const std::vector<int4>& a = b->sorted ? b->g1_sorted[h] : b->g1_natural[h];
    const std::vector<int4>& c = b->sorted ? b->g2_sorted[h] : b->g2_natural[h];
    BCHK(hipMemcpy(b->d_g1items, a.data(), a.size() * sizeof(int4), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(b->d_g2items, c.data(), c.size() * sizeof(int4), hipMemcpyHostToDevice));
    return ELPH_OK;
  }
  const std::vector<int4>& s1 = b->sorted ? b->s1_sorted : b->s1_natural;
  BCHK(hipMemcpy(b->d_s1items, s1.data(), s1.size() * sizeof(int4), hipMemcpyHostToDevice));
  for (auto& cl : b->cls) {
    const std::vector<int4>& it = b->sorted ? cl.sorted : cl.natural;
    BCHK(hipMemcpy(cl.d_items, it.data(), it.size() * sizeof(int4), hipMemcpyHostToDevice));
  }
  return ELPH_OK;
}

template <typename T, typename ST>
static elph_status batch_launch_step2(BatchImpl* b, BatchImpl::Cls& cl, int* counter) {
  const int nitems = (int)cl.natural.size();
  const unsigned grid = (unsigned)std::min<int64_t>(nitems, (int64_t)b->bpc * b->ncu);
  const S2Desc<T>* d = (const S2Desc<T>*)cl.d_desc;
#define S2P(NXV)                                                                                              \
  hipLaunchKernelGGL((k_step2_persist<T, ST, NXV>), dim3(grid), dim3(256), 0, b->stream, d, cl.d_items, nitems, \
                     counter)
  switch (cl.nx) {
    case 3: S2P(3); break;
    case 6: S2P(6); break;
    case 9: S2P(9); break;
    case 12: S2P(12); break;
    case 15: S2P(15); break;
    default: b->err = "unsupported branch count"; return ELPH_EINVAL;
  }
#undef S2P
  return ELPH_OK;
}


// GEMM forms: two persistent GEMM launches over all materials, each
// material's step-1 and step-2 epilogues, W_e from the store rows and W_ph.
template <typename T>
static elph_status batch_sequence_gemm(BatchImpl* b, double T_K, double* const* we, double* const* wph) {
  typedef T ST;
  typedef typename GemmOp<T>::type OP;
  const int n = (int)b->ctx.size();
  StreamSwap sw(b);
  for (int m = 0; m < n; ++m) fill_thermal(b->ctx[m], T_K, b->th[m], b->stream);
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, b->stream, b->d_counters, 64);
  const int h = b->wr == 2 ? 0 : 1;
  const int n1 = (int)b->g1_natural[h].size(), n2 = (int)b->g2_natural[h].size();
  const unsigned g1b = (unsigned)std::min<int64_t>(n1, (int64_t)b->bpc * b->ncu);
  const unsigned g2b = (unsigned)std::min<int64_t>(n2, (int64_t)b->bpc * b->ncu);
  if (b->wr == 2)
    hipLaunchKernelGGL((k_cgemm_persist<OP, 1, 2>), dim3(g1b), dim3(256), 0, b->stream, (const GemmArgs*)b->d_g1,
                       b->d_g1items, n1, b->d_counters);
  else
    hipLaunchKernelGGL((k_cgemm_persist<OP, 1, 4>), dim3(g1b), dim3(512), 0, b->stream, (const GemmArgs*)b->d_g1,
                       b->d_g1items, n1, b->d_counters);
  hipLaunchKernelGGL(k_step1_epi_persist<T>, dim3((unsigned)std::min<int64_t>(b->s1blocks, 8 * (int64_t)b->ncu)),
                     dim3(256), 0, b->stream, (const S1EpiDesc<T>*)b->d_s1epi, b->d_s1boff, n, b->s1blocks);
  if (b->wr == 2)
    hipLaunchKernelGGL((k_cgemm_persist<OP, 2, 2>), dim3(g2b), dim3(256), 0, b->stream, (const GemmArgs*)b->d_g2,
                       b->d_g2items, n2, b->d_counters + 1);
  else
    hipLaunchKernelGGL((k_cgemm_persist<OP, 2, 4>), dim3(g2b), dim3(512), 0, b->stream, (const GemmArgs*)b->d_g2,
                       b->d_g2items, n2, b->d_counters + 1);
  for (size_t ci = 0; ci < b->cls.size(); ++ci) {
    const unsigned eg = (unsigned)std::min<int64_t>(b->epi_items[ci], 8 * (int64_t)b->ncu);
    const EpiDesc<ST>* d = (const EpiDesc<ST>*)b->d_epi[ci];
#define EQP(NXV) \
  hipLaunchKernelGGL((k_epi_q_persist<ST, NXV>), dim3(eg), dim3(256), 0, b->stream, d, b->d_epi_items[ci], b->epi_items[ci])
    switch (b->cls[ci].nx) {
      case 3: EQP(3); break;
      case 6: EQP(6); break;
      case 9: EQP(9); break;
      case 12: EQP(12); break;
      case 15: EQP(15); break;
      default: b->err = "unsupported branch count"; return ELPH_EINVAL;
    }
#undef EQP
  }
  for (int m = 0; m < n; ++m) {
    elph_ctx c = b->ctx[m];
    launch_we_rows<ST>(c, (const ST*)c->d_Bp, (const ST*)c->d_Bm, b->th[m].lomf, b->th[m].nocc, c->d_we_part);
    double* wout = (we && we[m]) ? we[m] : b->we_tmp[m];
    hipLaunchKernelGGL(k_reduce_we, dim3(blocks_for(c->nstates, 256)), dim3(256), 0, b->stream, c->d_we_part,
                       (int64_t)1, c->m_pad, c->nstates, wout);
    if (wph && wph[m]) {
      launch_q_gather<ST, 1>(c, (const ST*)c->d_Bp, b->th[m].f, b->th[m].omf, nullptr, b->acc[m]);
      elph_status st = finalize_wph(c, b->th[m], b->acc[m], wph[m]);
      if (st != ELPH_OK) return st;
    }
  }
  BCHK(hipGetLastError());
  return ELPH_OK;
}

// The per-temperature sequence (no synchronisation, no allocation: safe to capture).
template <typename T>
static elph_status batch_sequence(BatchImpl* b, double T_K, double* const* we, double* const* wph) {
  typedef T ST;  // the store keeps the precision of the contraction
  if constexpr (UsesGemm<T>::value) return batch_sequence_gemm<T>(b, T_K, we, wph);
  const int n = (int)b->ctx.size();
  StreamSwap sw(b);
  for (int m = 0; m < n; ++m) fill_thermal(b->ctx[m], T_K, b->th[m], b->stream);
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, b->stream, b->d_counters, 64);
  const int n1 = (int)b->s1_natural.size();
  hipLaunchKernelGGL(k_step1_persist<T>, dim3((unsigned)std::min<int64_t>(n1, (int64_t)b->bpc * b->ncu)),
                     dim3(256), 0, b->stream, (const S1Desc<T>*)b->d_s1desc, b->d_s1items, n1, b->d_counters);
  for (size_t c = 0; c < b->cls.size(); ++c) {
    elph_status st = batch_launch_step2<T, ST>(b, b->cls[c], b->d_counters + 1 + c);
    if (st != ELPH_OK) return st;
  }
  for (int m = 0; m < n; ++m) {
    elph_ctx c = b->ctx[m];
    // W_e from the store rows, as elph_scatt_rates reduces it
    if (we && we[m])
      launch_we_rows<ST>(c, (const ST*)c->d_Bp, (const ST*)c->d_Bm, b->th[m].lomf, b->th[m].nocc, we[m]);
    if (wph && wph[m]) {
      launch_q_gather<ST, 1>(c, (const ST*)c->d_Bp, b->th[m].f, b->th[m].omf, nullptr, b->acc[m]);
      elph_status st = finalize_wph(c, b->th[m], b->acc[m], wph[m]);
      if (st != ELPH_OK) return st;
    }
  }
  BCHK(hipGetLastError());
  return ELPH_OK;
}

BatchImpl* batch_new(const std::vector<elph_ctx>& ctxs, std::string* err) {
  BatchImpl* b = new (std::nothrow) BatchImpl();
  if (!b) {
    *err = "host allocation failed";
    return nullptr;
  }
  b->ctx = ctxs;
  for (elph_ctx c : ctxs) b->saved_streams.push_back(c->stream);
  b->precision = ctxs[0]->precision;
  for (elph_ctx c : ctxs)
    if (c->precision != b->precision || c->hip_dead ||
        (b->precision != ELPH_FP64 && b->precision != ELPH_FP32)) {
      *err = "batch contexts must share the FP64 or the FP32 form and be usable";
      delete b;
      return nullptr;
    }
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    *err = "stream creation failed";
    delete b;
    return nullptr;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->ncu = prop.multiProcessorCount;
  return b;
}

void batch_free(BatchImpl* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* p : b->allocs) (void)hipFree(p);
  for (size_t m = 0; m < b->ctx.size(); ++m) {
    free_thermal(b->ctx[m], &b->th[m]);
    dev_free(b->ctx[m], b->acc[m]);
    dev_free(b->ctx[m], b->we_tmp[m]);
  }
  (void)hipStreamDestroy(b->stream);
  delete b;
}

static elph_status batch_prepare(BatchImpl* b) {
  if (b->prepared) return ELPH_OK;
  elph_status st = b->precision == ELPH_FP64 ? batch_prepare_t<double>(b) : batch_prepare_t<float>(b);
  if (st != ELPH_OK) return st;
  auto it = tune_cache().find(batch_signature(b));
  if (it != tune_cache().end()) {
    b->bpc = it->second.bpc;
    b->sorted = it->second.sorted;
    b->wr = it->second.wr;
    b->tuned = true;
  }
  return batch_upload_order(b);
}

static elph_status batch_run(BatchImpl* b, double T_K, double* const* we, double* const* wph) {
  return b->precision == ELPH_FP64 ? batch_sequence<double>(b, T_K, we, wph)
                                   : batch_sequence<float>(b, T_K, we, wph);
}

elph_status batch_rates(BatchImpl* b, double T_K, double* const* we, double* const* wph, bool use_graph) {
  elph_status st = batch_prepare(b);
  if (st != ELPH_OK) return st;
  const int n = (int)b->ctx.size();
  if (!use_graph) {
    st = batch_run(b, T_K, we, wph);
    if (st != ELPH_OK) return st;
  } else {
    std::vector<double*> key;
    for (int m = 0; m < n; ++m) {
      key.push_back(we ? we[m] : nullptr);
      key.push_back(wph ? wph[m] : nullptr);
    }
    if (!b->gexec || b->gT != T_K || key != b->gptrs) {
      if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->gexec = nullptr;
      b->graph = nullptr;
      BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      st = batch_run(b, T_K, we, wph);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (st != ELPH_OK) return st;
      BCHK(e);
      b->graph = g;
      BCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
      b->gT = T_K;
      b->gptrs = key;
    }
    BCHK(hipGraphLaunch(b->gexec, b->stream));
  }
  BCHK(hipStreamSynchronize(b->stream));
  for (elph_ctx c : b->ctx) c->store_ready = true;
  return ELPH_OK;
}

// Autotuner: time every launch shape of the persistent contractions (blocks
// per CU 1, 2, 4, 8 x item order x, in the GEMM forms, tile height 64 or
// 128 rows) on this batch and keep the fastest for its signature.  Every
// shape computes each output exactly as any other (the k order of a sum
// does not depend on the tile), so the choice changes time only.
static elph_status batch_time_shape(BatchImpl* b, double T_K, hipEvent_t e0, hipEvent_t e1, double* ms_out) {
  elph_status st = batch_upload_order(b);
  if (st != ELPH_OK) return st;
  st = batch_run(b, T_K, nullptr, nullptr);  // warm
  if (st != ELPH_OK) return st;
  BCHK(hipEventRecord(e0, b->stream));
  for (int rep = 0; rep < 2; ++rep) {
    st = batch_run(b, T_K, nullptr, nullptr);
    if (st != ELPH_OK) return st;
  }
  BCHK(hipEventRecord(e1, b->stream));
  BCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  BCHK(hipEventElapsedTime(&ms, e0, e1));
  *ms_out = ms / 2.0;
  return ELPH_OK;
}

elph_status batch_set_shape(BatchImpl* b, int bpc, bool sorted, int wr) {
  elph_status st = batch_prepare(b);
  if (st != ELPH_OK) return st;
  if ((bpc != 1 && bpc != 2 && bpc != 4 && bpc != 8) || (wr != 2 && wr != 4) || (!b->gemm && wr != kGemmWR)) {
    b->err = "launch shape: blocks per CU 1, 2, 4 or 8; tile rows 64 or 128 (FP32 batches; 128 in FP64)";
    return ELPH_EINVAL;
  }
  b->bpc = bpc;
  b->sorted = sorted;
  b->wr = wr;
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  return batch_upload_order(b);
}

elph_status batch_tune(BatchImpl* b, double T_K, int* choice, double* best_ms) {
  elph_status st = batch_prepare(b);
  if (st != ELPH_OK) return st;
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  double best = 1e300;
  BatchShape win{b->bpc, b->sorted, b->wr};
  const std::vector<int> heights = b->gemm ? std::vector<int>{2, 4} : std::vector<int>{kGemmWR};
  for (int wr : heights)
    for (int bpc : {1, 2, 4, 8})
      for (int so = 0; so < 2; ++so) {
        b->bpc = bpc;
        b->sorted = so == 1;
        b->wr = wr;
        double ms = 0.0;
        st = batch_time_shape(b, T_K, e0, e1, &ms);
        if (st != ELPH_OK) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return st;
        }
        if (ms < best) {
          best = ms;
          win = BatchShape{bpc, so == 1, wr};
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->bpc = win.bpc;
  b->sorted = win.sorted;
  b->wr = win.wr;
  b->tuned = true;
  tune_cache()[batch_signature(b)] = win;
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  if (choice) {
    choice[0] = win.bpc;
    choice[1] = win.sorted ? 1 : 0;
    choice[2] = 32 * win.wr;
  }
  if (best_ms) *best_ms = best;
  return batch_upload_order(b);
}

const std::string& batch_error(BatchImpl* b) { return b->err; }

}  // namespace elph
