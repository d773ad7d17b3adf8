// Internal device helpers shared by the vertex, rate and solver kernels.
#pragma once
#include "common.h"

namespace elph {

// Mesh index of q = k_j - k_i (mod the mesh); mesh indexes are below 2^31,
// so the arithmetic is 32-bit.
__device__ inline int q_between(int kj, int ki, int n0, int n1, int n2) {
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

// Mesh index of -q
__device__ inline int q_neg(int q, int n0, int n1, int n2) {
  const unsigned uq = (unsigned)q, u2 = (unsigned)n2, u1 = (unsigned)n1;
  const unsigned t = uq / u2;
  int c = (int)(uq - t * u2);
  const unsigned a0 = t / u1;
  int b = (int)(t - a0 * u1);
  int a = (int)a0;
  a = a ? n0 - a : 0;
  b = b ? n1 - b : 0;
  c = c ? n2 - c : 0;
  return (a * n1 + b) * n2 + c;
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

// Log code of the relative error estimate r of a stored |g|^2 in the GEMM
// forms: code 0 marks an exact (FP64-refined) term, code c >= 1 stands for
// r = 2^((c - 1)/6 - 42) (rounded up; 1.26 and above saturate at 255).  d2
// is the squared error scale of g and g2 = |g|^2: r = 2 sqrt(d2/g2) + d2/g2.
// An estimate needs no more than FP32 and the hardware log2.
__device__ inline uint32_t rho_encode(float d2, float g2) {
  if (!(g2 > 0.f)) return d2 > 0.f ? 255u : 1u;
  const float t = d2 / g2;
  const float r = 2.f * sqrtf(t) + t;
  if (!(r > 0.f)) return 1u;
  const float c = ceilf(6.f * (__log2f(r) + 42.f)) + 1.f;
  return (uint32_t)fminf(fmaxf(c, 1.f), 255.f);
}

// bytes per pair (i, j) of the code array for NX branches
template <int NX>
struct RhoStride {
  static constexpr int value = NX <= 8 ? 8 : 16;
};

// The codes of one pair, read with one 8- or 16-byte load
template <int NX>
struct PairCodes {
  uint32_t w[RhoStride<NX>::value / 4];
  __device__ inline void load(const uint8_t* p) {
    if constexpr (RhoStride<NX>::value == 8) {
      const uint2 v = *reinterpret_cast<const uint2*>(p);
      w[0] = v.x;
      w[1] = v.y;
    } else {
      const uint4 v = *reinterpret_cast<const uint4*>(p);
      w[0] = v.x;
      w[1] = v.y;
      w[2] = v.z;
      w[3] = v.w;
    }
  }
  __device__ inline unsigned operator[](int s) const { return (w[s >> 2] >> (8 * (s & 3))) & 255u; }
};

__device__ inline double rho_decode(unsigned c) { return c ? exp2((double)(c - 1) * (1.0 / 6.0) - 42.0) : 0.0; }


// Two adjacent values of T as one 8- or 16-byte access
template <typename T>
struct Two;
template <>
struct Two<float> {
  typedef float2 type;
};
template <>
struct Two<double> {
  typedef double2 type;
};

// v[0..N) converted to T and stored at p, in pairs when N is even (p is
// then aligned to two elements, as every row of N elements of an array of T
// is)
template <typename T, int N>
__device__ inline void store_row(T* p, const double (&v)[N]) {
  if constexpr (N % 2 == 0) {
    typedef typename Two<T>::type T2;
#pragma unroll
    for (int s = 0; s < N; s += 2) {
      T2 w;
      w.x = (T)v[s];
      w.y = (T)v[s + 1];
      *reinterpret_cast<T2*>(p + s) = w;
    }
  } else {
#pragma unroll
    for (int s = 0; s < N; ++s) p[s] = (T)v[s];
  }
}

}  // namespace elph
