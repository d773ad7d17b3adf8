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
