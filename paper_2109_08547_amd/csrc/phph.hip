// Three-phonon processes: the vertex V of Eq. 13, the transition rates W+-
// of Eq. 14 and the three-phonon part of the phonon RTA rate of Eq. 26.
//
// V-(q s, q' s', q'' s''), q'' = q - q', is a sum over the third-order force
// constants Psi(0 x_i, R_j x_j, R_k x_k) (x = 3 atom + Cartesian) of
//   E_q[x_i][s] exp(-2 pi i q'.R_j) E_{-q'}[x_j][s'] exp(-2 pi i q''.R_k) E_{-q''}[x_k][s'']
// with E = u / sqrt(M) the eigendisplacement columns (u the eigenvectors of
// D).  It is computed in two stages:
//   fold   (per mesh point P, per distinct R_j):
//     Phi[P][j][x_i][x_j][s''] = sum_{entries with R_j} exp(-2 pi i P.R_k)
//                                sum_{x_k} Psi[x_i][x_j][x_k] E_{-P}[x_k][s'']
//   rows   (per q, over every q'):
//     A[x_i][x_j][s''] = sum_j exp(-2 pi i q'.R_j) Phi[q - q'][j][x_i][x_j][s'']
//     B[x_i][s'][s'']  = sum_{x_j} E_{-q'}[x_j][s'] A[x_i][x_j][s'']
//     V[s][s'][s'']    = sum_{x_i} E_q[x_i][s] B[x_i][s'][s'']
// One V-(q, q') serves both processes of the row: the decay q -> q' + q''
// and, through |V+(q, -q', q'')| = |V-(q, q', q'')| (the identity the paper
// states below Eq. 13), the absorption q + (-q') -> q''; omega and n at -q'
// equal those at q'.
//
// Three row kernels evaluate the pair sums: k_phph_tile (one or two atoms, at
// most 32 distinct R_j: the slab of one q'' in registers, reused by a tile of
// 16 rows), k_phph_wide (one or two atoms, more R_j: the R_j sum in chunks)
// and k_phph_rows (any atom count: block per (q, q' chunk), the slab read per
// pair).  Each has a rates mode and a field mode (the in-scattering of Eq. 26).
#include "vertex.h"
#include "devutil.h"
#include "tables.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <vector>

namespace elph {

namespace {

constexpr int kFoldEnt = 64;   // entries of one R_j group staged in LDS per pass
constexpr int kMaxGroups = 256;  // distinct R_j

// hbar^5 e^3 / (amu^3 Angstrom^6) written through SI quantities:
// hbar[J s] hbar[eV s]^4 e[C]^2 / (amu[kg]^3 Angstrom[m]^6)
constexpr double kPhPhC =
    kHbarJs * kHbarEVs * kHbarEVs * kHbarEVs * kHbarEVs * kCharge * kCharge /
    (kAmuKg * kAmuKg * kAmuKg * kAngM * kAngM * kAngM * kAngM * kAngM * kAngM);

struct PhaseTab {
  const double2* t0;
  const double2* t1;
  const double2* t2;
  int n0, n1, n2;
  // exp(-2 pi i P . R) for the mesh point P (linear index) and integer R
  __device__ inline cd neg(int P, int r0, int r1, int r2) const {
    const int c = P % n2, t = P / n2, b = t % n1, a = t / n1;
    int i0 = (int)(((int64_t)a * r0) % n0); if (i0 < 0) i0 += n0;
    int i1 = (int)(((int64_t)b * r1) % n1); if (i1 < 0) i1 += n1;
    int i2 = (int)(((int64_t)c * r2) % n2); if (i2 < 0) i2 += n2;
    const double2 p0 = t0[i0], p1 = t1[i1], p2 = t2[i2];
    const cd z = cmul(cmul(cmake(p0.x, p0.y), cmake(p1.x, p1.y)), cmake(p2.x, p2.y));
    return cconj(z);
  }
};

// E[x][s] = u[x][s] / sqrt(M_x) from the table l_{x,s} u[x][s] (zero for
// modes below omega_min) and hbar omega: l = sqrt(C / (2 M hbar omega)).
__device__ inline cd edisp(const cd* Lq, const double* hw, int64_t q, int nbr, int x, int s) {
  const double w = hw[q * nbr + s];
  const cd L = Lq[(q * nbr + x) * nbr + s];
  return w > 0.0 ? cscale(L, sqrt(2.0 * w / kPhononC)) : cmake(0.0, 0.0);
}

// fold: block (P, j), threads over (x_i, x_j, s'')
template <int NBR>
__global__ __launch_bounds__(256) void k_ifc3_fold(PhaseTab ph, const int32_t* __restrict__ goff,
                                                   const int32_t* __restrict__ rk, const double* __restrict__ psi,
                                                   const cd* __restrict__ Lq, const double* __restrict__ hw,
                                                   int ng, cd* __restrict__ phi) {
  constexpr int N2 = NBR * NBR, N3 = N2 * NBR;
  __shared__ cd em[N2];          // E_{-P}[x_k][s'']
  __shared__ cd pe[kFoldEnt];    // exp(-2 pi i P.R_k) of the staged entries
  const int P = blockIdx.x, j = blockIdx.y;
  const MeshDims md{ph.n0, ph.n1, ph.n2};
  const int mP = q_neg(P, md.n0, md.n1, md.n2);
  for (int t = threadIdx.x; t < N2; t += blockDim.x) em[t] = edisp(Lq, hw, mP, NBR, t / NBR, t % NBR);
  const int e0 = goff[j], e1 = goff[j + 1];
  cd acc[(N3 + 255) / 256];
#pragma unroll
  for (int r = 0; r < (N3 + 255) / 256; ++r) acc[r] = cmake(0.0, 0.0);
  for (int eb = e0; eb < e1; eb += kFoldEnt) {
    const int ne = min(kFoldEnt, e1 - eb);
    __syncthreads();
    for (int t = threadIdx.x; t < ne; t += blockDim.x)
      pe[t] = ph.neg(P, rk[3 * (eb + t)], rk[3 * (eb + t) + 1], rk[3 * (eb + t) + 2]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (N3 + 255) / 256; ++r) {
      const int o = threadIdx.x + 256 * r;
      if (o < N3) {
        const int xij = o / NBR, s3 = o - xij * NBR;
        for (int e = 0; e < ne; ++e) {
          const double* row = psi + ((int64_t)(eb + e) * N2 + xij) * NBR;
          cd t = cmake(0.0, 0.0);
#pragma unroll
          for (int xk = 0; xk < NBR; ++xk) {
            const cd m = em[xk * NBR + s3];
            t.x += row[xk] * m.x;
            t.y += row[xk] * m.y;
          }
          acc[r] = cadd(acc[r], cmul(pe[e], t));
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < (N3 + 255) / 256; ++r) {
    const int o = threadIdx.x + 256 * r;
    if (o < N3) phi[((int64_t)P * ng + j) * N3 + o] = acc[r];
  }
}

// Shared stages of the row and vertex kernels for one pair (q, q'):
// V[s][s'][s''] into A (LDS, N3; A is free once B is formed), with
// eq = E_q and ex = E_{-q'} staged.
template <int NBR>
__device__ inline void pair_vertex(const PhaseTab& ph, int qp, int qpp, int ng, const int32_t* gr,
                                   const cd* __restrict__ phi, const cd* eq, const cd* ex, cd* pg, cd* A, cd* B) {
  constexpr int N2 = NBR * NBR, N3 = N2 * NBR;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) pg[g] = ph.neg(qp, gr[3 * g], gr[3 * g + 1], gr[3 * g + 2]);
  __syncthreads();
  const cd* src = phi + (int64_t)qpp * ng * N3;
  for (int o = threadIdx.x; o < N3; o += blockDim.x) {
    cd a = cmake(0.0, 0.0);
    for (int g = 0; g < ng; ++g) a = cadd(a, cmul(pg[g], src[(int64_t)g * N3 + o]));
    A[o] = a;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < N3; o += blockDim.x) {   // o = (x_i, s', s'')
    const int xi = o / N2, r = o - xi * N2, s2 = r / NBR, s3 = r - s2 * NBR;
    cd b = cmake(0.0, 0.0);
#pragma unroll
    for (int xj = 0; xj < NBR; ++xj) b = cadd(b, cmul(ex[xj * NBR + s2], A[(xi * NBR + xj) * NBR + s3]));
    B[o] = b;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < N3; o += blockDim.x) {   // o = (s, s', s'')
    const int s1 = o / N2, r = o - s1 * N2;
    cd v = cmake(0.0, 0.0);
#pragma unroll
    for (int xi = 0; xi < NBR; ++xi) v = cadd(v, cmul(eq[xi * NBR + s1], B[xi * N2 + r]));
    A[o] = v;
  }
  __syncthreads();
}

template <int NBR>
struct PairLds {
  cd eq[NBR * NBR];
  cd ex[NBR * NBR];
  cd pg[kMaxGroups];
  cd A[NBR * NBR * NBR];   // A, then V once B is formed
  cd B[NBR * NBR * NBR];
};

// |V-(q s, q' s', q'' s'')|^2 for a list of pairs: block per pair
template <int NBR>
__global__ __launch_bounds__(256) void k_phph_vertex(PhaseTab ph, int64_t npairs, const int32_t* __restrict__ qs,
                                                     const int32_t* __restrict__ qps, const int32_t* __restrict__ gr,
                                                     int ng, const cd* __restrict__ phi, const cd* __restrict__ Lq,
                                                     const double* __restrict__ hw, double* __restrict__ V2) {
  constexpr int N2 = NBR * NBR, N3 = N2 * NBR;
  __shared__ PairLds<NBR> L;
  const int64_t p = blockIdx.x;
  const int q = qs[p], qp = qps[p];
  const int nq = ph.n0 * ph.n1 * ph.n2;
  if (q < 0 || q >= nq || qp < 0 || qp >= nq) {   // uniform over the block: no barrier skipped
    for (int o = threadIdx.x; o < N3; o += blockDim.x) V2[p * N3 + o] = __builtin_nan("");
    return;
  }
  const MeshDims md{ph.n0, ph.n1, ph.n2};
  const int mqp = q_neg(qp, md.n0, md.n1, md.n2), qpp = q_between(q, qp, md.n0, md.n1, md.n2);
  for (int t = threadIdx.x; t < N2; t += blockDim.x) {
    L.eq[t] = edisp(Lq, hw, q, NBR, t / NBR, t % NBR);
    L.ex[t] = edisp(Lq, hw, mqp, NBR, t / NBR, t % NBR);
  }
  pair_vertex<NBR>(ph, qp, qpp, ng, gr, phi, L.eq, L.ex, L.pg, L.A, L.B);
  for (int o = threadIdx.x; o < N3; o += blockDim.x) V2[p * N3 + o] = cabs2(L.A[o]);
}

// Rates of one q over a chunk of q': block (q, chunk).  Thread t < NBR^2
// owns the branch pair (s', s'') = t and sums, per s, over the chunk
//   |V|^2 n'' [(1 + n') delta(E + E' - E'') + n' delta(E - E' - E'') / 2] / (E' E'')
// into part[chunk][q][s]; the constant factors follow in k_phph_finish.
// With NC = 3 the same terms weight the field F [nq][NBR][3] as the
// in-scattering of Eq. 26 does (part[chunk][q][s][c]).
template <int NBR, int NC>
__global__ __launch_bounds__(256) void k_phph_rows(PhaseTab ph, int nq, int chunk, const int32_t* __restrict__ gr,
                                                   int ng, const cd* __restrict__ phi, const cd* __restrict__ Lq,
                                                   const double* __restrict__ hw, double kT, double omega_min,
                                                   double sigma, const double* __restrict__ F,
                                                   double* __restrict__ part) {
  constexpr int N2 = NBR * NBR, NV = NC ? NC : 1;
  __shared__ PairLds<NBR> L;
  __shared__ double e1[NBR], e2[NBR], n2[NBR], e3[NBR], n3[NBR];
  __shared__ double f2[NBR * NV], f2m[NBR * NV], f3[NBR * NV];   // F at q', -q', q'' (NC > 0)
  const int q = blockIdx.x;
  const int c0 = blockIdx.y * chunk, c1 = min(nq, c0 + chunk);
  const MeshDims md{ph.n0, ph.n1, ph.n2};
  for (int t = threadIdx.x; t < N2; t += blockDim.x) L.eq[t] = edisp(Lq, hw, q, NBR, t / NBR, t % NBR);
  if (threadIdx.x < NBR) e1[threadIdx.x] = hw[(int64_t)q * NBR + threadIdx.x];
  const double inv2s2 = 0.5 / (sigma * sigma), dnorm = 1.0 / (sqrt(2.0 * kPi) * sigma);
  double acc[NBR * NV];
#pragma unroll
  for (int s = 0; s < NBR * NV; ++s) acc[s] = 0.0;
  for (int qp = c0; qp < c1; ++qp) {
    const int mqp = q_neg(qp, md.n0, md.n1, md.n2), qpp = q_between(q, qp, md.n0, md.n1, md.n2);
    __syncthreads();  // the previous pair's readers are done with ex, e2, e3
    for (int t = threadIdx.x; t < N2; t += blockDim.x) L.ex[t] = edisp(Lq, hw, mqp, NBR, t / NBR, t % NBR);
    if (threadIdx.x < NBR) {
      const int s = threadIdx.x;
      const double w2 = hw[(int64_t)qp * NBR + s], w3 = hw[(int64_t)qpp * NBR + s];
      e2[s] = w2 >= omega_min ? w2 : 0.0;
      e3[s] = w3 >= omega_min ? w3 : 0.0;
      n2[s] = w2 >= omega_min ? 1.0 / expm1(w2 / kT) : 0.0;
      n3[s] = w3 >= omega_min ? 1.0 / expm1(w3 / kT) : 0.0;
    }
    if constexpr (NC > 0) {
      for (int t = threadIdx.x; t < NBR * NC; t += blockDim.x) {
        f2[t] = F[(int64_t)qp * NBR * NC + t];
        f2m[t] = F[(int64_t)mqp * NBR * NC + t];
        f3[t] = F[(int64_t)qpp * NBR * NC + t];
      }
    }
    pair_vertex<NBR>(ph, qp, qpp, ng, gr, phi, L.eq, L.ex, L.pg, L.A, L.B);
    const int t = threadIdx.x;
    if (t < N2) {
      const int s2 = t / NBR, s3 = t - s2 * NBR;
      const double E2 = e2[s2], E3 = e3[s3];
      if (E2 > 0.0 && E3 > 0.0) {
        const double f = n3[s3] / (E2 * E3), np2 = n2[s2];
#pragma unroll
        for (int s1 = 0; s1 < NBR; ++s1) {
          const double E1 = e1[s1];
          const double dp = E1 + E2 - E3, dm = E1 - E2 - E3;
          const double b = cabs2(L.A[s1 * N2 + t]) * f * dnorm;
          const double wp = b * (1.0 + np2) * exp(-dp * dp * inv2s2);   // absorption with -q'
          const double wm = b * 0.5 * np2 * exp(-dm * dm * inv2s2);     // decay into q', half
          if constexpr (NC == 0) {
            acc[s1] += wp + wm;
          } else {
#pragma unroll
            for (int k = 0; k < NC; ++k)
              acc[s1 * NC + k] += wp * (f3[s3 * NC + k] - f2m[s2 * NC + k]) + wm * (f3[s3 * NC + k] + f2[s2 * NC + k]);
          }
        }
      }
    }
  }
  // sum over the branch pairs: the N2 <= 144 owners sit in the first waves
  __syncthreads();
  double* red = reinterpret_cast<double*>(L.B);   // 4 wave partials per value (2 N3 >= 4 NBR NV doubles)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < NBR * NV; ++s) {
    double x = acc[s];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[s * 4 + wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < NBR * NV) {
    const int s = threadIdx.x;
    part[((int64_t)blockIdx.y * nq + q) * NBR * NV + s] =
        (red[s * 4] + red[s * 4 + 1]) + (red[s * 4 + 2] + red[s * 4 + 3]);
  }
}

// a + b c in four fused multiply-adds
__device__ inline cd cfma(cd a, cd b, cd c) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(-b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(b.y, c.x, a.y);
  return a;
}

// n(hbar omega) of every mode, 0 below omega_min
__global__ void k_phph_bose(int64_t n, const double* __restrict__ hw, double kT, double omega_min,
                            double* __restrict__ nb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double w = hw[e];
  nb[e] = w >= omega_min ? 1.0 / expm1(w / kT) : 0.0;
}

// The same sums with the fold slab of one q'' held in registers: block
// (q tile, q'' range); for every q'' = P of its range each thread o < N3
// loads Phi[P][.][o] once, multiplies it by exp(2 pi i P.R_j) and reuses it
// for the TQ rows q of the tile, whose phases exp(-2 pi i q'.R_j) (q' = q - P)
// are then exp(-2 pi i q.R_j) (fixed for the block) times that factor.
// E_{-q'} (-q' = P - q), omega' and n' are staged for the whole tile per P;
// A, B and V pass through LDS QB = 4 rows at a time, and in the rate
// epilogue wave r owns row r (lanes over (s', s'')), reducing by shuffles.
// Partial sums per row and branch go to part[range][q][s].  For N3 = nbr^3
// <= 256 (one or two atoms).
constexpr int kTQ = 16, kQB = 4, kMaxG = 32;

template <int NBR, int NC, int NGP>
struct TileLds {
  cd exq[kTQ][NBR * NBR];      // E_q of the tile's rows
  cd exd[kTQ][NBR * NBR];      // E_{-q'} of the rows for the current q''
  cd tq[kTQ][NGP];             // exp(-2 pi i q.R_j) of the tile's rows (zero beyond ng)
  cd tP[NGP];                  // exp(+2 pi i P.R_j) (zero beyond ng)
  cd A[kQB][NBR * (NBR == 6 ? 38 : NBR * NBR)];  // A, then V; rows of x_i (or s) padded to 38 for bank spread
  cd B[kQB][NBR * NBR * NBR];
  double e1[kTQ][NBR];
  double e2[kTQ][NBR], n2[kTQ][NBR];
  double e3[NBR], n3[NBR];
  double acc[kTQ][NBR * (NC ? NC : 1)];
  double f3[NBR * (NC ? NC : 1)];                 // F at q'' (NC > 0)
  double f2[NC ? kTQ : 1][NBR * (NC ? NC : 1)];   // F at q'
  double f2m[NC ? kTQ : 1][NBR * (NC ? NC : 1)];  // F at -q'
};

template <int NBR, int NC, int NGP>
__global__ __launch_bounds__(256) void k_phph_tile(PhaseTab ph, int nq, int prange, const int32_t* __restrict__ gr,
                                                   int ng, const cd* __restrict__ phi, const cd* __restrict__ Lq,
                                                   const double* __restrict__ hw, const double* __restrict__ nbose,
                                                   double omega_min, double sigma, const double* __restrict__ F,
                                                   double* __restrict__ part) {
  constexpr int N2 = NBR * NBR, N3 = N2 * NBR, NV = NC ? NC : 1;
  constexpr int AS = NBR == 6 ? 38 : N2;  // stride of the leading index of A and V in LDS
  static_assert(N3 <= 256 && N2 <= 64 && kQB * 64 == 256, "one slab element per thread, one row per wave");
  __shared__ TileLds<NBR, NC, NGP> L;
  // rates: per-lane sums over the whole q'' range, one per sub-batch slot and branch
  double cacc[kTQ / kQB][NBR];
#pragma unroll
  for (int k = 0; k < kTQ / kQB; ++k)
#pragma unroll
    for (int s1 = 0; s1 < NBR; ++s1) cacc[k][s1] = 0.0;
  const int q0 = blockIdx.x * kTQ, nt = min(kTQ, nq - q0);
  const int P0 = blockIdx.y * prange, P1 = min(nq, P0 + prange);
  const MeshDims md{ph.n0, ph.n1, ph.n2};
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int t = tid; t < kTQ * N2; t += blockDim.x) {
    const int r = t / N2, e = t - r * N2;
    L.exq[r][e] = r < nt ? edisp(Lq, hw, q0 + r, NBR, e / NBR, e % NBR) : cmake(0.0, 0.0);
  }
  for (int t = tid; t < kTQ * NGP; t += blockDim.x) {
    const int r = t / NGP, g = t - r * NGP;
    L.tq[r][g] = (r < nt && g < ng) ? ph.neg(q0 + r, gr[3 * g], gr[3 * g + 1], gr[3 * g + 2]) : cmake(0.0, 0.0);
  }
  for (int t = tid; t < kTQ * NBR; t += blockDim.x) {
    const int r = t / NBR, s = t - r * NBR;
    L.e1[r][s] = r < nt ? hw[(int64_t)(q0 + r) * NBR + s] : 0.0;
  }
  for (int t = tid; t < kTQ * NBR * NV; t += blockDim.x) L.acc[t / (NBR * NV)][t % (NBR * NV)] = 0.0;
  const double inv2s2 = 0.5 / (sigma * sigma), dnorm = 1.0 / (sqrt(2.0 * kPi) * sigma);
  for (int P = P0; P < P1; ++P) {
    cd slab[NGP];
    const cd* src = phi + (int64_t)P * ng * N3 + tid;
#pragma unroll
    for (int g = 0; g < NGP; ++g) slab[g] = (g < ng && tid < N3) ? src[(int64_t)g * N3] : cmake(0.0, 0.0);
    __syncthreads();   // the previous q'' is done with exd, tP, e2, n2, e3, n3
    if (tid < NBR) {
      const double w3 = hw[(int64_t)P * NBR + tid];
      L.e3[tid] = w3 >= omega_min ? w3 : 0.0;
      L.n3[tid] = nbose[(int64_t)P * NBR + tid];
    }
    if (tid < NGP)
      L.tP[tid] = tid < ng ? cconj(ph.neg(P, gr[3 * tid], gr[3 * tid + 1], gr[3 * tid + 2])) : cmake(0.0, 0.0);
    for (int t = tid; t < kTQ * N2; t += blockDim.x) {
      const int r = t / N2, e = t - r * N2;
      cd v = cmake(0.0, 0.0);
      if (r < nt) v = edisp(Lq, hw, q_between(P, q0 + r, md.n0, md.n1, md.n2), NBR, e / NBR, e % NBR);
      L.exd[r][e] = v;
    }
    if constexpr (NC > 0) {
      for (int t = tid; t < NBR * NC; t += blockDim.x) L.f3[t] = F[(int64_t)P * NBR * NC + t];
      for (int t = tid; t < kTQ * NBR * NC; t += blockDim.x) {
        const int r = t / (NBR * NC), e = t - r * (NBR * NC);
        double a = 0.0, b = 0.0;
        if (r < nt) {
          a = F[(int64_t)q_between(q0 + r, P, md.n0, md.n1, md.n2) * NBR * NC + e];
          b = F[(int64_t)q_between(P, q0 + r, md.n0, md.n1, md.n2) * NBR * NC + e];
        }
        L.f2[r][e] = a;
        L.f2m[r][e] = b;
      }
    }
    for (int t = tid; t < kTQ * NBR; t += blockDim.x) {
      const int r = t / NBR, s = t - r * NBR;
      double w2 = 0.0, n2 = 0.0;
      if (r < nt) {
        const int64_t m = (int64_t)q_between(q0 + r, P, md.n0, md.n1, md.n2) * NBR + s;
        w2 = hw[m];
        n2 = nbose[m];
      }
      L.e2[r][s] = w2 >= omega_min ? w2 : 0.0;
      L.n2[r][s] = n2;
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NGP; ++g) slab[g] = cmul(L.tP[g], slab[g]);
    for (int rb = 0; rb < nt; rb += kQB) {
      if (tid < N3) {
#pragma unroll
        for (int r = 0; r < kQB; ++r) {
          cd a = cmake(0.0, 0.0);
#pragma unroll
          for (int g = 0; g < NGP; ++g) a = cfma(a, L.tq[rb + r][g], slab[g]);
          L.A[r][(tid / N2) * AS + tid % N2] = a;
        }
      }
      __syncthreads();
      for (int t = tid; t < kQB * N3; t += blockDim.x) {   // (r, x_i, s', s'')
        const int r = t / N3, o = t - r * N3;
        const int xi = o / N2, rr = o - xi * N2, s2 = rr / NBR, s3 = rr - s2 * NBR;
        cd b = cmake(0.0, 0.0);
#pragma unroll
        for (int xj = 0; xj < NBR; ++xj)
          b = cfma(b, L.exd[rb + r][xj * NBR + s2], L.A[r][xi * AS + xj * NBR + s3]);
        L.B[r][o] = b;
      }
      __syncthreads();
      for (int t = tid; t < kQB * N3; t += blockDim.x) {   // (r, s, s', s'')
        const int r = t / N3, o = t - r * N3;
        const int s1 = o / N2, rr = o - s1 * N2;
        cd v = cmake(0.0, 0.0);
#pragma unroll
        for (int xi = 0; xi < NBR; ++xi) v = cfma(v, L.exq[rb + r][xi * NBR + s1], L.B[r][xi * N2 + rr]);
        L.A[r][s1 * AS + rr] = v;
      }
      __syncthreads();
      {  // wave r: row rb + r, lane = (s', s'')
        const int r = wave;
        double c[NBR * NV];
#pragma unroll
        for (int k = 0; k < NBR * NV; ++k) c[k] = 0.0;
        if (lane < N2) {
          const int s2 = lane / NBR, s3 = lane - s2 * NBR;
          const double E2 = L.e2[rb + r][s2], E3 = L.e3[s3];
          if (E2 > 0.0 && E3 > 0.0) {
            const double f = L.n3[s3] / (E2 * E3) * dnorm, np2 = L.n2[rb + r][s2];
#pragma unroll
            for (int s1 = 0; s1 < NBR; ++s1) {
              const double E1 = L.e1[rb + r][s1];
              const double dp = E1 + E2 - E3, dm = E1 - E2 - E3;
              const double b = cabs2(L.A[r][s1 * AS + lane]) * f;
              const double wp = b * (1.0 + np2) * exp(-dp * dp * inv2s2);  // absorption with -q'
              const double wm = b * 0.5 * np2 * exp(-dm * dm * inv2s2);    // decay into q', half
              if constexpr (NC == 0) {
#pragma unroll
                for (int k = 0; k < kTQ / kQB; ++k) cacc[k][s1] += (k * kQB == rb) ? wp + wm : 0.0;
              } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                  const double F3 = L.f3[s3 * NC + k];
                  c[s1 * NC + k] = wp * (F3 - L.f2m[rb + r][s2 * NC + k]) + wm * (F3 + L.f2[rb + r][s2 * NC + k]);
                }
              }
            }
          }
        }
        if constexpr (NC > 0) {
#pragma unroll
          for (int k = 0; k < NBR * NV; ++k) {
            double x = c[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
            c[k] = x;
          }
        }
        if (NC > 0 && rb + r < nt) {
#pragma unroll
          for (int k0 = 0; k0 < NBR * NV; k0 += 64) {
            if (lane + k0 < NBR * NV) {
              double x = c[k0];
#pragma unroll
              for (int k = k0 + 1; k < NBR * NV && k < k0 + 64; ++k)
                if (lane + k0 == k) x = c[k];
              L.acc[rb + r][lane + k0] += x;
            }
          }
        }
      }
      __syncthreads();   // V (A) is rewritten by the next rows
    }
  }
  if constexpr (NC == 0) {
    // wave w holds row k kQB + w of every sub-batch slot k
#pragma unroll
    for (int k = 0; k < kTQ / kQB; ++k) {
#pragma unroll
      for (int s1 = 0; s1 < NBR; ++s1) {
        double x = cacc[k][s1];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        cacc[k][s1] = x;
      }
      const int row = k * kQB + wave;
      if (lane < NBR && row < nt) {
        double x = cacc[k][0];
#pragma unroll
        for (int s1 = 1; s1 < NBR; ++s1)
          if (lane == s1) x = cacc[k][s1];
        L.acc[row][lane] += x;
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < nt * NBR * NV; t += blockDim.x) {
    const int r = t / (NBR * NV), e = t - r * (NBR * NV);
    part[((int64_t)blockIdx.y * nq + q0 + r) * NBR * NV + e] = L.acc[r][e];
  }
}

// The tile scheme for more than 32 distinct R_j (up to 256): tiles of kTW
// rows; the R_j sum runs over chunks of 16 groups, each chunk's slab in
// registers and the A accumulators of the tile's rows in registers across
// the chunks; B, V and the epilogue as in k_phph_tile (per-row shuffles).
constexpr int kTW = 8, kWG = 16;  // rows per tile, R_j groups per chunk

template <int NBR, int NC>
struct WideLds {
  cd exq[kTW][NBR * NBR];
  cd exd[kTW][NBR * NBR];
  cd tq[kTW][kWG];             // exp(-2 pi i q.R_j) of the current chunk (zero beyond ng)
  cd tP[kWG];                  // exp(+2 pi i P.R_j) of the current chunk
  cd A[kTW][NBR * NBR * NBR];  // A of the tile's rows, then V
  cd B[kQB][NBR * NBR * NBR];
  double e1[kTW][NBR], e2[kTW][NBR], n2[kTW][NBR];
  double e3[NBR], n3[NBR];
  double acc[kTW][NBR * (NC ? NC : 1)];
  double f3[NBR * (NC ? NC : 1)];
  double f2[NC ? kTW : 1][NBR * (NC ? NC : 1)];
  double f2m[NC ? kTW : 1][NBR * (NC ? NC : 1)];
};

// exp(-2 pi i P.R) with 32-bit index arithmetic (|P_i R_i| stays far below 2^31)
__device__ inline cd phase_neg32(const PhaseTab& ph, int P, int r0, int r1, int r2) {
  const int c = P % ph.n2, t = P / ph.n2, b = t % ph.n1, a = t / ph.n1;
  int i0 = (a * r0) % ph.n0; if (i0 < 0) i0 += ph.n0;
  int i1 = (b * r1) % ph.n1; if (i1 < 0) i1 += ph.n1;
  int i2 = (c * r2) % ph.n2; if (i2 < 0) i2 += ph.n2;
  const double2 p0 = ph.t0[i0], p1 = ph.t1[i1], p2 = ph.t2[i2];
  return cconj(cmul(cmul(cmake(p0.x, p0.y), cmake(p1.x, p1.y)), cmake(p2.x, p2.y)));
}

template <int NBR, int NC>
__global__ __launch_bounds__(256) void k_phph_wide(PhaseTab ph, int nq, int prange, const int32_t* __restrict__ gr,
                                                   int ng, const cd* __restrict__ phi, const cd* __restrict__ Lq,
                                                   const double* __restrict__ hw, const double* __restrict__ nbose,
                                                   double omega_min, double sigma, const double* __restrict__ F,
                                                   double* __restrict__ part) {
  constexpr int N2 = NBR * NBR, N3 = N2 * NBR, NV = NC ? NC : 1;
  static_assert(N3 <= 256 && N2 <= 64 && kQB * 64 == 256 && kTW % kQB == 0, "tile shape");
  __shared__ WideLds<NBR, NC> L;
  const int q0 = blockIdx.x * kTW, nt = min(kTW, nq - q0);
  const int P0 = blockIdx.y * prange, P1 = min(nq, P0 + prange);
  const MeshDims md{ph.n0, ph.n1, ph.n2};
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int t = tid; t < kTW * N2; t += blockDim.x) {
    const int r = t / N2, e = t - r * N2;
    L.exq[r][e] = r < nt ? edisp(Lq, hw, q0 + r, NBR, e / NBR, e % NBR) : cmake(0.0, 0.0);
  }
  for (int t = tid; t < kTW * NBR; t += blockDim.x) {
    const int r = t / NBR, s = t - r * NBR;
    L.e1[r][s] = r < nt ? hw[(int64_t)(q0 + r) * NBR + s] : 0.0;
  }
  for (int t = tid; t < kTW * NBR * NV; t += blockDim.x) L.acc[t / (NBR * NV)][t % (NBR * NV)] = 0.0;
  const double inv2s2 = 0.5 / (sigma * sigma), dnorm = 1.0 / (sqrt(2.0 * kPi) * sigma);
  for (int P = P0; P < P1; ++P) {
    __syncthreads();   // the previous q'' is done with exd, e2, n2, e3, n3, f*, A
    if (tid < NBR) {
      const double w3 = hw[(int64_t)P * NBR + tid];
      L.e3[tid] = w3 >= omega_min ? w3 : 0.0;
      L.n3[tid] = nbose[(int64_t)P * NBR + tid];
    }
    for (int t = tid; t < kTW * N2; t += blockDim.x) {
      const int r = t / N2, e = t - r * N2;
      cd v = cmake(0.0, 0.0);
      if (r < nt) v = edisp(Lq, hw, q_between(P, q0 + r, md.n0, md.n1, md.n2), NBR, e / NBR, e % NBR);
      L.exd[r][e] = v;
    }
    for (int t = tid; t < kTW * NBR; t += blockDim.x) {
      const int r = t / NBR, s = t - r * NBR;
      double w2 = 0.0, n2 = 0.0;
      if (r < nt) {
        const int64_t m = (int64_t)q_between(q0 + r, P, md.n0, md.n1, md.n2) * NBR + s;
        w2 = hw[m];
        n2 = nbose[m];
      }
      L.e2[r][s] = w2 >= omega_min ? w2 : 0.0;
      L.n2[r][s] = n2;
    }
    if constexpr (NC > 0) {
      for (int t = tid; t < NBR * NC; t += blockDim.x) L.f3[t] = F[(int64_t)P * NBR * NC + t];
      for (int t = tid; t < kTW * NBR * NC; t += blockDim.x) {
        const int r = t / (NBR * NC), e = t - r * (NBR * NC);
        double a = 0.0, b = 0.0;
        if (r < nt) {
          a = F[(int64_t)q_between(q0 + r, P, md.n0, md.n1, md.n2) * NBR * NC + e];
          b = F[(int64_t)q_between(P, q0 + r, md.n0, md.n1, md.n2) * NBR * NC + e];
        }
        L.f2[r][e] = a;
        L.f2m[r][e] = b;
      }
    }
    cd a[kTW];
#pragma unroll
    for (int r = 0; r < kTW; ++r) a[r] = cmake(0.0, 0.0);
    for (int c0 = 0; c0 < ng; c0 += kWG) {
      cd slab[kWG];
      const cd* src = phi + ((int64_t)P * ng + c0) * N3 + tid;
#pragma unroll
      for (int g = 0; g < kWG; ++g)
        slab[g] = (c0 + g < ng && tid < N3) ? src[(int64_t)g * N3] : cmake(0.0, 0.0);
      __syncthreads();   // the previous chunk is done with tq and tP
      for (int t = tid; t < kTW * kWG; t += blockDim.x) {
        const int r = t / kWG, g = t - r * kWG, G = c0 + g;
        L.tq[r][g] = (r < nt && G < ng) ? phase_neg32(ph, q0 + r, gr[3 * G], gr[3 * G + 1], gr[3 * G + 2])
                                        : cmake(0.0, 0.0);
      }
      if (tid < kWG) {
        const int G = c0 + tid;
        L.tP[tid] = G < ng ? cconj(phase_neg32(ph, P, gr[3 * G], gr[3 * G + 1], gr[3 * G + 2])) : cmake(0.0, 0.0);
      }
      __syncthreads();
#pragma unroll
      for (int g = 0; g < kWG; ++g) slab[g] = cmul(L.tP[g], slab[g]);
#pragma unroll
      for (int r = 0; r < kTW; ++r)
#pragma unroll
        for (int g = 0; g < kWG; ++g) a[r] = cfma(a[r], L.tq[r][g], slab[g]);
    }
    if (tid < N3)
#pragma unroll
      for (int r = 0; r < kTW; ++r) L.A[r][tid] = a[r];
    __syncthreads();
    for (int rb = 0; rb < nt; rb += kQB) {
      for (int t = tid; t < kQB * N3; t += blockDim.x) {   // (r, x_i, s', s'')
        const int r = t / N3, o = t - r * N3;
        const int xi = o / N2, rr = o - xi * N2, s2 = rr / NBR, s3 = rr - s2 * NBR;
        cd b = cmake(0.0, 0.0);
#pragma unroll
        for (int xj = 0; xj < NBR; ++xj)
          b = cfma(b, L.exd[rb + r][xj * NBR + s2], L.A[rb + r][(xi * NBR + xj) * NBR + s3]);
        L.B[r][o] = b;
      }
      __syncthreads();
      for (int t = tid; t < kQB * N3; t += blockDim.x) {   // (r, s, s', s'')
        const int r = t / N3, o = t - r * N3;
        const int s1 = o / N2, rr = o - s1 * N2;
        cd v = cmake(0.0, 0.0);
#pragma unroll
        for (int xi = 0; xi < NBR; ++xi) v = cfma(v, L.exq[rb + r][xi * NBR + s1], L.B[r][xi * N2 + rr]);
        L.A[rb + r][o] = v;
      }
      __syncthreads();
      {  // wave r: row rb + r, lane = (s', s'')
        const int r = wave;
        double c[NBR * NV];
#pragma unroll
        for (int k = 0; k < NBR * NV; ++k) c[k] = 0.0;
        if (lane < N2) {
          const int s2 = lane / NBR, s3 = lane - s2 * NBR;
          const double E2 = L.e2[rb + r][s2], E3 = L.e3[s3];
          if (E2 > 0.0 && E3 > 0.0) {
            const double f = L.n3[s3] / (E2 * E3) * dnorm, np2 = L.n2[rb + r][s2];
#pragma unroll
            for (int s1 = 0; s1 < NBR; ++s1) {
              const double E1 = L.e1[rb + r][s1];
              const double dp = E1 + E2 - E3, dm = E1 - E2 - E3;
              const double b = cabs2(L.A[rb + r][s1 * N2 + lane]) * f;
              const double wp = b * (1.0 + np2) * exp(-dp * dp * inv2s2);  // absorption with -q'
              const double wm = b * 0.5 * np2 * exp(-dm * dm * inv2s2);    // decay into q', half
              if constexpr (NC == 0) {
                c[s1] = wp + wm;
              } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                  const double F3 = L.f3[s3 * NC + k];
                  c[s1 * NC + k] = wp * (F3 - L.f2m[rb + r][s2 * NC + k]) + wm * (F3 + L.f2[rb + r][s2 * NC + k]);
                }
              }
            }
          }
        }
#pragma unroll
        for (int k = 0; k < NBR * NV; ++k) {
          double x = c[k];
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
          c[k] = x;
        }
        if (rb + r < nt && lane < NBR * NV) {
          double x = c[0];
#pragma unroll
          for (int k = 1; k < NBR * NV; ++k)
            if (lane == k) x = c[k];
          L.acc[rb + r][lane] += x;
        }
      }
      __syncthreads();   // B is rewritten by the next rows
    }
  }
  __syncthreads();
  for (int t = tid; t < nt * NBR * NV; t += blockDim.x) {
    const int r = t / (NBR * NV), e = t - r * (NBR * NV);
    part[((int64_t)blockIdx.y * nq + q0 + r) * NBR * NV + e] = L.acc[r][e];
  }
}

// W[q][s] = pi C / (4 N_q) sum_chunks part / (E n), modes below omega_min 0
__global__ void k_phph_finish(int64_t nq, int nbr, int nv, int nchunk, const double* __restrict__ part,
                              const double* __restrict__ hw, double kT, double omega_min, double pref,
                              double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * nbr * nv) return;
  const double w = hw[e / nv];
  double sum = 0.0;
  for (int c = 0; c < nchunk; ++c) sum += part[(int64_t)c * nq * nbr * nv + e];
  W[e] = w >= omega_min ? pref * sum * expm1(w / kT) / w : 0.0;
}

PhaseTab phase_tab(elph_ctx ctx) {
  return PhaseTab{ctx->d_tab[0], ctx->d_tab[1], ctx->d_tab[2], ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
}

template <int NBR>
void launch_fold(elph_ctx ctx, cd* phi) {
  hipLaunchKernelGGL(k_ifc3_fold<NBR>, dim3((unsigned)ctx->nk, (unsigned)ctx->ng3), dim3(256), 0, ctx->stream,
                     phase_tab(ctx), ctx->d_i3_off, ctx->d_i3_rk, ctx->d_i3_psi, (const cd*)ctx->d_Lq, ctx->d_hw,
                     ctx->ng3, phi);
}

template <int NBR, int NC>
void launch_rows(elph_ctx ctx, int chunk, int nchunk, const cd* phi, double kT, double sigma, const double* F,
                 double* part) {
  hipLaunchKernelGGL((k_phph_rows<NBR, NC>), dim3((unsigned)ctx->nk, (unsigned)nchunk), dim3(256), 0, ctx->stream,
                     phase_tab(ctx), (int)ctx->nk, chunk, ctx->d_i3_rj, ctx->ng3, phi, (const cd*)ctx->d_Lq, ctx->d_hw,
                     kT, ctx->omega_min, sigma, F, part);
}

template <int NBR, int NC, int NGP>
void launch_tile_g(elph_ctx ctx, int prange, int nrange, const cd* phi, const double* nbose, double sigma,
                   const double* F, double* part) {
  hipLaunchKernelGGL((k_phph_tile<NBR, NC, NGP>), dim3((unsigned)((ctx->nk + kTQ - 1) / kTQ), (unsigned)nrange),
                     dim3(256), 0, ctx->stream, phase_tab(ctx), (int)ctx->nk, prange, ctx->d_i3_rj, ctx->ng3, phi,
                     (const cd*)ctx->d_Lq, ctx->d_hw, nbose, ctx->omega_min, sigma, F, part);
}

// the R_j count padded to 8, 16, 28 or 32 (zero phases and slab beyond ng)
template <int NBR, int NC>
void launch_tile(elph_ctx ctx, int prange, int nrange, const cd* phi, const double* nbose, double sigma,
                 const double* F, double* part) {
  if constexpr (NBR * NBR * NBR <= 256) {
    if (ctx->ng3 <= 8)
      launch_tile_g<NBR, NC, 8>(ctx, prange, nrange, phi, nbose, sigma, F, part);
    else if (ctx->ng3 <= 16)
      launch_tile_g<NBR, NC, 16>(ctx, prange, nrange, phi, nbose, sigma, F, part);
    else if (ctx->ng3 <= 28)
      launch_tile_g<NBR, NC, 28>(ctx, prange, nrange, phi, nbose, sigma, F, part);
    else
      launch_tile_g<NBR, NC, kMaxG>(ctx, prange, nrange, phi, nbose, sigma, F, part);
  }
}

template <int NBR, int NC>
void launch_wide(elph_ctx ctx, int prange, int nrange, const cd* phi, const double* nbose, double sigma,
                 const double* F, double* part) {
  if constexpr (NBR * NBR * NBR <= 256)
    hipLaunchKernelGGL((k_phph_wide<NBR, NC>), dim3((unsigned)((ctx->nk + kTW - 1) / kTW), (unsigned)nrange),
                       dim3(256), 0, ctx->stream, phase_tab(ctx), (int)ctx->nk, prange, ctx->d_i3_rj, ctx->ng3, phi,
                       (const cd*)ctx->d_Lq, ctx->d_hw, nbose, ctx->omega_min, sigma, F, part);
}

template <int NBR>
void launch_vertex(elph_ctx ctx, int64_t np, const int32_t* q, const int32_t* qp, const cd* phi, double* V2) {
  hipLaunchKernelGGL(k_phph_vertex<NBR>, dim3((unsigned)np), dim3(256), 0, ctx->stream, phase_tab(ctx), np, q, qp,
                     ctx->d_i3_rj, ctx->ng3, phi, (const cd*)ctx->d_Lq, ctx->d_hw, V2);
}

#define NBR_SWITCH(nbr, CALL)          \
  switch (nbr) {                       \
    case 3: CALL(3); break;            \
    case 6: CALL(6); break;            \
    case 9: CALL(9); break;            \
    case 12: CALL(12); break;          \
    default: break;                    \
  }

elph_status check_phph(elph_ctx ctx) {
  if (!ctx->d_i3_psi) {
    ctx->err = "no third-order force constants (elph_set_ifc3)";
    return ELPH_ESTATE;
  }
  if (ctx->nbr > 12) {
    ctx->err = "three-phonon processes support up to 4 atoms";
    return ELPH_EINVAL;
  }
  return ELPH_OK;
}

// the fold table for every mesh point: built once and kept on the context
// (it depends on the force constants and the phonon tables only; setting
// the force constants or dropping the tables releases it)
elph_status build_fold(elph_ctx ctx, cd** phi) {
  if (ctx->d_i3_fold) {
    *phi = (cd*)ctx->d_i3_fold;
    return ELPH_OK;
  }
  const int64_t n3 = (int64_t)ctx->nbr * ctx->nbr * ctx->nbr;
  ALLOC(*phi, ctx->nk * ctx->ng3 * n3 * sizeof(cd));
#define FOLD(N) launch_fold<N>(ctx, *phi)
  NBR_SWITCH(ctx->nbr, FOLD)
#undef FOLD
  HIPCHK(hipGetLastError());
  ctx->d_i3_fold = *phi;
  return ELPH_OK;
}

}  // namespace

elph_status phph_set_ifc3(elph_ctx ctx, int32_t n, const int32_t* rj, const int32_t* rk, const double* psi) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  void** ptrs[] = {(void**)&ctx->d_i3_rj, (void**)&ctx->d_i3_off, (void**)&ctx->d_i3_rk, (void**)&ctx->d_i3_psi,
                   (void**)&ctx->d_i3_fold};
  for (void** p : ptrs) {
    dev_free(ctx, *p);
    *p = nullptr;
  }
  ctx->n3 = ctx->ng3 = 0;
  if (n == 0 || !psi) return ELPH_OK;
  if (n < 0 || !rj || !rk) {
    ctx->err = "elph_set_ifc3: bad entry count or null cell arrays";
    return ELPH_EINVAL;
  }
  const int na = ctx->na, nbr = ctx->nbr;
  const int64_t blk = (int64_t)nbr * nbr * nbr;
  for (int64_t i = 0; i < (int64_t)n * blk; ++i)
    if (!std::isfinite(psi[i])) {
      ctx->err = "elph_set_ifc3: psi is not finite";
      return ELPH_EINVAL;
    }
  // entries grouped by R_j (stable), Psi reordered to [x_i][x_j][x_k]
  std::map<std::array<int32_t, 3>, std::vector<int>> groups;
  for (int e = 0; e < n; ++e) groups[{rj[3 * e], rj[3 * e + 1], rj[3 * e + 2]}].push_back(e);
  if ((int)groups.size() > kMaxGroups) {
    ctx->err = "elph_set_ifc3: more than 256 distinct R_j";
    return ELPH_EINVAL;
  }
  std::vector<int32_t> hg, hoff, hrk;
  std::vector<double> hpsi((size_t)n * blk);
  hoff.push_back(0);
  int pos = 0;
  for (auto& kv : groups) {
    hg.insert(hg.end(), kv.first.begin(), kv.first.end());
    for (int e : kv.second) {
      hrk.insert(hrk.end(), {rk[3 * e], rk[3 * e + 1], rk[3 * e + 2]});
      const double* src = psi + (int64_t)e * blk;   // [ti][tj][tk][a][b][c]
      double* dst = hpsi.data() + (int64_t)pos * blk;
      for (int ti = 0; ti < na; ++ti)
        for (int tj = 0; tj < na; ++tj)
          for (int tk = 0; tk < na; ++tk)
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c)
                  dst[((3 * ti + a) * nbr + 3 * tj + b) * nbr + 3 * tk + c] =
                      src[((((ti * na + tj) * na + tk) * 3 + a) * 3 + b) * 3 + c];
      ++pos;
    }
    hoff.push_back(pos);
  }
  ctx->n3 = n;
  ctx->ng3 = (int)groups.size();
  ALLOC(ctx->d_i3_rj, hg.size() * sizeof(int32_t));
  ALLOC(ctx->d_i3_off, hoff.size() * sizeof(int32_t));
  ALLOC(ctx->d_i3_rk, hrk.size() * sizeof(int32_t));
  ALLOC(ctx->d_i3_psi, hpsi.size() * sizeof(double));
  HIPCHK(hipMemcpy(ctx->d_i3_rj, hg.data(), hg.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ctx->d_i3_off, hoff.data(), hoff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ctx->d_i3_rk, hrk.data(), hrk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ctx->d_i3_psi, hpsi.data(), hpsi.size() * sizeof(double), hipMemcpyHostToDevice));
  return ELPH_OK;
}

elph_status phph_vertex(elph_ctx ctx, int64_t npairs, const int32_t* q, const int32_t* qp, double* V2) {
  elph_status st = check_phph(ctx);
  if (st != ELPH_OK) return st;
  if (npairs < 0 || (npairs > 0 && (!q || !qp || !V2))) {
    ctx->err = "elph_phph_vertex: bad pair list";
    return ELPH_EINVAL;
  }
  if (npairs == 0) return ELPH_OK;
  if (npairs > 0x7fffffff) {
    ctx->err = "elph_phph_vertex: too many pairs for one call";
    return ELPH_EINVAL;
  }
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  cd* phi = nullptr;
  st = build_fold(ctx, &phi);
  if (st != ELPH_OK) return st;
#define VTX(N) launch_vertex<N>(ctx, npairs, q, qp, phi, V2)
  NBR_SWITCH(ctx->nbr, VTX)
#undef VTX
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ELPH_OK;
}

// One pass over every (q, q') pair: the rates (F = NULL) or the in-scattering
// sums of a field F [nq][nbr][3] (Eq. 26), into out [nq][nbr] or [nq][nbr][3].
static elph_status phph_pass(elph_ctx ctx, const char* name, double T_K, double sigma_eV, const double* F,
                             double* out) {
  elph_status st = check_phph(ctx);
  if (st != ELPH_OK) return st;
  if (!(sigma_eV > 0) || !std::isfinite(sigma_eV) || !out) {
    ctx->err = std::string(name) + ": sigma must be positive and the output non-null";
    return ELPH_EINVAL;
  }
  if (ctx->nk > 0x7fffffff) {
    ctx->err = std::string(name) + ": mesh too large";
    return ELPH_EINVAL;
  }
  const int64_t nq = ctx->nk;
  const bool tile = ctx->nbr <= 6 && ctx->ng3 <= kMaxG;
  const bool wide = ctx->nbr <= 6 && ctx->ng3 > kMaxG;
  const int nv = F ? 3 : 1;
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  cd* phi = nullptr;
  st = build_fold(ctx, &phi);
  if (st != ELPH_OK) return st;
  int nchunk, chunk;
  if (tile || wide) {
    // q'' ranges: about 4096 blocks in all, at least 8 q'' per block
    const int64_t ntile = (nq + (wide ? kTW : kTQ) - 1) / (wide ? kTW : kTQ);
    nchunk = (int)std::max<int64_t>(1, std::min<int64_t>((nq + 7) / 8, (4096 + ntile - 1) / ntile));
  } else {
    // chunks of q' so that the grid holds at least ~4096 blocks
    nchunk = (int)std::min<int64_t>(nq, std::max<int64_t>(1, (4096 + nq - 1) / nq));
  }
  chunk = (int)((nq + nchunk - 1) / nchunk);
  nchunk = (int)((nq + chunk - 1) / chunk);
  double* part = nullptr;
  ALLOC(part, (size_t)nchunk * nq * ctx->nbr * nv * sizeof(double));
  const double kT = kBoltzEVK * T_K;
  double* nbose = nullptr;
  if (tile || wide) {
    ALLOC(nbose, (size_t)nq * ctx->nbr * sizeof(double));
    hipLaunchKernelGGL(k_phph_bose, dim3(blocks_for(nq * ctx->nbr, 256)), dim3(256), 0, ctx->stream,
                       nq * ctx->nbr, ctx->d_hw, kT, ctx->omega_min, nbose);
  }
  mark(ctx, 4);  // the row kernel is reported in the step-2 timing window
  if (wide && !F) {
#define WIDE(N) launch_wide<N, 0>(ctx, chunk, nchunk, phi, nbose, sigma_eV, nullptr, part)
    NBR_SWITCH(ctx->nbr, WIDE)
#undef WIDE
  } else if (wide) {
#define WIDE(N) launch_wide<N, 3>(ctx, chunk, nchunk, phi, nbose, sigma_eV, F, part)
    NBR_SWITCH(ctx->nbr, WIDE)
#undef WIDE
  } else if (tile && !F) {
#define TILE(N) launch_tile<N, 0>(ctx, chunk, nchunk, phi, nbose, sigma_eV, nullptr, part)
    NBR_SWITCH(ctx->nbr, TILE)
#undef TILE
  } else if (tile) {
#define TILE(N) launch_tile<N, 3>(ctx, chunk, nchunk, phi, nbose, sigma_eV, F, part)
    NBR_SWITCH(ctx->nbr, TILE)
#undef TILE
  } else if (!F) {
#define ROWS(N) launch_rows<N, 0>(ctx, chunk, nchunk, phi, kT, sigma_eV, nullptr, part)
    NBR_SWITCH(ctx->nbr, ROWS)
#undef ROWS
  } else {
#define ROWS(N) launch_rows<N, 3>(ctx, chunk, nchunk, phi, kT, sigma_eV, F, part)
    NBR_SWITCH(ctx->nbr, ROWS)
#undef ROWS
  }
  mark(ctx, 5);
  HIPCHK(hipGetLastError());
  const double pref = kPi / (4.0 * (double)nq) * kPhPhC;
  hipLaunchKernelGGL(k_phph_finish, dim3(blocks_for(nq * ctx->nbr * nv, 256)), dim3(256), 0, ctx->stream, nq,
                     ctx->nbr, nv, nchunk, part, ctx->d_hw, kT, ctx->omega_min, pref, out);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dev_free(ctx, part);
  dev_free(ctx, nbose);
  return ELPH_OK;
}

elph_status phph_rates(elph_ctx ctx, double T_K, double sigma_eV, double* W) {
  return phph_pass(ctx, "elph_phph_rates", T_K, sigma_eV, nullptr, W);
}

elph_status phph_inscatter(elph_ctx ctx, double T_K, double sigma_eV, const double* F, double* S) {
  if (!F) {
    ctx->err = "elph_phph_inscatter: F is null";
    return ELPH_EINVAL;
  }
  return phph_pass(ctx, "elph_phph_inscatter", T_K, sigma_eV, F, S);
}

}  // namespace elph
