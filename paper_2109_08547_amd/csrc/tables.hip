// Electron and phonon tables on the device:
//  * per-axis phase tables and Fourier sums H(k), grad H(k), D(q), grad D(q)
//    (Eqs. 1 and 3 of "The elphbolt ab initio solver ...", short-range part),
//  * a batched FP64 cyclic Jacobi eigensolver for Hermitian matrices up to
//    16 x 16 (eigenvalues ascending, eigenvectors as columns),
//  * the transport window and its compaction into kept k and active states,
//  * band and branch velocities (Eqs. 2 and 5) and the phonon factors of
//    Eq. 6 (l_{x,s} u_q[x,s], with l = sqrt(C / (2 M hbar omega))), the
//    phonons diagonalised at one q of each +-q pair (time reversal), with
//    the non-analytic term of Eq. 4 for polar materials.
#include "devutil.h"
#include "tables.h"

#include <algorithm>
#include <utility>
#include <vector>

namespace elph {

// ---------------------------------------------------------------------------
// phases

__global__ void k_axis_table(int n, double2* tab) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)n, &s, &c);
  tab[j] = make_double2(c, s);
}

struct MeshPhase {
  const double2* t0;
  const double2* t1;
  const double2* t2;
  int n0, n1, n2;
  // exp(2 pi i k . R) for k = (a/n0, b/n1, c/n2) and integer R
  __device__ inline cd operator()(int a, int b, int c, int r0, int r1, int r2) const {
    int i0 = (int)(((int64_t)a * r0) % n0); if (i0 < 0) i0 += n0;
    int i1 = (int)(((int64_t)b * r1) % n1); if (i1 < 0) i1 += n1;
    int i2 = (int)(((int64_t)c * r2) % n2); if (i2 < 0) i2 += n2;
    double2 p0 = t0[i0], p1 = t1[i1], p2 = t2[i2];
    cd z = cmul(cmake(p0.x, p0.y), cmake(p1.x, p1.y));
    return cmul(z, cmake(p2.x, p2.y));
  }
};

static MeshPhase mesh_phase(elph_ctx c) {
  return MeshPhase{c->d_tab[0], c->d_tab[1], c->d_tab[2], c->mesh[0], c->mesh[1], c->mesh[2]};
}

__device__ inline void mesh_coords(int64_t lin, int n1, int n2, int& a, int& b, int& c) {
  c = (int)(lin % n2);
  int64_t t = lin / n2;
  b = (int)(t % n1);
  a = (int)(t / n1);
}

// Fourier sum over R for a list of mesh points: out[p][a][b] = sum_R w_R e^{ik.R} M(R)[a][b]
// and optionally grad[p][c][a][b] = sum_R i R_cart[c] w_R e^{ik.R} M(R)[a][b].
// The same sums as a complex GEMM on the 16x16x4 FP64 MFMA:
// out[p][col] = sum_r A[p][r] M[r][col] with A[p][r] = w_r e^{2 pi i k_p.R_r}.
// A wavefront owns 16 points x 16 columns; lane l supplies A[l%16][r0 + l/16]
// (its phase computed from the per-axis tables) and M[r0 + l/16][col0 + l%16];
// the gradient is three more products with A scaled by i R_cart.  The
// accumulator of lane l holds rows l/16 + 4r, column l%16.
typedef double d4f __attribute__((ext_vector_type(4)));

__device__ inline d4f mma64(double a, double b, d4f c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// exp(2 pi i k.R) from the per-axis tables with 32-bit index arithmetic
// (|a R| < 2^31 for the meshes and R sets here)
__device__ inline cd phase32(const MeshPhase& ph, int a, int b, int c, int r0, int r1, int r2) {
  int i0 = (a * r0) % ph.n0; if (i0 < 0) i0 += ph.n0;
  int i1 = (b * r1) % ph.n1; if (i1 < 0) i1 += ph.n1;
  int i2 = (c * r2) % ph.n2; if (i2 < 0) i2 += ph.n2;
  const double2 p0 = ph.t0[i0], p1 = ph.t1[i1], p2 = ph.t2[i2];
  return cmul(cmul(cmake(p0.x, p0.y), cmake(p1.x, p1.y)), cmake(p2.x, p2.y));
}

// CT column tiles of 16 per wavefront share each computed phase.
template <bool REAL_IN, bool GRAD, int CT>
__global__ void __launch_bounds__(256) k_fourier_mfma(MeshPhase ph, const int32_t* __restrict__ pts, int64_t base,
                                                      int64_t npts, const int32_t* __restrict__ R,
                                                      const double* __restrict__ w, int nR,
                                                      const double* __restrict__ lat, const double* __restrict__ Min,
                                                      int nn, cd* __restrict__ out, cd* __restrict__ grad) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (p0 >= npts) return;  // whole wavefront
  const int colb = blockIdx.y * 16 * CT;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t p = p0 + lr;
  const bool pv = p < npts;
  int a = 0, b = 0, c = 0;
  if (pv) mesh_coords(pts ? (int64_t)pts[p] : base + p, ph.n1, ph.n2, a, b, c);
  constexpr int NG = GRAD ? 3 : 0;
  const d4f zero = {0.0, 0.0, 0.0, 0.0};
  d4f vr[CT], vi[CT], gr[CT][NG > 0 ? NG : 1], gi[CT][NG > 0 ? NG : 1];
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    vr[t] = zero;
    vi[t] = zero;
#pragma unroll
    for (int d = 0; d < (NG > 0 ? NG : 1); ++d) gr[t][d] = gi[t][d] = zero;
  }
  for (int r0 = 0; r0 < nR; r0 += 4) {
    const int r = r0 + lk;
    cd z = cmake(0.0, 0.0);
    double rc[3] = {0.0, 0.0, 0.0};
    const bool rv = r < nR;
    if (rv) {
      const int R0 = R[3 * r], R1 = R[3 * r + 1], R2 = R[3 * r + 2];
      if (pv) {
        z = phase32(ph, a, b, c, R0, R1, R2);
        if (w) z = cscale(z, w[r]);
      }
      if (GRAD)
#pragma unroll
        for (int d = 0; d < 3; ++d) rc[d] = R0 * lat[d] + R1 * lat[3 + d] + R2 * lat[6 + d];
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = colb + 16 * t + lr;
      double mr = 0.0, mi = 0.0;
      if (rv && col < nn) {
        if (REAL_IN) {
          mr = Min[(int64_t)r * nn + col];
        } else {
          mr = Min[2 * ((int64_t)r * nn + col)];
          mi = Min[2 * ((int64_t)r * nn + col) + 1];
        }
      }
      vr[t] = mma64(z.x, mr, vr[t]);
      vi[t] = mma64(z.y, mr, vi[t]);
      if (!REAL_IN) {
        vr[t] = mma64(-z.y, mi, vr[t]);
        vi[t] = mma64(z.x, mi, vi[t]);
      }
      if (GRAD) {
#pragma unroll
        for (int d = 0; d < NG; ++d) {
          const double zr = -rc[d] * z.y, zi = rc[d] * z.x;  // i R_cart z
          gr[t][d] = mma64(zr, mr, gr[t][d]);
          gi[t][d] = mma64(zi, mr, gi[t][d]);
          if (!REAL_IN) {
            gr[t][d] = mma64(-zi, mi, gr[t][d]);
            gi[t][d] = mma64(zr, mi, gi[t][d]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int col = colb + 16 * t + lr;
    if (col >= nn) continue;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t pp = p0 + lk + 4 * rr;
      if (pp >= npts) continue;
      out[pp * nn + col] = cmake(vr[t][rr], vi[t][rr]);
      if (GRAD)
#pragma unroll
        for (int d = 0; d < NG; ++d) grad[(pp * 3 + d) * nn + col] = cmake(gr[t][d][rr], gi[t][d][rr]);
    }
  }
}

// ---------------------------------------------------------------------------
// Batched cyclic Jacobi for Hermitian n x n (n <= P <= 16).
//
// A group of P lanes owns one matrix: lane j holds column j of A and of the
// accumulated rotation V in registers.  Each sweep runs the P-1 rounds of a
// round-robin tournament; in a round the P/2 disjoint pairs (p, q) rotate in
// parallel with the unitary J = [[c, s e^{i phi}], [-s e^{-i phi}, c]] that
// zeroes A[p][q] (phi = arg A[p][q], t = tan(theta) from the classical
// symmetric Jacobi formula): columns with the partner lane's column, rows
// with the pair parameters broadcast from the owning lanes.  Padded
// rows/columns carry a large diagonal and zero coupling, so they never
// rotate and sort last.

__host__ __device__ constexpr int rr_partner(int i, int rho, int P) {
  // round-robin (circle method) schedule over P players, rounds 0..P-2
  return (i == P - 1) ? ((rho * (P / 2)) % (P - 1))
                      : ((((rho - i) % (P - 1) + (P - 1)) % (P - 1)) == i
                             ? P - 1
                             : (((rho - i) % (P - 1) + (P - 1)) % (P - 1)));
}

__device__ inline double shfl_d(double v, int src) { return __shfl(v, src, 64); }
__device__ inline cd shfl_c(cd v, int src) { return cmake(__shfl(v.x, src, 64), __shfl(v.y, src, 64)); }

// Wave-private LDS: column storage col[lane][r] (row stride P+1 against bank
// conflicts) and the rotation parameters of each lane.
template <int P>
struct JacobiLds {
  cd col[64][P + 1];
  double c[64];
  cd se[64];
};

template <int P, int RHO, int p>
__device__ __forceinline__ void jacobi_row_pair(cd (&a)[P], const JacobiLds<P>& L, int base) {
  constexpr int q = rr_partner(p, RHO, P);
  if constexpr (p < q) {
    const double cp = L.c[base + p];
    const cd sp = L.se[base + p];
    const cd ap = a[p], aq = a[q];
    a[p] = csub(cscale(ap, cp), cmul(sp, aq));
    a[q] = cadd(cmul(cconj(sp), ap), cscale(aq, cp));
  }
}

template <int P, int RHO, int... PS>
__device__ __forceinline__ void jacobi_rows(cd (&a)[P], const JacobiLds<P>& L, int base,
                                            std::integer_sequence<int, PS...>) {
  (jacobi_row_pair<P, RHO, PS>(a, L, base), ...);
}

// One round RHO of the tournament.  Register arrays are indexed statically;
// the lane-dependent reads (own diagonal, partner column) go through LDS.
template <int P, bool VECS, int RHO>
__device__ __forceinline__ void jacobi_round(cd (&a)[P], cd (&v)[P], int j, int lane, int base,
                                             JacobiLds<P>& L) {
  const int pj = rr_partner(j, RHO, P);
  const bool isp = j < pj;
#pragma unroll
  for (int r = 0; r < P; ++r) L.col[lane][r] = a[r];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const cd ajj = L.col[lane][j];
  const cd ajp = L.col[lane][pj];
  const double dpart = L.col[base + pj][pj].x;
  const cd opart = L.col[base + pj][j];
  const double app = isp ? ajj.x : dpart;
  const double aqq = isp ? dpart : ajj.x;
  const cd apq = isp ? opart : ajp;  // A[p][q] lives in column q
  double c = 1.0;
  cd se = cmake(0, 0);
  const double habs = sqrt(cabs2(apq));
  if (habs > 1.0e-300) {
    const double tau = (aqq - app) / (2.0 * habs);
    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + t * t);
    const double s = t * c;
    se = cscale(apq, s / habs);  // s e^{i phi}
  }
  // columns: A <- A J, V <- V J
  const cd wgt = isp ? cmake(-se.x, se.y) /* -conj(se) */ : se;
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const cd pa = L.col[base + pj][r];
    a[r] = cadd(cscale(a[r], c), cmul(wgt, pa));
    if (VECS) {
      const cd pv = shfl_c(v[r], base + pj);
      v[r] = cadd(cscale(v[r], c), cmul(wgt, pv));
    }
  }
  L.c[lane] = c;
  L.se[lane] = se;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // rows: A <- J^H A, pair parameters from the lane owning row p
  jacobi_rows<P, RHO>(a, L, base, std::make_integer_sequence<int, P>{});
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

template <int P, bool VECS, int... RHO>
__device__ __forceinline__ void jacobi_sweep(cd (&a)[P], cd (&v)[P], int j, int lane, int base,
                                             JacobiLds<P>& L, std::integer_sequence<int, RHO...>) {
  (jacobi_round<P, VECS, RHO>(a, v, j, lane, base, L), ...);
}

template <int P, bool VECS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_jacobi(const cd* __restrict__ Ain, int64_t nmat, int n,
                                                       double* __restrict__ evals, cd* __restrict__ evecs,
                                                       int max_sweeps) {
  __shared__ JacobiLds<P> lds[WAVES];
  JacobiLds<P>& L = lds[threadIdx.x / 64];
  const int lane = threadIdx.x & 63;
  const int j = lane % P;
  const int base = lane - j;
  const int64_t mat = ((int64_t)blockIdx.x * WAVES + threadIdx.x / 64) * (64 / P) + lane / P;
  const bool valid = mat < nmat;
  const int64_t nn = (int64_t)n * n;

  cd a[P], v[P];
  double frob = 0.0;
#pragma unroll
  for (int r = 0; r < P; ++r) {
    cd x = cmake(0, 0);
    if (valid && r < n && j < n) x = Ain[mat * nn + (int64_t)r * n + j];
    frob += cabs2(x);
    a[r] = x;
    v[r] = cmake(r == j ? 1.0 : 0.0, 0.0);
  }
  // padded (or absent) columns: distinct large diagonal, no coupling
  if (!(valid && j < n)) {
#pragma unroll
    for (int r = 0; r < P; ++r)
      if (r == j) a[r] = cmake(1.0e200 * (1.0 + j), 0.0);
  }
  // Frobenius norm^2 of the group's matrix
#pragma unroll
  for (int o = 1; o < P; o <<= 1) frob += __shfl_xor(frob, o, 64);
  const double tol2 = 1.0e-30 * frob;

  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    jacobi_sweep<P, VECS>(a, v, j, lane, base, L, std::make_integer_sequence<int, P - 1>{});
    // convergence: off-diagonal norm of the whole group
    double off = 0.0;
#pragma unroll
    for (int r = 0; r < P; ++r)
      if (r != j) off += cabs2(a[r]);
#pragma unroll
    for (int o = 1; o < P; o <<= 1) off += __shfl_xor(off, o, 64);
    const bool done = !(off > tol2);
    if (__all(done)) break;
  }

  // sort ascending
#pragma unroll
  for (int r = 0; r < P; ++r) L.col[lane][r] = a[r];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const double dj = L.col[lane][j].x;
  int rank = 0;
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const double dr = shfl_d(dj, base + r);
    rank += (dr < dj || (dr == dj && r < j)) ? 1 : 0;
  }
  if (valid && j < n && rank < n) {
    if (evals) evals[mat * n + rank] = dj;
    if (VECS) {
#pragma unroll
      for (int r = 0; r < P; ++r)
        if (r < n) evecs[mat * nn + (int64_t)r * n + rank] = v[r];
    }
  }
}

template <bool VECS>
static void launch_jacobi_t(const cd* A, int64_t nmat, int n, double* ev, cd* U, hipStream_t s) {
  if (n <= 4) {
    constexpr int W = 4;
    hipLaunchKernelGGL((k_jacobi<4, VECS, W>), dim3(blocks_for(nmat, W * 16)), dim3(64 * W), 0, s, A, nmat, n, ev,
                       U, 12);
  } else if (n <= 8) {
    constexpr int W = 4;
    hipLaunchKernelGGL((k_jacobi<8, VECS, W>), dim3(blocks_for(nmat, W * 8)), dim3(64 * W), 0, s, A, nmat, n, ev,
                       U, 12);
  } else {
    constexpr int W = 2;
    hipLaunchKernelGGL((k_jacobi<16, VECS, W>), dim3(blocks_for(nmat, W * 4)), dim3(64 * W), 0, s, A, nmat, n,
                       ev, U, 14);
  }
}

void launch_jacobi(const cd* A, int64_t nmat, int n, double* evals, cd* evecs, hipStream_t s) {
  if (nmat <= 0) return;
  if (evecs) launch_jacobi_t<true>(A, nmat, n, evals, evecs, s);
  else launch_jacobi_t<false>(A, nmat, n, evals, nullptr, s);
}

// ---------------------------------------------------------------------------
// window and compaction

__global__ void k_window(const double* __restrict__ eps, int64_t nk, int nb, double mu, double window,
                         int32_t* __restrict__ nact, int32_t* __restrict__ kept_flag) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  int c = 0;
  for (int m = 0; m < nb; ++m) c += (fabs(eps[k * nb + m] - mu) <= window) ? 1 : 0;
  nact[k] = c;
  kept_flag[k] = c > 0 ? 1 : 0;
}

// exclusive scan, three phases; block size 1024
__global__ void k_scan_block(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ out,
                             int32_t* __restrict__ block_sums) {
  __shared__ int32_t s[1024];
  int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int32_t x = i < n ? in[i] : 0;
  s[threadIdx.x] = x;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int32_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - x;
  if (threadIdx.x == 1023) block_sums[blockIdx.x] = s[1023];
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ block_pref) {
  int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < n) out[i] += block_pref[blockIdx.x];
}

// exclusive scan of in[0..n) into out[0..n); total written to out_total (device, 1 int)
void scan_exclusive(elph_ctx ctx, const int32_t* in, int64_t n, int32_t* out, int32_t* out_total,
                    int32_t* scratch, hipStream_t s) {
  int64_t nblk = (n + 1023) / 1024;
  if (nblk == 0) {
    (void)hipMemsetAsync(out_total, 0, sizeof(int32_t), s);  // errors surface at the caller's next check
    return;
  }
  int32_t* bsum = scratch;          // [nblk]
  int32_t* bpref = scratch + nblk;  // [nblk]
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nblk), dim3(1024), 0, s, in, n, out, bsum);
  if (nblk == 1) {
    (void)hipMemsetAsync(bpref, 0, sizeof(int32_t), s);
    (void)hipMemcpyAsync(out_total, bsum, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    return;
  }
  int32_t* tot2 = scratch + 2 * nblk;
  scan_exclusive(ctx, bsum, nblk, bpref, tot2, scratch + 2 * nblk + 1, s);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nblk), dim3(1024), 0, s, out, n, bpref);
  (void)hipMemcpyAsync(out_total, tot2, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
}

__global__ void k_compact_kept(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos, int64_t nk,
                               int32_t* __restrict__ kidx, int32_t* __restrict__ kept,
                               const int32_t* __restrict__ nact_mesh, int32_t* __restrict__ nact_kept) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  if (flag[k]) {
    kidx[k] = pos[k];
    kept[pos[k]] = (int32_t)k;
    nact_kept[pos[k]] = nact_mesh[k];
  } else {
    kidx[k] = -1;
  }
}

__global__ void k_fill_states(const int32_t* __restrict__ kept, int64_t nkept, const int32_t* __restrict__ soff,
                              const double* __restrict__ eps_all, int nb, double mu, double window,
                              int32_t* __restrict__ st_k, int32_t* __restrict__ st_kidx,
                              int32_t* __restrict__ st_m, double* __restrict__ st_eps) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nkept) return;
  int32_t km = kept[t];
  int32_t o = soff[t];
  for (int m = 0; m < nb; ++m) {
    double e = eps_all[(int64_t)km * nb + m];
    if (fabs(e - mu) <= window) {
      st_k[o] = km;
      st_kidx[o] = (int32_t)t;
      st_m[o] = m;
      st_eps[o] = e;
      ++o;
    }
  }
}

// ---------------------------------------------------------------------------
// velocities

// Electron: v[m] = Re(U[:,m]^H dH_c U[:,m]) (A eV -> m/s), averaged over
// degenerate groups of eps, written for active states of each kept k.
__global__ void k_electron_vd(int64_t nkept, int nb, const cd* __restrict__ U, const cd* __restrict__ dH,
                              double* __restrict__ vd) {
  // thread per (kept k t, direction c, band m): u_m^+ (dH/dk_c) u_m / hbar
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nkept * 3 * nb) return;
  const int64_t t = e / (3 * nb);
  const int cm = (int)(e - t * 3 * nb), c = cm / nb, m = cm - c * nb;
  const int64_t nn = (int64_t)nb * nb;
  const cd* u = U + t * nn;
  const cd* h = dH + (t * 3 + c) * nn;
  double acc = 0.0;
  for (int a = 0; a < nb; ++a) {
    cd row = cmake(0, 0);
    for (int b = 0; b < nb; ++b) row = cadd(row, cmul(h[a * nb + b], u[b * nb + m]));
    acc += cmul(cconj(u[a * nb + m]), row).x;
  }
  vd[(t * nb + m) * 3 + c] = acc * (kAngM / kHbarEVs);
}

// average over degenerate bands, then keep the active states' velocities
__global__ void k_electron_vel(int64_t nkept, int nb, const double* __restrict__ vdin,
                               const double* __restrict__ eps_all, const int32_t* __restrict__ kept,
                               const int32_t* __restrict__ soff, double mu, double window, double degen,
                               double* __restrict__ vel) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nkept) return;
  double vd[kMaxBands][3];
  for (int m = 0; m < nb; ++m)
    for (int c = 0; c < 3; ++c) vd[m][c] = vdin[(t * nb + m) * 3 + c];
  const double* e = eps_all + (int64_t)kept[t] * nb;
  int start = 0;
  for (int b = 1; b <= nb; ++b) {
    if (b == nb || e[b] - e[b - 1] >= degen) {
      if (b - start > 1) {
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int m = start; m < b; ++m) s += vd[m][c];
          s /= (double)(b - start);
          for (int m = start; m < b; ++m) vd[m][c] = s;
        }
      }
      start = b;
    }
  }
  int o = soff[t];
  for (int m = 0; m < nb; ++m) {
    if (fabs(e[m] - mu) <= window) {
      for (int c = 0; c < 3; ++c) vel[(int64_t)o * 3 + c] = vd[m][c];
      ++o;
    }
  }
}

// Phonon factors per element: hbar omega_s = sqrt(C max(lambda_s, 0)) and
// Lq[q][x][s] = l_{x,s} u_q[x][s] with l = sqrt(C / (2 M_x hbar omega_s))
// (zero for modes below omega_min); thread per (q, x, s).
// Mesh index of -q
__device__ inline int64_t mesh_neg(int64_t q, int n0, int n1, int n2) {
  const int64_t c = q % n2, t = q / n2;
  const int64_t b = t % n1, a = t / n1;
  return ((a ? n0 - a : 0) * n1 + (b ? n1 - b : 0)) * n2 + (c ? n2 - c : 0);
}

// The force constants are real, so D(-q) = D(q)^* (time reversal): the
// modes at -q are those at q with conjugated eigenvectors, the same
// frequencies and opposite velocities.  The phonon tables are therefore
// diagonalised at one q of each +-q pair (pts) and written at both.

// hbar omega = sqrt(C lambda) and L[q][x][s] = u_xs sqrt(C / (2 M_x omega))
// (Eq. 6 prefactor); thread per (point, x, s) of the chunk, also written at -q
__global__ void k_phonon_hw_L(int64_t nq, int nbr, MeshDims md, const int32_t* __restrict__ pts,
                              const double* __restrict__ lam, const cd* __restrict__ u,
                              const double* __restrict__ mass_x, double omega_min, double* __restrict__ hw,
                              cd* __restrict__ Lq) {
  const int64_t nn = (int64_t)nbr * nbr;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * nn) return;
  const int64_t p = e / nn;
  const int xs = (int)(e - p * nn), x = xs / nbr, s = xs - x * nbr;
  const int64_t q = pts[p], mq = mesh_neg(q, md.n0, md.n1, md.n2);
  const double l = lam[p * nbr + s];
  const double w = sqrt(kPhononC * (l > 0.0 ? l : 0.0));
  const cd L = (w >= omega_min) ? cscale(u[e], sqrt(kPhononC / (2.0 * mass_x[x] * w))) : cmake(0.0, 0.0);
  if (x == 0) hw[q * nbr + s] = w;
  Lq[q * nn + xs] = L;
  if (mq != q) {
    if (x == 0) hw[mq * nbr + s] = w;
    Lq[mq * nn + xs] = cconj(L);
  }
}

// Branch velocities (Eq. 5) v_c = (C / (2 hbar omega)) u_s^+ (dD/dq_c) u_s / hbar
// before degenerate averaging; thread per (point, c, s) of the chunk, result
// in vph at q = pts[point].
__global__ void k_phonon_vel(int64_t nq, int nbr, const int32_t* __restrict__ pts, const double* __restrict__ hw,
                             const cd* __restrict__ u, const cd* __restrict__ dD, double omega_min,
                             double* __restrict__ vph) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * 3 * nbr) return;
  const int64_t p = e / (3 * nbr);
  const int cs = (int)(e - p * 3 * nbr), c = cs / nbr, s = cs - c * nbr;
  const int64_t nn = (int64_t)nbr * nbr;
  const int64_t q = pts[p];
  const double w = hw[q * nbr + s];
  double acc = 0.0;
  if (w >= omega_min) {
    const cd* d = dD + (p * 3 + c) * nn;
    const cd* uq = u + p * nn;
    for (int a = 0; a < nbr; ++a) {
      cd row = cmake(0, 0);
      for (int b = 0; b < nbr; ++b) row = cadd(row, cmul(d[a * nbr + b], uq[b * nbr + s]));
      acc += cmul(cconj(uq[a * nbr + s]), row).x;
    }
    acc = kPhononC * acc / (2.0 * w) * (kAngM / kHbarEVs);
  }
  vph[(q * nbr + s) * 3 + c] = acc;
}

// Average the branch velocities at q = pts[point] over groups of
// (near-)degenerate branches, then write their negatives at -q.
__global__ void k_phonon_degen(int64_t nq, int nbr, MeshDims md, const int32_t* __restrict__ pts,
                               const double* __restrict__ hw, double degen, double* __restrict__ vph) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nq) return;
  const int64_t q = pts[p], mq = mesh_neg(q, md.n0, md.n1, md.n2);
  const double* w = hw + q * nbr;
  double* v = vph + q * nbr * 3;
  int start = 0;
  for (int b = 1; b <= nbr; ++b) {
    if (b == nbr || w[b] - w[b - 1] >= degen) {
      if (b - start > 1) {
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int m = start; m < b; ++m) s += v[m * 3 + c];
          s /= (double)(b - start);
          for (int m = start; m < b; ++m) v[m * 3 + c] = s;
        }
      }
      start = b;
    }
  }
  if (mq != q) {
    double* vm = vph + mq * nbr * 3;
    for (int e = 0; e < nbr * 3; ++e) vm[e] = -v[e];
  }
}

// phase tables of kept k: Ee[t][r] = w_r e^{2 pi i k.Re_r}, Ep[t][r] = e^{2 pi i k.Rp_r}
__global__ void k_kept_phases(MeshPhase ph, const int32_t* __restrict__ kept, int64_t nkept,
                              const int32_t* __restrict__ R, const double* __restrict__ w, int nR,
                              cd* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nkept * nR) return;
  int64_t t = e / nR;
  int r = (int)(e % nR);
  int a, b, c;
  mesh_coords(kept[t], ph.n1, ph.n2, a, b, c);
  cd z = ph(a, b, c, R[3 * r], R[3 * r + 1], R[3 * r + 2]);
  out[e] = cscale(z, w ? w[r] : 1.0);
}

__global__ void k_max_reduce(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double s[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, x[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

// Eq. 4, the non-analytic (dipole-dipole) part of D(q) for polar materials,
// added to the chunk's D and its Cartesian gradient: coef (q.Z_t)_a
// (q.Z_t')_b / (q.eps.q) / sqrt(m_t m_t') with (q.Z_t)_b = sum_a q_a Z_t[a][b],
// q the image of the mesh point nearest Gamma (fractional coordinates in
// [-1/2, 1/2), 2 pi included), averaged over the two images of a coordinate
// at exactly 1/2 so that the term stays even in q; nothing at Gamma.
// Thread per (point, x, y).
__global__ void k_nac_add(int64_t npts, int nbr, MeshDims md, const int32_t* __restrict__ pts,
                          const double* __restrict__ nac, double coef, const double* __restrict__ mass_x,
                          cd* __restrict__ D, cd* __restrict__ G) {
  const int64_t nn = (int64_t)nbr * nbr;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npts * nn) return;
  const int64_t p = e / nn;
  const int xy = (int)(e - p * nn), x = xy / nbr, y = xy - x * nbr;
  const int na = nbr / 3;
  const int tx = x / 3, ax = x % 3, ty = y / 3, ay = y % 3;
  const double* Z = nac;
  const double* eps = nac + 9 * na;
  const double* B = eps + 9;
  const int64_t k = pts ? (int64_t)pts[p] : p;
  const int c = (int)(k % md.n2), t = (int)(k / md.n2), b = t % md.n1, a = t / md.n1;
  const int idx[3] = {a, b, c}, nd[3] = {md.n0, md.n1, md.n2};
  double f[3];
  bool half[3];
  int nimg = 1;
  for (int d = 0; d < 3; ++d) {
    half[d] = 2 * idx[d] == nd[d];
    f[d] = (double)idx[d] / nd[d];
    if (2 * idx[d] >= nd[d]) f[d] -= 1.0;
    if (half[d]) nimg *= 2;
  }
  const double s = coef / sqrt(mass_x[x] * mass_x[y]) / nimg;
  double dsum = 0.0, gsum[3] = {0.0, 0.0, 0.0};
  for (int im = 0; im < 8; ++im) {
    // image im: bit d set moves a coordinate at -1/2 to +1/2
    bool skip = false;
    double g[3];
    for (int d = 0; d < 3; ++d) {
      const bool up = (im >> d) & 1;
      if (up && !half[d]) skip = true;
      g[d] = f[d] + (up ? 1.0 : 0.0);
    }
    if (skip) continue;
    double q[3];
    for (int d = 0; d < 3; ++d) q[d] = g[0] * B[d] + g[1] * B[3 + d] + g[2] * B[6 + d];
    double eq[3], Q = 0.0;
    for (int d = 0; d < 3; ++d) {
      eq[d] = eps[3 * d] * q[0] + eps[3 * d + 1] * q[1] + eps[3 * d + 2] * q[2];
      Q += q[d] * eq[d];
    }
    if (!(Q > 0.0)) continue;
    double A = 0.0, Bv = 0.0;  // (q.Z_tx)_ax, (q.Z_ty)_ay
    for (int d = 0; d < 3; ++d) {
      A += q[d] * Z[(tx * 3 + d) * 3 + ax];
      Bv += q[d] * Z[(ty * 3 + d) * 3 + ay];
    }
    dsum += A * Bv / Q;
    for (int d = 0; d < 3; ++d)
      gsum[d] += (Z[(tx * 3 + d) * 3 + ax] * Bv + A * Z[(ty * 3 + d) * 3 + ay]) / Q - 2.0 * eq[d] * A * Bv / (Q * Q);
  }
  D[p * nn + xy].x += s * dsum;
  if (G)
    for (int d = 0; d < 3; ++d) G[(p * 3 + d) * nn + xy].x += s * gsum[d];
}

// Eq. 7 without its electron overlap: F_s(q) = i (e^2 / (eps_0 V)) sum_t
// sum_{G != -q} ((q+G).Z_t.lu_t,s) / ((q+G).eps.(q+G)) exp(-i (q+G).r_t)
// exp(-(q+G).eps.(q+G) / (4 alpha)), alpha = 1 Bohr^-2, over the G of a box
// with (q+G).eps.(q+G) / (4 alpha) <= 40; lu = l u, the phonon factors of
// Eq. 6 (Angstrom).  Thread per point; every G term serves all branches.
// The box is walked in rows along the third reciprocal vector, where Q is
// a quadratic in the row index (only its range inside the cutoff is
// visited) and the phases advance by one fixed factor per step.
constexpr double kBohrA = 0.529177210903;
constexpr double kEwaldInv4a = kBohrA * kBohrA / 4.0;  // 1 / (4 alpha), Angstrom^2
constexpr double kEwaldCut = 40.0;

__global__ void __launch_bounds__(256) k_frohlich(int64_t npts, int nbr, MeshDims md, const int32_t* __restrict__ pts,
                                                  const double* __restrict__ nac, double coef, int g0, int g1, int g2,
                                                  const cd* __restrict__ Lq, cd* __restrict__ F) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const int na = nbr / 3;
  const double* Z = nac;
  const double* eps = nac + 9 * na;
  const double* B = eps + 9;
  const double* tau = B + 9;
  const int64_t k = pts ? (int64_t)pts[p] : p;
  const int c = (int)(k % md.n2), t = (int)(k / md.n2), b = t % md.n1, a = t / md.n1;
  const double f[3] = {(double)a / md.n0, (double)b / md.n1, (double)c / md.n2};
  const cd* lu = Lq + p * nbr * nbr;
  const double qmax = kEwaldCut / kEwaldInv4a;  // (q+G).eps.(q+G) bound of the kept terms
  // along a row of the box, q + G = P + l B2: Q(l) = qa l^2 + qb l + qc
  double eB2[3];
  for (int d = 0; d < 3; ++d) eB2[d] = eps[3 * d] * B[6] + eps[3 * d + 1] * B[7] + eps[3 * d + 2] * B[8];
  const double qa = B[6] * eB2[0] + B[7] * eB2[1] + B[8] * eB2[2];
  // per atom, W_t = sum_G w_G ((q+G).Z_t) with the complex weight
  // w_G = exp(-i (q+G).r_t) exp(-Q/(4 alpha)) / Q; F_s = i coef sum_t W_t . lu_t,s
  double wr[5][3], wi[5][3];
#pragma unroll
  for (int at = 0; at < 5; ++at)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) wr[at][bb] = wi[at][bb] = 0.0;
  for (int i = -g0; i <= g0; ++i)
    for (int j = -g1; j <= g1; ++j) {
      const double h0 = f[0] + i, h1 = f[1] + j;
      double P[3];
      for (int d = 0; d < 3; ++d) P[d] = h0 * B[d] + h1 * B[3 + d] + f[2] * B[6 + d];
      double eP[3];
      for (int d = 0; d < 3; ++d) eP[d] = eps[3 * d] * P[0] + eps[3 * d + 1] * P[1] + eps[3 * d + 2] * P[2];
      const double qb = 2.0 * (B[6] * eP[0] + B[7] * eP[1] + B[8] * eP[2]);
      const double qc = P[0] * eP[0] + P[1] * eP[1] + P[2] * eP[2];
      // l range of Q(l) <= qmax (widened by one; every term is still tested)
      const double disc = qb * qb - 4.0 * qa * (qc - qmax);
      if (disc < 0.0) continue;
      const double sq = sqrt(disc);
      int l0 = (int)floor((-qb - sq) / (2.0 * qa)) - 1, l1 = (int)ceil((-qb + sq) / (2.0 * qa)) + 1;
      l0 = l0 < -g2 ? -g2 : l0;
      l1 = l1 > g2 ? g2 : l1;
      if (l0 > l1) continue;
#pragma unroll
      for (int at = 0; at < 5; ++at) {
        if (at >= na) break;
        // exp(-i (P + l B2).r) from its value at l0 and the per-step factor
        const double* r = tau + 3 * at;
        const double br = B[6] * r[0] + B[7] * r[1] + B[8] * r[2];
        double s0, c0, s1, c1;
        sincos(P[0] * r[0] + P[1] * r[1] + P[2] * r[2] + l0 * br, &s0, &c0);
        sincos(br, &s1, &c1);
        double phr = c0, phi = -s0;
        const double str = c1, sti = -s1;
        // (q+G).Z_t = P.Z_t + l B2.Z_t
        double pz[3], bz[3];
        for (int bb = 0; bb < 3; ++bb) {
          pz[bb] = P[0] * Z[(at * 3 + 0) * 3 + bb] + P[1] * Z[(at * 3 + 1) * 3 + bb] + P[2] * Z[(at * 3 + 2) * 3 + bb];
          bz[bb] = B[6] * Z[(at * 3 + 0) * 3 + bb] + B[7] * Z[(at * 3 + 1) * 3 + bb] + B[8] * Z[(at * 3 + 2) * 3 + bb];
        }
        for (int l = l0; l <= l1; ++l) {
          const double Q = (qa * l + qb) * l + qc;
          if (Q > 0.0 && Q * kEwaldInv4a <= kEwaldCut) {
            const double damp = exp(-Q * kEwaldInv4a) / Q;
            const double pr = phr * damp, pi = phi * damp;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
              const double z = pz[bb] + l * bz[bb];
              wr[at][bb] += pr * z;
              wi[at][bb] += pi * z;
            }
          }
          const double nr = phr * str - phi * sti;
          phi = phr * sti + phi * str;
          phr = nr;
        }
      }
    }
  for (int s = 0; s < nbr; ++s) {
    double xr = 0.0, xi = 0.0;
#pragma unroll
    for (int at = 0; at < 5; ++at) {
      if (at >= na) break;
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        const cd u = lu[(3 * at + bb) * nbr + s];
        xr += wr[at][bb] * u.x - wi[at][bb] * u.y;
        xi += wr[at][bb] * u.y + wi[at][bb] * u.x;
      }
    }
    F[p * nbr + s] = cmake(-coef * xi, coef * xr);  // i coef sum
  }
}

__global__ void k_fill_ustate(int64_t M, int nb, const int32_t* __restrict__ st_kidx, const int32_t* __restrict__ st_m,
                              const cd* __restrict__ U, cd* __restrict__ us) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * nb) return;
  const int64_t i = e / nb;
  const int w = (int)(e - i * nb);
  us[e] = U[((int64_t)st_kidx[i] * nb + w) * nb + st_m[i]];
}

void launch_frohlich(elph_ctx ctx, const int32_t* pts, int64_t npts, const cd* Lq, cd* F, hipStream_t s) {
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  hipLaunchKernelGGL(k_frohlich, dim3(blocks_for(npts, 256)), dim3(256), 0, s, npts, ctx->nbr, md, pts, ctx->d_nac,
                     ctx->nac_coef, ctx->fr_box[0], ctx->fr_box[1], ctx->fr_box[2], Lq, F);
}

// ---------------------------------------------------------------------------
// host drivers


template <bool REAL_IN, bool GRAD>
static void launch_fourier(elph_ctx ctx, const int32_t* pts, int64_t base, int64_t npts, const int32_t* R,
                           const double* w, int nR, const double* Min, int n, cd* out, cd* grad) {
  const int nn = n * n;
  constexpr int CT = GRAD ? 1 : 4;  // column tiles per wavefront
  hipLaunchKernelGGL((k_fourier_mfma<REAL_IN, GRAD, CT>),
                     dim3(blocks_for(npts, 64), (unsigned)((nn + 16 * CT - 1) / (16 * CT))), dim3(256), 0,
                     ctx->stream, mesh_phase(ctx), pts, base, npts, R, w, nR, ctx->d_lat, Min, nn, out, grad);
}

elph_status build_tables(elph_ctx ctx) {
  if (ctx->tables_ready) return ELPH_OK;
  mark(ctx, 0);
  hipStream_t s = ctx->stream;
  const int nb = ctx->nb, nbr = ctx->nbr;
  const int64_t nk = ctx->nk;
  const int64_t chunk = 1 << 16;

  // ---- electrons on the whole mesh: eigenvalues decide the window (Eq. 1)
  ALLOC(ctx->d_eps_all, nk * nb * sizeof(double));
  cd* hbuf = nullptr;
  const int nmaxb = nb > nbr ? nb : nbr;
  ALLOC(hbuf, chunk * (int64_t)nmaxb * nmaxb * sizeof(cd));
  cd* gbuf = nullptr;
  ALLOC(gbuf, chunk * 3 * (int64_t)nmaxb * nmaxb * sizeof(cd));
  for (int64_t k0 = 0; k0 < nk; k0 += chunk) {
    int64_t cnt = (nk - k0 < chunk) ? nk - k0 : chunk;
    launch_fourier<false, false>(ctx, nullptr, k0, cnt, ctx->d_re, ctx->d_wre, ctx->nre, ctx->d_hr, nb, hbuf,
                                 nullptr);
    launch_jacobi(hbuf, cnt, nb, ctx->d_eps_all + k0 * nb, nullptr, s);
  }
  HIPCHK(hipGetLastError());

  // ---- window and compaction
  int32_t *nact_mesh = nullptr, *flag = nullptr, *pos = nullptr, *scr = nullptr, *tot = nullptr;
  ALLOC(nact_mesh, nk * sizeof(int32_t));
  ALLOC(flag, nk * sizeof(int32_t));
  ALLOC(pos, nk * sizeof(int32_t));
  ALLOC(scr, (4 * ((nk + 1023) / 1024) + 64) * sizeof(int32_t));
  ALLOC(tot, 2 * sizeof(int32_t));
  hipLaunchKernelGGL(k_window, dim3(blocks_for(nk, 256)), dim3(256), 0, s, ctx->d_eps_all, nk, nb, ctx->mu,
                     ctx->window, nact_mesh, flag);
  scan_exclusive(ctx, flag, nk, pos, tot, scr, s);
  int32_t h_nkept = 0;
  HIPCHK(hipMemcpyAsync(&h_nkept, tot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->nkept = h_nkept;
  if (ctx->nkept == 0) {
    ctx->err = "no electron state inside the transport window";
    return ELPH_EINVAL;
  }
  ALLOC(ctx->d_kidx, nk * sizeof(int32_t));
  ALLOC(ctx->d_kept, ctx->nkept * sizeof(int32_t));
  int32_t* nact_kept = nullptr;
  ALLOC(nact_kept, (ctx->nkept + 1) * sizeof(int32_t));
  ALLOC(ctx->d_soff, (ctx->nkept + 1) * sizeof(int32_t));
  hipLaunchKernelGGL(k_compact_kept, dim3(blocks_for(nk, 256)), dim3(256), 0, s, flag, pos, nk, ctx->d_kidx,
                     ctx->d_kept, nact_mesh, nact_kept);
  scan_exclusive(ctx, nact_kept, ctx->nkept, ctx->d_soff, tot + 1, scr, s);
  HIPCHK(hipMemcpyAsync(ctx->d_soff + ctx->nkept, tot + 1, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  int32_t h_ns = 0;
  HIPCHK(hipMemcpyAsync(&h_ns, tot + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->nstates = h_ns;
  const int64_t M = ctx->nstates;
  ALLOC(ctx->d_state_k, M * sizeof(int32_t));
  ALLOC(ctx->d_state_kidx, M * sizeof(int32_t));
  ALLOC(ctx->d_state_m, M * sizeof(int32_t));
  ALLOC(ctx->d_eps, M * sizeof(double));
  ALLOC(ctx->d_vel, M * 3 * sizeof(double));
  hipLaunchKernelGGL(k_fill_states, dim3(blocks_for(ctx->nkept, 256)), dim3(256), 0, s, ctx->d_kept, ctx->nkept,
                     ctx->d_soff, ctx->d_eps_all, nb, ctx->mu, ctx->window, ctx->d_state_k, ctx->d_state_kidx,
                     ctx->d_state_m, ctx->d_eps);

  // ---- eigenvectors and velocities of kept k (Eqs. 1, 2)
  ALLOC(ctx->d_U, ctx->nkept * (int64_t)nb * nb * sizeof(cd));
  double* vdbuf = nullptr;
  ALLOC(vdbuf, std::min<int64_t>(chunk, ctx->nkept) * nb * 3 * sizeof(double));
  for (int64_t k0 = 0; k0 < ctx->nkept; k0 += chunk) {
    int64_t cnt = (ctx->nkept - k0 < chunk) ? ctx->nkept - k0 : chunk;
    launch_fourier<false, true>(ctx, ctx->d_kept + k0, 0, cnt, ctx->d_re, ctx->d_wre, ctx->nre, ctx->d_hr, nb, hbuf,
                                gbuf);
    launch_jacobi(hbuf, cnt, nb, nullptr, (cd*)ctx->d_U + k0 * nb * nb, s);
    hipLaunchKernelGGL(k_electron_vd, dim3(blocks_for(cnt * 3 * nb, 256)), dim3(256), 0, s, cnt, nb,
                       (const cd*)ctx->d_U + k0 * nb * nb, gbuf, vdbuf);
    hipLaunchKernelGGL(k_electron_vel, dim3(blocks_for(cnt, 64)), dim3(64), 0, s, cnt, nb, vdbuf, ctx->d_eps_all,
                       ctx->d_kept + k0, ctx->d_soff + k0, ctx->mu, ctx->window, 1.0e-6, ctx->d_vel);
  }
  HIPCHK(hipGetLastError());

  // ---- phonons on the whole q mesh (Eqs. 3, 5, 6 prefactor)
  ALLOC(ctx->d_hw, nk * nbr * sizeof(double));
  ALLOC(ctx->d_Lq, nk * (int64_t)nbr * nbr * sizeof(cd));
  ALLOC(ctx->d_vph, nk * nbr * 3 * sizeof(double));
  double* lam = nullptr;
  cd* ubuf = nullptr;
  ALLOC(lam, chunk * nbr * sizeof(double));
  ALLOC(ubuf, chunk * (int64_t)nbr * nbr * sizeof(cd));
  const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
  for (int64_t r0 = 0; r0 < ctx->nqrep; r0 += chunk) {
    const int64_t cnt = (ctx->nqrep - r0 < chunk) ? ctx->nqrep - r0 : chunk;
    const int32_t* pts = ctx->d_qrep + r0;  // one q of each +-q pair; -q follows by time reversal
    launch_fourier<true, true>(ctx, pts, 0, cnt, ctx->d_rp, ctx->d_wrp, ctx->nrp, ctx->d_dr, nbr, hbuf, gbuf);
    if (ctx->d_nac)
      hipLaunchKernelGGL(k_nac_add, dim3(blocks_for(cnt * nbr * nbr, 256)), dim3(256), 0, s, cnt, nbr, md, pts,
                         ctx->d_nac, ctx->nac_coef, ctx->d_mass_x, hbuf, gbuf);
    launch_jacobi(hbuf, cnt, nbr, lam, ubuf, s);
    hipLaunchKernelGGL(k_phonon_hw_L, dim3(blocks_for(cnt * nbr * nbr, 256)), dim3(256), 0, s, cnt, nbr, md, pts,
                       lam, ubuf, ctx->d_mass_x, ctx->omega_min, ctx->d_hw, (cd*)ctx->d_Lq);
    hipLaunchKernelGGL(k_phonon_vel, dim3(blocks_for(cnt * 3 * nbr, 256)), dim3(256), 0, s, cnt, nbr, pts,
                       ctx->d_hw, ubuf, gbuf, ctx->omega_min, ctx->d_vph);
    hipLaunchKernelGGL(k_phonon_degen, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, cnt, nbr, md, pts, ctx->d_hw,
                       1.0e-6, ctx->d_vph);
  }
  HIPCHK(hipGetLastError());

  // ---- the active states' eigenvectors (state overlaps of Eq. 7, error
  // estimates and FP64 refinement of the GEMM forms) and, for polar
  // materials, F_s(q) of Eq. 7
  ALLOC(ctx->d_ustate, ctx->nstates * nb * sizeof(cd));
  hipLaunchKernelGGL(k_fill_ustate, dim3(blocks_for(ctx->nstates * nb, 256)), dim3(256), 0, s, ctx->nstates, nb,
                     ctx->d_state_kidx, ctx->d_state_m, (const cd*)ctx->d_U, (cd*)ctx->d_ustate);
  HIPCHK(hipGetLastError());
  if (ctx->frohlich) {
    ALLOC(ctx->d_frohlich, nk * nbr * sizeof(cd));
    mark(ctx, 8);
    launch_frohlich(ctx, nullptr, nk, (const cd*)ctx->d_Lq, (cd*)ctx->d_frohlich, s);
    mark(ctx, 9);
  }

  // ---- hw_max
  double* red = nullptr;
  ALLOC(red, 256 * sizeof(double));
  hipLaunchKernelGGL(k_max_reduce, dim3(256), dim3(256), 0, s, ctx->d_hw, nk * nbr, red);
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, red, 256, red);
  HIPCHK(hipMemcpyAsync(&ctx->hw_max, red, sizeof(double), hipMemcpyDeviceToHost, s));

  // ---- phases of kept k
  ALLOC(ctx->d_Ee, ctx->nkept * ctx->nre * sizeof(cd));
  ALLOC(ctx->d_Ep, ctx->nkept * ctx->nrp * sizeof(cd));
  hipLaunchKernelGGL(k_kept_phases, dim3(blocks_for(ctx->nkept * ctx->nre, 256)), dim3(256), 0, s,
                     mesh_phase(ctx), ctx->d_kept, ctx->nkept, ctx->d_re, ctx->d_wre, ctx->nre, (cd*)ctx->d_Ee);
  hipLaunchKernelGGL(k_kept_phases, dim3(blocks_for(ctx->nkept * ctx->nrp, 256)), dim3(256), 0, s,
                     mesh_phase(ctx), ctx->d_kept, ctx->nkept, ctx->d_rp, nullptr, ctx->nrp, (cd*)ctx->d_Ep);
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());

  // scratch no longer needed
  dev_free(ctx, hbuf);
  dev_free(ctx, gbuf);
  dev_free(ctx, nact_mesh);
  dev_free(ctx, flag);
  dev_free(ctx, pos);
  dev_free(ctx, scr);
  dev_free(ctx, tot);
  dev_free(ctx, nact_kept);
  dev_free(ctx, vdbuf);
  dev_free(ctx, lam);
  dev_free(ctx, ubuf);
  dev_free(ctx, red);
  mark(ctx, 1);
  ctx->tables_ready = true;
  return ELPH_OK;
}

elph_status make_axis_tables(elph_ctx ctx) {
  for (int d = 0; d < 3; ++d) {
    ALLOC(ctx->d_tab[d], ctx->mesh[d] * sizeof(double2));
    hipLaunchKernelGGL(k_axis_table, dim3(blocks_for(ctx->mesh[d], 256)), dim3(256), 0, ctx->stream,
                       ctx->mesh[d], ctx->d_tab[d]);
  }
  HIPCHK(hipGetLastError());
  // one q of each +-q pair of the mesh (the smaller mesh index)
  const int64_t n0 = ctx->mesh[0], n1 = ctx->mesh[1], n2 = ctx->mesh[2], nk = n0 * n1 * n2;
  std::vector<int32_t> rep;
  rep.reserve((size_t)(nk / 2 + 8));
  for (int64_t a = 0; a < n0; ++a)
    for (int64_t b = 0; b < n1; ++b)
      for (int64_t c = 0; c < n2; ++c) {
        const int64_t q = (a * n1 + b) * n2 + c;
        const int64_t mq = ((a ? n0 - a : 0) * n1 + (b ? n1 - b : 0)) * n2 + (c ? n2 - c : 0);
        if (q <= mq) rep.push_back((int32_t)q);
      }
  ctx->nqrep = (int64_t)rep.size();
  ALLOC(ctx->d_qrep, rep.size() * sizeof(int32_t));
  HIPCHK(hipMemcpy(ctx->d_qrep, rep.data(), rep.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return ELPH_OK;
}

// H(k) (and optionally eigen-decomposition) for an arbitrary list of mesh points
elph_status fourier_points(elph_ctx ctx, bool phonon, const int32_t* pts, int64_t npts, cd* out) {
  if (phonon) {
    launch_fourier<true, false>(ctx, pts, 0, npts, ctx->d_rp, ctx->d_wrp, ctx->nrp, ctx->d_dr, ctx->nbr, out,
                                nullptr);
    if (ctx->d_nac) {
      const MeshDims md{ctx->mesh[0], ctx->mesh[1], ctx->mesh[2]};
      hipLaunchKernelGGL(k_nac_add, dim3(blocks_for(npts * ctx->nbr * ctx->nbr, 256)), dim3(256), 0, ctx->stream,
                         npts, ctx->nbr, md, pts, ctx->d_nac, ctx->nac_coef, ctx->d_mass_x, out, (cd*)nullptr);
    }
  }
  else
    launch_fourier<false, false>(ctx, pts, 0, npts, ctx->d_re, ctx->d_wre, ctx->nre, ctx->d_hr, ctx->nb, out,
                                 nullptr);
  HIPCHK(hipGetLastError());
  return ELPH_OK;
}

}  // namespace elph
