// Screening MLP on gfx950.  Hidden layers z_l = a_{l-1} W_l + b_l and
// a_l = GELU(z_l) = z_l Phi(z_l) (the erf form), output y = a_L w + b, loss =
// mean squared error.  Matrix products take BF16 operands on the 16x16x32
// BF16 MFMA with FP32 accumulation; weights are kept as FP32 masters (Adam
// updates them) with BF16 copies for the products; pre-activations are kept
// in FP32 for the GELU derivative, activations and backward signals in BF16.
// Every reduction runs in a fixed order, so results are deterministic.
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#define MCHK(x)                                                                            \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      m->err = std::string("HIP error ") + hipGetErrorString(e_) + " at " + __FILE__ + ":" + \
               std::to_string(__LINE__);                                                   \
      m->hip_dead = true;                                                                  \
      return ELPH_EHIP;                                                                    \
    }                                                                                      \
  } while (0)

namespace elph {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ inline unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------
// C(m, n) = sum_k A(m, k) B(k, n).  A(m, k) = A[m lda + k] when AK (k
// contiguous) else A[k lda + m]; B(k, n) = B[n ldb + k] when BK else
// B[k ldb + n].  Block tile 64 x 64 staged through LDS as [row][k], k step 32;
// four wavefronts of 32 x 32 (2 x 2 MFMA tiles).  Host-checked requirements:
// K and the per-block k range are multiples of 32; an operand read
// contiguously along m (n) has M (N) a multiple of 8; leading dimensions are
// multiples of 8.
enum { EPI_STORE = 0, EPI_FWD = 1, EPI_BWD = 2 };

struct GemmP {
  int M, N, K, kchunk;
  const unsigned short* A;
  int64_t lda;
  const unsigned short* B;
  int64_t ldb;
  int64_t ldc;
  float* C;                  // EPI_STORE: partials [blockIdx.z][M][ldc]
  const float* bias;         // EPI_FWD
  float* zout;               // EPI_FWD, may be null: FP32 pre-activations
  unsigned short* hout;      // EPI_FWD: BF16 GELU(z); EPI_BWD: BF16 acc * GELU'(zprev)
  const float* zprev;        // EPI_BWD
};

template <bool AK, bool BK, int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmP p) {
  __shared__ __attribute__((aligned(16))) unsigned short As[64][40];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[64][40];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * p.kchunk;
  const int ke = min(p.K, kb + p.kchunk);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lq = (lane >> 4) * 8;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  const us8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    if (AK) {
      const int r = tid >> 2, kq = (tid & 3) * 8;
      us8 v = zero8;
      if (m0 + r < p.M) v = *(const us8*)(p.A + (int64_t)(m0 + r) * p.lda + k0 + kq);
      *(us8*)&As[r][kq] = v;
    } else {
      const int kk = tid >> 3, mr = (tid & 7) * 8;
      us8 v = zero8;
      if (m0 + mr < p.M) v = *(const us8*)(p.A + (int64_t)(k0 + kk) * p.lda + m0 + mr);
#pragma unroll
      for (int t = 0; t < 8; ++t) As[mr + t][kk] = v[t];
    }
    if (BK) {
      const int r = tid >> 2, kq = (tid & 3) * 8;
      us8 v = zero8;
      if (n0 + r < p.N) v = *(const us8*)(p.B + (int64_t)(n0 + r) * p.ldb + k0 + kq);
      *(us8*)&Bs[r][kq] = v;
    } else {
      const int kk = tid >> 3, nr = (tid & 7) * 8;
      us8 v = zero8;
      if (n0 + nr < p.N) v = *(const us8*)(p.B + (int64_t)(k0 + kk) * p.ldb + n0 + nr);
#pragma unroll
      for (int t = 0; t < 8; ++t) Bs[nr + t][kk] = v[t];
    }
    __syncthreads();
    bf8 af[2], bfr[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) af[a] = __builtin_bit_cast(bf8, *(const us8*)&As[wm + 16 * a + lr][lq]);
#pragma unroll
    for (int b = 0; b < 2; ++b) bfr[b] = __builtin_bit_cast(bf8, *(const us8*)&Bs[wn + 16 * b + lr][lq]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mm = m0 + wm + 16 * a + (lane >> 4) * 4 + r;
        const int nn = n0 + wn + 16 * b + lr;
        if (mm >= p.M || nn >= p.N) continue;
        const float v = acc[a][b][r];
        const int64_t o = (int64_t)mm * p.ldc + nn;
        if (EPI == EPI_STORE) {
          p.C[(int64_t)blockIdx.z * p.M * p.ldc + o] = v;
        } else if (EPI == EPI_FWD) {
          const float z = v + p.bias[nn];
          if (p.zout) p.zout[o] = z;
          p.hout[o] = f2bf(gelu(z));
        } else {
          p.hout[o] = f2bf(v * gelu_grad(p.zprev[o]));
        }
      }
}

// ---------------------------------------------------------------------------
// small kernels

__global__ void k_x_to_bf(int64_t n, int nin, int in_pad, const float* __restrict__ x,
                          unsigned short* __restrict__ xb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * in_pad) return;
  const int64_t r = t / in_pad;
  const int c = (int)(t - r * in_pad);
  xb[t] = c < nin ? f2bf(x[r * nin + c]) : (unsigned short)0;
}

// BF16 copies of W_l ([K][W] and [W][K], rows/columns >= fan_in zero) and of
// the output weights
__global__ void k_refresh(const float* __restrict__ Wsrc, int fan_in, int K, int W, unsigned short* __restrict__ Wb,
                          unsigned short* __restrict__ Wtb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)K * W) return;
  const int k = (int)(t / W), j = (int)(t - (int64_t)k * W);
  const unsigned short v = k < fan_in ? f2bf(Wsrc[(int64_t)k * W + j]) : (unsigned short)0;
  if (Wb) Wb[t] = v;
  if (Wtb) Wtb[(int64_t)j * K + k] = v;
}

// y[r] = sum_k h[r][k] w[k] + b (one wavefront per row)
__global__ void __launch_bounds__(256) k_out_fwd(int64_t n, int W, const unsigned short* __restrict__ h,
                                                 const unsigned short* __restrict__ w, const float* __restrict__ b,
                                                 float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  float s = 0.f;
  for (int k = lane; k < W; k += 64) s += bf2f(h[r * W + k]) * bf2f(w[k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) y[r] = s + b[0];
}

// dy[r] = 2 (y - t) / n; dz[r][k] = BF16(dy w[k] GELU'(z[r][k])); lpart[block] = sum (y - t)^2
__global__ void __launch_bounds__(256) k_out_bwd(int64_t n, int W, const float* __restrict__ y,
                                                 const float* __restrict__ t, const unsigned short* __restrict__ w,
                                                 const float* __restrict__ z, float* __restrict__ dy,
                                                 unsigned short* __restrict__ dz, float* __restrict__ lpart) {
  __shared__ float sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 4 + wave;
  float l2 = 0.f;
  if (r < n) {
    const float e = y[r] - t[r];
    const float d = 2.f * e / (float)n;
    l2 = e * e;
    if (lane == 0) dy[r] = d;
    for (int k = lane; k < W; k += 64) dz[r * W + k] = f2bf(d * bf2f(w[k]) * gelu_grad(z[r * W + k]));
  }
  if (lane == 0) sh[wave] = l2;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// part[block][c] = sum over the block's rows r of src[r][c] (* scale[r])
__global__ void __launch_bounds__(256) k_colsum(int64_t n, int W, const unsigned short* __restrict__ src,
                                                const float* __restrict__ scale, float* __restrict__ part) {
  for (int c = threadIdx.x; c < W; c += 256) {
    float s = 0.f;
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) s += bf2f(src[r * W + c]) * (scale ? scale[r] : 1.f);
    part[(int64_t)blockIdx.x * W + c] = s;
  }
}

// out[i] = sum_s part[s * stride + i], s in order
__global__ void k_sum_parts(int64_t len, int nparts, int64_t stride, const float* __restrict__ part,
                            float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int k = 0; k < nparts; ++k) s += part[(int64_t)k * stride + i];
  out[i] = s;
}

// out[0] = sum of a[0..n) (one block; strided partial sums, then a fixed tree)
__global__ void __launch_bounds__(256) k_sum_f32(const float* __restrict__ a, int64_t n, float* __restrict__ out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += a[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ ve, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * mo[i] + (1.f - b1) * gi;
  const float vi = b2 * ve[i] + (1.f - b2) * gi * gi;
  mo[i] = mi;
  ve[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// host side

static elph_status malloc_m(elph_mlp m, void** p, size_t bytes) {
  *p = nullptr;
  if (hipMalloc(p, bytes > 0 ? bytes : 1) != hipSuccess) {
    (void)hipGetLastError();
    m->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
    return ELPH_ENOMEM;
  }
  m->allocs.push_back(*p);
  return ELPH_OK;
}

static void free_m(elph_mlp m, void* p) {
  if (!p) return;
  auto it = std::find(m->allocs.begin(), m->allocs.end(), p);
  if (it != m->allocs.end()) {
    m->allocs.erase(it);
    (void)hipFree(p);
  }
}

static int layer_k(elph_mlp m, int l) { return l == 0 ? m->in_pad : m->width; }

static elph_status refresh_bf16(elph_mlp m) {
  const int W = m->width;
  for (int l = 0; l < m->depth; ++l) {
    const int K = layer_k(m, l);
    hipLaunchKernelGGL(k_refresh, dim3(nblk((int64_t)K * W, 256)), dim3(256), 0, m->stream,
                       m->d_params + m->w_off[l], m->fan_in[l], K, W, m->d_W[l], m->d_Wt[l]);
  }
  hipLaunchKernelGGL(k_refresh, dim3(nblk(W, 256)), dim3(256), 0, m->stream, m->d_params + m->w_off[m->depth], W, W,
                     1, m->d_wout, (unsigned short*)nullptr);
  MCHK(hipGetLastError());
  return ELPH_OK;
}

elph_status mlp_reserve(elph_mlp m, int64_t n) {
  if (n <= m->cap) return ELPH_OK;
  free_m(m, m->d_x);
  for (auto p : m->d_h) free_m(m, p);
  for (auto p : m->d_z) free_m(m, p);
  free_m(m, m->d_dz[0]);
  free_m(m, m->d_dz[1]);
  free_m(m, m->d_y);
  m->cap = 0;
  const int64_t cap = ((n + 63) / 64) * 64;
  const int W = m->width;
  elph_status st;
  if ((st = malloc_m(m, (void**)&m->d_x, (size_t)cap * m->in_pad * 2)) != ELPH_OK) return st;
  for (int l = 0; l < m->depth; ++l) {
    if ((st = malloc_m(m, (void**)&m->d_h[l], (size_t)cap * W * 2)) != ELPH_OK) return st;
    if ((st = malloc_m(m, (void**)&m->d_z[l], (size_t)cap * W * 4)) != ELPH_OK) return st;
  }
  for (int b = 0; b < 2; ++b)
    if ((st = malloc_m(m, (void**)&m->d_dz[b], (size_t)cap * W * 2)) != ELPH_OK) return st;
  if ((st = malloc_m(m, (void**)&m->d_y, (size_t)cap * 2 * 4)) != ELPH_OK) return st;  // y and dy
  m->cap = cap;
  return ELPH_OK;
}

static elph_status ensure_part(elph_mlp m, int64_t len) {
  if (len <= m->part_len) return ELPH_OK;
  free_m(m, m->d_part);
  m->part_len = 0;
  elph_status st = malloc_m(m, (void**)&m->d_part, (size_t)len * 4);
  if (st != ELPH_OK) return st;
  m->part_len = len;
  return ELPH_OK;
}

static GemmP gemm_p(int M, int N, int K, const unsigned short* A, int64_t lda, const unsigned short* B, int64_t ldb,
                    int64_t ldc) {
  GemmP p;
  std::memset(&p, 0, sizeof(p));
  p.M = M;
  p.N = N;
  p.K = K;
  p.kchunk = K;
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.ldc = ldc;
  return p;
}

elph_status mlp_forward_rows(elph_mlp m, int64_t n, bool keep, float* y) {
  const int W = m->width;
  if (n == 0) return ELPH_OK;
  for (int l = 0; l < m->depth; ++l) {
    const int K = layer_k(m, l);
    const unsigned short* A = l == 0 ? m->d_x : m->d_h[l - 1];
    GemmP p = gemm_p((int)n, W, K, A, K, m->d_Wt[l], K, W);
    p.bias = m->d_params + m->b_off[l];
    p.zout = keep ? m->d_z[l] : nullptr;
    p.hout = m->d_h[l];
    hipLaunchKernelGGL((k_gemm_bf16<true, true, EPI_FWD>), dim3(nblk(W, 64), nblk(n, 64), 1), dim3(256), 0,
                       m->stream, p);
  }
  hipLaunchKernelGGL(k_out_fwd, dim3(nblk(n, 4)), dim3(256), 0, m->stream, n, W, m->d_h[m->depth - 1], m->d_wout,
                     m->d_params + m->b_off[m->depth], y);
  MCHK(hipGetLastError());
  return ELPH_OK;
}

// gradient of the mean squared error into m->d_grad; loss to *loss (host)
static elph_status mlp_backward(elph_mlp m, int64_t n, const float* t, double* loss) {
  const int W = m->width, L = m->depth;
  float* y = m->d_y;
  float* dy = m->d_y + m->cap;
  const unsigned lb = nblk(n, 4);
  const int ncs = (int)std::min<int64_t>(256, (n + 63) / 64);  // column-sum blocks
  int nsplit = (int)std::min<int64_t>(32, n / 256);
  if (nsplit < 1) nsplit = 1;
  int64_t kchunk = ((n + nsplit - 1) / nsplit + 31) / 32 * 32;
  nsplit = (int)((n + kchunk - 1) / kchunk);
  const int64_t part_need =
      std::max<int64_t>(std::max<int64_t>((int64_t)lb + 1, (int64_t)ncs * W), (int64_t)nsplit * m->in_pad * W);
  elph_status st = ensure_part(m, std::max<int64_t>(part_need, (int64_t)nsplit * W * W));
  if (st != ELPH_OK) return st;
  if (!m->h_pin) MCHK(hipHostMalloc((void**)&m->h_pin, 64 * sizeof(float), hipHostMallocDefault));
  // output layer
  unsigned short* dz = m->d_dz[0];
  unsigned short* dz2 = m->d_dz[1];
  hipLaunchKernelGGL(k_out_bwd, dim3(lb), dim3(256), 0, m->stream, n, W, y, t, m->d_wout, m->d_z[L - 1], dy, dz,
                     m->d_part);
  // loss = sum of the block partials / n (device tree, one word to the host)
  float* lsum = m->d_part + lb;
  hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, m->stream, m->d_part, (int64_t)lb, lsum);
  MCHK(hipMemcpyAsync(m->h_pin, lsum, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MCHK(hipStreamSynchronize(m->stream));
  if (loss) *loss = (double)m->h_pin[0] / (double)n;
  // dW_out = sum_r h_L[r] dy[r]; db_out = sum dy
  hipLaunchKernelGGL(k_colsum, dim3(ncs), dim3(256), 0, m->stream, n, W, m->d_h[L - 1], dy, m->d_part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(W, 256)), dim3(256), 0, m->stream, (int64_t)W, ncs, (int64_t)W,
                     m->d_part, m->d_grad + m->w_off[L]);
  hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, m->stream, dy, n, m->d_grad + m->b_off[L]);
  for (int l = L - 1; l >= 0; --l) {
    const int K = layer_k(m, l);
    const unsigned short* A = l == 0 ? m->d_x : m->d_h[l - 1];
    // dW_l = A^T dz (split over the batch, partials summed in split order)
    GemmP p = gemm_p(K, W, (int)n, A, K, dz, W, W);
    p.kchunk = (int)kchunk;
    p.C = m->d_part;
    hipLaunchKernelGGL((k_gemm_bf16<false, false, EPI_STORE>), dim3(nblk(W, 64), nblk(K, 64), nsplit), dim3(256),
                       0, m->stream, p);
    hipLaunchKernelGGL(k_sum_parts, dim3(nblk((int64_t)m->fan_in[l] * W, 256)), dim3(256), 0, m->stream,
                       (int64_t)m->fan_in[l] * W, nsplit, (int64_t)K * W, m->d_part, m->d_grad + m->w_off[l]);
    // db_l = column sums of dz
    hipLaunchKernelGGL(k_colsum, dim3(ncs), dim3(256), 0, m->stream, n, W, dz, (const float*)nullptr, m->d_part);
    hipLaunchKernelGGL(k_sum_parts, dim3(nblk(W, 256)), dim3(256), 0, m->stream, (int64_t)W, ncs, (int64_t)W,
                       m->d_part, m->d_grad + m->b_off[l]);
    if (l > 0) {
      // dz_{l-1} = (dz W_l^T) * GELU'(z_{l-1})
      GemmP q = gemm_p((int)n, W, W, dz, W, m->d_W[l], W, W);
      q.hout = dz2;
      q.zprev = m->d_z[l - 1];
      hipLaunchKernelGGL((k_gemm_bf16<true, true, EPI_BWD>), dim3(nblk(W, 64), nblk(n, 64), 1), dim3(256), 0,
                         m->stream, q);
      std::swap(dz, dz2);
    }
  }
  MCHK(hipGetLastError());
  return ELPH_OK;
}

}  // namespace elph

using namespace elph;

static thread_local std::string g_mlp_create_err;

#define CHECK_M(m)                                 \
  do {                                             \
    if (!(m)) return ELPH_EINVAL;                  \
    if ((m)->hip_dead) {                           \
      (m)->err = "MLP unusable after a HIP error"; \
      return ELPH_ESTATE;                          \
    }                                              \
    (m)->err.clear();                              \
  } while (0)

extern "C" elph_status elph_mlp_create(int32_t nin, int32_t width, int32_t depth, const float* params,
                                       void* hip_stream, elph_mlp* out) {
  if (!out) return ELPH_EINVAL;
  *out = nullptr;
  if (nin < 1 || nin > 1024 || width < 64 || width > 1024 || width % 64 != 0 || depth < 1 || depth > 8 || !params) {
    g_mlp_create_err = "need 1 <= nin <= 1024, width a multiple of 64 in [64, 1024], 1 <= depth <= 8, params";
    return ELPH_EINVAL;
  }
  elph_mlp m = new elph_mlp_s();
  m->stream = (hipStream_t)hip_stream;
  m->nin = nin;
  m->in_pad = (nin + 31) / 32 * 32;
  m->width = width;
  m->depth = depth;
  int64_t o = 0;
  for (int l = 0; l <= depth; ++l) {
    const int fi = l == 0 ? nin : width, fo = l == depth ? 1 : width;
    m->fan_in.push_back(fi);
    m->fan_out.push_back(fo);
    m->w_off.push_back(o);
    o += (int64_t)fi * fo;
    m->b_off.push_back(o);
    o += fo;
  }
  m->nparams = o;
  for (size_t i = 0; i < (size_t)o; ++i)
    if (!std::isfinite(params[i])) {
      g_mlp_create_err = "non-finite parameter";
      delete m;
      return ELPH_EINVAL;
    }
  m->d_W.assign(depth, nullptr);
  m->d_Wt.assign(depth, nullptr);
  m->d_h.assign(depth, nullptr);
  m->d_z.assign(depth, nullptr);
  const size_t pb = (size_t)o * 4;
  bool okm = malloc_m(m, (void**)&m->d_params, pb) == ELPH_OK && malloc_m(m, (void**)&m->d_grad, pb) == ELPH_OK &&
             malloc_m(m, (void**)&m->d_m, pb) == ELPH_OK && malloc_m(m, (void**)&m->d_v, pb) == ELPH_OK &&
             malloc_m(m, (void**)&m->d_wout, (size_t)width * 2) == ELPH_OK;
  for (int l = 0; okm && l < depth; ++l) {
    const size_t kb = (size_t)layer_k(m, l) * width * 2;
    okm = malloc_m(m, (void**)&m->d_W[l], kb) == ELPH_OK && malloc_m(m, (void**)&m->d_Wt[l], kb) == ELPH_OK;
  }
  if (!okm || hipMemcpy(m->d_params, params, pb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(m->d_m, 0, pb, m->stream) != hipSuccess ||
      hipMemsetAsync(m->d_v, 0, pb, m->stream) != hipSuccess || refresh_bf16(m) != ELPH_OK ||
      hipStreamSynchronize(m->stream) != hipSuccess) {
    g_mlp_create_err = m->err.empty() ? "MLP setup failed" : m->err;
    elph_mlp_destroy(m);
    return ELPH_ENOMEM;
  }
  *out = m;
  return ELPH_OK;
}

extern "C" void elph_mlp_destroy(elph_mlp m) {
  if (!m) return;
  if (!m->hip_dead) (void)hipStreamSynchronize(m->stream);
  for (void* p : m->allocs) (void)hipFree(p);
  if (m->h_pin) (void)hipHostFree(m->h_pin);
  delete m;
}

extern "C" const char* elph_mlp_last_error(elph_mlp m) { return m ? m->err.c_str() : g_mlp_create_err.c_str(); }

extern "C" int64_t elph_mlp_nparams(elph_mlp m) { return m ? m->nparams : 0; }

extern "C" elph_status elph_mlp_get_params(elph_mlp m, float* params) {
  CHECK_M(m);
  if (!params) {
    m->err = "null output";
    return ELPH_EINVAL;
  }
  MCHK(hipMemcpyAsync(params, m->d_params, m->nparams * 4, hipMemcpyDeviceToHost, m->stream));
  MCHK(hipStreamSynchronize(m->stream));
  return ELPH_OK;
}

extern "C" elph_status elph_mlp_set_params(elph_mlp m, const float* params) {
  CHECK_M(m);
  if (!params) {
    m->err = "null input";
    return ELPH_EINVAL;
  }
  for (int64_t i = 0; i < m->nparams; ++i)
    if (!std::isfinite(params[i])) {
      m->err = "non-finite parameter";
      return ELPH_EINVAL;
    }
  MCHK(hipMemcpyAsync(m->d_params, params, m->nparams * 4, hipMemcpyHostToDevice, m->stream));
  MCHK(hipMemsetAsync(m->d_m, 0, m->nparams * 4, m->stream));
  MCHK(hipMemsetAsync(m->d_v, 0, m->nparams * 4, m->stream));
  m->step = 0;
  elph_status st = refresh_bf16(m);
  if (st != ELPH_OK) return st;
  MCHK(hipStreamSynchronize(m->stream));
  return ELPH_OK;
}

static elph_status load_x(elph_mlp m, int64_t n, const float* x) {
  elph_status st = mlp_reserve(m, n);
  if (st != ELPH_OK) return st;
  hipLaunchKernelGGL(k_x_to_bf, dim3(nblk(n * m->in_pad, 256)), dim3(256), 0, m->stream, n, m->nin, m->in_pad, x,
                     m->d_x);
  MCHK(hipGetLastError());
  return ELPH_OK;
}

extern "C" elph_status elph_mlp_forward(elph_mlp m, int64_t n, const float* x, float* y) {
  CHECK_M(m);
  if (n < 0 || (n > 0 && (!x || !y))) {
    m->err = "bad sizes or null pointers";
    return ELPH_EINVAL;
  }
  if (n == 0) return ELPH_OK;
  elph_status st = load_x(m, n, x);
  if (st != ELPH_OK) return st;
  return mlp_forward_rows(m, n, false, y);
}

static elph_status grads(elph_mlp m, int64_t n, const float* x, const float* t, double* loss) {
  if (n < 64 || n % 64 != 0 || !x || !t) {
    m->err = "training batches need n a positive multiple of 64 and device x, t";
    return ELPH_EINVAL;
  }
  elph_status st = load_x(m, n, x);
  if (st != ELPH_OK) return st;
  st = mlp_forward_rows(m, n, true, m->d_y);
  if (st != ELPH_OK) return st;
  return mlp_backward(m, n, t, loss);
}

extern "C" elph_status elph_mlp_gradients(elph_mlp m, int64_t n, const float* x, const float* t, float* grad,
                                          double* loss) {
  CHECK_M(m);
  elph_status st = grads(m, n, x, t, loss);
  if (st != ELPH_OK) return st;
  if (grad) MCHK(hipMemcpyAsync(grad, m->d_grad, m->nparams * 4, hipMemcpyDeviceToDevice, m->stream));
  MCHK(hipStreamSynchronize(m->stream));
  return ELPH_OK;
}

extern "C" elph_status elph_mlp_train_step(elph_mlp m, int64_t n, const float* x, const float* t, float lr,
                                           double* loss) {
  CHECK_M(m);
  if (!(lr > 0.f) || !std::isfinite(lr)) {
    m->err = "learning rate must be positive";
    return ELPH_EINVAL;
  }
  elph_status st = grads(m, n, x, t, loss);
  if (st != ELPH_OK) return st;
  m->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 - std::pow(b1, (double)m->step));
  const float bc2 = (float)(1.0 - std::pow(b2, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3(nblk(m->nparams, 256)), dim3(256), 0, m->stream, m->nparams, m->d_params,
                     m->d_grad, m->d_m, m->d_v, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2);
  MCHK(hipGetLastError());
  st = refresh_bf16(m);
  if (st != ELPH_OK) return st;
  return ELPH_OK;
}
