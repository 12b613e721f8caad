// The warm-start network (a multilayer perceptron from instance parameters to a primal trajectory
// and equality multipliers): d_in -> H -> H -> H -> d_out, GELU after each hidden layer.
// Weights and activations enter the matrix products in BF16, every product accumulates in FP32
// on the matrix cores (v_mfma_f32_16x16x32_bf16); biases, pre-activations, the loss, gradients
// and the Adam state are FP32.  Inputs and targets are normalised per column with statistics
// stored in the model buffer.
//
// Model buffer (FP32): per layer l = 1..4 the weight W_l [out][in] (row major) then the bias b_l
// [out]; then in_mu[d_in], in_sd[d_in], out_mu[d_out], out_sd[d_out].  The BF16 copy of the
// weights (no biases) follows the same order and is what the products read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hipipm_mlp.h"

namespace hipipm_mlp {

constexpr int WAVE = 64;
constexpr int NL = 4;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Dims {
  int din, h, dout;
  int in[NL], out[NL];
  long long w[NL], b[NL], wb[NL];      // offsets: weights / biases in the model, weights in the BF16 copy
  long long n_params, n_weights, in_mu, in_sd, out_mu, out_sd, model_len;
};

static Dims dims_of(int din, int h, int dout) {
  Dims d;
  d.din = din; d.h = h; d.dout = dout;
  const int io[NL + 1] = {din, h, h, h, dout};
  long long o = 0, ow = 0;
  for (int l = 0; l < NL; ++l) {
    d.in[l] = io[l];
    d.out[l] = io[l + 1];
    d.w[l] = o; o += (long long)d.in[l] * d.out[l];
    d.b[l] = o; o += d.out[l];
    d.wb[l] = ow; ow += (long long)d.in[l] * d.out[l];
  }
  d.n_params = o;
  d.n_weights = ow;
  d.in_mu = o; d.in_sd = o + din; d.out_mu = o + 2 * din; d.out_sd = o + 2 * din + dout;
  d.model_len = o + 2 * din + 2 * dout;
  return d;
}

// ---------------------------------------------------------------------------- BF16 helpers
__device__ __forceinline__ uint16_t to_bf16(float f) {
  // round to nearest even; NaN stays NaN
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// ---------------------------------------------------------------------------- GEMM
// C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn] (BF16),
// C FP32 row major (ldc).  A workgroup of four wavefronts owns a 64 x 64 tile of C, each wavefront
// a 32 x 32 quarter as 2 x 2 MFMA blocks of 16 x 16; K advances 32 at a time on gfx950's
// v_mfma_f32_16x16x32_bf16.  Operand layout: lane l holds A(i, k) and B(k, j) for i = j = l % 16
// and k = 8 (l / 16) + 0..7, and receives C(4 (l / 16) + 0..3, l % 16).
// AK / BK: the operand is contiguous along k with rows aligned to 4 elements and K % 4 == 0, so a
// lane's eight k values are two 8-byte loads (the network's forward products); otherwise eight
// 2-byte loads.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
template <bool CONTIG>
__device__ __forceinline__ bf16x8 load_k8(const uint16_t* __restrict__ P, int row, int rows, long long srow,
                                          long long sk, int k, int K) {
  bf16x4 lo = {0, 0, 0, 0}, hi = {0, 0, 0, 0};
  if constexpr (CONTIG) {
    // K % 4 == 0: each half is wholly inside or wholly outside [0, K)
    if (row < rows && k < K) lo = *reinterpret_cast<const bf16x4*>(P + row * srow + k);
    if (row < rows && k + 4 < K) hi = *reinterpret_cast<const bf16x4*>(P + row * srow + k + 4);
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      lo[t] = (row < rows && k + t < K) ? (short)P[row * srow + (k + t) * sk] : (short)0;
      hi[t] = (row < rows && k + 4 + t < K) ? (short)P[row * srow + (k + 4 + t) * sk] : (short)0;
    }
  }
  const short __attribute__((ext_vector_type(8))) v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
}
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t* __restrict__ A, long long sam,
                                              long long sak, const uint16_t* __restrict__ B, long long sbk,
                                              long long sbn, float* __restrict__ C, long long ldc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (wv >> 1) * 32, n0 = blockIdx.x * 64 + (wv & 1) * 32;
  const int r16 = lane & 15, k8 = (lane >> 4) * 8, c4 = (lane >> 4) * 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = load_k8<AK>(A, m0 + 16 * i + r16, M, sam, sak, k0 + k8, K);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = load_k8<BK>(B, n0 + 16 * j + r16, N, sbn, sbk, k0 + k8, K);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + 16 * i + c4 + t, n = n0 + 16 * j + r16;
        if (m < M && n < N) C[m * ldc + n] = acc[i][j][t];
      }
}

static bool k_contig(const uint16_t* p, long long s_k, long long s_row, int K) {
  return s_k == 1 && s_row % 4 == 0 && K % 4 == 0 && ((uintptr_t)p & 7) == 0;
}

static void gemm(hipStream_t st, int M, int N, int K, const uint16_t* A, long long sam, long long sak,
                 const uint16_t* B, long long sbk, long long sbn, float* C, long long ldc) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  const bool ak = k_contig(A, sak, sam, K), bk = k_contig(B, sbk, sbn, K);
  if (ak && bk)
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc);
  else if (ak)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc);
  else if (bk)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc);
  else
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc);
}

// ---------------------------------------------------------------------------- elementwise
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// normalised input rows (optionally gathered through idx) in BF16
__global__ void k_input(int B, int din, const double* __restrict__ x, const int32_t* __restrict__ idx,
                        const float* __restrict__ model, long long mu, long long sd, uint16_t* __restrict__ xb) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)B * din) return;
  const int r = (int)(q / din), c = (int)(q % din);
  const long long src = idx ? idx[r] : r;
  xb[q] = to_bf16((float)((x[src * din + c] - model[mu + c]) / model[sd + c]));
}

// z = c + b (kept for the backward pass), a = GELU(z) in BF16
__global__ void k_bias_gelu(int B, int n, const float* __restrict__ c, const float* __restrict__ bias,
                            float* __restrict__ z, uint16_t* __restrict__ a) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)B * n) return;
  const float v = c[q] + bias[q % n];
  z[q] = v;
  a[q] = to_bf16(gelu(v));
}

// network output: y = c + b (normalised); de-normalised to FP64 out when out != null
__global__ void k_bias_out(int B, int n, float* __restrict__ c, const float* __restrict__ bias,
                           const float* __restrict__ model, long long mu, long long sd, double* __restrict__ out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)B * n) return;
  const int col = (int)(q % n);
  const float v = c[q] + bias[col];
  c[q] = v;
  if (out) out[q] = (double)v * model[sd + col] + model[mu + col];
}

// mean squared error in normalised space: dy = 2 (y - t) / (B n) in BF16, per-block partial sums
__global__ void k_loss(int B, int n, const float* __restrict__ y, const double* __restrict__ t,
                       const int32_t* __restrict__ idx, const float* __restrict__ model, long long mu, long long sd,
                       uint16_t* __restrict__ dy, float* __restrict__ part) {
  __shared__ float red[256];
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float e2 = 0.f;
  if (q < (long long)B * n) {
    const int r = (int)(q / n), col = (int)(q % n);
    const long long src = idx ? idx[r] : r;
    const float tn = (float)((t[src * n + col] - model[mu + col]) / model[sd + col]);
    const float e = y[q] - tn;
    e2 = e * e;
    dy[q] = to_bf16(2.0f * e / ((float)B * (float)n));
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dz = da * GELU'(z) in BF16
__global__ void k_gelu_back(int B, int n, const float* __restrict__ da, const float* __restrict__ z,
                            uint16_t* __restrict__ dz) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)B * n) return;
  dz[q] = to_bf16(da[q] * gelu_d(z[q]));
}

// bias gradient: column sums of dz.  A workgroup owns 64 columns (lane = column, so each row is
// one coalesced read per wavefront); its CS_WAVES wavefronts take every CS_WAVES-th row and their
// partial sums are added in wavefront order (deterministic).
constexpr int CS_WAVES = 8;
__global__ __launch_bounds__(CS_WAVES * 64) void k_colsum(int B, int n, const uint16_t* __restrict__ dz,
                                                         float* __restrict__ g) {
  __shared__ float part[CS_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (col < n) {
    // eight independent loads in flight per lane, summed in row order
    int r = wv;
    for (; r + 7 * CS_WAVES < B; r += 8 * CS_WAVES) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = from_bf16(dz[(long long)(r + u * CS_WAVES) * n + col]);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; r < B; r += CS_WAVES) s += from_bf16(dz[(long long)r * n + col]);
  }
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && col < n) {
    float t = 0.f;
    for (int w = 0; w < CS_WAVES; ++w) t += part[w][lane];
    g[col] = t;
  }
}

// Adam on the parameters (FP32 master), then the BF16 copy of the weights
__global__ void k_adam(long long np, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}
__global__ void k_to_bf16(long long n, const float* __restrict__ src, uint16_t* __restrict__ dst) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = to_bf16(src[q]);
}

// column mean and standard deviation (floored at 1e-6) of an FP64 [rows][cols] array; the same
// column-tile layout as k_colsum with CT_WAVES wavefronts over the rows, FP64 sums
constexpr int CT_WAVES = 16;
__global__ __launch_bounds__(CT_WAVES * 64) void k_colstats(long long rows, int cols, const double* __restrict__ x,
                                                           float* __restrict__ mu, float* __restrict__ sd) {
  __shared__ double p1[CT_WAVES][64], p2[CT_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  double s = 0.0, s2 = 0.0;
  if (col < cols) {
    long long r = wv;
    for (; r + 7 * CT_WAVES < rows; r += 8 * CT_WAVES) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = x[(r + u * CT_WAVES) * cols + col];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s += v[u];
        s2 += v[u] * v[u];
      }
    }
    for (; r < rows; r += CT_WAVES) {
      const double v = x[r * cols + col];
      s += v;
      s2 += v * v;
    }
  }
  p1[wv][lane] = s;
  p2[wv][lane] = s2;
  __syncthreads();
  if (wv == 0 && col < cols) {
    double t = 0.0, t2 = 0.0;
    for (int w = 0; w < CT_WAVES; ++w) { t += p1[w][lane]; t2 += p2[w][lane]; }
    const double m = t / (double)rows;
    const double var = t2 / (double)rows - m * m;
    mu[col] = (float)m;
    sd[col] = (float)fmax(sqrt(fmax(var, 0.0)), 1e-6);
  }
}

static inline unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// activation workspace carve-up for a batch of B rows
struct Act {
  uint16_t *xb, *a[3], *dy, *dz0, *dz1;
  float *z[3], *y, *da, *part;
};
static size_t act_bytes(const Dims& d, int B) {
  const size_t h = (size_t)B * d.h, o = (size_t)B * d.dout;
  size_t bytes = 0;
  bytes += 2 * (size_t)B * d.din;                 // xb
  bytes += 3 * 2 * h;                              // a1..a3
  bytes += 2 * o;                                  // dy
  bytes += 2 * 2 * h;                              // dz0, dz1
  bytes += 3 * 4 * h;                              // z1..z3
  bytes += 4 * o;                                  // y
  bytes += 4 * h;                                  // da
  bytes += 4 * ((o + 255) / 256 + 1);              // loss partial sums
  return bytes + 16 * 16;                          // alignment slack
}
static Act carve(const Dims& d, int B, void* base) {
  char* p = (char*)base;
  auto take = [&](size_t n) {
    char* r = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    p = r + n;
    return (void*)r;
  };
  const size_t h = (size_t)B * d.h, o = (size_t)B * d.dout;
  Act a;
  a.xb = (uint16_t*)take(2 * (size_t)B * d.din);
  for (int l = 0; l < 3; ++l) a.a[l] = (uint16_t*)take(2 * h);
  a.dy = (uint16_t*)take(2 * o);
  a.dz0 = (uint16_t*)take(2 * h);
  a.dz1 = (uint16_t*)take(2 * h);
  for (int l = 0; l < 3; ++l) a.z[l] = (float*)take(4 * h);
  a.y = (float*)take(4 * o);
  a.da = (float*)take(4 * h);
  a.part = (float*)take(4 * ((o + 255) / 256 + 1));
  return a;
}

// forward pass into the workspace (y normalised); out (FP64, de-normalised) if non-null
static void forward(hipStream_t st, const Dims& d, const float* model, const uint16_t* wb, const double* x,
                    const int32_t* idx, int B, const Act& a, double* out) {
  hipLaunchKernelGGL(k_input, dim3(blocks((long long)B * d.din, 256)), dim3(256), 0, st, B, d.din, x, idx, model,
                     d.in_mu, d.in_sd, a.xb);
  const uint16_t* prev = a.xb;
  for (int l = 0; l < 3; ++l) {
    gemm(st, B, d.out[l], d.in[l], prev, d.in[l], 1, wb + d.wb[l], 1, d.in[l], a.z[l], d.out[l]);
    hipLaunchKernelGGL(k_bias_gelu, dim3(blocks((long long)B * d.h, 256)), dim3(256), 0, st, B, d.h, a.z[l],
                       model + d.b[l], a.z[l], a.a[l]);
    prev = a.a[l];
  }
  gemm(st, B, d.dout, d.h, prev, d.h, 1, wb + d.wb[3], 1, d.h, a.y, d.dout);
  hipLaunchKernelGGL(k_bias_out, dim3(blocks((long long)B * d.dout, 256)), dim3(256), 0, st, B, d.dout, a.y,
                     model + d.b[3], model, d.out_mu, d.out_sd, out);
}

// loss and gradient (FP32, model layout; the statistics part of grad is left untouched)
static void backward(hipStream_t st, const Dims& d, const float* model, const uint16_t* wb, const double* target,
                     const int32_t* idx, int B, const Act& a, float* grad) {
  const long long no = (long long)B * d.dout;
  hipLaunchKernelGGL(k_loss, dim3(blocks(no, 256)), dim3(256), 0, st, B, d.dout, a.y, target, idx, model,
                     d.out_mu, d.out_sd, a.dy, a.part);
  const uint16_t* dz = a.dy;
  uint16_t* dzn[2] = {a.dz0, a.dz1};
  for (int l = 3; l >= 0; --l) {
    const int nout = d.out[l], nin = d.in[l];
    const uint16_t* ain = (l == 0) ? a.xb : a.a[l - 1];
    // dW_l[o][i] = sum_b dz[b][o] ain[b][i];  db_l = column sums of dz
    gemm(st, nout, nin, B, dz, 1, nout, ain, nin, 1, grad + d.w[l], nin);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(nout, 64)), dim3(CS_WAVES * 64), 0, st, B, nout, dz, grad + d.b[l]);
    if (l == 0) break;
    // da[b][i] = sum_o dz[b][o] W_l[o][i], then dz_{l-1} = da * GELU'(z_{l-1})
    gemm(st, B, nin, nout, dz, nout, 1, wb + d.wb[l], nin, 1, a.da, nin);
    uint16_t* nz = dzn[l & 1];
    hipLaunchKernelGGL(k_gelu_back, dim3(blocks((long long)B * nin, 256)), dim3(256), 0, st, B, nin, a.da,
                       a.z[l - 1], nz);
    dz = nz;
  }
}

static void weights_to_bf16(hipStream_t st, const Dims& d, const float* model, uint16_t* wb) {
  for (int l = 0; l < NL; ++l) {
    const long long n = (long long)d.in[l] * d.out[l];
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n, 256)), dim3(256), 0, st, n, model + d.w[l], wb + d.wb[l]);
  }
}

static bool dims_ok(int din, int h, int dout) { return din > 0 && h > 0 && dout > 0 && din <= 4096 && h <= 4096 && dout <= 8192; }

}  // namespace hipipm_mlp

using namespace hipipm_mlp;

extern "C" {

int hipipm_mlp_sizes(int32_t d_in, int32_t hidden, int32_t d_out, int32_t batch, int64_t* model_len,
                     int64_t* n_params, int64_t* n_weights, int64_t* act_bytes_out) {
  if (!dims_ok(d_in, hidden, d_out) || batch < 0) return -1;
  const Dims d = dims_of(d_in, hidden, d_out);
  if (model_len) *model_len = d.model_len;
  if (n_params) *n_params = d.n_params;
  if (n_weights) *n_weights = d.n_weights;
  if (act_bytes_out) *act_bytes_out = (int64_t)act_bytes(d, batch);
  return 0;
}

int hipipm_mlp_weights_bf16(int32_t d_in, int32_t hidden, int32_t d_out, const float* model, uint16_t* w_bf16,
                            void* stream) {
  if (!dims_ok(d_in, hidden, d_out) || !model || !w_bf16) return -1;
  hipStream_t st = (hipStream_t)stream;
  weights_to_bf16(st, dims_of(d_in, hidden, d_out), model, w_bf16);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int hipipm_mlp_normalizer(int32_t d_in, int32_t hidden, int32_t d_out, int64_t rows, const double* inputs,
                          const double* targets, float* model, void* stream) {
  if (!dims_ok(d_in, hidden, d_out) || rows <= 0 || !inputs || !targets || !model) return -1;
  const Dims d = dims_of(d_in, hidden, d_out);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_colstats, dim3(blocks(d.din, 64)), dim3(CT_WAVES * 64), 0, st, (long long)rows, d.din, inputs,
                     model + d.in_mu, model + d.in_sd);
  hipLaunchKernelGGL(k_colstats, dim3(blocks(d.dout, 64)), dim3(CT_WAVES * 64), 0, st, (long long)rows, d.dout, targets,
                     model + d.out_mu, model + d.out_sd);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int hipipm_mlp_forward(int32_t d_in, int32_t hidden, int32_t d_out, const float* model, const uint16_t* w_bf16,
                       const double* inputs, double* outputs, int32_t batch, void* act, void* stream) {
  if (!dims_ok(d_in, hidden, d_out) || batch < 0 || !model || !w_bf16 || !act) return -1;
  if (batch == 0) return 0;
  if (!inputs || !outputs) return -1;
  const Dims d = dims_of(d_in, hidden, d_out);
  hipStream_t st = (hipStream_t)stream;
  forward(st, d, model, w_bf16, inputs, nullptr, batch, carve(d, batch, act), outputs);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int hipipm_mlp_backward(int32_t d_in, int32_t hidden, int32_t d_out, const float* model, const uint16_t* w_bf16,
                        const double* inputs, const double* targets, const int32_t* rows, int32_t batch,
                        void* act, float* grad, float* loss_parts, void* stream) {
  if (!dims_ok(d_in, hidden, d_out) || batch <= 0 || !model || !w_bf16 || !inputs || !targets || !act || !grad)
    return -1;
  const Dims d = dims_of(d_in, hidden, d_out);
  hipStream_t st = (hipStream_t)stream;
  const Act a = carve(d, batch, act);
  forward(st, d, model, w_bf16, inputs, rows, batch, a, nullptr);
  backward(st, d, model, w_bf16, targets, rows, batch, a, grad);
  if (loss_parts) {
    const long long nb = blocks((long long)batch * d.dout, 256);
    if (hipMemcpyAsync(loss_parts, a.part, nb * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess) return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int hipipm_mlp_adam(int32_t d_in, int32_t hidden, int32_t d_out, float* model, uint16_t* w_bf16, const float* grad,
                    float* adam_m, float* adam_v, int32_t step, float lr, float beta1, float beta2, float eps,
                    void* stream) {
  if (!dims_ok(d_in, hidden, d_out) || !model || !w_bf16 || !grad || !adam_m || !adam_v || step < 1) return -1;
  const Dims d = dims_of(d_in, hidden, d_out);
  hipStream_t st = (hipStream_t)stream;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(d.n_params, 256)), dim3(256), 0, st, (long long)d.n_params, model, grad,
                     adam_m, adam_v, lr, beta1, beta2, eps, c1, c2);
  weights_to_bf16(st, d, model, w_bf16);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
