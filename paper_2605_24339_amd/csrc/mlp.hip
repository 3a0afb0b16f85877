// Per-vertex MLP for the learned warm start: 9 -> 128 -> 128 -> 128 -> 3,
// SiLU activations, inputs padded to 16 features and outputs to 16.
// Dense layers run on the matrix cores: v_mfma_f32_32x32x16_bf16 with bf16
// operands (converted from the float32 tensors while staging tiles in LDS)
// and float32 accumulation; bias and SiLU are fused into the GEMM epilogue.
// Weight gradients (a reduction over the batch) use split-K partials summed
// in a fixed order, so training is deterministic.
//
// Parameter layout (float32, contiguous):
//   W1 [16][128], b1 [128], W2 [128][128], b2 [128], W3 [128][128], b3 [128],
//   W4 [128][16], b4 [16]
// Saved activations for the backward pass ("act", float32, [B][768]):
//   Z1 | H1 | Z2 | H2 | Z3 | H3, 128 columns each, row-major per row block.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/gmcp_mlp.h"
#include "common.h"

// Scratch of gmcp_mlp_mse_noalloc (the per-block partial losses), in static
// device memory: every GPU the library runs on holds its own copy until the
// process ends.  Host code must not pass this name to a kernel (on the host
// it is only a stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returns for each device.
constexpr int64_t kMseScratch = int64_t(1) << 20;  // floats, 4 MiB per GPU
static __device__ __align__(256) float scratch[kMseScratch];

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int IN = 16, HID = 128, OUT = 16;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
                  OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * HID, OFF_W4 = OFF_B3 + HID,
                  OFF_B4 = OFF_W4 + HID * OUT, N_PARAMS = OFF_B4 + OUT;
constexpr int ACT = 6 * HID;  // saved activations per row

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2 };

__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_grad(float z) {
  float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C = op(A) op(B) (+ bias, SiLU), op(A) is M x K, op(B) is K x N.
// A(m,k) = transA ? A[k*lda + m] : A[m*lda + k]; B(k,n) likewise.
// Block tile 64 x 64 (four waves of 32 x 32), K step 32 (two MFMAs).
// Split-K (EPI_STORE): block z handles k in [z*kc, (z+1)*kc) and writes
// its partial product at C + z * split_stride.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float *__restrict__ A, int lda, int transA,
                                               const float *__restrict__ B, int ldb, int transB, int M, int N, int K,
                                               int kc, const float *__restrict__ bias, float *__restrict__ C,
                                               int ldc, float *__restrict__ C2, int64_t split_stride) {
  __shared__ __bf16 As[64][32 + 8];
  __shared__ __bf16 Bs[32][64 + 8];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  f32x16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    for (int e = tid; e < 64 * 32; e += 256) {
      int r = e >> 5, kk = e & 31, m = m0 + r, k = k0 + kk;
      float v = (m < M && k < ke) ? (transA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k]) : 0.0f;
      As[r][kk] = (__bf16)v;
    }
    for (int e = tid; e < 32 * 64; e += 256) {
      int kk = e >> 6, cc = e & 63, k = k0 + kk, n = n0 + cc;
      float v = (k < ke && n < N) ? (transB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n]) : 0.0f;
      Bs[kk][cc] = (__bf16)v;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 a, b;
      const int kq = h * 16 + 8 * (lane >> 5);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        a[j] = As[wm * 32 + (lane & 31)][kq + j];
        b[j] = Bs[kq + j][wn * 32 + (lane & 31)];
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int n = n0 + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    if (m >= M || n >= N) continue;
    float v = acc[r];
    if (EPI == EPI_STORE) {
      C[blockIdx.z * split_stride + (int64_t)m * ldc + n] = v;
    } else if (EPI == EPI_BIAS) {
      C[(int64_t)m * ldc + n] = v + bias[n];
    } else {
      float z = v + bias[n];
      C[(int64_t)m * ldc + n] = z;
      C2[(int64_t)m * ldc + n] = silu(z);
    }
  }
}

// out[i] = sum_s part[s][i] (fixed order)
__global__ void k_reduce_split(const float *__restrict__ part, int S, int64_t n, float *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int z = 0; z < S; ++z) s += part[z * n + i];
  out[i] = s;
}

// column sums of X [B][ld] (first ncol columns) into out [ncol], two levels
__global__ void k_colsum_partial(const float *__restrict__ X, int64_t B, int ld, int ncol, int rows_per,
                                 float *__restrict__ part) {
  int c = threadIdx.x;
  if (c >= ncol) return;
  int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = min(B, r0 + rows_per);
  float s = 0.0f;
  for (int64_t r = r0; r < r1; ++r) s += X[r * ld + c];
  part[(int64_t)blockIdx.x * ncol + c] = s;
}

// dZ = dH * silu'(Z)   (all [B][ld], first 128 columns)
__global__ void k_silu_bwd(const float *__restrict__ dH, int ldh, const float *__restrict__ Z, int ldz,
                           float *__restrict__ dZ, int ldd, int64_t B) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * HID) return;
  int64_t r = i / HID;
  int c = (int)(i % HID);
  dZ[r * ldd + c] = dH[r * ldh + c] * silu_grad(Z[r * ldz + c]);
}

// dY = 2 (Y - T) / (B n_out) on the first n_out columns, 0 on the padding;
// loss partials per block
__global__ void k_mse(const float *__restrict__ Y, const float *__restrict__ T, int64_t B, int n_out,
                      float *__restrict__ dY, float *__restrict__ part) {
  __shared__ float s[256];
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (i < B * OUT) {
    int c = (int)(i % OUT);
    float d = c < n_out ? Y[i] - T[i] : 0.0f;
    dY[i] = c < n_out ? 2.0f * d / (float)(B * n_out) : 0.0f;
    l = d * d / (float)(B * n_out);
  }
  s[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_sum(const float *__restrict__ part, int64_t n, float *out) {
  __shared__ float s[256];
  float v = 0.0f;
  for (int64_t j = threadIdx.x; j < n; j += 256) v += part[j];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nb(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <int EPI>
hipError_t gemm(hipStream_t s, const float *A, int lda, int tA, const float *B, int ldb, int tB, int M, int N, int K,
                const float *bias, float *C, int ldc, float *C2, int splits = 1, int64_t split_stride = 0) {
  int kc = (K + splits - 1) / splits;
  kc = (kc + 31) / 32 * 32;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)splits);
  hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(256), 0, s, A, lda, tA, B, ldb, tB, M, N, K, kc, bias, C, ldc, C2,
                     split_stride);
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(hipStream_t s, float **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMCP_E_HIP;
  if (s) {
    hipDevice_t sd = 0;
    if (hipStreamGetDevice(s, &sd) != hipSuccess) return GMCP_E_HIP;
    if ((int)sd != dev) return GMCP_E_ARG;  // the stream must belong to the current device
  }
  if (dev < 0 || dev >= kMaxDevices) return GMCP_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GMCP_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = (float *)g_scratch_ptr[dev];
  return GMCP_OK;
}

constexpr int kSplitRows = 4096;  // batch rows per split-K chunk of a weight gradient

int splits_for(int64_t B) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (B + kSplitRows - 1) / kSplitRows)); }

}  // namespace

extern "C" {

int64_t gmcp_mlp_param_count(void) { return N_PARAMS; }

size_t gmcp_mlp_work_bytes(int64_t B) {
  int S = splits_for(B);
  // two [B][128] gradient buffers, split partials for the largest weight,
  // column-sum partials, loss partials
  return sizeof(float) * ((size_t)2 * B * HID + (size_t)S * HID * HID + (size_t)((B + 255) / 256 + 1) * HID +
                          (size_t)(B * OUT + 255) / 256 + 64);
}

int gmcp_mlp_forward(const float *params, const float *x, int64_t B, float *y, float *act, void *stream) {
  if (!params || !x || !y || B <= 0 || B > (int64_t(1) << 30)) return GMCP_E_ARG;
  if (!act) return GMCP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const float *P = params;
  const int ld = ACT;
  float *Z1 = act, *H1 = act + HID, *Z2 = act + 2 * HID, *H2 = act + 3 * HID, *Z3 = act + 4 * HID,
        *H3 = act + 5 * HID;
  if (gemm<EPI_BIAS_SILU>(s, x, IN, 0, P + OFF_W1, HID, 0, (int)B, HID, IN, P + OFF_B1, Z1, ld, H1) != hipSuccess ||
      gemm<EPI_BIAS_SILU>(s, H1, ld, 0, P + OFF_W2, HID, 0, (int)B, HID, HID, P + OFF_B2, Z2, ld, H2) != hipSuccess ||
      gemm<EPI_BIAS_SILU>(s, H2, ld, 0, P + OFF_W3, HID, 0, (int)B, HID, HID, P + OFF_B3, Z3, ld, H3) != hipSuccess ||
      gemm<EPI_BIAS>(s, H3, ld, 0, P + OFF_W4, OUT, 0, (int)B, OUT, HID, P + OFF_B4, y, OUT, nullptr) != hipSuccess)
    return GMCP_E_HIP;
  return GMCP_OK;
}

int gmcp_mlp_backward(const float *params, const float *x, const float *act, const float *dy, int64_t B, float *grad,
                      void *work, size_t work_bytes, void *stream) {
  if (!params || !x || !act || !dy || !grad || !work || B <= 0 || B > (int64_t(1) << 30)) return GMCP_E_ARG;
  if (work_bytes < gmcp_mlp_work_bytes(B)) return GMCP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const float *P = params;
  const int S = splits_for(B);
  float *dA = (float *)work;                 // [B][128]
  float *dB = dA + (size_t)B * HID;          // [B][128]
  float *part = dB + (size_t)B * HID;        // [S][128][128]
  float *cpart = part + (size_t)S * HID * HID;
  const int rows_per = 256;
  const unsigned cblocks = (unsigned)((B + rows_per - 1) / rows_per);
  const float *Z1 = act, *H1 = act + HID, *Z2 = act + 2 * HID, *H2 = act + 3 * HID, *Z3 = act + 4 * HID,
              *H3 = act + 5 * HID;
  const int ld = ACT;
  hipError_t e = hipSuccess;
  auto wgrad = [&](const float *Hin, int ldh, int fin, const float *dZ, int ldz, int fout, float *dW) {
    // dW [fin][fout] = Hin^T dZ over the batch, split-K partials then a fixed-order sum
    if (e == hipSuccess)
      e = gemm<EPI_STORE>(s, Hin, ldh, 1, dZ, ldz, 0, fin, fout, (int)B, nullptr, part, fout, nullptr, S,
                          (int64_t)fin * fout);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_reduce_split, dim3(nb((int64_t)fin * fout)), dim3(256), 0, s, part, S,
                         (int64_t)fin * fout, dW);
      e = hipGetLastError();
    }
  };
  auto bgrad = [&](const float *dZ, int ldz, int ncol, float *db) {
    if (e != hipSuccess) return;
    hipLaunchKernelGGL(k_colsum_partial, dim3(cblocks), dim3(HID), 0, s, dZ, B, ldz, ncol, rows_per, cpart);
    hipLaunchKernelGGL(k_reduce_split, dim3(1), dim3(HID), 0, s, cpart, (int)cblocks, (int64_t)ncol, db);
    e = hipGetLastError();
  };
  // layer 4: Y = H3 W4 + b4
  wgrad(H3, ld, HID, dy, OUT, OUT, grad + OFF_W4);
  bgrad(dy, OUT, OUT, grad + OFF_B4);
  if (e == hipSuccess) e = gemm<EPI_STORE>(s, dy, OUT, 0, P + OFF_W4, OUT, 1, (int)B, HID, OUT, nullptr, dA, HID, nullptr);
  // layer 3
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_silu_bwd, dim3(nb(B * HID)), dim3(256), 0, s, dA, HID, Z3, ld, dB, HID, B);
    e = hipGetLastError();
  }
  wgrad(H2, ld, HID, dB, HID, HID, grad + OFF_W3);
  bgrad(dB, HID, HID, grad + OFF_B3);
  if (e == hipSuccess) e = gemm<EPI_STORE>(s, dB, HID, 0, P + OFF_W3, HID, 1, (int)B, HID, HID, nullptr, dA, HID, nullptr);
  // layer 2
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_silu_bwd, dim3(nb(B * HID)), dim3(256), 0, s, dA, HID, Z2, ld, dB, HID, B);
    e = hipGetLastError();
  }
  wgrad(H1, ld, HID, dB, HID, HID, grad + OFF_W2);
  bgrad(dB, HID, HID, grad + OFF_B2);
  if (e == hipSuccess) e = gemm<EPI_STORE>(s, dB, HID, 0, P + OFF_W2, HID, 1, (int)B, HID, HID, nullptr, dA, HID, nullptr);
  // layer 1
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_silu_bwd, dim3(nb(B * HID)), dim3(256), 0, s, dA, HID, Z1, ld, dB, HID, B);
    e = hipGetLastError();
  }
  wgrad(x, IN, IN, dB, HID, HID, grad + OFF_W1);
  bgrad(dB, HID, HID, grad + OFF_B1);
  return e == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int gmcp_mlp_mse(const float *y, const float *t, int64_t B, int n_out, float *loss, float *dy, void *work,
                 size_t work_bytes, void *stream) {
  if (!y || !t || !loss || !dy || !work || B <= 0 || n_out < 1 || n_out > OUT) return GMCP_E_ARG;
  int64_t blocks = (B * OUT + 255) / 256;
  if (work_bytes < sizeof(float) * (size_t)blocks) return GMCP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mse, dim3((unsigned)blocks), dim3(256), 0, s, y, t, B, n_out, dy, (float *)work);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, (const float *)work, blocks, loss);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int64_t gmcp_mlp_mse_noalloc_max_rows(void) { return kMseScratch * 256 / OUT; }

int gmcp_mlp_mse_noalloc(const float *y, const float *t, int64_t B, int n_out, float *loss, float *dy,
                         void *stream) {
  if (!y || !t || !loss || !dy || B <= 0 || n_out < 1 || n_out > OUT) return GMCP_E_ARG;
  if (B > gmcp_mlp_mse_noalloc_max_rows()) return GMCP_E_ARG;
  const int64_t blocks = (B * OUT + 255) / 256;  // <= kMseScratch partials
  hipStream_t s = (hipStream_t)stream;
  float *part = nullptr;
  const int rc = scratch_address(s, &part);
  if (rc != GMCP_OK) return rc;
  // k_mse writes every partial it reads back, so nothing needs clearing
  hipLaunchKernelGGL(k_mse, dim3((unsigned)blocks), dim3(256), 0, s, y, t, B, n_out, dy, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, (const float *)part, blocks, loss);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int gmcp_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                  float eps, int step, void *stream) {
  if (!params || !grad || !m || !v || n <= 0 || step < 1) return GMCP_E_ARG;
  float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, n, lr, beta1, beta2,
                     eps, c1, c2);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
}

int gmcp_gemm_bf16(const float *A, int lda, int transA, const float *B, int ldb, int transB, int M, int N, int K,
                   float *C, int ldc, void *stream) {
  if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0) return GMCP_E_ARG;
  return gemm<EPI_STORE>((hipStream_t)stream, A, lda, transA, B, ldb, transB, M, N, K, nullptr, C, ldc, nullptr) ==
                 hipSuccess
             ? GMCP_OK
             : GMCP_E_HIP;
}

}  // extern "C"
