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

using gmcp::kWave;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int IN = 16, HID = 128, OUT = 16;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
                  OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID * HID, OFF_W4 = OFF_B3 + HID,
                  OFF_B4 = OFF_W4 + HID * OUT, N_PARAMS = OFF_B4 + OUT;
constexpr int ACT = 6 * HID;  // saved activations per row

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_SILU_BWD = 3 };

__device__ inline float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ inline float silu_grad(float z) {
  float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C = op(A) op(B) (+ bias, SiLU), op(A) is M x K, op(B) is K x N.
// A(m,k) = transA ? A[k*lda + m] : A[m*lda + k]; B(k,n) likewise.
// Block tile 64 x 64 (four waves of 32 x 32), K step 32 (two MFMAs).
// Split-K (EPI_STORE): block z handles k in [z*kc, (z+1)*kc) and writes
// its partial product at C + z * split_stride.  EPI_SILU_BWD multiplies the
// product by silu'(Z) (Z [M][ldz], the layer's pre-activations): the
// backward pass's dZ = (dH W^T) * silu'(Z) in the GEMM's epilogue.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float *__restrict__ A, int lda, int transA,
                                               const float *__restrict__ B, int ldb, int transB, int M, int N, int K,
                                               int kc, const float *__restrict__ bias, float *__restrict__ C,
                                               int ldc, float *__restrict__ C2, int64_t split_stride,
                                               const float *__restrict__ Z, int ldz) {
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
    } else if (EPI == EPI_SILU_BWD) {
      C[(int64_t)m * ldc + n] = v * silu_grad(Z[(int64_t)m * ldz + n]);
    } else {
      float z = v + bias[n];
      C[(int64_t)m * ldc + n] = z;
      C2[(int64_t)m * ldc + n] = silu(z);
    }
  }
}

// out[i] = sum_s part[s][i], 64 outputs per block of 1024 threads: thread
// group g (of 16) adds the partials s = g, g + 16, ... in that order, then
// the 16 group sums are added in group order (a fixed order, so runs agree
// bitwise; sixteen short chains of loads instead of one long one)
constexpr int kRedGroups = 16;
__global__ __launch_bounds__(kWave *kRedGroups) void k_reduce_split(const float *__restrict__ part, int S, int64_t n,
                                                                     float *__restrict__ out) {
  __shared__ float red[kRedGroups][kWave];
  const int e = threadIdx.x & (kWave - 1), g = threadIdx.x / kWave;
  const int64_t i = (int64_t)blockIdx.x * kWave + e;
  float s = 0.0f;
  if (i < n)
    for (int z = g; z < S; z += kRedGroups) s += part[(int64_t)z * n + i];
  red[g][e] = s;
  __syncthreads();
  if (g == 0 && i < n) {
    float t = 0.0f;
    for (int k = 0; k < kRedGroups; ++k) t += red[k][e];
    out[i] = t;
  }
}

// column sums of X [B][ld] (the first ncol <= 128 columns) over chunks of
// rows_per rows, one chunk per block of 256 threads: thread (h, c) adds
// column c over the chunk's rows h, h + 2, ... in order, and the two halves
// are added in LDS (fixed order); part [chunks][ncol]
constexpr int kColRows = 64;  // rows per chunk
__global__ __launch_bounds__(2 * HID) void k_colsum_partial(const float *__restrict__ X, int64_t B, int ld, int ncol,
                                                             int rows_per, float *__restrict__ part) {
  __shared__ float half[HID];
  const int c = threadIdx.x & (HID - 1), h = threadIdx.x / HID;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = min(B, r0 + rows_per);
  float s = 0.0f;
  if (c < ncol)
    for (int64_t r = r0 + h; r < r1; r += 2) s += X[r * ld + c];
  if (h == 1) half[c] = s;
  __syncthreads();
  if (h == 0 && c < ncol) part[(int64_t)blockIdx.x * ncol + c] = s + half[c];
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

// ---------------------------------------------------------------- fused forward
// The whole network for 32 rows per wave, activations in registers.  Each
// layer is computed transposed, out^T (features x rows) = W^T (features x
// k) . in^T (k x rows), on v_mfma_f32_32x32x16_bf16, so the accumulator of
// a 32-feature output tile holds, in lane l, row (l & 31) and features
// (r >> 2) * 8 + 4 (l >> 5) + (r & 3) of its register r.  Those registers
// are exactly the B operand of the next layer's k-steps if the k slots are
// taken in that order: slot j of lane half h in k-step s stands for input
// feature 16 s + (j >> 2) * 8 + 4 h + (j & 3).  The weights are staged once
// per block into LDS as bf16 A fragments in the same slot order (64 lanes x
// 8 values, one 16-byte read per lane and MFMA), so the activations never
// leave the registers between layers.
constexpr int kFrag = kWave * 8;                     // bf16 per A fragment
constexpr int kFragL1 = 4, kFragL2 = 32, kFragL3 = 32, kFragL4 = 8;  // 32-feature tiles x k-steps
constexpr int kFragAll = kFragL1 + kFragL2 + kFragL3 + kFragL4;      // 76 fragments, 76 KB
constexpr int kFusedWaves = 8;

__device__ inline int slot_feature(int s, int h, int j) { return 16 * s + (j >> 2) * 8 + 4 * h + (j & 3); }

template <bool SAVE>
__global__ __launch_bounds__(kWave *kFusedWaves) void k_mlp_fwd(const float *__restrict__ P,
                                                                const float *__restrict__ x, int64_t B,
                                                                float *__restrict__ y, float *__restrict__ act) {
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16 *wf = reinterpret_cast<__bf16 *>(smem);  // [kFragAll][64 lanes][8]
  // stage: fragment f of layer L = (tile t, k-step s), lane l, slot j holds
  // W_L[k = slot_feature(s, l >> 5, j)][n = 32 t + (l & 31)] (0 beyond N).
  // A fragment is the 16 x 32 block of W_L at rows 16 s.., columns 32 t..;
  // consecutive threads read consecutive columns of a row (coalesced) and
  // place each value at its lane and slot
  // (eight loads in flight per thread: the staging is latency-bound)
  constexpr int kStage = kFragAll * kFrag, kBatch = 8;
  for (int e0 = threadIdx.x; e0 < kStage; e0 += kBatch * blockDim.x) {
    float v[kBatch];
    int dst[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * blockDim.x;
      v[u] = 0.0f;
      dst[u] = -1;
      if (e < kStage) {
        const int f = e / kFrag, kl = (e % kFrag) / 32, nl = e % 32;
        int ff, S, N, K;
        int64_t off;
        if (f < kFragL1) { ff = f; S = 1; N = HID; K = IN; off = OFF_W1; }
        else if (f < kFragL1 + kFragL2) { ff = f - kFragL1; S = 8; N = HID; K = HID; off = OFF_W2; }
        else if (f < kFragL1 + kFragL2 + kFragL3) { ff = f - kFragL1 - kFragL2; S = 8; N = HID; K = HID; off = OFF_W3; }
        else { ff = f - kFragL1 - kFragL2 - kFragL3; S = 8; N = OUT; K = HID; off = OFF_W4; }
        const int t = ff / S, sk = ff % S;
        const int n = 32 * t + nl, k = 16 * sk + kl;
        // k local = (j >> 2) * 8 + 4 h + (j & 3)  <=>  h = (kl >> 2) & 1, j = (kl >> 3) * 4 + (kl & 3)
        const int h = (kl >> 2) & 1, j = ((kl >> 3) << 2) | (kl & 3);
        dst[u] = f * kFrag + (nl + 32 * h) * 8 + j;
        if (n < N && k < K) v[u] = P[off + (int64_t)k * N + n];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (dst[u] >= 0) wf[dst[u]] = (__bf16)v[u];
  }
  __syncthreads();
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int h = lane >> 5;
  const int64_t tiles = (B + 31) / 32;
  const bf16x8 *frag = reinterpret_cast<const bf16x8 *>(wf);  // frag[f * 64 + lane]
  for (int64_t tile = (int64_t)blockIdx.x * kFusedWaves + w; tile < tiles; tile += (int64_t)gridDim.x * kFusedWaves) {
    const int64_t row = tile * 32 + (lane & 31);
    const bool live = row < B;
    // layer 1 input: x features {4h..4h+3, 8+4h..8+4h+3} of the lane's row
    bf16x8 bin;
    {
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), c = a;
      if (live) {
        a = *reinterpret_cast<const float4 *>(x + row * IN + 4 * h);
        c = *reinterpret_cast<const float4 *>(x + row * IN + 8 + 4 * h);
      }
      bin[0] = (__bf16)a.x; bin[1] = (__bf16)a.y; bin[2] = (__bf16)a.z; bin[3] = (__bf16)a.w;
      bin[4] = (__bf16)c.x; bin[5] = (__bf16)c.y; bin[6] = (__bf16)c.z; bin[7] = (__bf16)c.w;
    }
    // a layer's output as the next layer's B operands (one per k-step);
    // tiles run one at a time (not unrolled, so few fragments are in flight)
    // and their operands are placed by selects, keeping every index static
    bf16x8 hcur[8], hnext[8];
    // bias + SiLU on the accumulator of output tile t, optional save of Z and
    // H, and the bf16 operands of k-steps 2t (lo) and 2t + 1 (hi)
    auto epilogue = [&](const f32x16 &acc, int t, const float *bias, int save_off) {
      bf16x8 lo, hi;
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // four groups of four consecutive features
        const int f0 = 32 * t + q * 8 + 4 * h;
        float z[4], hv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          z[i] = acc[4 * q + i] + bias[f0 + i];
          hv[i] = silu(z[i]);
          if (q < 2) lo[4 * q + i] = (__bf16)hv[i];
          else hi[4 * (q - 2) + i] = (__bf16)hv[i];
        }
        if (SAVE && live) {
          *reinterpret_cast<float4 *>(act + row * ACT + save_off + f0) = make_float4(z[0], z[1], z[2], z[3]);
          *reinterpret_cast<float4 *>(act + row * ACT + save_off + HID + f0) =
              make_float4(hv[0], hv[1], hv[2], hv[3]);
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k == 2 * t) hnext[k] = lo;
        if (k == 2 * t + 1) hnext[k] = hi;
      }
    };
    // layer 1: K = 16, one k-step
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
      f32x16 zero = {};
      const f32x16 a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag[t * kWave + lane], bin, zero, 0, 0, 0);
      epilogue(a, t, P + OFF_B1, 0);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) hcur[k] = hnext[k];
    // layers 2 and 3: K = 128, eight k-steps per output tile
#pragma unroll 1
    for (int L = 0; L < 2; ++L) {
      const int fbase = kFragL1 + L * kFragL2;
#pragma unroll 1
      for (int t = 0; t < 4; ++t) {
        f32x16 a = {};
#pragma unroll
        for (int sk = 0; sk < 8; ++sk)
          a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag[(fbase + t * 8 + sk) * kWave + lane], hcur[sk], a, 0, 0,
                                                      0);
        epilogue(a, t, P + (L == 0 ? OFF_B2 : OFF_B3), (L + 1) * 2 * HID);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) hcur[k] = hnext[k];
    }
    // layer 4: one 32-feature tile, the first 16 are the outputs
    {
      const int fbase = kFragL1 + kFragL2 + kFragL3;
      f32x16 a = {};
#pragma unroll
      for (int sk = 0; sk < 8; ++sk)
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag[(fbase + sk) * kWave + lane], hcur[sk], a, 0, 0, 0);
      if (live) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int f0 = q * 8 + 4 * h;
          const float *b4 = P + OFF_B4;
          *reinterpret_cast<float4 *>(y + row * OUT + f0) =
              make_float4(a[4 * q] + b4[f0], a[4 * q + 1] + b4[f0 + 1], a[4 * q + 2] + b4[f0 + 2],
                          a[4 * q + 3] + b4[f0 + 3]);
        }
      }
    }
  }
}

inline unsigned nb(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <int EPI>
hipError_t gemm(hipStream_t s, const float *A, int lda, int tA, const float *B, int ldb, int tB, int M, int N, int K,
                const float *bias, float *C, int ldc, float *C2, int splits = 1, int64_t split_stride = 0,
                const float *Z = nullptr, int ldz = 0) {
  int kc = (K + splits - 1) / splits;
  kc = (kc + 31) / 32 * 32;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)splits);
  hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(256), 0, s, A, lda, tA, B, ldb, tB, M, N, K, kc, bias, C, ldc, C2,
                     split_stride, Z, ldz);
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

constexpr int kSplitRows = 512;  // batch rows per split-K chunk of a weight gradient (enough blocks to fill the device)

int splits_for(int64_t B) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (B + kSplitRows - 1) / kSplitRows)); }

}  // namespace

extern "C" {

int64_t gmcp_mlp_param_count(void) { return N_PARAMS; }

size_t gmcp_mlp_work_bytes(int64_t B) {
  int S = splits_for(B);
  // two [B][128] gradient buffers, split partials for the largest weight,
  // column-sum partials, loss partials
  return sizeof(float) * ((size_t)2 * B * HID + (size_t)S * HID * HID + (size_t)((B + kColRows - 1) / kColRows + 1) * HID +
                          (size_t)(B * OUT + 255) / 256 + 64);
}

int gmcp_mlp_forward(const float *params, const float *x, int64_t B, float *y, float *act, void *stream) {
  if (!params || !x || !y || B <= 0 || B > (int64_t(1) << 30)) return GMCP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  // one fused launch: every wave runs the whole network on 32 rows at a
  // time (weights staged once per block); two blocks fit a CU's LDS
  // persistent grid: two blocks per compute unit (their LDS), each walking
  // many row tiles, so the weights are staged once per block
  static int n_cu[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GMCP_E_HIP;
  if (n_cu[dev] == 0 && (hipDeviceGetAttribute(&n_cu[dev], hipDeviceAttributeMultiprocessorCount, dev) !=
                             hipSuccess || n_cu[dev] < 1))
    n_cu[dev] = 256;
  const int64_t tiles = (B + 31) / 32;
  const int64_t want = (tiles + kFusedWaves - 1) / kFusedWaves;
  const unsigned grid = (unsigned)std::min<int64_t>(want, 2 * (int64_t)n_cu[dev]);
  const size_t lds = (size_t)kFragAll * kFrag * sizeof(__bf16);
  if (act)
    hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(grid), dim3(kWave * kFusedWaves), lds, s, params, x, B, y, act);
  else
    hipLaunchKernelGGL(k_mlp_fwd<false>, dim3(grid), dim3(kWave * kFusedWaves), lds, s, params, x, B, y, act);
  return hipGetLastError() == hipSuccess ? GMCP_OK : GMCP_E_HIP;
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
  const int rows_per = kColRows;
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
      hipLaunchKernelGGL(k_reduce_split, dim3(nb((int64_t)fin * fout, kWave)), dim3(kWave * kRedGroups), 0, s, part,
                         S, (int64_t)fin * fout, dW);
      e = hipGetLastError();
    }
  };
  auto bgrad = [&](const float *dZ, int ldz, int ncol, float *db) {
    if (e != hipSuccess) return;
    hipLaunchKernelGGL(k_colsum_partial, dim3(cblocks), dim3(2 * HID), 0, s, dZ, B, ldz, ncol, rows_per, cpart);
    hipLaunchKernelGGL(k_reduce_split, dim3(nb(ncol, kWave)), dim3(kWave * kRedGroups), 0, s, cpart, (int)cblocks,
                       (int64_t)ncol, db);
    e = hipGetLastError();
  };
  // layer 4: Y = H3 W4 + b4; each dZ of the layers below comes out of the
  // GEMM with silu'(Z) applied in its epilogue (dA and dB alternate)
  wgrad(H3, ld, HID, dy, OUT, OUT, grad + OFF_W4);
  bgrad(dy, OUT, OUT, grad + OFF_B4);
  if (e == hipSuccess)
    e = gemm<EPI_SILU_BWD>(s, dy, OUT, 0, P + OFF_W4, OUT, 1, (int)B, HID, OUT, nullptr, dB, HID, nullptr, 1, 0, Z3,
                           ld);
  // layer 3
  wgrad(H2, ld, HID, dB, HID, HID, grad + OFF_W3);
  bgrad(dB, HID, HID, grad + OFF_B3);
  if (e == hipSuccess)
    e = gemm<EPI_SILU_BWD>(s, dB, HID, 0, P + OFF_W3, HID, 1, (int)B, HID, HID, nullptr, dA, HID, nullptr, 1, 0, Z2,
                           ld);
  // layer 2
  wgrad(H1, ld, HID, dA, HID, HID, grad + OFF_W2);
  bgrad(dA, HID, HID, grad + OFF_B2);
  if (e == hipSuccess)
    e = gemm<EPI_SILU_BWD>(s, dA, HID, 0, P + OFF_W2, HID, 1, (int)B, HID, HID, nullptr, dB, HID, nullptr, 1, 0, Z1,
                           ld);
  // layer 1
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
