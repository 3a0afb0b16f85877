// Device-wide exclusive scan, fills and status resets.
#include "common.h"

namespace gmcp {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;  // 1024 elements per block

__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int t = __shfl_up(v, d, kWave);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan of one 1024-element block; block totals to sums[blockIdx].
__global__ __launch_bounds__(kScanThreads) void k_scan_block(const int32_t *__restrict__ in,
                                                              int32_t *__restrict__ out,
                                                              int32_t *__restrict__ sums, int64_t n) {
  __shared__ int wsum[kScanThreads / kWave];
  int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * kScanPer;
  int v[kScanPer];
  int run = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    int64_t j = base + i;
    v[i] = j < n ? in[j] : 0;
    run += v[i];
  }
  int incl = wave_incl_scan(run, lane);
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int woff = 0;
  for (int i = 0; i < w; ++i) woff += wsum[i];
  int ex = woff + incl - run;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    int64_t j = base + i;
    if (j < n) out[j] = ex;
    ex += v[i];
  }
  if (tid == kScanThreads - 1 && sums) sums[blockIdx.x] = ex;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t *__restrict__ out,
                                                            const int32_t *__restrict__ offs, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int add = offs[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i, j += kScanThreads)
    if (j < n) out[j] += add;
}

// Second launch of the two-launch scan (up to kScanTop blocks): block b
// adds the sum of the block totals before it (its threads split them, wave
// butterflies, the wave sums in LDS) to its 1024 elements.
constexpr int64_t kScanTop = 1024;

__global__ __launch_bounds__(kScanThreads) void k_scan_add_top(int32_t *__restrict__ out,
                                                                const int32_t *__restrict__ sums, int64_t n) {
  __shared__ int wsum[kScanThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int b = blockIdx.x;
  int s = 0;
  for (int i = tid; i < b; i += kScanThreads) s += sums[i];
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane == 0) wsum[w] = s;
  __syncthreads();
  int add = 0;
  for (int i = 0; i < kScanThreads / kWave; ++i) add += wsum[i];
  int64_t j = (int64_t)b * kScanBlock + tid;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i, j += kScanThreads)
    if (j < n) out[j] += add;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_stage_init(DevStatus *st, StageInit a, int n_env) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) {
    if (a.which & 1) st->n_cand = 0;  // broad phase
    if (a.which & 2) {                // assembly
      st->n_active = 0;
      st->n_pairs = 0;
      st->nnzb = 0;
      st->mortar_alloc = 0;
    }
    if (a.which & 4) st->n_swept = 0;  // step bound
  }
  if (blockIdx.x == 0)
    for (int k = 0; k < 3; ++k)
      if (a.zero[k] && (int)threadIdx.x < a.nzero[k]) a.zero[k][threadIdx.x] = 0;
  if (e < n_env) {
    if (a.box)
      for (int d = 0; d < 3; ++d) {
        a.box[6 * e + d] = 0xffffffffu;  // min: largest ordered value
        a.box[6 * e + 3 + d] = 0u;       // max: smallest ordered value
      }
    if (a.alpha) a.alpha[e] = 0x7f800000u;  // +inf
  }
}

}  // namespace

hipError_t scan_exclusive(gmcp_ctx *c, const int32_t *in, int32_t *out, int64_t n, bool side) {
  int32_t *const scratch = side ? c->b.scan_tmp2 : c->b.scan_tmp;
  // levels: out <- scan(in); block sums in tmp, scanned recursively in place
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb <= 0) return hipSuccess;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(kScanThreads), 0, c->stream, in, out, nullptr, n);
    return hipGetLastError();
  }
  if (nb <= kScanTop) {  // two launches: block scans + totals, then each block's offset
    if (nb > (int64_t)c->scan_tmp_elems) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kScanThreads), 0, c->stream, in, out, scratch, n);
    hipLaunchKernelGGL(k_scan_add_top, dim3((unsigned)nb), dim3(kScanThreads), 0, c->stream, out,
                       (const int32_t *)scratch, n);
    return hipGetLastError();
  }
  // the scratch holds every level's block sums back to back
  int32_t *lvl_in[8], *lvl_out[8];
  int64_t lvl_n[8];
  int depth = 0;
  int32_t *tmp = scratch;
  int64_t used = 0;
  int64_t cur = n;
  const int32_t *src = in;
  int32_t *dst = out;
  for (;;) {
    int64_t blocks = (cur + kScanBlock - 1) / kScanBlock;
    int32_t *sums = blocks > 1 ? tmp + used : nullptr;
    if (blocks > 1) {
      if (used + 2 * blocks > (int64_t)c->scan_tmp_elems || depth >= 8) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)blocks), dim3(kScanThreads), 0, c->stream, src, dst,
                       sums, cur);
    lvl_in[depth] = dst;
    lvl_out[depth] = sums;
    lvl_n[depth] = cur;
    ++depth;
    if (blocks == 1) break;
    int32_t *sums_scanned = tmp + used + blocks;
    used += 2 * blocks;
    src = sums;
    dst = sums_scanned;
    cur = blocks;
  }
  // propagate block offsets down: level d's sums were scanned into level d+1's dst
  for (int d = depth - 2; d >= 0; --d) {
    int64_t blocks = (lvl_n[d] + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)blocks), dim3(kScanThreads), 0, c->stream, lvl_in[d],
                       lvl_in[d + 1], lvl_n[d]);
  }
  (void)lvl_out;
  return hipGetLastError();
}

hipError_t fill_i32(gmcp_ctx *c, int32_t *p, int32_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, c->stream, p, v, n);
  return hipGetLastError();
}

hipError_t stage_init(gmcp_ctx *c, const StageInit &a) {
  for (int k = 0; k < 3; ++k)
    if (a.nzero[k] > 64) return hipErrorInvalidValue;
  const int blocks = c->n_env > 64 ? (c->n_env + 63) / 64 : 1;
  hipLaunchKernelGGL(k_stage_init, dim3(blocks), dim3(64), 0, c->stream, c->b.status, a, c->n_env);
  return hipGetLastError();
}

}  // namespace gmcp
