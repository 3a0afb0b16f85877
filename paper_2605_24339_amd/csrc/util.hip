// Device-wide exclusive scan, fills and status resets.
#include "common.h"

namespace gmcp {

namespace {

// When all tiles run at once, inclusive prefixes cross the array at one
// look-back window per memory round trip: a window of 1024 descriptors (the
// whole block reads) and 16 K elements per tile keep that rate far above the
// array's read and write time.  (A 64-descriptor window over 4 K-element
// tiles scanned the 64.6 M cells of a 256-environment grid at 2 TB/s.)
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 16;                         // consecutive elements per thread
constexpr int kScanTile = kScanThreads * kScanPer;  // 16384 elements per tile
// bound on the polls of one look-back window: a predecessor tile publishes
// its sum right after its own loads, so a wait this long means the state
// was corrupted; the kernel then reports an error instead of waiting on
constexpr int kScanSpin = 1 << 20;

__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int t = __shfl_up(v, d, kWave);
    if (lane >= d) v += t;
  }
  return v;
}

// Tile descriptors of the single-pass scan: epoch (30 bits, the call) |
// state (2 bits: 1 = the tile's own sum, 2 = its inclusive prefix) | value.
// A descriptor of another epoch reads as "not yet published".
__device__ inline unsigned long long scan_desc(uint32_t epoch, uint32_t state, int32_t v) {
  return ((unsigned long long)(epoch & 0x3fffffffu) << 34) | ((unsigned long long)state << 32) | (uint32_t)v;
}

// Exclusive scan in one launch (decoupled look-back, Merrill and Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016).
// Tiles are numbered in the order blocks start (a ticket counter), so every
// tile a block waits on belongs to a block already running.  The ticket word
// holds the epoch (high 32 bits) and the tickets taken (low 32); the block
// that takes the last ticket moves it to the next epoch with no tickets, so
// the state is ready for the next call without a clearing pass, and the
// descriptors of earlier calls no longer match.
//
// Grid scans (grid != nullptr): the cells of environment e are
// [cell0_e, cell0_e + budget_e) and only the first nx ny nz of them are
// used this call; the others hold zero counts and nobody reads their
// starts.  A tile that meets no used range (nor the element after one, nor
// the last element) publishes a zero sum and stops: its successors look
// back past it.
__device__ inline bool scan_tile_used(int64_t t0, int64_t t1, int64_t n, const GridEnv *grid, const EnvInfo *env,
                                      int n_env) {
  if (t1 >= n) return true;  // the total
  int lo = 0, hi = n_env - 1;  // the last environment starting at or before t0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (env[mid].cell0 <= t0) lo = mid;
    else hi = mid - 1;
  }
  for (int e = lo; e < n_env && env[e].cell0 < t1; ++e) {
    const GridEnv &g = grid[e];
    const int64_t used = g.valid ? (int64_t)g.nx * g.ny * g.nz : 0;
    if (env[e].cell0 + used >= t0) return true;  // [cell0, cell0 + used] meets [t0, t1)
  }
  return false;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_lookback(const int32_t *__restrict__ in,
                                                                int32_t *__restrict__ out, int64_t n,
                                                                int64_t ntiles, unsigned long long *ticket,
                                                                unsigned long long *desc, DevStatus *st,
                                                                const GridEnv *__restrict__ grid,
                                                                const EnvInfo *__restrict__ env, int n_env) {
  __shared__ uint32_t s_tile, s_epoch;
  __shared__ int s_used;
  __shared__ int wsum[kScanPer / 4][kScanThreads / kWave];
  __shared__ int lb_first[kScanThreads / kWave], lb_wait[kScanThreads / kWave], lb_sum[kScanThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  if (tid == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    const uint32_t t = (uint32_t)(tk & 0xffffffffull);
    if ((int64_t)t == ntiles - 1) atomicAdd(ticket, (1ull << 32) - (unsigned long long)ntiles);
    s_tile = t;
    s_epoch = (uint32_t)(tk >> 32) & 0x3fffffffu;
    s_used = (int64_t)t >= ntiles || !grid ||
             scan_tile_used((int64_t)t * kScanTile, ((int64_t)t + 1) * kScanTile, n, grid, env, n_env);
  }
  __syncthreads();
  const int64_t tile = (int64_t)s_tile;  // 0 .. 2^32 - 1
  if (tile >= ntiles) {  // only if the ticket word was corrupted: no descriptor to write
    if (tid == 0) set_error(st, GMCP_E_TIMEOUT, (unsigned long long)tile);
    return;
  }
  const uint32_t epoch = s_epoch;
  if (!s_used) {  // unused cells: a zero sum (tile 0: its prefix), nothing loaded or written
    if (tid == 0)
      __hip_atomic_store(&desc[tile], scan_desc(epoch, tile == 0 ? 2u : 1u, 0), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  // coalesced loads: group k of the tile is elements [k * 4 * kScanThreads,
  // (k + 1) * 4 * kScanThreads), four consecutive ones per thread
  constexpr int kGroups = kScanPer / 4;
  int4 q[kGroups];
  int gs[kGroups], gi[kGroups];
#pragma unroll
  for (int k = 0; k < kGroups; ++k) {
    const int64_t e0 = tile * kScanTile + ((int64_t)k * kScanThreads + tid) * 4;
    if (e0 + 4 <= n) {
      q[k] = reinterpret_cast<const int4 *>(in)[e0 >> 2];
    } else {
      q[k].x = e0 < n ? in[e0] : 0;
      q[k].y = e0 + 1 < n ? in[e0 + 1] : 0;
      q[k].z = e0 + 2 < n ? in[e0 + 2] : 0;
      q[k].w = 0;
    }
    gs[k] = q[k].x + q[k].y + q[k].z + q[k].w;
    gi[k] = wave_incl_scan(gs[k], lane);
    if (lane == kWave - 1) wsum[k][w] = gi[k];
  }
  __syncthreads();
  // offset of (group k, wave w) in the tile, and the tile's sum
  int goff[kGroups], agg = 0;
#pragma unroll
  for (int k = 0; k < kGroups; ++k) {
    goff[k] = agg;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
      if (i < w) goff[k] += wsum[k][i];
      agg += wsum[k][i];
    }
  }
  if (tid == 0)
    __hip_atomic_store(&desc[tile], scan_desc(epoch, tile == 0 ? 2u : 1u, agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  // look back over windows of kScanThreads predecessors (thread k reads
  // tile i - k) until one holds its inclusive prefix; tiles before 0 read as
  // prefix 0.  The whole block takes each decision from the waves' summaries
  // in LDS, so the loop is uniform.
  int prefix = 0;
  if (tile > 0) {
    int spins = 0;
    for (int64_t i = tile - 1;;) {
      const int64_t j = i - tid;
      const unsigned long long d =
          j >= 0 ? __hip_atomic_load(&desc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : scan_desc(epoch, 2u, 0);
      const uint32_t state = (uint32_t)(d >> 34) == epoch ? (uint32_t)(d >> 32) & 3u : 0u;
      const uint64_t pm = __ballot(state == 2u), zm = __ballot(state == 0u);
      const int first = pm ? __ffsll((unsigned long long)pm) - 1 : kWave;  // the wave's nearest prefix
      const uint64_t need = first >= kWave - 1 ? ~0ull : (2ull << first) - 1;
      int c = lane <= first ? (int)(uint32_t)d : 0;
      for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
      if (lane == 0) {
        lb_first[w] = first;
        lb_wait[w] = (zm & need) != 0;
        lb_sum[w] = c;
      }
      __syncthreads();
      bool wait = false, found = false;
      int add = 0;
      for (int k = 0; k < kScanThreads / kWave && !found; ++k) {
        wait = wait || lb_wait[k];
        add += lb_sum[k];
        found = lb_first[k] < kWave;
      }
      __syncthreads();  // the summaries are read before the next window's writes
      if (wait) {
        if (++spins > kScanSpin) {
          if (tid == 0) set_error(st, GMCP_E_TIMEOUT, (unsigned long long)tile);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      prefix += add;
      if (found) break;
      i -= kScanThreads;
    }
    if (tid == 0)
      __hip_atomic_store(&desc[tile], scan_desc(epoch, 2u, prefix + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
#pragma unroll
  for (int k = 0; k < kGroups; ++k) {
    const int64_t e0 = tile * kScanTile + ((int64_t)k * kScanThreads + tid) * 4;
    int4 o;
    o.x = prefix + goff[k] + gi[k] - gs[k];
    o.y = o.x + q[k].x;
    o.z = o.y + q[k].y;
    o.w = o.z + q[k].z;
    if (e0 + 4 <= n) {
      reinterpret_cast<int4 *>(out)[e0 >> 2] = o;
    } else {
      if (e0 < n) out[e0] = o.x;
      if (e0 + 1 < n) out[e0 + 1] = o.y;
      if (e0 + 2 < n) out[e0 + 2] = o.z;
    }
  }
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

hipError_t scan_exclusive(gmcp_ctx *c, const int32_t *in, int32_t *out, int64_t n, bool side, const GridEnv *grid) {
  // one state per stream that scans (the side stream scans the swept grid):
  // the ticket word, then one descriptor per tile
  int32_t *const scratch = side ? c->b.scan_tmp2 : c->b.scan_tmp;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles <= 0) return hipSuccess;
  if (2 * (ntiles + 1) > (int64_t)c->scan_tmp_elems || ntiles >= (int64_t(1) << 31) ||
      ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15))
    return hipErrorInvalidValue;
  unsigned long long *ticket = reinterpret_cast<unsigned long long *>(scratch);
  hipLaunchKernelGGL(k_scan_lookback, dim3((unsigned)ntiles), dim3(kScanThreads), 0, c->stream, in, out, n, ntiles,
                     ticket, ticket + 1, c->b.status, grid, c->b.env, c->n_env);
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
