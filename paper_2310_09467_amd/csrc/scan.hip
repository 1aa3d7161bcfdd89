// scan.hip -- device-wide prefix scans (sum and max over uint32) and fills.
//
// Two launches: per-tile reductions, then a per-tile rescan from a carry
// that each workgroup sums from the aggregates itself.  A tile is 256 threads x
// 16 items, staged through LDS so that global accesses stay coalesced while
// each thread scans 16 consecutive items.  (A single pass with decoupled
// look-back measured slower here: device-scope status polls across the XCDs
// cost about a microsecond each.)  Sums wrap mod 2^32, so differences of
// prefix values inside any segment whose own total stays below 2^32 are
// exact.
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;
constexpr int kPad = kTile + kTile / 32;
constexpr uint32_t kStateWords = 16;  // reserved words in front of the tile aggregates

struct OpSum {
  static __device__ __forceinline__ uint32_t f(uint32_t a, uint32_t b) { return a + b; }
  static constexpr uint32_t id = 0u;
};
struct OpMax {
  static __device__ __forceinline__ uint32_t f(uint32_t a, uint32_t b) { return a > b ? a : b; }
  static constexpr uint32_t id = 0u;
};

__device__ __forceinline__ uint32_t get_n(const uint32_t *d_n, uint32_t n_max) {
  if (!d_n) return n_max;
  uint32_t n = *d_n;
  return n < n_max ? n : n_max;
}

__device__ __forceinline__ int padi(int j) { return j + (j >> 5); }

// Workgroup scan of one value per thread: inclusive and exclusive prefix of
// this thread, and the workgroup total.
template <typename Op>
__device__ void block_scan(uint32_t v, uint32_t *sh_wave, uint32_t &incl, uint32_t &excl, uint32_t &total) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t o = __shfl_up(x, d);
    if (lane >= d) x = Op::f(o, x);
  }
  uint32_t xe = __shfl_up(x, 1);
  if (lane == 0) xe = Op::id;
  if (lane == kWave - 1) sh_wave[wave] = x;
  __syncthreads();
  uint32_t carry = Op::id, t = Op::id;
  for (int w = 0; w < nwaves; w++) {
    if (w < wave) carry = Op::f(carry, sh_wave[w]);
    t = Op::f(t, sh_wave[w]);
  }
  __syncthreads();
  incl = Op::f(carry, x);
  excl = Op::f(carry, xe);
  total = t;
}

// Phase 1: per-tile reductions over a capped grid.
template <typename Op>
__global__ __launch_bounds__(kThreads) void k_reduce(const uint32_t *in, const uint32_t *d_n, uint32_t n_max,
                                                     uint32_t *aggs) {
  __shared__ uint32_t sh_wave[kThreads / kWave];
  const uint32_t n = get_n(d_n, n_max);
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t base = (uint64_t)tile * kTile;
    uint32_t acc = Op::id;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
      const uint64_t j = base + (uint64_t)i * kThreads + threadIdx.x;
      if (j < n) acc = Op::f(acc, in[j]);
    }
    uint32_t inc, exc, total;
    block_scan<Op>(acc, sh_wave, inc, exc, total);
    if (threadIdx.x == 0) aggs[tile] = total;
  }
}

// Phase 2: each workgroup reduces the aggregates in front of its tile
// itself (a few KB from L2; later tiles of the same workgroup extend the
// sum), then rescans its items from that carry.
template <typename Op, bool kInclusive>
__global__ __launch_bounds__(kThreads) void k_downsweep(const uint32_t *in, uint32_t *out, const uint32_t *d_n,
                                                        uint32_t n_max, const uint32_t *aggs, uint32_t *d_total) {
  __shared__ uint32_t tile_buf[kPad];
  __shared__ uint32_t sh_wave[kThreads / kWave];
  const uint32_t n = get_n(d_n, n_max);
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0 && d_total) *d_total = Op::id;
  uint32_t carry = Op::id, counted = 0;  // carry = Op over aggs[0, counted)
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    uint32_t part = Op::id;
    for (uint32_t j = counted + threadIdx.x; j < tile; j += kThreads) part = Op::f(part, aggs[j]);
    uint32_t inc, exc, total;
    block_scan<Op>(part, sh_wave, inc, exc, total);
    carry = Op::f(carry, total);
    counted = tile;
    const uint64_t base = (uint64_t)tile * kTile;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
      const int j = i * kThreads + threadIdx.x;
      const uint64_t g = base + j;
      tile_buf[padi(j)] = g < n ? in[g] : Op::id;
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t acc = Op::id;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
      v[i] = tile_buf[padi(threadIdx.x * kItems + i)];
      acc = Op::f(acc, v[i]);
    }
    block_scan<Op>(acc, sh_wave, inc, exc, total);
    uint32_t run = Op::f(carry, exc);
#pragma unroll
    for (int i = 0; i < kItems; i++) {
      const uint32_t nv = Op::f(run, v[i]);
      tile_buf[padi(threadIdx.x * kItems + i)] = kInclusive ? nv : run;
      run = nv;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; i++) {
      const int j = i * kThreads + threadIdx.x;
      const uint64_t g = base + j;
      if (g < n) out[g] = tile_buf[padi(j)];
    }
    if (tile == ntiles - 1 && d_total && threadIdx.x == 0) *d_total = Op::f(carry, total);
    __syncthreads();
  }
}

__global__ void k_copy1(uint32_t *dst, const uint32_t *src) { *dst = *src; }

__global__ void k_fill(uint32_t *p, uint32_t v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

template <typename Op, bool kInclusive>
void run_scan(const uint32_t *in, uint32_t *out, const uint32_t *d_n, uint32_t n_max, void *tmp, uint32_t *d_total,
              hipStream_t s) {
  if (n_max == 0) {
    if (d_total) fill_u32(d_total, 0, 1, s);
    return;
  }
  const uint32_t ntiles = (n_max + kTile - 1) / kTile;
  const uint32_t grid = ntiles < 2048 ? ntiles : 2048;  // persistent grid; tiles come from the device count
  uint32_t *aggs = (uint32_t *)tmp + kStateWords;
  PCBZ_LAUNCH((k_reduce<Op>), dim3(grid), dim3(kThreads), 0, s, in, d_n, n_max, aggs);
  PCBZ_LAUNCH((k_downsweep<Op, kInclusive>), dim3(grid), dim3(kThreads), 0, s, in, out, d_n, n_max, aggs, d_total);
}

}  // namespace

size_t scan_tmp_bytes(size_t n_max) {
  return (kStateWords + (n_max + kTile - 1) / kTile + 1) * sizeof(uint32_t);
}


void scan_exclusive_u32(const uint32_t *in, uint32_t *out, const uint32_t *d_n, uint32_t n_max, void *tmp,
                        uint32_t *d_total, hipStream_t s) {
  run_scan<OpSum, false>(in, out, d_n, n_max, tmp, d_total, s);
}

void scan_inclusive_max_u32(const uint32_t *in, uint32_t *out, const uint32_t *d_n, uint32_t n_max, void *tmp,
                            hipStream_t s) {
  run_scan<OpMax, true>(in, out, d_n, n_max, tmp, nullptr, s);
}

void copy_u32(uint32_t *dst, const uint32_t *src, hipStream_t s) {
  PCBZ_LAUNCH(k_copy1, dim3(1), dim3(1), 0, s, dst, src);
}

void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  PCBZ_LAUNCH(k_fill, dim3((uint32_t)blocks), dim3(256), 0, s, p, v, n);
}

}  // namespace pcbz
