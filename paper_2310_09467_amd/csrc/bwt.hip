// bwt.hip -- Burrows-Wheeler transform of every block by prefix doubling.
//
// All blocks of a batch are sorted together.  A rotation's rank is the
// position in the final suffix order where its group (rotations sharing the
// compared prefix) starts, so ranks of different blocks never collide.
//   round 0: key = (block, first four bytes of the rotation, cyclic)
//   round r: key = (rank[g], rank[start + (g - start + h) mod m]) for the
//            rotations still in groups of two or more, h = 4 * 2^(r-1)
// After each stable sort the group starts give new ranks; groups of one are
// final, and a block is final once the compared prefix length reaches its
// length m (equal rotations of a periodic block are then ordered by start
// index, which the stable sort preserved from the initial index order).
//
// Sorting is a least-significant-digit radix sort (8-bit digits) on 64-bit
// keys with 32-bit values: per-tile digit counts, one exclusive scan over
// the digit-major count table, then a stable scatter that ranks equal digits
// inside each wavefront with ballot matching.
#include <cstdio>
#include <cstdlib>

#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;

__device__ __forceinline__ uint32_t dev_n(const uint32_t *d_n, uint32_t n_max) {
  if (!d_n) return n_max;
  uint32_t n = *d_n;
  return n < n_max ? n : n_max;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t *keys, const uint32_t *d_n, uint32_t n_max,
                                                        int shift, uint32_t *counts, uint32_t stride) {
  __shared__ uint32_t h[kRsThreads / kWave][256];
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < (kRsThreads / kWave) * 256; i += kRsThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint32_t n = dev_n(d_n, n_max);
  const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
  if (base < n) {
#pragma unroll 4
    for (int it = 0; it < kRsItems; it++) {
      uint64_t j = base + (uint64_t)it * kRsThreads + threadIdx.x;
      if (j < n) atomicAdd(&h[w][(uint32_t)(keys[j] >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  uint32_t d = threadIdx.x;
  uint32_t c = 0;
  for (int k = 0; k < kRsThreads / kWave; k++) c += h[k][d];
  counts[(size_t)d * stride + blockIdx.x] = c;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t *keys_in, const uint32_t *vals_in,
                                                           uint64_t *keys_out, uint32_t *vals_out,
                                                           const uint32_t *d_n, uint32_t n_max, int shift,
                                                           const uint32_t *offsets, uint32_t stride) {
  __shared__ uint32_t base_d[256];
  __shared__ uint32_t wcnt[kRsThreads / kWave][256];
  const uint32_t n = dev_n(d_n, n_max);
  const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
  if (base >= n) return;
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  base_d[threadIdx.x] = offsets[(size_t)threadIdx.x * stride + blockIdx.x];
  for (int k = 0; k < kRsThreads / kWave; k++) wcnt[k][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  for (int it = 0; it < kRsItems; it++) {
    const uint64_t j = base + (uint64_t)it * kRsThreads + threadIdx.x;
    const bool valid = j < n;
    uint64_t key = 0;
    uint32_t val = 0, d = 0;
    if (valid) {
      key = keys_in[j];
      val = vals_in[j];
      d = (uint32_t)(key >> shift) & 255u;
    }
    const uint64_t act = ballot64(valid);
    const uint64_t peers = match_any8(d, act);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base_d[d] + rank;
      for (int k = 0; k < w; k++) pos += wcnt[k][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    {
      const uint32_t dd = threadIdx.x;
      uint32_t add = 0;
      for (int k = 0; k < kRsThreads / kWave; k++) {
        add += wcnt[k][dd];
        wcnt[k][dd] = 0;
      }
      base_d[dd] += add;
    }
    __syncthreads();
    (void)lane;
  }
}

// ---------------------------------------------------------------- doubling steps
__device__ __forceinline__ uint32_t block_of(const uint32_t *blk_start, uint32_t nb, uint32_t g) {
  return upper_index(blk_start, nb, g);
}

__global__ void k_bwt_init(const uint8_t *rle, uint32_t N, const uint32_t *blk_start, uint32_t nb, uint64_t *keys,
                           uint32_t *vals, uint32_t *slot) {
  for (uint64_t gi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < N; gi += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = (uint32_t)gi;
    const uint32_t k = block_of(blk_start, nb, g);
    const uint32_t s = blk_start[k], m = blk_start[k + 1] - s, i = g - s;
    uint32_t v = 0;
    for (uint32_t t = 0; t < 4; t++) v = (v << 8) | rle[s + (i + t) % m];
    keys[g] = ((uint64_t)k << 32) | v;
    vals[g] = g;
    slot[g] = g;
  }
}

// Group-start markers (the slot of each group's first element), for a
// max-scan that yields every element's new rank.
__global__ void k_bwt_heads(const uint64_t *keys, const uint32_t *slot, uint32_t U, uint32_t *mark) {
  for (uint64_t ki = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ki < U; ki += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)ki;
    mark[k] = (k == 0 || keys[k] != keys[k - 1]) ? slot[k] : 0u;
  }
}

// Writes ranks and suffix-array entries; flags elements that stay unresolved.
__global__ void k_bwt_update(const uint64_t *keys, const uint32_t *vals, const uint32_t *slot,
                             const uint32_t *newrank, uint32_t U, const uint32_t *blk_start, uint32_t nb,
                             uint32_t compared, uint32_t *rank, uint32_t *sa, uint32_t *unres) {
  for (uint64_t ki = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ki < U; ki += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)ki;
    const uint32_t g = vals[k];
    rank[g] = newrank[k];
    sa[slot[k]] = g;
    const bool first = (k == 0) || keys[k] != keys[k - 1];
    const bool last = (k + 1 == U) || keys[k + 1] != keys[k];
    const uint32_t b = block_of(blk_start, nb, g);
    const uint32_t m = blk_start[b + 1] - blk_start[b];
    unres[k] = (first && last) || m <= compared ? 0u : 1u;
  }
}

__global__ void k_bwt_compact(const uint32_t *vals, const uint32_t *slot, const uint32_t *unres,
                              const uint32_t *pos, uint32_t U, uint32_t *vals2, uint32_t *slot2) {
  for (uint64_t ki = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ki < U; ki += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)ki;
    if (unres[k]) {
      vals2[pos[k]] = vals[k];
      slot2[pos[k]] = slot[k];
    }
  }
}

__global__ void k_bwt_keys(const uint32_t *vals, uint32_t U, const uint32_t *rank, const uint32_t *blk_start,
                           uint32_t nb, uint32_t h, int bits, uint64_t *keys) {
  for (uint64_t ki = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ki < U; ki += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = vals[ki];
    const uint32_t b = block_of(blk_start, nb, g);
    const uint32_t s = blk_start[b], m = blk_start[b + 1] - s;
    const uint32_t g2 = s + (uint32_t)(((uint64_t)(g - s) + h) % m);
    keys[ki] = ((uint64_t)rank[g] << bits) | rank[g2];
  }
}

__global__ void k_bwt_emit(const uint32_t *sa, const uint8_t *rle, uint32_t N, const uint32_t *blk_start, uint32_t nb,
                           uint8_t *L, BlockCode *codes) {
  for (uint64_t ji = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; ji < N; ji += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = (uint32_t)ji;
    const uint32_t g = sa[j];
    const uint32_t b = block_of(blk_start, nb, j);
    const uint32_t s = blk_start[b], e = blk_start[b + 1];
    L[j] = rle[g == s ? e - 1 : g - 1];
    if (g == s) codes[b].orig_ptr = j - s;
  }
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) b++;
  return b;
}

uint32_t grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (uint32_t)g;
}

}  // namespace

size_t radix_counts_words(uint32_t n_max) { return (size_t)256 * ((n_max + kRsTile - 1) / kRsTile + 1); }

// Sorts (keys[0], vals[0]) by the low `bits` bits of the key; returns the
// buffer index holding the result.
int radix_sort(uint64_t *keys[2], uint32_t *vals[2], uint32_t n, int bits, uint32_t *counts, void *scan_tmp,
               hipStream_t s) {
  int cur = 0;
  if (n <= 1 || bits <= 0) return cur;
  const uint32_t ntiles = (n + kRsTile - 1) / kRsTile;
  for (int shift = 0; shift < bits; shift += 8) {
    PCBZ_LAUNCH(k_rs_hist, dim3(ntiles), dim3(kRsThreads), 0, s, keys[cur], nullptr, n, shift, counts, ntiles);
    scan_exclusive_u32(counts, counts, nullptr, 256u * ntiles, scan_tmp, nullptr, s);
    PCBZ_LAUNCH(k_rs_scatter, dim3(ntiles), dim3(kRsThreads), 0, s, keys[cur], vals[cur], keys[cur ^ 1],
                       vals[cur ^ 1], nullptr, n, shift, counts, ntiles);
    // a scatter pass reads and writes every 8-byte key and 4-byte value once
    trace_bytes("k_rs_scatter", 24ull * n);
    cur ^= 1;
  }
  return cur;
}

// Eager prefix doubling: reads the unresolved count back after each round.
int run_bwt(const uint8_t *rle, uint32_t N, uint32_t nb, const uint32_t *blk_start, BwtWork w, uint32_t *sa,
            uint8_t *L, BlockCode *codes, uint32_t *pinned_u, hipStream_t s) {
  if (N == 0) return 0;
  uint64_t *keys[2] = {w.key[0], w.key[1]};
  uint32_t *vals[2] = {w.val[0], w.val[1]};
  uint32_t *slot = w.slot, *slot2 = w.slot2;
  PCBZ_LAUNCH(k_bwt_init, dim3(grid_for(N)), dim3(256), 0, s, rle, N, blk_start, nb, keys[0], vals[0], slot);
  int cur = radix_sort(keys, vals, N, 32 + bits_for(nb - 1), w.counts, w.scan_tmp, s);
  const int rbits = bits_for(N - 1);
  uint32_t U = N;
  uint32_t compared = 4;
  int rounds = 0;
  for (;;) {
    // new ranks: max-scan of group-start slots
    PCBZ_LAUNCH(k_bwt_heads, dim3(grid_for(U)), dim3(256), 0, s, keys[cur], slot, U, w.flag);
    scan_inclusive_max_u32(w.flag, w.flag, nullptr, U, w.scan_tmp, s);
    PCBZ_LAUNCH(k_bwt_update, dim3(grid_for(U)), dim3(256), 0, s, keys[cur], vals[cur], slot, w.flag, U,
                       blk_start, nb, compared, w.rank, sa, w.flag2);
    scan_exclusive_u32(w.flag2, w.flag, nullptr, U, w.scan_tmp, w.d_u, s);
    PCBZ_LAUNCH(k_bwt_compact, dim3(grid_for(U)), dim3(256), 0, s, vals[cur], slot, w.flag2, w.flag, U,
                       vals[cur ^ 1], slot2);
    hipMemcpyAsync(pinned_u, w.d_u, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    U = *pinned_u;
    rounds++;
    if (getenv("PCBZ_DEBUG_BWT")) fprintf(stderr, "pcbz bwt: N=%u round %d compared=%u unresolved=%u\n", N, rounds, compared, U);
    if (U == 0) break;
    if (rounds > 40 || compared >= (1u << 31)) return -1;  // doubling must finish once 2h reaches the block length
    // compact list is now in (vals[cur^1], slot2)
    cur ^= 1;
    uint32_t *t = slot;
    slot = slot2;
    slot2 = t;
    const uint32_t h = compared;
    PCBZ_LAUNCH(k_bwt_keys, dim3(grid_for(U)), dim3(256), 0, s, vals[cur], U, w.rank, blk_start, nb, h, rbits,
                       keys[cur]);
    // sort keys[cur]/vals[cur]; radix_sort sorts buffer 0, so arrange the pair
    uint64_t *kk[2] = {keys[cur], keys[cur ^ 1]};
    uint32_t *vv[2] = {vals[cur], vals[cur ^ 1]};
    int r = radix_sort(kk, vv, U, 2 * rbits, w.counts, w.scan_tmp, s);
    if (r == 1) cur ^= 1;
    compared = compared * 2;
  }
  PCBZ_LAUNCH(k_bwt_emit, dim3(grid_for(N)), dim3(256), 0, s, sa, rle, N, blk_start, nb, L, codes);
  return rounds;
}

}  // namespace pcbz
