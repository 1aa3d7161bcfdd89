// bwt.hip -- Burrows-Wheeler transform of every block by prefix doubling.
//
// All blocks of a batch are sorted together.  A rotation's rank is the
// position in the final suffix order where its group (rotations sharing the
// compared prefix) starts, so ranks of different blocks never collide.
//   round 0: key = (block, first b bytes of the rotation, cyclic), b = 7
//            (6 above 256 blocks per call, 4 above 65536)
//   round r: key = (rank[g], rank[start + (g - start + h) mod m]) for the
//            rotations still in groups of two or more, h = b * 2^(r-1)
// After each stable sort the group starts give new ranks; groups of one are
// final, and a block is final once the compared prefix length reaches its
// length m (equal rotations of a periodic block are then ordered by start
// index, which the stable sort preserved from the initial index order).
//
// Round 0 and any round with a group larger than kSegMaxGroup use a
// least-significant-digit radix sort (8-bit digits) on 64-bit keys with
// 32-bit values: per-tile digit counts, an exclusive scan of each
// digit's row of counts (one workgroup per digit, which also yields the
// digit totals), then a stable scatter.  The scatter ranks
// equal digits inside each wavefront with ballot matching, sorts the tile by
// digit in LDS, and writes each digit's run with consecutive threads.
//
// The other rounds sort each group on its own (k_seg_sort): the unresolved
// list is already ordered by group, so only the second rank has to be
// ordered inside each group.  A workgroup owns the groups whose first element
// lies in its tile of kSegTile positions, stages them (at most kSegCap
// elements) in LDS, sorts every 64-element chunk in registers, and places
// each element by counting, with a binary search per chunk its group spans,
// the elements that precede it.
//
// Every count (elements, blocks, unresolved rotations) is read from device
// memory and every kernel loops over its work with a capped grid, so the
// whole sort can be enqueued without reading anything back: a caller either
// reads the unresolved count after each round to stop early, or enqueues a
// fixed number of rounds (after which the count must be zero).
#include <cstdio>
#include <cstdlib>

#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr int kRsThreads = 256;
constexpr uint32_t kGridCap = 2048;  // workgroups of the grid-stride kernels

__device__ __forceinline__ uint32_t dev_n(const uint32_t *d_n, uint32_t n_max) {
  if (!d_n) return n_max;
  const uint32_t n = *d_n;
  return n < n_max ? n : n_max;
}

// Tiles of a sort.  Unsegmented (blk null): tile t covers [t TILE,
// min(n, (t + 1) TILE)).  Segmented: every pass keeps each block's elements
// inside the block's range (a stable sort within each block, so no pass is
// spent on the block id) and tiles never straddle a block: tile t of block b
// (tile_base[b] <= t < tile_base[b + 1]) covers TILE elements from
// blk[b] + (t - tile_base[b]) TILE, cut at the block's end.
struct RsSeg {
  const uint32_t *blk;        // block starts [nb + 1], or null
  const uint32_t *tile_base;  // first tile of each block [nb + 1]
  const uint32_t *d_nb;
};
struct RsTile {
  uint32_t base, tn, b, tb0, tb1;  // tb0, tb1: the block's first tile and the next block's
};
// With fewer than 64 blocks a lane holds block lane's start and first tile
// (loaded once per workgroup), and a tile's block is one ballot.
struct RsLanes {
  uint32_t nb, bs, tbl;
  bool on;
};
__device__ __forceinline__ RsLanes rs_lanes(const RsSeg &sg) {
  RsLanes L{0u, 0u, 0xFFFFFFFFu, false};
  if (!sg.blk) return L;
  L.nb = *sg.d_nb;
  L.on = L.nb < (uint32_t)kWave;
  const uint32_t lane = lane_id();
  if (L.on && lane <= L.nb) {
    L.bs = sg.blk[lane];
    L.tbl = lane < L.nb ? sg.tile_base[lane] : 0xFFFFFFFFu;
  }
  return L;
}
__device__ __forceinline__ uint32_t rs_tiles(const RsSeg &sg, uint32_t n, uint32_t tile_len) {
  return sg.blk ? sg.tile_base[*sg.d_nb] : (n + tile_len - 1) / tile_len;
}
__device__ __forceinline__ RsTile rs_tile(const RsSeg &sg, const RsLanes &L, uint32_t n, uint32_t nt,
                                          uint32_t tile_len, uint32_t t) {
  if (!sg.blk) {
    const uint32_t base = t * tile_len;
    return {base, min(tile_len, n - base), 0u, 0u, nt};
  }
  uint32_t b, s0, s1, tb0, tb1;
  if (L.on) {  // uniform: every lane holds the same t
    b = (uint32_t)__popcll(ballot64(L.tbl <= t)) - 1u;
    s0 = (uint32_t)__builtin_amdgcn_readlane((int)L.bs, (int)b);
    s1 = (uint32_t)__builtin_amdgcn_readlane((int)L.bs, (int)b + 1);
    tb0 = (uint32_t)__builtin_amdgcn_readlane((int)L.tbl, (int)b);
    tb1 = b + 1 < L.nb ? (uint32_t)__builtin_amdgcn_readlane((int)L.tbl, (int)b + 1) : nt;
  } else {
    b = upper_index(sg.tile_base, L.nb, t);
    s0 = sg.blk[b];
    s1 = sg.blk[b + 1];
    tb0 = sg.tile_base[b];
    tb1 = sg.tile_base[b + 1];
  }
  const uint32_t base = s0 + (t - tb0) * tile_len;
  return {base, min(tile_len, s1 - base), b, tb0, tb1};
}

// first tile of each block: exclusive scan of ceil(block length / tile_len).
// One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_rs_tile_base(const uint32_t *blk, const uint32_t *d_nb, uint32_t tile_len,
                                                      uint32_t *tile_base) {
  __shared__ uint32_t sh[256];
  const uint32_t nb = *d_nb, t = threadIdx.x;
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += 256) {
    const uint32_t b = c0 + t;
    const uint32_t v = b < nb ? (blk[b + 1] - blk[b] + tile_len - 1) / tile_len : 0u;
    sh[t] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 256; d <<= 1) {
      const uint32_t x = t >= d ? sh[t - d] : 0u;
      __syncthreads();
      sh[t] += x;
      __syncthreads();
    }
    if (b < nb) tile_base[b] = carry + sh[t] - v;
    carry += sh[255];
    __syncthreads();
  }
  if (t == 0) tile_base[nb] = carry;
}

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t *keys, const uint32_t *d_n, uint32_t n_max,
                                                        RsSeg sg, int shift, uint32_t *counts, uint32_t *d_count_n) {
  constexpr uint32_t TILE = kRsThreads * ITEMS;
  __shared__ uint32_t h[kRsThreads / kWave][256];
  const uint32_t n = dev_n(d_n, n_max);
  const uint32_t nt = rs_tiles(sg, n, TILE);
  if (blockIdx.x == 0 && threadIdx.x == 0) *d_count_n = 256u * nt;
  const int w = threadIdx.x / kWave;
  const RsLanes RL = rs_lanes(sg);
  for (XcdWalk wk(nt); wk.t < wk.end; wk.t += wk.step) {
    const uint32_t tile = wk.t;
    const RsTile T = rs_tile(sg, RL, n, nt, TILE, tile);
    const uint32_t te = T.base + T.tn;
    for (int i = threadIdx.x; i < (kRsThreads / kWave) * 256; i += kRsThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    // a thread counts ITEMS consecutive keys (vector loads) and adds each run
    // of equal digits once; a digit shared by the whole wavefront (the block
    // id, the mostly-zero high bytes) is added once per wavefront
    const uint64_t j0 = (uint64_t)T.base + (uint64_t)threadIdx.x * ITEMS;
    uint32_t dig[ITEMS];
    if (j0 + ITEMS <= te && (j0 & 1) == 0) {  // 16-byte loads need an even start
      const uint4 *q = (const uint4 *)(keys + j0);
#pragma unroll
      for (int i = 0; i < ITEMS / 2; i++) {
        const uint4 t = q[i];
        dig[2 * i] = (uint32_t)((((uint64_t)t.y << 32) | t.x) >> shift) & 255u;
        dig[2 * i + 1] = (uint32_t)((((uint64_t)t.w << 32) | t.z) >> shift) & 255u;
      }
    } else if (j0 + ITEMS <= te) {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) dig[i] = (uint32_t)(keys[j0 + i] >> shift) & 255u;
    } else {
#pragma unroll
      for (int i = 0; i < ITEMS; i++) dig[i] = j0 + i < te ? (uint32_t)(keys[j0 + i] >> shift) & 255u : 256u;
    }
    uint32_t cur = dig[0], run = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
      if (dig[i] != cur) {
        if (cur < 256u) atomicAdd(&h[w][cur], run);
        cur = dig[i];
        run = 0;
      }
      run++;
    }
    const bool valid = cur < 256u;
    const uint64_t vm = ballot64(valid);
    if (vm) {  // uniform: every lane of the wavefront takes the same branches below
      const uint32_t dv = (uint32_t)__builtin_amdgcn_readlane((int)cur, (int)__builtin_ctzll(vm));
      if (__all(!valid || cur == dv)) {
        uint32_t r = valid ? run : 0u;
        for (int dd = kWave / 2; dd > 0; dd >>= 1) r += (uint32_t)__shfl_xor((int)r, dd);
        if (lane_id() == 0) atomicAdd(&h[w][dv], r);
      } else if (valid) {
        atomicAdd(&h[w][cur], run);
      }
    }
    __syncthreads();
    const uint32_t d = threadIdx.x;
    uint32_t c = 0;
    for (int k = 0; k < kRsThreads / kWave; k++) c += h[k][d];
    counts[(size_t)d * nt + tile] = c;
    __syncthreads();
  }
}

// Exclusive scan of one digit's row of per-tile counts, in place; the row
// total goes to totals[digit].  One workgroup per digit.
template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_rowscan(uint32_t *counts, const uint32_t *d_n, uint32_t n_max,
                                                           RsSeg sg, uint32_t *totals) {
  constexpr uint32_t TILE = kRsThreads * ITEMS;
  constexpr uint32_t kPer = 16;  // consecutive row entries per thread
  __shared__ uint32_t wsum[kRsThreads / kWave];
  const uint32_t n = dev_n(d_n, n_max);
  const uint32_t nt = rs_tiles(sg, n, TILE);
  uint32_t *row = counts + (size_t)blockIdx.x * nt;
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < nt; c0 += kRsThreads * kPer) {
    const uint32_t b = c0 + threadIdx.x * kPer;
    uint32_t v[kPer], sum = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPer; i++) {
      v[i] = b + i < nt ? row[b + i] : 0u;
      sum += v[i];
    }
    uint32_t incl = sum;
    for (int dd = 1; dd < kWave; dd <<= 1) {
      const uint32_t t = __shfl_up(incl, dd);
      if (lane >= dd) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = carry, chunk = 0;
    for (int k = 0; k < kRsThreads / kWave; k++) {
      if (k < w) before += wsum[k];
      chunk += wsum[k];
    }
    uint32_t run = before + incl - sum;
#pragma unroll
    for (uint32_t i = 0; i < kPer; i++) {
      if (b + i < nt) row[b + i] = run;
      run += v[i];
    }
    carry += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t *keys_in, const uint32_t *vals_in,
                                                           uint64_t *keys_out, uint32_t *vals_out,
                                                           const uint32_t *d_n, uint32_t n_max, RsSeg sg, int shift,
                                                           const uint32_t *offsets, const uint32_t *totals) {
  constexpr uint32_t TILE = kRsThreads * ITEMS;
  __shared__ uint64_t skey[TILE];
  __shared__ uint32_t sval[TILE];
  __shared__ uint32_t gbase[256];   // global position of each digit's run in this tile
  __shared__ uint32_t lstart[256];  // start of each digit's run inside the tile
  __shared__ uint32_t wcnt[kRsThreads / kWave][256];
  __shared__ uint32_t wsum[kRsThreads / kWave];
  __shared__ uint32_t bsum[kRsThreads / kWave];
  const uint32_t n = dev_n(d_n, n_max);
  const uint32_t nt = rs_tiles(sg, n, TILE);
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t d0 = threadIdx.x;
  // first output position of each digit: exclusive scan of the digit totals
  uint32_t dbase;
  {
    const uint32_t tot = totals[d0];
    uint32_t incl = tot;
    for (int dd = 1; dd < kWave; dd <<= 1) {
      const uint32_t t = __shfl_up(incl, dd);
      if (lane >= dd) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    dbase = incl - tot;
    for (int k = 0; k < w; k++) dbase += wsum[k];
    __syncthreads();
  }
  const uint32_t dend = dbase + totals[d0];
  const RsLanes RL = rs_lanes(sg);
  for (XcdWalk wk(nt); wk.t < wk.end; wk.t += wk.step) {
    const uint32_t tile = wk.t;
    const RsTile T = rs_tile(sg, RL, n, nt, TILE, tile);
    const uint64_t base = T.base;
    const uint32_t tn = T.tn;
    // wavefront w holds the tile's elements [w * ITEMS * 64, (w + 1) * ITEMS * 64)
    // as ITEMS rows of 64, all loaded before the first barrier
    const uint32_t wfirst = (uint32_t)w * (kWave * ITEMS);
    uint64_t tkey[ITEMS];
    uint32_t tval[ITEMS], trank[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
      const uint32_t li = wfirst + (uint32_t)it * kWave + lane;
      tkey[it] = li < tn ? keys_in[base + li] : 0ull;
      tval[it] = li < tn ? (vals_in ? vals_in[base + li] : (uint32_t)(base + li)) : 0u;  // null: value = position
    }
    // tile-local digit counts follow from the row-scanned table: the next
    // entry of the digit's row is the successor of (digit, tile)
    const size_t at = (size_t)d0 * nt + tile;
    uint32_t here, next;
    if (sg.blk) {
      // the block's count of each digit (row entries at its first tile and
      // after its last), their exclusive scan over the digits, and the
      // digit's count in the block's earlier tiles
      const uint32_t tb0 = T.tb0, tb1 = T.tb1;
      const uint32_t c0 = offsets[(size_t)d0 * nt + tb0];
      const uint32_t c1 = tb1 < nt ? offsets[(size_t)d0 * nt + tb1] : totals[d0];
      const uint32_t cb = c1 - c0;
      uint32_t bi = cb;
      for (int dd = 1; dd < kWave; dd <<= 1) {
        const uint32_t t = __shfl_up(bi, dd);
        if (lane >= dd) bi += t;
      }
      if (lane == kWave - 1) bsum[w] = bi;
      __syncthreads();
      uint32_t bb = T.base - (tile - tb0) * TILE + bi - cb;  // block start + digits before
      for (int k = 0; k < w; k++) bb += bsum[k];
      here = bb + offsets[at] - c0;
      next = bb + (tile + 1 < tb1 ? offsets[at + 1] - c0 : cb);
    } else {
      here = dbase + offsets[at];
      next = tile == nt - 1 ? dend : dbase + offsets[at + 1];
    }
    const uint32_t cnt = next - here;
    gbase[d0] = here;
    // exclusive scan of the 256 counts (one per thread)
    uint32_t incl = cnt;
    for (int dd = 1; dd < kWave; dd <<= 1) {
      const uint32_t t = __shfl_up(incl, dd);
      if (lane >= dd) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    for (int k = 0; k < kRsThreads / kWave; k++) wcnt[k][d0] = 0;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; k++) before += wsum[k];
    const uint32_t lfirst = before + incl - cnt;
    lstart[d0] = lfirst;
    // stable rank of each element among its wavefront's elements of the same
    // digit; only this wavefront touches its counter row, so the rows need no
    // barrier between them
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
      const bool valid = wfirst + (uint32_t)it * kWave + lane < tn;
      const uint32_t d = valid ? (uint32_t)(tkey[it] >> shift) & 255u : 0u;
      const uint64_t peers = match_any8(d, ballot64(valid));
      const uint32_t seen = valid ? wcnt[w][d] : 0u;
      trank[it] = seen + (uint32_t)__popcll(peers & lt);
      if (valid && (peers & lt) == 0) wcnt[w][d] = seen + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // a wavefront's run of digit d starts after the tile's earlier digits and
    // after the earlier wavefronts' elements of digit d
    {
      uint32_t acc = lfirst;
      for (int k = 0; k < kRsThreads / kWave; k++) {
        const uint32_t c = wcnt[k][d0];
        wcnt[k][d0] = acc;
        acc += c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; it++) {
      if (wfirst + (uint32_t)it * kWave + lane < tn) {
        const uint32_t pos = wcnt[w][(uint32_t)(tkey[it] >> shift) & 255u] + trank[it];
        skey[pos] = tkey[it];
        sval[pos] = tval[it];
      }
    }
    __syncthreads();
    // each digit's run is contiguous in LDS and in the output
    for (uint32_t i = threadIdx.x; i < tn; i += kRsThreads) {
      const uint64_t key = skey[i];
      const uint32_t d = (uint32_t)(key >> shift) & 255u;
      const uint32_t gp = gbase[d] + (i - lstart[d]);
      keys_out[gp] = key;
      vals_out[gp] = sval[i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- doubling steps
__device__ __forceinline__ uint32_t block_of(const uint32_t *blk_start, uint32_t nb, uint32_t g) {
  return upper_index(blk_start, nb, g);
}

__global__ void k_iota(uint32_t *v, const uint32_t *d_n, uint32_t n_max) {
  const uint32_t n = dev_n(d_n, n_max);
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) v[k] = k;
}

// key = (block, the first `nbytes` bytes of the rotation, cyclic), the block
// in the bits above 8 * nbytes.  A thread builds 8 consecutive keys: when
// their windows stay inside one block they come from one 16-byte load
// (byte-reversed, then shifted per key), else position by position.  A
// wavefront's 512 keys are staged in LDS and stored in 1 KB runs (a thread's
// own 64 bytes would be four 16-byte stores 64 bytes apart across the lanes).
__device__ __forceinline__ uint64_t bwt_init_one(const uint8_t *rle, const uint32_t *blk_start, uint32_t nb,
                                                 int nbytes, uint32_t g) {
  const uint32_t k = block_of(blk_start, nb, g);
  const uint32_t s = blk_start[k], m = blk_start[k + 1] - s, i = g - s;
  uint64_t v = 0;
  uint32_t j = i;
  for (int t = 0; t < nbytes; t++) {
    v = (v << 8) | rle[s + j];
    j = j + 1 == m ? 0u : j + 1;
  }
  return ((uint64_t)k << (8 * nbytes)) | v;
}

constexpr int kInitThreads = 256;
constexpr uint32_t kInitStride = 9;  // LDS words of 8 bytes per lane (8 keys and a pad against bank conflicts)

__global__ __launch_bounds__(kInitThreads) void k_bwt_init(const uint8_t *rle, const uint32_t *d_N,
                                                           const uint32_t *blk_start, const uint32_t *d_nb,
                                                           int nbytes, uint64_t *keys, uint32_t *d_u) {
  __shared__ uint64_t stage[kInitThreads / kWave][kWave * kInitStride];
  const uint32_t N = *d_N, nb = *d_nb;
  if (blockIdx.x == 0 && threadIdx.x == 0) *d_u = N;
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  uint64_t *st = stage[wv];
  // the block table in one register per lane when it fits a wavefront
  const bool lane_tab = nb < (uint32_t)kWave;
  const uint32_t bs = lane_tab && (uint32_t)lane <= nb ? blk_start[lane] : 0u;
  const int kbits = 8 * nbytes;  // nbytes <= 7
  const uint32_t waves = gridDim.x * (kInitThreads / kWave);
  // every lane of a wavefront takes every step (the stores are shared)
  for (uint64_t wbase = (uint64_t)(blockIdx.x * (kInitThreads / kWave) + wv) * 512; wbase < N;
       wbase += (uint64_t)waves * 512) {
    const uint32_t g0 = (uint32_t)wbase + 8u * (uint32_t)lane;
    uint64_t kk[8];
    if (g0 < N) {
      uint32_t k = 0;
      if (lane_tab) {
        for (uint32_t j = 1; j < nb; j++) k += g0 >= (uint32_t)__builtin_amdgcn_readlane((int)bs, (int)j) ? 1u : 0u;
      } else {
        k = block_of(blk_start, nb, g0);
      }
      const uint32_t e = blk_start[k + 1];
      // bytes g0 .. g0 + 7 + nbytes - 1 all inside block k (no wrap); the 16
      // loaded bytes end below N + 8, inside the buffer's padding
      if ((uint64_t)g0 + 8 <= N && (uint64_t)g0 + 7 + (uint32_t)nbytes <= e) {
        const uint64_t hi = __builtin_bswap64(*(const uint64_t *)(rle + g0));
        const uint64_t lo = __builtin_bswap64(*(const uint64_t *)(rle + g0 + 8));
        const uint64_t top = (uint64_t)k << kbits;
#pragma unroll
        for (int o = 0; o < 8; o++) {
          const uint64_t w64 = o == 0 ? hi : (hi << (8 * o)) | (lo >> (64 - 8 * o));  // bytes g0 + o .. g0 + o + 7
          kk[o] = top | (w64 >> (64 - kbits));
        }
      } else {
#pragma unroll
        for (int o = 0; o < 8; o++) kk[o] = g0 + o < N ? bwt_init_one(rle, blk_start, nb, nbytes, g0 + o) : 0ull;
      }
    }
#pragma unroll
    for (int o = 0; o < 8; o++) st[lane * kInitStride + o] = kk[o];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // store q: keys 2 (64 q + lane) and the one after, of lane (64 q + lane) / 4
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const uint32_t kx = 2u * (64u * (uint32_t)q + (uint32_t)lane);
      const uint32_t at = (kx >> 3) * kInitStride + (kx & 7u);
      const uint64_t a = st[at], b2 = st[at + 1];
      const uint64_t gk = wbase + kx;
      if (gk + 2 <= N) {
        *(uint4 *)(keys + gk) = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b2, (uint32_t)(b2 >> 32));
      } else if (gk < N) {
        keys[gk] = a;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

constexpr int kSegThreads = 1024;
constexpr uint32_t kSegCap = 8192;                     // elements staged per workgroup
constexpr uint32_t kSegTile = 4096;                    // positions whose group starts a workgroup owns
constexpr uint32_t kSegMaxGroup = kSegCap - kSegTile;  // largest group the in-tile sort takes

// ---------------------------------------------------------------- one doubling round
// A round turns the sorted list into ranks in two launches over tiles of
// 4096 elements (256 threads x 16):
//   k_rnd_marks    per-tile maximum of the group-start marks (a group start
//                  is marked with its slot, other elements with 0) and
//                  per-tile count of the elements that stay unresolved (both
//                  follow from the keys and slots alone);
//   k_rnd_update   max-scan of the marks (each element's rank = its group's
//                  first slot), rank and suffix-array writes, and the
//                  compaction of the unresolved elements (exclusive scan of
//                  the counts).
// Each scan takes its carry by reducing the tile aggregates in front of its
// tile itself (no look-back: see the tile-scan helpers).
constexpr int kRThreads = kTThreads;
constexpr int kRItems = kTItems;
constexpr uint32_t kRTile = kTTile;

// 16 consecutive 32- or 64-bit values from k0 (vector loads when all are in
// range)
__device__ __forceinline__ void load16(const uint32_t *a, uint32_t k0, uint32_t n, uint32_t *v) {
  if (k0 + kTItems <= n) {
    const uint4 *q = (const uint4 *)(a + k0);
#pragma unroll
    for (int j = 0; j < kTItems / 4; j++) {
      const uint4 t = q[j];
      v[4 * j] = t.x;
      v[4 * j + 1] = t.y;
      v[4 * j + 2] = t.z;
      v[4 * j + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kTItems; i++) v[i] = k0 + i < n ? a[k0 + i] : 0u;
  }
}
__device__ __forceinline__ void load16(const uint64_t *a, uint32_t k0, uint32_t n, uint64_t *v) {
  if (k0 + kTItems <= n) {
    const uint4 *q = (const uint4 *)(a + k0);
#pragma unroll
    for (int j = 0; j < kTItems / 2; j++) {
      const uint4 t = q[j];
      v[2 * j] = ((uint64_t)t.y << 32) | t.x;
      v[2 * j + 1] = ((uint64_t)t.w << 32) | t.z;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kTItems; i++) v[i] = k0 + i < n ? a[k0 + i] : 0ull;
  }
}
// slots of 16 consecutive list elements; a null list means slot = position
__device__ __forceinline__ void load_slots(const uint32_t *slot, uint32_t k0, uint32_t n, uint32_t *v) {
  if (slot) {
    load16(slot, k0, n, v);
  } else {
#pragma unroll
    for (int i = 0; i < kTItems; i++) v[i] = k0 + i;
  }
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src), hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Group boundaries around a thread's 16 consecutive list elements: bit i of
// the result is set where element i starts a group (its key differs from the
// one before); *ends: the last element's key differs from the next one.
__device__ __forceinline__ uint32_t group_starts(const uint64_t *keys, uint32_t k0, uint32_t U, int lane,
                                                 const uint64_t *key, bool &ends) {
  uint64_t before = shfl64(key[kRItems - 1], lane - 1), after = shfl64(key[0], lane + 1);
  if (lane == 0) before = k0 > 0 && k0 - 1 < U ? keys[k0 - 1] : 0ull;
  if (lane == kWave - 1) after = k0 + kRItems < U ? keys[k0 + kRItems] : 0ull;
  uint32_t diff = 0;
#pragma unroll
  for (int i = 0; i < kRItems; i++) {
    const uint64_t pk = i == 0 ? before : key[i - 1];
    if (k0 + i == 0 || key[i] != pk) diff |= 1u << i;
  }
  ends = k0 + kRItems >= U || after != key[kRItems - 1];
  return diff;
}

// The elements that leave the list this round (bit i for element k0 + i):
// groups of one, and every element of a block whose rotations are compared
// in full.  A slot lies in its rotation's block (the suffix-array slots of a
// block are the block's own range of positions).  Bit i + 16: element i ends
// its group.
__device__ __forceinline__ uint32_t resolved(uint32_t diff, bool ends, const uint32_t *sl, uint32_t k0, uint32_t U,
                                             bool any_short, const uint32_t *blk_start, uint32_t nb,
                                             uint32_t compared) {
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < kRItems; i++) {
    const uint32_t k = k0 + i;
    if (k >= U) continue;
    const bool last = k + 1 == U || (i + 1 < kRItems ? ((diff >> (i + 1)) & 1u) != 0 : ends);
    bool done = ((diff >> i) & 1u) && last;
    if (!done && any_short) {
      const uint32_t b = block_of(blk_start, nb, sl[i]);
      done = blk_start[b + 1] - blk_start[b] <= compared;
    }
    m |= (done ? 1u : 0u) << i;
    m |= (last ? 1u : 0u) << (i + 16);
  }
  return m;
}

__global__ __launch_bounds__(kRThreads) void k_rnd_marks(const uint64_t *keys, const uint32_t *slot,
                                                         const uint32_t *d_u, const uint32_t *blk_start,
                                                         const uint32_t *d_nb, const uint32_t *d_min_m,
                                                         uint32_t compared, uint32_t *aggs_m, uint32_t *aggs_s,
                                                         uint32_t *d_maxg) {
  __shared__ uint32_t sh[kRThreads / kWave];
  const uint32_t U = *d_u, nb = *d_nb;
  const uint32_t nt = (U + kRTile - 1) / kRTile;
  const bool any_short = compared >= *d_min_m;  // else no block is fully compared yet
  const int lane = lane_id();
  if (blockIdx.x == 0 && threadIdx.x == 0) *d_maxg = 0;
  for (XcdWalk wk(nt); wk.t < wk.end; wk.t += wk.step) {
    const uint32_t tile = wk.t;
    const uint32_t k0 = tile * kRTile + threadIdx.x * kRItems;
    uint64_t key[kRItems];
    uint32_t sl[kRItems];
    load16(keys, k0, U, key);
    load_slots(slot, k0, U, sl);
    bool ends;
    const uint32_t diff = group_starts(keys, k0, U, lane, key, ends);
    // slots grow along the list: the last group start of the thread has the largest mark
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kRItems; i++)
      if (k0 + i < U && ((diff >> i) & 1u)) m = sl[i];
    const uint32_t res = resolved(diff, ends, sl, k0, U, any_short, blk_start, nb, compared);
    const uint32_t valid = k0 >= U ? 0u : k0 + kRItems <= U ? 0xFFFFu : (1u << (U - k0)) - 1u;
    const uint32_t cnt = (uint32_t)__popc(valid & ~res & 0xFFFFu);
    m = block_reduce<true>(m, sh);
    const uint32_t c = block_reduce<false>(cnt, sh);
    if (threadIdx.x == 0) {
      aggs_m[tile] = m;
      aggs_s[tile] = c;
    }
  }
}

// Ranks, suffix-array entries of the elements now resolved, and the list of
// the unresolved ones moved to the front (their order kept) with the compact
// position of each one's group start; writes the new count.  Also the
// largest group that stays unresolved (its last element knows the size:
// slots of a group are consecutive and its rank is the first slot), and the
// in-group sort's tile boundaries: the last element of each unresolved group
// sets bound[t] = the first group start at or after t * kSegTile, which for
// every t * kSegTile inside (group start, group end] is this group's end.
// A thread owns 16 consecutive elements (vector loads); keys next to them
// come from the neighbouring lanes.  The compact list is staged per
// wavefront in LDS and stored in runs of consecutive positions.  From the
// second round on, bits old_bits and up of a key hold the rank the key was
// built from, which rank[] still holds: the random rank write is skipped
// where the new rank equals it (the first part of every group that splits).
__global__ __launch_bounds__(kRThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_rnd_update(
    const uint64_t *keys, const uint32_t *vals, const uint32_t *slot, const uint32_t *d_u, const uint32_t *aggs_m,
    const uint32_t *aggs_s, const uint32_t *blk_start, const uint32_t *d_nb, const uint32_t *d_min_m,
    uint32_t compared, int old_bits, uint32_t *rank, uint32_t *sa, uint32_t *vals2, uint32_t *slot2,
    uint32_t *gstart2, uint32_t *bound, uint32_t *d_unew, uint32_t *d_maxg) {
  __shared__ uint32_t buf[kRTile + kRTile / 32];
  __shared__ uint32_t oldr[kRTile + kRTile / 32];
  __shared__ uint32_t sh[kRThreads / kWave];
  __shared__ uint32_t shw[kRThreads / kWave];
  const uint32_t U = *d_u, nb = *d_nb;
  const uint32_t nt = (U + kRTile - 1) / kRTile;
  const bool any_short = compared >= *d_min_m;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bound[0] = 0;
    if (nt == 0) *d_unew = 0;
  }
  uint32_t carry = 0, counted = 0, ccarry = 0, ccounted = 0, gmax = 0;
  for (XcdWalk wk(nt); wk.t < wk.end; wk.t += wk.step) {
    const uint32_t tile = wk.t;
    const uint32_t base = tile * kRTile;
    const uint32_t k0 = base + threadIdx.x * kRItems;
    uint32_t sl[kRItems], g[kRItems], diff;
    bool ends;
    {
      uint64_t key[kRItems];
      load16(keys, k0, U, key);
      diff = group_starts(keys, k0, U, lane, key, ends);
      // the rank each key was built from, kept in LDS (registers are the
      // limit on this kernel's occupancy)
#pragma unroll
      for (int i = 0; i < kRItems; i++)
        oldr[tpad(threadIdx.x * kRItems + i)] = old_bits ? (uint32_t)(key[i] >> old_bits) : 0xFFFFFFFFu;
    }
    load_slots(slot, k0, U, sl);
    load16(vals, k0, U, g);
    carry = tile_carry<true>(aggs_m, counted, tile, carry, sh);
    ccarry = tile_carry<false>(aggs_s, ccounted, tile, ccarry, sh);
#pragma unroll
    for (int i = 0; i < kRItems; i++)
      buf[tpad(threadIdx.x * kRItems + i)] = k0 + i < U && ((diff >> i) & 1u) ? sl[i] : 0u;
    __syncthreads();
    tile_scan<true, true>(buf, carry, sh);
    const uint32_t res = resolved(diff, ends, sl, k0, U, any_short, blk_start, nb, compared);
    const uint32_t valid = k0 >= U ? 0u : k0 + kRItems <= U ? 0xFFFFu : (1u << (U - k0)) - 1u;
    const uint32_t unres = valid & ~res & 0xFFFFu;
    uint32_t off[kRItems];
#pragma unroll
    for (int i = 0; i < kRItems; i++) {
      const uint32_t k = k0 + i;
      off[i] = 0;
      if (k >= U) continue;
      const uint32_t nr = buf[tpad(threadIdx.x * kRItems + i)];
      if (nr != oldr[tpad(threadIdx.x * kRItems + i)]) rank[g[i]] = nr;  // rank[g] already holds the rank the key was built from
      if ((res >> i) & 1u) sa[sl[i]] = g[i];  // final position; unresolved ones are written in a later round
      off[i] = sl[i] - nr;
      if (((unres >> i) & 1u) && ((res >> (i + 16)) & 1u)) gmax = max(gmax, off[i] + 1u);
    }
    // compact positions: the tile's carry, the waves before, the lanes before
    const uint32_t cnt = (uint32_t)__popc(unres);
    uint32_t x = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)x, d);
      if (lane >= d) x += o;
    }
    const uint32_t lane_before = x - cnt, wave_total = (uint32_t)__shfl((int)x, kWave - 1);
    if (lane == 0) shw[wave] = wave_total;
    __syncthreads();
    uint32_t wave_before = 0, tile_total = 0;
    for (int w = 0; w < kRThreads / kWave; w++) {
      wave_before += w < wave ? shw[w] : 0u;
      tile_total += shw[w];
    }
    const uint32_t q_wave = ccarry + wave_before;
    if (tile == nt - 1 && threadIdx.x == 0) *d_unew = ccarry + tile_total;
    // each wavefront stages its elements in its own quarter of buf (it read
    // its ranks from there already), then stores runs of 64
    uint32_t *stage = buf + tpad((uint32_t)wave * (kRTile / (kRThreads / kWave)));
#pragma unroll
    for (int a = 0; a < 3; a++) {
      uint32_t j = lane_before;
#pragma unroll
      for (int i = 0; i < kRItems; i++) {
        if (!((unres >> i) & 1u)) continue;
        const uint32_t q = q_wave + j;
        stage[tpad(j)] = a == 0 ? g[i] : a == 1 ? sl[i] : q - off[i];
        if (a == 2 && ((res >> (i + 16)) & 1u)) {  // last of its group
          const uint32_t head = q - off[i], end = q + 1u;
          for (uint32_t t = head / kSegTile + 1; (uint64_t)t * kSegTile <= end; t++) bound[t] = end;
        }
        j++;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      uint32_t *dst = a == 0 ? vals2 : a == 1 ? slot2 : gstart2;
      for (uint32_t r = (uint32_t)lane; r < wave_total; r += kWave) dst[q_wave + r] = stage[tpad(r)];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  gmax = block_reduce<true>(gmax, sh);
  if (threadIdx.x == 0 && gmax) atomicMax(d_maxg, gmax);
}

__global__ void k_bwt_keys(const uint32_t *vals, const uint32_t *d_u, const uint32_t *rank, const uint32_t *blk_start,
                           const uint32_t *d_nb, uint32_t h, int bits, uint64_t *keys) {
  const uint32_t U = *d_u, nb = *d_nb;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < U; k += gridDim.x * blockDim.x) {
    const uint32_t g = vals[k];
    const uint32_t b = block_of(blk_start, nb, g);
    const uint32_t s = blk_start[b], m = blk_start[b + 1] - s;
    const uint32_t g2 = s + (uint32_t)(((uint64_t)(g - s) + h) % m);
    keys[k] = ((uint64_t)rank[g] << bits) | rank[g2];
  }
}

// ---------------------------------------------------------------- in-group sort

// sorting network for 8 values in registers (19 compare-exchanges)
__device__ __forceinline__ void cx(uint64_t &a, uint64_t &b) {
  const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}
__device__ __forceinline__ void sort8(uint64_t *v) {
  cx(v[0], v[2]); cx(v[1], v[3]); cx(v[4], v[6]); cx(v[5], v[7]);
  cx(v[0], v[4]); cx(v[1], v[5]); cx(v[2], v[6]); cx(v[3], v[7]);
  cx(v[0], v[1]); cx(v[2], v[3]); cx(v[4], v[5]); cx(v[6], v[7]);
  cx(v[2], v[4]); cx(v[3], v[5]);
  cx(v[1], v[4]); cx(v[3], v[6]);
  cx(v[1], v[2]); cx(v[3], v[4]); cx(v[5], v[6]);
}

// The rotation h positions after g, inside g's block [s, s + m); h < m for
// every rotation that is still unresolved (a block is final once h >= m).
__device__ __forceinline__ uint32_t rot_ahead(uint32_t g, uint32_t s, uint32_t m, uint32_t h) {
  uint32_t t = (g - s) + h;
  if (t >= m) t -= m;
  if (t >= m) t %= m;  // only for an invalid list
  return s + t;
}

// Sorts every unresolved group by the rank h positions further on, stably.
// Input: the unresolved list (vals = rotation, slot = its position in the
// suffix array, gstart = position of its group's first element), ordered by
// group; rank[] holds each rotation's group rank.
// Output: vals_out in the new order and keys_out = (rank << rbits) | rank2,
// the keys the radix path would have sorted.  A group above kSegMaxGroup
// sets *d_fail and its workgroup copies its range unsorted (the result of
// the call is then invalid, every index stays in range).
//
// In LDS each element is the composite (group start, rank2, position): the
// range is already ordered by group start, so sorting the composites sorts
// each group and keeps equal ranks in position order.  Each thread sorts 8
// consecutive composites in registers, then sorted runs are merged pairwise
// (8 -> 16 -> ... -> 8192) along merge paths: a thread finds where its 8
// outputs start with one binary search on its diagonal and merges them
// sequentially.  A level is skipped when no group crosses the middle of a
// window of that level (its merge would move nothing).
// one tile of the in-group sort (every exit is uniform over the workgroup)
__device__ __forceinline__ void seg_sort_tile(uint32_t tile, uint32_t U, uint32_t nb, const uint32_t *vals,
                                              const uint32_t *slot, const uint32_t *gstart, const uint32_t *rank,
                                              const uint32_t *bound, const uint32_t *blk_start, uint32_t h, int rbits,
                                              uint32_t *vals_out, uint64_t *keys_out, uint32_t *d_fail,
                                              uint64_t *scomp, uint16_t *sgs) {
  constexpr int kPer = (int)(kSegCap / kSegThreads);  // 8 consecutive elements per thread
  constexpr int kLevels = 10;                         // runs of 8 << i, i < 10
  const uint64_t t0 = (uint64_t)tile * kSegTile;
  if (t0 >= U) return;
  const uint32_t R0 = min(bound[tile], U);
  const uint32_t R1 = t0 + kSegTile >= U ? U : min(bound[tile + 1], U);
  if (R1 <= R0) return;  // a group from an earlier tile covers this one
  const uint32_t len = R1 - R0;
  if (len > kSegCap) {
    if (threadIdx.x == 0) *d_fail = 1u;
    for (uint32_t k = R0 + threadIdx.x; k < R1; k += kSegThreads) {
      vals_out[k] = vals[k];
      keys_out[k] = 0;
    }
    return;
  }
  const int w = threadIdx.x / kWave, lane = lane_id();
  // the block table in one register per lane when it fits a wavefront
  const bool lane_tab = nb < (uint32_t)kWave;
  const uint32_t bs = lane_tab && (uint32_t)lane <= nb ? blk_start[lane] : 0u;
  // coalesced loads: element x = threadIdx.x + i * kSegThreads
#pragma unroll
  for (int i = 0; i < kPer; i++) {
    const uint32_t x = threadIdx.x + (uint32_t)i * kSegThreads;
    const bool in = x < len;
    const uint32_t k = R0 + (in ? x : 0u);
    const uint32_t g = vals[k];
    const uint32_t gh = gstart[k];
    const uint32_t gsx = gh >= R0 && gh - R0 <= x ? gh - R0 : 0u;
    uint32_t s0, s1;
    if (lane_tab) {
      uint32_t b = 0;
      for (uint32_t j = 1; j < nb; j++) b += g >= (uint32_t)__builtin_amdgcn_readlane((int)bs, (int)j) ? 1u : 0u;
      s0 = (uint32_t)__shfl((int)bs, (int)b);
      s1 = (uint32_t)__shfl((int)bs, (int)b + 1);
    } else {
      const uint32_t b = block_of(blk_start, nb, g);
      s0 = blk_start[b];
      s1 = blk_start[b + 1];
    }
    const uint32_t k2 = rank[rot_ahead(g, s0, s1 - s0, h)];
    scomp[x] = in ? ((uint64_t)gsx << 45) | ((uint64_t)k2 << 13) | x : ~0ull;  // padding sorts last
    sgs[x] = (uint16_t)(in ? gsx : 0u);
  }
  __syncthreads();
  // from here on a thread owns the 8 consecutive elements x0 .. x0 + 7
  const uint32_t x0 = threadIdx.x * kPer;
  uint64_t v[kPer];
  uint32_t gs[kPer];
#pragma unroll
  for (int i = 0; i < kPer; i++) {
    v[i] = scomp[x0 + i];
    gs[i] = sgs[x0 + i];
  }
  // the last element of each group records the group's end at its start
  bool last[kPer];
#pragma unroll
  for (int i = 0; i < kPer; i++) {
    const uint32_t x = x0 + i;
    last[i] = x < len && (x + 1 == len || sgs[x + 1] == x + 1);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kPer; i++)
    if (last[i]) sgs[gs[i]] = (uint16_t)(x0 + i + 1);
  __syncthreads();
  // Level l (runs of L = 8 << l) can move something only if a group holds a
  // multiple of L strictly inside, which needs L <= the highest bit where
  // its first and last positions differ.
  uint32_t levels = 0;
#pragma unroll
  for (int i = 0; i < kPer; i++) {
    const uint32_t x = x0 + i;
    if (x < len && x == gs[i]) {
      const uint32_t diff = x ^ (sgs[x] - 1u);
      const int hb = diff ? 31 - __builtin_clz(diff) : -1;
      if (hb >= 3) levels |= (2u << min(hb - 3, kLevels - 1)) - 1u;
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) levels |= (uint32_t)__shfl_xor((int)levels, d);
  // scratch words in scomp: this thread's composites are in registers
  uint32_t *red = (uint32_t *)scomp;
  __syncthreads();
  if (lane == 0) red[w] = levels;
  __syncthreads();
  levels = 0;
  for (int i = 0; i < kSegThreads / kWave; i++) levels |= red[i];
  __syncthreads();
  sort8(v);
#pragma unroll
  for (int i = 0; i < kPer; i++) scomp[x0 + i] = v[i];
  __syncthreads();
  // sgs now maps positions to groups: sgs[p] is p's group start, except at a
  // group start, where it holds the group end (> p)
  for (int l = 0; l < kLevels; l++) {
    if (!((levels >> l) & 1u)) continue;
    const uint32_t L = 8u << l;
    const uint32_t d = x0 & (2 * L - 1);  // diagonal of this thread inside its window
    const uint32_t W = x0 - d;
    // only the group holding the window's middle can cross it; threads whose
    // outputs miss that group keep their elements
    const uint32_t mid = W + L;
    bool work = false;
    if (mid < len) {
      const uint32_t sm = sgs[mid];
      if (sm < mid) work = x0 < sgs[sm] && x0 + kPer > sm;
    }
    uint64_t o[kPer];
    if (work) {
      const uint64_t *A = scomp + W, *B = scomp + W + L;
      uint32_t lo = d > L ? d - L : 0u, hi = d < L ? d : L;
      while (lo < hi) {  // A elements among the window's first d outputs (A first on ties)
        const uint32_t m = (lo + hi) >> 1;
        if (A[m] <= B[d - 1 - m]) lo = m + 1;
        else hi = m;
      }
      uint32_t ia = lo, ib = d - lo;
      uint64_t a = ia < L ? A[ia] : ~0ull, b = ib < L ? B[ib] : ~0ull;
#pragma unroll
      for (int i = 0; i < kPer; i++) {
        // an exhausted run reads as all ones; ties with padding give the same value
        const bool take_a = a <= b;
        o[i] = take_a ? a : b;
        const uint32_t na = ia + (take_a ? 1u : 0u), nb = ib + (take_a ? 0u : 1u);
        const uint32_t at = take_a ? na : L + nb;
        const bool in = take_a ? na < L : nb < L;
        const uint64_t nx = scomp[W + (in ? at : 0u)];
        ia = na;
        ib = nb;
        if (take_a) a = in ? nx : ~0ull;
        else b = in ? nx : ~0ull;
      }
    }
    __syncthreads();
    if (work) {
#pragma unroll
      for (int i = 0; i < kPer; i++) scomp[x0 + i] = o[i];
    }
    __syncthreads();
  }
  // sorted position p holds the composite of the element that goes there
  for (uint32_t p = threadIdx.x; p < len; p += kSegThreads) {
    const uint64_t c = scomp[p];
    const uint32_t x = (uint32_t)c & (kSegCap - 1);
    const uint32_t gsp = (uint32_t)(c >> 45);
    const uint32_t k2 = (uint32_t)(c >> 13);
    vals_out[R0 + p] = vals[R0 + x];
    keys_out[R0 + p] = ((uint64_t)slot[R0 + gsp] << rbits) | k2;
  }
}

// The tiles come from an XCD-aware walk over a capped grid, so a round with
// few unresolved rotations (or none: a round of a fixed schedule past the
// data's need) costs a few workgroups, not one per tile of the bound.
constexpr uint32_t kSegGridCap = 512;  // two workgroups of 80 KB LDS per CU

__global__ __launch_bounds__(kSegThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_seg_sort(
    const uint32_t *vals, const uint32_t *slot, const uint32_t *gstart, const uint32_t *rank, const uint32_t *d_u,
    const uint32_t *bound,
    const uint32_t *blk_start, const uint32_t *d_nb, uint32_t h, int rbits, uint32_t *vals_out, uint64_t *keys_out,
    uint32_t *d_fail) {
  __shared__ uint64_t scomp[kSegCap];  // composites, in runs sorted so far
  __shared__ uint16_t sgs[kSegCap];    // group starts, then group ends at each start
  const uint32_t U = *d_u, nb = *d_nb;
  const uint32_t nt = (U + kSegTile - 1) / kSegTile;
  for (XcdWalk wk(nt); wk.t < wk.end; wk.t += wk.step) {
    seg_sort_tile(wk.t, U, nb, vals, slot, gstart, rank, bound, blk_start, h, rbits, vals_out, keys_out, d_fail,
                  scomp, sgs);
    __syncthreads();  // the next tile reuses the LDS
  }
}

__global__ void k_bwt_left(const uint32_t *d_u, const uint32_t *d_fail, uint32_t *d_left) {
  *d_left = *d_u + *d_fail;
}

__global__ void k_min_block(const uint32_t *blk_start, const uint32_t *d_nb, uint32_t *d_min_m) {
  __shared__ uint32_t red[256];
  const uint32_t nb = *d_nb;
  uint32_t mn = 0xFFFFFFFFu;
  for (uint32_t b = threadIdx.x; b < nb; b += 256) mn = min(mn, blk_start[b + 1] - blk_start[b]);
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *d_min_m = red[0];
}

// L[j] = the byte before rotation sa[j] (cyclic in its block); the slot of
// each block's rotation 0 is its orig_ptr.  Tiles of 4096 positions, 16
// consecutive per thread: one vector load of sa, the block from the tile's
// block table, 16 independent byte gathers in flight, one 16-byte store.
__global__ __launch_bounds__(kTThreads) void k_bwt_emit(const uint32_t *sa, const uint8_t *rle, const uint32_t *d_N,
                                                        const uint32_t *blk_start, const uint32_t *d_nb, uint8_t *L,
                                                        BlockCode *codes) {
  const uint32_t N = *d_N, nb = *d_nb;
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  for (XcdWalk wk(nt); wk.t < wk.end; wk.t += wk.step) {
    const uint32_t tile = wk.t;
    const TileBlocks tb(blk_start, nb, tile * kTTile);
    const uint32_t j0 = tile * kTTile + threadIdx.x * kTItems;
    uint32_t g[kTItems], src[kTItems];
    load16(sa, j0, N, g);
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t j = j0 + i;
      src[i] = 0;
      if (j < N) {
        uint32_t s, e;
        const uint32_t b = tb.find(j, s, e);
        // a slot left unresolved by a capped round budget (the call is then
        // redone) may hold any value: keep the read inside the block
        const uint32_t gi = g[i] >= s && g[i] < e ? g[i] : s;
        src[i] = gi == s ? e - 1 : gi - 1;
        if (g[i] == s) codes[b].orig_ptr = j - s;
      }
    }
    uint32_t c[kTItems];
#pragma unroll
    for (int i = 0; i < kTItems; i++) c[i] = j0 + i < N ? rle[src[i]] : 0u;
    if (j0 + kTItems <= N) {
      uint32_t wv[4];
#pragma unroll
      for (int q = 0; q < 4; q++)
        wv[q] = c[4 * q] | (c[4 * q + 1] << 8) | (c[4 * q + 2] << 16) | (c[4 * q + 3] << 24);
      *(uint4 *)(L + j0) = make_uint4(wv[0], wv[1], wv[2], wv[3]);
    } else {
#pragma unroll
      for (int i = 0; i < kTItems; i++)
        if (j0 + i < N) L[j0 + i] = (uint8_t)c[i];
    }
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
  if (g > kGridCap) g = kGridCap;
  return (uint32_t)g;
}

template <int ITEMS>
int radix_sort_t(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *d_n, uint32_t n_max, int bits, bool iota_vals,
                 const uint32_t *blk_start, const uint32_t *d_nb, uint32_t nb_max, uint32_t *counts,
                 uint32_t *d_count_n, hipStream_t s) {
  constexpr uint32_t TILE = kRsThreads * ITEMS;
  int cur = 0;
  if (n_max <= 1 || bits <= 0) {
    if (iota_vals) PCBZ_LAUNCH(k_iota, dim3(grid_for(n_max)), dim3(256), 0, s, vals[0], d_n, n_max);
    return cur;
  }
  // count table for at most ntiles tiles, then the digit totals, then the
  // blocks' first tiles (segmented)
  const uint32_t nseg = blk_start ? nb_max : 0u;
  const uint32_t ntiles = (n_max + TILE - 1) / TILE + nseg;
  uint32_t *totals = counts + (size_t)256 * (ntiles + 1);
  RsSeg sg{blk_start, blk_start ? totals + 256 : nullptr, d_nb};
  if (blk_start)
    PCBZ_LAUNCH(k_rs_tile_base, dim3(1), dim3(256), 0, s, blk_start, d_nb, TILE, (uint32_t *)sg.tile_base);
  const uint32_t grid = std::min<uint32_t>(ntiles, kGridCap);
  // algorithmic bytes of the scatter passes: each reads and writes every
  // 8-byte key and 4-byte value once (24 B per element a pass; the first
  // pass of a sort whose values are the positions reads none: 20 B), counted
  // at this point of the stream (later rounds reuse the count's slot)
  trace_bytes_count("k_rs_scatter<ITEMS>", 24ull * (uint64_t)((bits + 7) / 8) - (iota_vals ? 4u : 0u), d_n, s);
  for (int shift = 0; shift < bits; shift += 8) {
    PCBZ_LAUNCH(k_rs_hist<ITEMS>, dim3(grid), dim3(kRsThreads), 0, s, keys[cur], d_n, n_max, sg, shift, counts,
                d_count_n);
    PCBZ_LAUNCH(k_rs_rowscan<ITEMS>, dim3(256), dim3(kRsThreads), 0, s, counts, d_n, n_max, sg, totals);
    PCBZ_LAUNCH(k_rs_scatter<ITEMS>, dim3(grid), dim3(kRsThreads), 0, s, keys[cur],
                iota_vals && shift == 0 ? nullptr : vals[cur], keys[cur ^ 1],
                vals[cur ^ 1], d_n, n_max, sg, shift, counts, totals);
    cur ^= 1;
  }
  return cur;
}

}  // namespace

size_t seg_bound_words(uint32_t n_max) { return (size_t)n_max / kSegTile + 2; }

size_t rnd_aggs_words(uint32_t n_max) { return 2 * ((size_t)n_max / kRTile + 2); }

size_t radix_counts_words(uint32_t n_max, uint32_t nb_max) {
  // tiles of at least 2048 elements, one more per block when segmented;
  // the digit totals; the blocks' first tiles
  return (size_t)256 * ((n_max + 2047) / 2048 + nb_max + 1) + 256 + nb_max + 2;
}

// Sorts (keys[0], vals[0]) by the low `bits` bits of the key (n read from
// d_n); returns the buffer index holding the result.  With iota_vals the
// values are the positions 0..n-1 and vals[0] is not read.
int radix_sort(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *d_n, uint32_t n_max, int bits, int items,
               bool iota_vals, const uint32_t *blk_start, const uint32_t *d_nb, uint32_t nb_max, uint32_t *counts,
               uint32_t *d_count_n, hipStream_t s) {
  if (items <= 8)
    return radix_sort_t<8>(keys, vals, d_n, n_max, bits, iota_vals, blk_start, d_nb, nb_max, counts, d_count_n, s);
  return radix_sort_t<16>(keys, vals, d_n, n_max, bits, iota_vals, blk_start, d_nb, nb_max, counts, d_count_n, s);
}

// Prefix doubling over every block.  With `pinned_u` the unresolved count and
// the largest group are read back after each round (pinned_u[0..6] receive
// d_u[0..6]), the loop stops when nothing is left (at most max_rounds), and a
// round whose groups all fit kSegMaxGroup is sorted group by group; *seg_mask
// receives the rounds sorted that way (bit r - 1 for the sort after round r).
// Without it exactly max_rounds rounds are enqueued, the rounds in *seg_mask
// are sorted group by group (a group that does not fit sets the fail word),
// and the final unresolved count plus the fail word is left in *d_left.
// Returns the rounds enqueued.
int run_bwt(const uint8_t *rle, const uint32_t *d_N, uint32_t n_max, const uint32_t *d_nb, uint32_t nb_max,
            const uint32_t *blk_start, BwtWork w, uint32_t *sa, uint8_t *L, BlockCode *codes, int max_rounds,
            int items, uint32_t *pinned_u, uint64_t *seg_mask, uint32_t *d_left, hipStream_t s) {
  if (n_max == 0) return 0;
  uint64_t *keys[2] = {w.key[0], w.key[1]};
  uint32_t *vals[2] = {w.val[0], w.val[1]};
  uint32_t *slot = w.slot, *slot2 = w.slot2;
  uint32_t *du[2] = {w.d_u, w.d_u + 1};
  const uint32_t g = grid_for(n_max);
  const uint64_t mask_in = seg_mask ? *seg_mask : 0ull;
  uint64_t mask_out = 0;
  // first prefix: 7 bytes under an 8-bit block id, or 6 bytes under a 16-bit
  // one (noisy 16-bit data leaves most rotations tied after 4 bytes, far
  // fewer after 7)
  const int nbytes = nb_max <= 256 ? 7 : nb_max <= 65536 ? 6 : 4;
  PCBZ_LAUNCH(k_bwt_init, dim3(g), dim3(256), 0, s, rle, d_N, blk_start, d_nb, nbytes, keys[0], du[0]);
  PCBZ_LAUNCH(k_min_block, dim3(1), dim3(256), 0, s, blk_start, d_nb, w.d_min_m);
  // the values are the rotations, i.e. the positions: the first pass makes them
  // sorted block by block (segmented), so the passes cover the bytes only
  int cur = radix_sort(keys, vals, du[0], n_max, 8 * nbytes, items, true, blk_start, d_nb, nb_max,
                       w.counts, w.d_count_n, s);
  const int rbits = bits_for(n_max - 1);
  const ptrdiff_t maxg_at = w.d_maxg - w.d_u;  // read back together with the counts
  int u = 0;  // which count slot holds the current unresolved count
  uint32_t compared = (uint32_t)nbytes;
  int rounds = 0;
  uint32_t n_cur = n_max;  // bound on the unresolved count (exact when read back)
  uint32_t maxg = 0xFFFFFFFFu;
  for (;;) {
    // new ranks (max-scan of group-start slots) and the compaction
    const uint32_t gt = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kGridCap, (n_cur + kRTile - 1) / kRTile));
    uint32_t *aggs_m = w.aggs, *aggs_s = w.aggs + rnd_aggs_words(n_max) / 2;
    // after the first sort, list position k is suffix-array slot k
    const uint32_t *slot_in = rounds == 0 ? nullptr : slot;
    PCBZ_LAUNCH(k_rnd_marks, dim3(gt), dim3(kRThreads), 0, s, keys[cur], slot_in, du[u], blk_start, d_nb, w.d_min_m,
                compared, aggs_m, aggs_s, w.d_maxg);
    PCBZ_LAUNCH(k_rnd_update, dim3(gt), dim3(kRThreads), 0, s, keys[cur], vals[cur], slot_in, du[u], aggs_m, aggs_s,
                blk_start, d_nb, w.d_min_m, compared, rounds == 0 ? 0 : rbits, w.rank, sa, vals[cur ^ 1], slot2,
                w.gstart, w.seg_bound, du[u ^ 1], w.d_maxg);
    u ^= 1;
    rounds++;
    if (pinned_u) {
      // a failed read-back ends the rounds; the caller's error check reports it
      if (hipMemcpyAsync(pinned_u, w.d_u, (size_t)(maxg_at + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        break;
      n_cur = pinned_u[u];
      maxg = pinned_u[maxg_at];
      if (getenv("PCBZ_DEBUG_BWT"))
        fprintf(stderr, "pcbz bwt: round %d compared=%u unresolved=%u largest group=%u\n", rounds, compared, n_cur,
                maxg);
      if (n_cur == 0) break;
    }
    if (rounds >= max_rounds || compared >= (1u << 30)) break;
    // the compact list is now in (vals[cur^1], slot2)
    cur ^= 1;
    uint32_t *t = slot;
    slot = slot2;
    slot2 = t;
    const bool seg = pinned_u ? maxg <= kSegMaxGroup : rounds <= 64 && ((mask_in >> (rounds - 1)) & 1ull);
    if (seg) {
      if (rounds <= 64) mask_out |= 1ull << (rounds - 1);
      const uint32_t gs = xcd_grid((uint32_t)std::max<uint64_t>(
          1, std::min<uint64_t>(kSegGridCap, (n_cur + kSegTile - 1) / kSegTile)));
      PCBZ_LAUNCH(k_seg_sort, dim3(gs), dim3(kSegThreads), 0, s, vals[cur], slot, w.gstart, w.rank, du[u], w.seg_bound,
                  blk_start, d_nb, compared, rbits, vals[cur ^ 1], keys[cur ^ 1], w.d_fail);
      cur ^= 1;
    } else {
      PCBZ_LAUNCH(k_bwt_keys, dim3(grid_for(n_cur)), dim3(256), 0, s, vals[cur], du[u], w.rank, blk_start, d_nb,
                  compared, rbits, keys[cur]);
      uint64_t *kk[2] = {keys[cur], keys[cur ^ 1]};
      uint32_t *vv[2] = {vals[cur], vals[cur ^ 1]};
      if (radix_sort(kk, vv, du[u], n_cur, 2 * rbits, items, false, nullptr, nullptr, 0, w.counts, w.d_count_n,
                     s) == 1)
        cur ^= 1;
    }
    compared *= 2;
  }
  if (d_left) PCBZ_LAUNCH(k_bwt_left, dim3(1), dim3(1), 0, s, du[u], w.d_fail, d_left);
  if (seg_mask && pinned_u) *seg_mask = mask_out;
  PCBZ_LAUNCH(k_bwt_emit, dim3(std::max<uint32_t>(1, std::min<uint32_t>(kGridCap, (n_max + kTTile - 1) / kTTile))),
              dim3(kTThreads), 0, s, sa, rle, d_N, blk_start, d_nb, L, codes);
  return rounds;
}

}  // namespace pcbz
