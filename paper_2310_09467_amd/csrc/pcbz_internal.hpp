// pcbz_internal.hpp -- shared declarations of the HIP library (device structs,
// wave64 helpers and the launchers each kernel file exports to the runtime).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stddef.h>
#include <stdint.h>

namespace pcbz {

constexpr int kWave = 64;
constexpr int kNumCand = 16;            // RASTER, VIEW, VIEW_DX, VIEW_DT, then the predictor family (ids 4..15)
constexpr int kNumBasic = 4;            // ids the rearrangement kernel writes (and the selector predicts)
constexpr uint32_t kNone16 = 0xFFFFu;   // "no byte" marker in 16-bit tables
constexpr int kMaxAlpha = 258;          // bzip2 alphabet bound (256 byte ranks + RUNA/RUNB... + EOB)
constexpr int kMaxGroups = 6;
constexpr int kMaxCodeLen = 17;
constexpr int kGroupSize = 50;          // symbols per selector group
constexpr uint32_t kPrefixWords = 6144; // 24 KB of header bits per block (bounded below)
constexpr uint32_t kMaxSelectors = 18002;  // ceil((899981 + 1) / 50) for the largest block, plus slack

// One band of one frame (whole lens rows).
struct BandDesc {
  const uint16_t *frame;  // frame base (H x W, row-major)
  const uint16_t *prev;   // previous frame of the stream or nullptr
  uint32_t W, pitch, Nt;  // width, lenslet pitch, lens columns
  uint32_t Rb;            // lens rows in this band
  uint32_t y0;            // first pixel row of the band
  uint32_t frame_id;      // index of the frame in the batch
  uint32_t band_in_frame;
  uint32_t cand_mask;     // candidates the judge scores
  uint32_t level;         // bzip2 level 1..9 (block limit 100000*level-19)
  uint32_t n;             // band bytes = 2*Rb*pitch*W
  uint64_t off;           // first byte of the band in the concatenated byte space
  uint32_t blk_slot;      // first block slot of this band
  uint32_t blk_slots;     // block slots reserved for this band
};

// Lens-row work item for the rearrangement kernel.
struct RowItem {
  uint32_t band;
  uint32_t s;  // lens row inside the band
};

// One (band, candidate) entropy-judgement task.
struct JudgeTask {
  uint32_t band;
  uint32_t cand;
  uint32_t n;         // bytes
  uint32_t seg_base;  // first 4096-byte segment of this task in the segment tables
  uint64_t x_off;     // offset of the candidate bytes in the candidate buffer
};

// A bzip2 block after the first run-length stage (dense list, device-built).
struct BlockDesc {
  uint32_t band;
  uint32_t frame_id;
  uint32_t raw_start, raw_end;  // global raw byte positions covered
  uint32_t rle_start, rle_end;  // global positions of its first-stage output
  uint32_t level;
  uint32_t crc;                 // CRC-32/BZIP2 of the raw bytes
};

// Per-block coding state (device-built).
struct BlockCode {
  uint32_t n_in_use;
  uint32_t alpha;
  uint32_t n_mtf;      // symbols including end-of-block
  uint32_t sym_start;  // first symbol in the global symbol array
  uint32_t n_groups;
  uint32_t n_sel;
  uint32_t sel_start;  // first selector in the global selector array
  uint32_t orig_ptr;
  uint32_t prefix_bits;
  uint32_t data_bits;
  uint32_t stream_bytes;
  uint32_t stream_off;  // byte offset inside its frame's container
  uint32_t word_start;  // first 32-bit output word of this stream in the writer's index space
  uint32_t chunk_start; // first 4096-symbol MTF chunk of this block
  uint32_t n_chunks;
  uint32_t pad;
};

// ---------------------------------------------------------------- wave64 helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }

// Lanes of `active` whose 8-bit value equals this lane's value: for each
// bit, the ballot of that bit where this lane's bit is set, its complement
// where it is clear, i.e. ~(ballot ^ t) with t = the bit spread over a word
// (one xnor-and per 32-bit half instead of a per-lane select of 64-bit masks).
__device__ __forceinline__ uint64_t match_any8(uint32_t v, uint64_t active) {
  uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
#pragma unroll
  for (int b = 0; b < 8; b++) {
    uint32_t t = (uint32_t)((int32_t)(v << (31 - b)) >> 31);
    asm volatile("" : "+v"(t));  // the ballot compares t itself (no second shift)
    const uint64_t bal = ballot64(t != 0u);
    lo &= ~((uint32_t)bal ^ t);
    hi &= ~((uint32_t)(bal >> 32) ^ t);
  }
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_read(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// ---------------------------------------------------------------- tile scans
// Building blocks of the fused scans (a scan whose input is computed on the
// fly and whose consumer runs in the same kernel): tiles of 4096 elements,
// 256 threads x 16; the carry of a tile is the reduction of the tile
// aggregates in front of it, which each workgroup sums itself.  (A single
// pass with decoupled look-back measured slower: device-scope status polls
// across the XCDs cost about a microsecond each.)  Sums wrap mod 2^32, so
// differences of prefix values inside any segment whose own total stays
// below 2^32 are exact.
constexpr int kTThreads = 256;
constexpr int kTItems = 16;
constexpr uint32_t kTTile = kTThreads * kTItems;
constexpr uint32_t kTPad = kTTile + kTTile / 32;  // LDS words of a padded tile

__device__ __forceinline__ int tpad(int j) { return j + (j >> 5); }

template <bool kMax>
__device__ __forceinline__ uint32_t top(uint32_t a, uint32_t b) { return kMax ? (a > b ? a : b) : a + b; }

// Workgroup reduction of one value per thread (all threads get the result).
template <bool kMax>
__device__ __forceinline__ uint32_t block_reduce(uint32_t v, uint32_t *sh) {
  for (int d = kWave / 2; d > 0; d >>= 1) v = top<kMax>(v, (uint32_t)__shfl_xor((int)v, d));
  __syncthreads();
  if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  uint32_t t = 0;
  for (int i = 0; i < kTThreads / kWave; i++) t = top<kMax>(t, sh[i]);
  return t;
}

// Scan (inclusive or exclusive) of 16 consecutive LDS values per thread, in
// place, from a carry; returns the tile total (without the carry).
template <bool kMax, bool kInclusive>
__device__ __forceinline__ uint32_t tile_scan(uint32_t *buf, uint32_t carry, uint32_t *sh) {
  uint32_t v[kTItems], acc = 0;
#pragma unroll
  for (int i = 0; i < kTItems; i++) {
    v[i] = buf[tpad(threadIdx.x * kTItems + i)];
    acc = top<kMax>(acc, v[i]);
  }
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  uint32_t x = acc;
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)x, d);
    if (lane >= d) x = top<kMax>(o, x);
  }
  uint32_t xe = (uint32_t)__shfl_up((int)x, 1);
  if (lane == 0) xe = 0;
  __syncthreads();
  if (lane == kWave - 1) sh[wave] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < kTThreads / kWave; w++) {
    if (w < wave) before = top<kMax>(before, sh[w]);
    total = top<kMax>(total, sh[w]);
  }
  uint32_t run = top<kMax>(carry, top<kMax>(before, xe));
#pragma unroll
  for (int i = 0; i < kTItems; i++) {
    const uint32_t nv = top<kMax>(run, v[i]);
    buf[tpad(threadIdx.x * kTItems + i)] = kInclusive ? nv : run;
    run = nv;
  }
  __syncthreads();
  return total;
}

// Stores a tile's values from buf (tile order, as tile_scan leaves them) at
// out[tile_base + j] for tile_base + j < n, consecutive threads taking
// consecutive positions (a thread's own 16 values would be four 16-byte
// stores 64 bytes apart across the lanes).  buf must stay unchanged until
// the next barrier.
__device__ __forceinline__ void tile_store(const uint32_t *buf, uint32_t *out, uint32_t tile_base, uint32_t n) {
#pragma unroll
  for (int i = 0; i < kTItems; i++) {
    const uint32_t j = (uint32_t)(i * kTThreads) + threadIdx.x;
    if (tile_base + j < n) out[tile_base + j] = buf[tpad((int)j)];
  }
}

// carry over aggs[counted, tile), extending a running carry
template <bool kMax>
__device__ __forceinline__ uint32_t tile_carry(const uint32_t *aggs, uint32_t &counted, uint32_t tile,
                                               uint32_t carry, uint32_t *sh) {
  uint32_t part = 0;
  for (uint32_t j = counted + threadIdx.x; j < tile; j += kTThreads) part = top<kMax>(part, aggs[j]);
  counted = tile;
  return top<kMax>(carry, block_reduce<kMax>(part, sh));
}

// XCD-aware tile walk.  The dispatcher deals the workgroups of a launch to
// the eight XCDs round robin (workgroup i to XCD i mod 8), and each XCD has
// its own L2.  Workgroup i takes the tiles of the (i mod 8)-th eighth of
// [0, nt), so neighbouring tiles (consecutive list elements, mostly one
// block's, whose scattered accesses stay inside that block's part of an
// array) share one L2.  A workgroup's tiles come in increasing order, every
// tile is taken once; with fewer than eight workgroups it is a plain stride.
constexpr uint32_t kXcds = 8;
struct XcdWalk {
  uint32_t t, end, step;
  __device__ __forceinline__ explicit XcdWalk(uint32_t nt) {
    const uint32_t per = gridDim.x / kXcds;  // workgroups per XCD (the grid's remainder idles)
    if (per == 0) {
      t = blockIdx.x;
      end = nt;
      step = gridDim.x;
      return;
    }
    const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    t = (uint32_t)((uint64_t)nt * x / kXcds) + j;
    end = j < per ? (uint32_t)((uint64_t)nt * (x + 1) / kXcds) : 0u;
    step = per;
  }
};
// A grid of whole XCD groups (grids of eight or more workgroups are rounded
// up to a multiple of eight, so no XCD idles in XcdWalk).
inline uint32_t xcd_grid(uint32_t tiles) { return tiles < kXcds ? tiles : (tiles + kXcds - 1) / kXcds * kXcds; }

// Binary search: largest i in [0, n) with a[i] <= key (a sorted ascending, a[0] <= key).
template <typename T>
__device__ __forceinline__ uint32_t upper_index(const T *a, uint32_t n, T key) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= key) lo = mid; else hi = mid;
  }
  return lo;
}

// The blocks a tile touches: the first one's bounds are kept in registers,
// positions past it (tiles that cross a block end) search forward.
struct TileBlocks {
  const uint32_t *blk_start;
  uint32_t nb, b0, s0, e0;
  __device__ __forceinline__ TileBlocks(const uint32_t *bs, uint32_t n, uint32_t base) : blk_start(bs), nb(n) {
    if (n < (uint32_t)kWave) {  // one load per lane instead of a chain of dependent ones
      const int lane = lane_id();
      const uint32_t mine = (uint32_t)lane <= n ? bs[lane] : 0xFFFFFFFFu;
      b0 = (uint32_t)__popcll(ballot64((uint32_t)lane < n && mine <= base)) - 1u;
      s0 = (uint32_t)__shfl((int)mine, (int)b0);
      e0 = (uint32_t)__shfl((int)mine, (int)b0 + 1);
    } else {
      b0 = upper_index(bs, n, base);
      s0 = bs[b0];
      e0 = bs[b0 + 1];
    }
  }
  // block of p (p >= the tile base), with its start and end
  __device__ __forceinline__ uint32_t find(uint32_t p, uint32_t &s, uint32_t &e) const {
    if (p < e0) {
      s = s0;
      e = e0;
      return b0;
    }
    uint32_t b = b0;
    while (b + 1 < nb && blk_start[b + 1] <= p) b++;
    s = blk_start[b];
    e = blk_start[b + 1];
    return b;
  }
};

// Copies n elements from global memory into LDS with the whole workgroup,
// keeping 16 loads in flight per thread (a plain strided loop waits for each
// load before the next).
template <typename T>
__device__ __forceinline__ void stage_to_lds(T *dst, const T *src, uint32_t n) {
  constexpr uint32_t kInFlight = 16;
  const uint32_t step = blockDim.x;
  for (uint32_t base = 0; base < n; base += step * kInFlight) {
    T v[kInFlight];
#pragma unroll
    for (uint32_t k = 0; k < kInFlight; k++) {
      const uint32_t i = base + k * step + threadIdx.x;
      if (i < n) v[k] = src[i];
    }
#pragma unroll
    for (uint32_t k = 0; k < kInFlight; k++) {
      const uint32_t i = base + k * step + threadIdx.x;
      if (i < n) dst[i] = v[k];
    }
  }
}

// ---------------------------------------------------------------- tracing
// Optional HIP-event timing of named kernel launches (see pcbz_trace_*).
// When tracing is off these are a single branch.
extern bool g_trace_on;
// Stage label recorded with traced launches ("stage|kernel"); nullptr = none.
extern thread_local const char *g_trace_stage;
inline void trace_stage(const char *stage) { g_trace_stage = stage; }
void trace_begin_impl(const char *name, hipStream_t s);
void trace_end_impl(const char *name, hipStream_t s);
inline void trace_begin(const char *name, hipStream_t s) {
  if (g_trace_on) trace_begin_impl(name, s);
}
inline void trace_end(const char *name, hipStream_t s) {
  if (g_trace_on) trace_end_impl(name, s);
}
// Adds algorithmic bytes (what the step must read and write) to a kernel's
// trace record; the name is the kernel's launch spelling.
void trace_bytes_impl(const char *name, uint64_t bytes);
inline void trace_bytes(const char *name, uint64_t bytes) {
  if (g_trace_on) trace_bytes_impl(name, bytes);
}
// The same with the element count in device memory (launches sized by a
// bound): a one-thread kernel on s copies *d_count as it is at this point of
// the stream, and per_elem times that count is added when trace_settle reads
// the copies back after the call's results (the call ends with a sync anyway).
void trace_bytes_count_impl(const char *name, uint64_t per_elem, const uint32_t *d_count, hipStream_t s);
inline void trace_bytes_count(const char *name, uint64_t per_elem, const uint32_t *d_count, hipStream_t s) {
  if (g_trace_on) trace_bytes_count_impl(name, per_elem, d_count, s);
}
void trace_settle_impl(hipStream_t s);
inline void trace_settle(hipStream_t s) {
  if (g_trace_on) trace_settle_impl(s);
}
#define PCBZ_LAUNCH(kernel, grid, block, lds, stream, ...)                  \
  do {                                                                      \
    ::pcbz::trace_begin(#kernel, stream);                                   \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);      \
    ::pcbz::trace_end(#kernel, stream);                                     \
  } while (0)

// ---------------------------------------------------------------- launchers
struct CandBufs {
  uint8_t *p[kNumCand];
};

// Per-frame output description for the container writer.
struct FrameOut {
  uint8_t *out;           // caller's device output buffer
  const uint8_t *forced;  // caller's forced ids (device, n_bands) or nullptr
  uint64_t cap;  // its capacity in bytes
  uint32_t h, w, pitch, level;
  uint32_t n_bands;
  uint32_t band_base;  // first band of this frame in the band table
};

// fill.hip
// Word ranges cleared by one launch.
struct ZeroSpans {
  uint32_t *p[8];
  size_t n[8];
  int count = 0;
  void add(void *ptr, size_t words) {
    if (ptr && words && count < 8) {
      p[count] = (uint32_t *)ptr;
      n[count] = words;
      count++;
    }
  }
};
void zero_spans(const ZeroSpans &z, hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
void copy_u32(uint32_t *dst, const uint32_t *src, hipStream_t s);  // one word, device to device, as a kernel

// judge.hip
size_t remap_lds_bytes(uint32_t pitch, uint32_t lens_per_wg);
size_t predict_lds_bytes(uint32_t pitch, uint32_t lens_per_wg);
// Residuals of the predictor family (ids 4..15) of every band that enables or is forced to one.
void launch_predict(const BandDesc *bands, const RowItem *rows, uint32_t n_rows, uint32_t max_chunks,
                    uint32_t lens_per_wg, uint32_t pitch_max, CandBufs cb, const uint8_t *forced, hipStream_t s);
void launch_remap2(const BandDesc *bands, const RowItem *rows, uint32_t n_rows, uint32_t max_chunks,
                   uint32_t lens_per_wg, uint32_t pitch_max, CandBufs cb, const uint8_t *forced,
                   uint32_t write_mask, hipStream_t s);
// forced (may be nullptr): tasks of bands whose id is not 0xFF are skipped.
void launch_judge2(const JudgeTask *tasks, uint32_t n_tasks, const uint32_t *tile_task, const uint32_t *tile_local,
                   uint32_t n_tiles, CandBufs cb, uint16_t *seg_first, uint16_t *seg_last, uint32_t *hist,
                   const int64_t *tq, unsigned long long *score, const uint8_t *forced, hipStream_t s);
void launch_choose2(const BandDesc *bands, uint32_t n_bands, const int32_t *task_of,
                    const unsigned long long *score, const JudgeTask *tasks, const uint8_t *forced, uint8_t *choice,
                    double *entropy, int64_t *score_out, hipStream_t s);
void launch_gather2(const uint32_t *band_start, uint32_t n_bands, CandBufs cb, const uint8_t *choice,
                    uint8_t *chosen, uint64_t total, hipStream_t s);
void launch_validate_forced(const BandDesc *bands, uint32_t n_bands, uint8_t *forced, uint32_t *err,
                            hipStream_t s);
void launch_gather_forced(const FrameOut *frames, uint32_t n_frames, uint8_t *forced, hipStream_t s);

// rle1.hip
// d_total (may be null) also receives the output length, off[N]
void launch_rle1_2(const uint32_t *band_start, uint32_t n_bands, const uint8_t *x, uint32_t N, uint32_t *runstart,
                   uint32_t *len, uint32_t *off, uint8_t *rle, uint32_t *d_total, hipStream_t s);
void launch_cut2(const BandDesc *bands, uint32_t n_bands, const uint32_t *band_start, uint32_t N,
                 const uint32_t *runstart, const uint32_t *off, BlockDesc *slots, uint32_t *slot_count,
                 uint32_t *err, BlockDesc *blocks, uint32_t *blk_raw_start, uint32_t *blk_rle_start,
                 uint32_t *crc_chunk_base, uint32_t *d_n_blocks, uint32_t *d_crc_chunks, hipStream_t s);
void launch_crc2(const uint8_t *x, uint32_t N, BlockDesc *blocks, const uint32_t *d_n_blocks, uint32_t max_blocks,
                 const uint32_t *blk_raw_start, const uint32_t *xpow_chunk, const uint32_t *xpow_byte,
                 const uint32_t *xpow2, uint32_t *crc_acc, hipStream_t s);

// bwt.hip
struct BwtWork {
  uint64_t *key[2];
  uint32_t *val[2];
  uint32_t *slot;
  uint32_t *slot2;
  uint32_t *rank;
  uint32_t *counts;     // radix tile counts
  uint32_t *d_u;        // [2] unresolved counts (device)
  uint32_t *d_count_n;  // size of the current count table (device)
  uint32_t *d_min_m;    // length of the shortest block (device)
  uint32_t *d_maxg;     // largest unresolved group of the last round (device, d_u + 6)
  uint32_t *d_fail;     // set when a group did not fit the in-group sort (device)
  uint32_t *seg_bound;  // [seg_bound_words] tile boundaries of the in-group sort
  uint32_t *gstart;     // [N+1] compact position of each unresolved element's group start
  uint32_t *aggs;       // [rnd_aggs_words] tile aggregates of a doubling round's two scans
};
size_t radix_counts_words(uint32_t n_max, uint32_t nb_max);
size_t seg_bound_words(uint32_t n_max);
size_t rnd_aggs_words(uint32_t n_max);
int radix_sort(uint64_t *keys[2], uint32_t *vals[2], const uint32_t *d_n, uint32_t n_max, int bits, int items,
               bool iota_vals, const uint32_t *blk_start, const uint32_t *d_nb, uint32_t nb_max, uint32_t *counts,
               uint32_t *d_count_n, hipStream_t s);
int run_bwt(const uint8_t *rle, const uint32_t *d_N, uint32_t n_max, const uint32_t *d_nb, uint32_t nb_max,
            const uint32_t *blk_start, BwtWork w, uint32_t *sa, uint8_t *L, BlockCode *codes, int max_rounds,
            int items, uint32_t *pinned_u, uint64_t *seg_mask, uint32_t *d_left, hipStream_t s);

// mtf.hip
constexpr uint32_t kMtfSegs = 64;    // segments per block in the move-to-front list chain
constexpr uint32_t kMtfChunk = 256;  // positions per move-to-front chunk (one wavefront replays one)
constexpr uint32_t kMtfMaxBlock = 899981;  // longest first-stage block (level 9)
// chunks per segment of the longest block
constexpr uint32_t kMtfUnits = ((kMtfMaxBlock + kMtfChunk - 1) / kMtfChunk + kMtfSegs - 1) / kMtfSegs;
struct MtfWork {
  uint32_t *used;        // [max_blocks * 8] used-byte bitmaps
  uint32_t *chunk_block; // [max_chunks + 1] first chunk of each block
  uint8_t *plist;        // [max_chunks * 256] chunk partial lists
  uint32_t *plen;        // [max_chunks]
  uint8_t *inlist;       // [max_chunks * 256]
  uint8_t *seglist;      // [max_blocks * kMtfSegs * 256] segment partial lists, then segment incoming lists
  uint32_t *seglen;      // [max_blocks * kMtfSegs]
  uint8_t *idx;          // [N] MTF indices
  uint32_t *zs;          // [N] zero-run segment start of each position
  uint32_t *aggs;        // [2 * (N / kTTile + 2)] tile aggregates of the zero-run scans
  uint32_t *d_n_chunks;
};
void launch_mtf2(const uint8_t *L, const uint32_t *d_N, uint32_t N, const uint32_t *blk_start, const uint32_t *d_nb, uint32_t max_blocks,
                 uint32_t max_chunks, MtfWork w, BlockCode *codes, uint16_t *sym, uint32_t *freq,
                 uint32_t *d_n_sym, hipStream_t s);

// huff.hip
void launch_huff2(const uint16_t *sym, const uint32_t *d_nb, uint32_t max_blocks, uint32_t max_groups,
                  BlockCode *codes, const uint32_t *freq, uint8_t *cost, uint32_t *tfreq, uint32_t *group_base,
                  uint32_t *d_n_groups, uint8_t *sel, uint8_t *lens, uint32_t *code_words, hipStream_t s);

// pack.hip
// Header bits of every block (the stream header, used-byte map, selectors
// and code lengths) into prefix; sets codes[b].prefix_bits.
void launch_pack_prefix(const uint32_t *d_nb, uint32_t max_blocks, const BlockDesc *blocks, BlockCode *codes,
                        const uint32_t *used, const uint8_t *sel, const uint8_t *lens, uint32_t *prefix,
                        hipStream_t s);
// Symbol bit lengths and offsets, stream layout, the words of every stream
// and the container headers.  The layout waits for prefix_ready (when given:
// the event recorded after launch_pack_prefix on another stream).
void launch_pack2(const uint32_t *d_nb, uint32_t max_blocks, const BlockDesc *blocks, BlockCode *codes,
                  const uint8_t *sel, const uint8_t *lens, const uint32_t *code_words, const uint16_t *sym,
                  const uint32_t *d_n_sym, uint32_t max_sym, const uint32_t *prefix, uint32_t *sym_bits,
                  uint32_t *sym_off, uint32_t *blk_sym_start, const FrameOut *frames,
                  uint32_t n_frames, const BandDesc *bands, const uint8_t *choice, uint32_t *band_len,
                  uint64_t *frame_len, uint32_t *word_start, uint32_t *d_words, uint32_t max_words,
                  hipEvent_t prefix_ready, hipStream_t s);

// ---------------------------------------------------------------- decompression
// One band of a decompression call (host-built).
struct DecBand {
  const uint8_t *src;      // the band's bzip2 streams inside the container (device)
  uint16_t *out;           // the frame being written (device)
  const uint16_t *prev;    // previous frame (VIEW_DT) or nullptr
  uint32_t src_len;        // bytes of the band's streams
  uint32_t id;             // arrangement id
  uint32_t W, pitch, Nt, Rb, y0;
  uint32_t n;              // raw bytes of the band (2 * Rb * pitch * W)
  uint32_t raw_off;        // first byte of the band in the call's raw byte space
  uint32_t slot0, nslots;  // block slots of the band
  uint32_t level;          // container level (block limit 100000 * level)
  uint32_t sym_base, sym_end;  // the band's range of the symbol space
  uint32_t blk_cap;        // bound on the band's block bytes (n + n / 4 + 8)
  uint32_t col0_off;       // first value of the band's first-lens-column sums (VIEW_DX)
};

// One block slot of a decompression call (device-built).
struct DecSlot {
  uint32_t valid;         // a stream was decoded into this slot
  uint32_t band;
  uint32_t start_byte;    // first byte of the stream in its band
  uint32_t end_byte;      // first byte after the stream
  uint32_t crc;           // stored block CRC
  uint32_t orig_ptr;
  uint32_t n_in_use;
  uint32_t n_sym;         // symbols including the end-of-block symbol
  uint32_t sym_off;       // first symbol in the symbol space
  uint32_t m;             // block length (inverse move-to-front output)
  uint32_t l_off;         // first byte of the block in the packed block space
  uint32_t raw_len;       // bytes once the first run-length stage is undone
  uint32_t raw_off;       // first byte in the call's raw byte space (0xFFFFFFFF: band failed)
  uint32_t chunk0, n_chunks;  // move-to-front chunks
  uint32_t seg0, n_segs;      // segments of 32 chunks
  uint32_t blk;               // index among the valid slots
  uint32_t cyc;               // length of the inverse-BWT cycle through the origin row (divides m)
};

constexpr uint32_t kDecChunk = 1024;      // symbols per inverse move-to-front chunk
constexpr uint32_t kDecSeg = 32;          // chunks per segment of the list chain
constexpr uint32_t kDecSplit = 64;        // stride of the inverse-BWT splitters
constexpr uint32_t kDecTile = 4096;       // positions per inverse run-length tile
constexpr uint32_t kDecHeadBytes = 24576; // bytes staged for a stream header (it is shorter)
constexpr uint32_t kDecMaxBlock = 900000; // the format's largest block (level 9)
constexpr uint32_t kDecMaxSpl = kDecMaxBlock / kDecSplit + 2;  // splitters of one block

// Error bits of a decompression call (word 0 of its counters).
enum : uint32_t {
  kDecErrStream = 1u,    // malformed stream header or Huffman data
  kDecErrMtf = 2u,       // bad move-to-front index, run or block length
  kDecErrBwt = 4u,       // the inverse BWT permutation is not one cycle
  kDecErrLen = 8u,       // a band decodes to the wrong number of bytes
  kDecErrCrc = 16u,      // block CRC mismatch
  kDecErrSlots = 32u,    // streams left over in a band, or none
};

// Counter words of a decompression call.
enum : uint32_t {
  kDcErr = 0, kDcBand = 1, kDcBlocks = 2, kDcChunks = 3, kDcN = 4, kDcSpl = 5, kDcTiles = 6, kDcSegs = 7,
  kDcCountN = 8, kDcWords = 16
};

struct DecWork {
  DecBand *bands;
  DecSlot *slots;
  uint32_t *ctr;          // kDcWords counter words
  uint8_t *seq;           // [slots][256] byte of each symbol-map rank
  uint16_t *sym;          // [sym_total] symbols, band by band
  uint8_t *tok;           // [sym_total] placeholder tokens
  uint32_t *chunk_slot;   // [max_chunks]
  uint32_t *chunk_tot;    // [max_chunks] bytes a chunk expands to
  uint32_t *chunk_off;    // [max_chunks] its first byte inside the block
  uint8_t *chunk_fin;     // [max_chunks][256] list permutation at the chunk's end
  uint8_t *chunk_in;      // [max_chunks][256] incoming list
  uint32_t *seg_slot;     // [max_segs]
  uint8_t *seg_perm;      // [max_segs][256]
  uint8_t *seg_in;        // [max_segs][256]
  uint32_t *seg_tot;      // [max_segs]
  uint32_t *seg_off;      // [max_segs]
  uint8_t *L;             // [n_max + 16] block space
  uint8_t *T;             // [n_max + 16]
  uint64_t *key[2];
  uint32_t *val[2];
  uint32_t *E;            // [n_max] successor << 8 | byte
  uint32_t *counts;       // radix counts
  uint32_t *blk_start;    // [n_slots + 1] dense blocks in the block space
  uint32_t *blk_slot;     // [n_slots] slot of each dense block
  uint32_t *blk_spl0;     // [n_slots + 1] first splitter of each dense block
  uint32_t *blk_tile0;    // [n_slots + 1] first run-length tile of each dense block
  uint32_t *spl_nxt, *spl_len, *spl_pos;  // [max_spl]
  uint32_t *tile_agg;     // [max_tiles][6] map + five lengths
  uint32_t *tile_in;      // [max_tiles][2] in-state, first raw byte
  uint8_t *raw;           // [raw_total + 16] raw band bytes
  uint16_t *col0;         // [col0_total] running sums down the first lens column of every view (VIEW_DX)
  BlockDesc *blocks;      // [n_slots + 1] dense blocks' raw ranges and computed CRCs
  uint32_t *blk_raw_start;  // [n_slots + 1]
  uint32_t *crc_acc;      // [n_slots + 1]
  uint32_t sym_total, max_chunks, max_segs, n_max, max_spl, max_tiles, raw_total, n_slots, n_bands, max_nslots;
  uint32_t col0_total;
  RowItem *rows;          // [n_rows] (band, lens row) of every band
  uint32_t n_rows;
  uint32_t pred_pixel;    // some band uses a pixel-neighbour predictor
  uint32_t pred_lines;    // some band uses a lens or phase-space predictor
  uint32_t pred_sets;     // most line sets of such a band
  uint32_t nt_max;        // most lens columns of such a band
};

// decode.hip: the stages of one decompression call, in stream order.  The
// host reads the counters back after launch_dec_front (the block-space
// layout and any error) and sizes the later launches from them.
void launch_dec_front(const DecWork &w, hipStream_t s);
// hc: the counters as read back (kDcWords words).
void launch_dec_back(const DecWork &w, const uint32_t *hc, int radix_items, const uint32_t *xpow_chunk,
                     const uint32_t *xpow_byte, const uint32_t *xpow2, hipStream_t s);

// ---------------------------------------------------------------- learned selector
}  // namespace pcbz
struct pcbz_selector;
struct pcbz_ctx;
namespace pcbz {
constexpr uint32_t kFeatCells = 4096;  // 64 x 64 cells per band
constexpr uint32_t kFeatChan = 4;
// Per-band features [n_bands][64][64][4] (FP32) from the raw frames.
void launch_features(const BandDesc *bands, uint32_t n_bands, float *feat, hipStream_t s);
// Generation of the selector's device buffers (changes whenever one moves).
uint64_t selector_gen(const pcbz_selector *S);
int context_device(const pcbz_ctx *ctx);
// Logits of n feature maps: one fused inference kernel (capturable).
int selector_forward(pcbz_selector *S, const float *feat, uint32_t n, float *logits, hipStream_t s);
// Bands with forced == 0xFF take the network's argmax over their enabled
// candidates if its softmax probability is >= min_conf, else stay 0xFF (judged).
void launch_select(const float *logits, uint32_t n_bands, const BandDesc *bands, float min_conf, uint8_t *forced,
                   uint32_t *n_fallback, hipStream_t s);
}  // namespace pcbz
