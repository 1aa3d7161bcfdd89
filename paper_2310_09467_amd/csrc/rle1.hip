// rle1.hip -- bzip2's first run-length stage, greedy block cuts and block CRCs.
//
// Runs of equal bytes never cross a band.  A position's offset k inside its
// run comes from an inclusive max-scan of run-start positions; pieces are
// k / 255, and a piece of length L emits min(L,4) copies plus, when L >= 4,
// a count byte L-4 (written by the piece's fourth position).  Output offsets
// are an exclusive sum-scan of the per-position output lengths.
//
// Block cut: pieces are appended while the block stays within
// 100000*level-19 bytes.  Output ends e(i) = off[i] + len[i] are monotone, so
// the first piece that does not fit is found by binary search.
//
// CRC-32/BZIP2 of each block's raw bytes: every 256-byte chunk, counted back
// from the block end, gets its zero-init register value R (table-driven,
// MSB-first, polynomial 0x04C11DB7); the block register is the XOR of
// R_j * x^(8*256*j) mod P over chunks, plus 0xFFFFFFFF * x^(8m) for the
// initial value; the final XOR with 0xFFFFFFFF gives the CRC.
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr uint32_t kPoly = 0x04C11DB7u;
constexpr int kCrcChunk = 64;  // bytes per thread: short table-lookup chains, many threads

__device__ __forceinline__ uint32_t piece_len_out(uint32_t o) { return o < 3 ? 1u : (o == 3 ? 2u : 0u); }

// The stage runs in three launches over tiles of 4096 positions (256 threads
// x 16 consecutive positions; each scan takes its carry by reducing the tile
// aggregates in front of its tile):
//   k_r1_marks   per-tile maximum of the run-start marks (a position that
//                starts a run is marked with itself, others with 0);
//   k_r1_counts  max-scan of the marks = each position's run start (kept for
//                the block cut), and per-tile sums of the output lengths;
//   k_r1_write   exclusive scan of the output lengths = output offsets (kept
//                for the block cut, total at off[N]) and the output bytes.

// 16 bytes from p0 (16-byte aligned; the buffer has 16 bytes of slack past N)
// and the run-start marks of those positions.
struct R1Bytes {
  uint32_t w[4];
  __device__ __forceinline__ uint32_t at(int i) const { return (w[i >> 2] >> (8 * (i & 3))) & 255u; }
};
__device__ __forceinline__ R1Bytes r1_load(const uint8_t *x, uint32_t p0) {
  const uint4 q = *(const uint4 *)(x + p0);
  return R1Bytes{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ void r1_marks(const R1Bytes &z, const uint8_t *x, const uint32_t *band_start,
                                         uint32_t n_bands, uint32_t p0, uint32_t N, uint32_t *mk) {
  uint32_t b = upper_index(band_start, n_bands, p0);
  uint32_t prevc = p0 > 0 ? x[p0 - 1] : 0u;
#pragma unroll
  for (int i = 0; i < kTItems; i++) {
    const uint32_t p = p0 + i;
    while (b + 1 < n_bands && band_start[b + 1] <= p) b++;  // bands can be shorter than 16 bytes
    const uint32_t c = z.at(i);
    mk[i] = p < N && (p == band_start[b] || c != prevc) ? p : 0u;
    prevc = c;
  }
}

__global__ __launch_bounds__(kTThreads) void k_r1_marks(const uint32_t *band_start, uint32_t n_bands,
                                                        const uint8_t *x, uint32_t N, uint32_t *aggs_m) {
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t p0 = tile * kTTile + threadIdx.x * kTItems;
    uint32_t m = 0;
    if (p0 < N) {
      uint32_t mk[kTItems];
      r1_marks(r1_load(x, p0), x, band_start, n_bands, p0, N, mk);
#pragma unroll
      for (int i = 0; i < kTItems; i++) m = max(m, mk[i]);
    }
    m = block_reduce<true>(m, sh);
    if (threadIdx.x == 0) aggs_m[tile] = m;
  }
}

__global__ __launch_bounds__(kTThreads) void k_r1_counts(const uint32_t *band_start, uint32_t n_bands,
                                                         const uint8_t *x, uint32_t N, const uint32_t *aggs_m,
                                                         uint32_t *runstart, uint32_t *aggs_s) {
  __shared__ uint32_t buf[kTPad];
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  uint32_t carry = 0, counted = 0;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t p0 = tile * kTTile + threadIdx.x * kTItems;
    uint32_t mk[kTItems];
    if (p0 < N) {
      r1_marks(r1_load(x, p0), x, band_start, n_bands, p0, N, mk);
    } else {
#pragma unroll
      for (int i = 0; i < kTItems; i++) mk[i] = 0;
    }
    carry = tile_carry<true>(aggs_m, counted, tile, carry, sh);
#pragma unroll
    for (int i = 0; i < kTItems; i++) buf[tpad(threadIdx.x * kTItems + i)] = mk[i];
    __syncthreads();
    tile_scan<true, true>(buf, carry, sh);
    uint32_t rs[kTItems], cnt = 0;
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      rs[i] = buf[tpad(threadIdx.x * kTItems + i)];
      if (p0 + i < N) cnt += piece_len_out((p0 + i - rs[i]) % 255u);
    }
    tile_store(buf, runstart, tile * kTTile, N);
    cnt = block_reduce<false>(cnt, sh);
    if (threadIdx.x == 0) aggs_s[tile] = cnt;
  }
}

__global__ __launch_bounds__(kTThreads) void k_r1_write(const uint32_t *band_start, uint32_t n_bands,
                                                        const uint8_t *x, uint32_t N, const uint32_t *runstart,
                                                        const uint32_t *aggs_s, uint32_t *off, uint8_t *rle,
                                                        uint32_t *d_total) {
  __shared__ uint32_t buf[kTPad];
  __shared__ uint32_t sh[kTThreads / kWave];
  __shared__ uint8_t stage[2 * kTTile];  // the tile's output bytes (at most two a position)
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  uint32_t carry = 0, counted = 0;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t p0 = tile * kTTile + threadIdx.x * kTItems;
    uint32_t o[kTItems];  // offset inside the run's 255-byte piece (above 3: no output)
    R1Bytes z{{0u, 0u, 0u, 0u}};
    if (p0 + kTItems <= N) {
      const uint4 *q = (const uint4 *)(runstart + p0);
#pragma unroll
      for (int k = 0; k < kTItems / 4; k++) {
        const uint4 r = q[k];
        o[4 * k] = (p0 + 4 * k - r.x) % 255u;
        o[4 * k + 1] = (p0 + 4 * k + 1 - r.y) % 255u;
        o[4 * k + 2] = (p0 + 4 * k + 2 - r.z) % 255u;
        o[4 * k + 3] = (p0 + 4 * k + 3 - r.w) % 255u;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kTItems; i++) o[i] = p0 + i < N ? (p0 + i - runstart[p0 + i]) % 255u : 255u;
    }
    if (p0 < N) z = r1_load(x, p0);
    carry = tile_carry<false>(aggs_s, counted, tile, carry, sh);
#pragma unroll
    for (int i = 0; i < kTItems; i++) buf[tpad(threadIdx.x * kTItems + i)] = p0 + i < N ? piece_len_out(o[i]) : 0u;
    __syncthreads();
    const uint32_t total = tile_scan<false, false>(buf, carry, sh);
    uint32_t q[kTItems];
#pragma unroll
    for (int i = 0; i < kTItems; i++) q[i] = buf[tpad(threadIdx.x * kTItems + i)];
    tile_store(buf, off, tile * kTTile, N);
    // the tile's output is one run from `carry`: staged, then stored with
    // consecutive threads on consecutive bytes
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t p = p0 + i;
      if (p >= N || o[i] > 3) continue;
      const uint32_t c = z.at(i);
      stage[q[i] - carry] = (uint8_t)c;
      if (o[i] == 3) {  // the piece's count byte: equal bytes after the fourth, at most 251, inside the band
        const uint32_t b = upper_index(band_start, n_bands, p);
        const uint32_t bend = b + 1 < n_bands ? band_start[b + 1] : N;
        const uint32_t lim = min(bend, p + 252u);
        uint32_t j = p + 1;
        while (j < lim && x[j] == c) j++;
        stage[q[i] - carry + 1] = (uint8_t)(j - p - 1);
      }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < total; j += kTThreads) rle[carry + j] = stage[j];
    if (tile == nt - 1 && threadIdx.x == 0) {
      off[N] = carry + total;
      if (d_total) *d_total = carry + total;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t out_end(const uint32_t *runstart, const uint32_t *off, uint32_t i) {
  return off[i] + piece_len_out((i - runstart[i]) % 255u);
}

// One thread per band: greedy cuts into block slots.
__global__ void k_cut(const BandDesc *bands, uint32_t n_bands, const uint32_t *band_start, uint32_t /*N*/,
                      const uint32_t *runstart, const uint32_t *off, BlockDesc *slots, uint32_t *slot_count,
                      uint32_t *err) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bands) return;
  const BandDesc B = bands[b];
  const uint32_t s0 = band_start[b], e0 = s0 + B.n;
  const uint32_t lim = 100000u * B.level - 19u;
  uint32_t P = s0, q = off[s0], k = 0;
  for (;;) {
    const uint32_t limit = q + lim;
    uint32_t cut = e0;
    if (off[e0] > limit) {
      uint32_t lo = P, hi = e0 - 1;  // out_end(hi) = off[e0] > limit
      while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (out_end(runstart, off, mid) > limit) hi = mid; else lo = mid + 1;
      }
      cut = lo - (lo - runstart[lo]) % 255u;
      if (cut <= P) {  // cannot happen for consistent offsets; never loop without progress
        atomicOr(err, 2u);
        break;
      }
    }
    if (k < B.blk_slots) {
      BlockDesc d;
      d.band = b;
      d.frame_id = B.frame_id;
      d.raw_start = P;
      d.raw_end = cut;
      d.rle_start = q;
      d.rle_end = off[cut];
      d.level = B.level;
      d.crc = 0;
      slots[B.blk_slot + k] = d;
    } else {
      atomicOr(err, 1u);
    }
    k++;
    if (cut >= e0) break;
    P = cut;
    q = off[cut];
  }
  slot_count[b] = min(k, B.blk_slots);
}

// Dense block list in band order, with CRC chunk bases.  One workgroup.
__global__ __launch_bounds__(1024) void k_blocks_compact(const BandDesc *bands, uint32_t n_bands,
                                                         const BlockDesc *slots, const uint32_t *slot_count,
                                                         BlockDesc *blocks, uint32_t *blk_raw_start,
                                                         uint32_t *blk_rle_start, uint32_t *crc_chunk_base,
                                                         uint32_t *d_n_blocks, uint32_t *d_crc_chunks) {
  __shared__ uint32_t sh[1024];
  __shared__ uint32_t carry_blocks;
  if (threadIdx.x == 0) carry_blocks = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n_bands; base += 1024) {
    uint32_t b = base + threadIdx.x;
    uint32_t cnt = b < n_bands ? slot_count[b] : 0;
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      uint32_t v = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
      __syncthreads();
      sh[threadIdx.x] += v;
      __syncthreads();
    }
    uint32_t excl = carry_blocks + sh[threadIdx.x] - cnt;
    if (b < n_bands)
      for (uint32_t k = 0; k < cnt; k++) blocks[excl + k] = slots[bands[b].blk_slot + k];
    __syncthreads();
    if (threadIdx.x == 1023) carry_blocks += sh[1023];
    __syncthreads();
  }
  const uint32_t nb = carry_blocks;
  // raw / rle starts and CRC chunk bases (serial over blocks, cheap)
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t k = 0; k < nb; k++) {
      blk_raw_start[k] = blocks[k].raw_start;
      blk_rle_start[k] = blocks[k].rle_start;
      crc_chunk_base[k] = acc;
      acc += (blocks[k].raw_end - blocks[k].raw_start + kCrcChunk - 1) / kCrcChunk;
    }
    crc_chunk_base[nb] = acc;
    blk_raw_start[nb] = nb ? blocks[nb - 1].raw_end : 0;
    blk_rle_start[nb] = nb ? blocks[nb - 1].rle_end : 0;
    *d_n_blocks = nb;
    *d_crc_chunks = acc;
  }
}

__device__ uint32_t gf_mulmod(uint32_t a, uint32_t b) {
  uint32_t r = 0;
  for (int i = 31; i >= 0; i--) {
    r = (r & 0x80000000u) ? (r << 1) ^ kPoly : (r << 1);
    if ((b >> i) & 1u) r ^= a;
  }
  return r;
}

// One thread per aligned 256-byte chunk of the raw byte space.  A chunk
// inside one block is folded four bytes at a time with slice-by-4 tables
// (T[k][v] = v * x^(32+8k) mod P); a chunk that crosses block edges is folded
// byte by byte per block part.  Each part's register is carried to its block
// end by x^(8d) mod P, d = bytes after the part = 256 q + r, from the tables
// x^(2048 q) and x^(8 r).
__global__ __launch_bounds__(256) void k_crc_chunks(const uint8_t *x, uint32_t N, const uint32_t *d_n_blocks,
                                                    const uint32_t *blk_raw_start, const uint32_t *xpow_chunk,
                                                    const uint32_t *xpow_byte, uint32_t *crc_acc) {
  __shared__ uint32_t T[4][256];
  {
    uint32_t r = (uint32_t)threadIdx.x << 24;
    for (int k = 0; k < 8; k++) r = (r & 0x80000000u) ? (r << 1) ^ kPoly : (r << 1);
    T[0][threadIdx.x] = r;
    for (int t = 1; t < 4; t++) {
      for (int k = 0; k < 8; k++) r = (r & 0x80000000u) ? (r << 1) ^ kPoly : (r << 1);
      T[t][threadIdx.x] = r;
    }
  }
  // XOR accumulators for the first blocks this workgroup touches; parts of
  // later blocks (only with many tiny blocks) go straight to global memory
  constexpr uint32_t kSlots = 16;
  __shared__ uint32_t acc[kSlots];
  const uint32_t nb = *d_n_blocks;
  const uint32_t nchunks = (N + kCrcChunk - 1) / kCrcChunk;
  const uint32_t cfirst = blockIdx.x * blockDim.x;
  const uint32_t kfirst = cfirst < nchunks ? upper_index(blk_raw_start, nb, cfirst * kCrcChunk) : 0;
  if (threadIdx.x < kSlots) acc[threadIdx.x] = 0;
  __syncthreads();
  {
    const uint32_t c = cfirst + threadIdx.x;
    if (c >= nchunks) goto flush;
    const uint32_t c0 = c * kCrcChunk, c1 = min(N, c0 + kCrcChunk);
    uint32_t k = upper_index(blk_raw_start, nb, c0);
    for (;;) {
      const uint32_t bs = blk_raw_start[k], be = blk_raw_start[k + 1];
      const uint32_t lo = max(c0, bs), hi = min(c1, be);
      uint32_t r = 0;
      if (lo == c0 && hi == c0 + kCrcChunk) {
        const uint4 *p = (const uint4 *)(x + c0);
        constexpr int kVec = kCrcChunk / 16;
        uint4 v[kVec];
#pragma unroll
        for (int i = 0; i < kVec; i++) v[i] = p[i];
#pragma unroll
        for (int i = 0; i < kVec; i++) {
          const uint32_t wds[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
          for (int q = 0; q < 4; q++) {
            r ^= __builtin_bswap32(wds[q]);
            r = T[0][r & 255u] ^ T[1][(r >> 8) & 255u] ^ T[2][(r >> 16) & 255u] ^ T[3][r >> 24];
          }
        }
      } else {
        for (uint32_t i = lo; i < hi; i++) r = (r << 8) ^ T[0][(r >> 24) ^ x[i]];
      }
      const uint32_t d = be - hi;
      r = gf_mulmod(gf_mulmod(r, xpow_chunk[d >> 8]), xpow_byte[d & 255u]);
      if (k - kfirst < kSlots)
        atomicXor(&acc[k - kfirst], r);
      else
        atomicXor(&crc_acc[k], r);
      if (be >= c1 || k + 1 >= nb) break;
      k++;
    }
  }
flush:
  __syncthreads();
  if (threadIdx.x < kSlots && kfirst + threadIdx.x < nb && acc[threadIdx.x])
    atomicXor(&crc_acc[kfirst + threadIdx.x], acc[threadIdx.x]);
}

__device__ uint32_t xpow8_bytes(uint32_t m, const uint32_t *xpow2) {
  // x^(8m) mod P from x^(2^k) mod P, k = 0..63
  uint64_t e = (uint64_t)m * 8u;
  uint32_t r = 1u;  // x^0
  for (int k = 0; e; k++, e >>= 1)
    if (e & 1u) r = gf_mulmod(r, xpow2[k]);
  return r;
}

__global__ void k_crc_final(BlockDesc *blocks, const uint32_t *d_n_blocks, const uint32_t *crc_acc,
                            const uint32_t *xpow2) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= *d_n_blocks) return;
  const uint32_t m = blocks[k].raw_end - blocks[k].raw_start;
  const uint32_t init = gf_mulmod(0xFFFFFFFFu, xpow8_bytes(m, xpow2));
  blocks[k].crc = crc_acc[k] ^ init ^ 0xFFFFFFFFu;
}

}  // namespace

void launch_rle1_2(const uint32_t *band_start, uint32_t n_bands, const uint8_t *x, uint32_t N, uint32_t *runstart,
                   uint32_t *len, uint32_t *off, uint8_t *rle, uint32_t *d_total, hipStream_t s) {
  if (!N) return;
  // the per-position length array is not needed: it holds the two scans'
  // tile aggregates (2 * (tiles + 1) <= N + 5 words)
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  uint32_t *aggs_m = len, *aggs_s = len + nt + 1;
  const uint32_t gt = std::max<uint32_t>(1, std::min<uint32_t>(2048, nt));
  PCBZ_LAUNCH(k_r1_marks, dim3(gt), dim3(kTThreads), 0, s, band_start, n_bands, x, N, aggs_m);
  PCBZ_LAUNCH(k_r1_counts, dim3(gt), dim3(kTThreads), 0, s, band_start, n_bands, x, N, aggs_m, runstart, aggs_s);
  PCBZ_LAUNCH(k_r1_write, dim3(gt), dim3(kTThreads), 0, s, band_start, n_bands, x, N, runstart, aggs_s, off, rle,
              d_total);
}

void launch_cut2(const BandDesc *bands, uint32_t n_bands, const uint32_t *band_start, uint32_t N,
                 const uint32_t *runstart, const uint32_t *off, BlockDesc *slots, uint32_t *slot_count,
                 uint32_t *err, BlockDesc *blocks, uint32_t *blk_raw_start, uint32_t *blk_rle_start,
                 uint32_t *crc_chunk_base, uint32_t *d_n_blocks, uint32_t *d_crc_chunks, hipStream_t s) {
  PCBZ_LAUNCH(k_cut, dim3((n_bands + 63) / 64), dim3(64), 0, s, bands, n_bands, band_start, N, runstart, off,
                     slots, slot_count, err);
  PCBZ_LAUNCH(k_blocks_compact, dim3(1), dim3(1024), 0, s, bands, n_bands, slots, slot_count, blocks,
                     blk_raw_start, blk_rle_start, crc_chunk_base, d_n_blocks, d_crc_chunks);
}

void launch_crc2(const uint8_t *x, uint32_t N, BlockDesc *blocks, const uint32_t *d_n_blocks, uint32_t max_blocks,
                 const uint32_t *blk_raw_start, const uint32_t *xpow_chunk, const uint32_t *xpow_byte,
                 const uint32_t *xpow2, uint32_t *crc_acc, hipStream_t s) {
  const uint32_t chunks = (N + kCrcChunk - 1) / kCrcChunk;
  const uint32_t grid = (chunks + 255) / 256;  // one chunk per thread
  if (!grid) return;
  PCBZ_LAUNCH(k_crc_chunks, dim3(grid), dim3(256), 0, s, x, N, d_n_blocks, blk_raw_start, xpow_chunk, xpow_byte,
              crc_acc);
  PCBZ_LAUNCH(k_crc_final, dim3((max_blocks + 255) / 256), dim3(256), 0, s, blocks, d_n_blocks, crc_acc,
                     xpow2);
}

}  // namespace pcbz
