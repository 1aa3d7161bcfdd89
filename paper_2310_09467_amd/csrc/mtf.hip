// mtf.hip -- move-to-front and the zero-run stage of bzip2.
//
// Move-to-front is sequential per block, so each block is cut into chunks of
// kMtfChunk positions.  The list after a chunk depends on the list before it only
// through a fixed rule: the chunk's distinct symbols in order of last
// occurrence (most recent first) move to the front, the rest keep their
// order.  So (1) every chunk computes that partial list, (2) the partial lists
// are chained (in three shallow steps) into each chunk's incoming list, and
// (3) every chunk replays move-to-front from its incoming list (ranks in
// registers, see k_mtf_run).
//
// Zero runs: a run of r zero indices becomes the bijective base-2 digits of
// r, least significant first (RUNA = 0 for digit 1, RUNB = 1 for digit 2); a
// non-zero index v becomes v + 1; each block ends with nInUse + 1.
#include <algorithm>

#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr uint32_t kChunk = kMtfChunk;

__device__ __forceinline__ void chunk_range(uint32_t c, const uint32_t *chunk_base, const uint32_t *blk_start,
                                            uint32_t nb, uint32_t &b, uint32_t &p0, uint32_t &p1, uint32_t &bs,
                                            uint32_t &be) {
  b = upper_index(chunk_base, nb, c);
  bs = blk_start[b];
  be = blk_start[b + 1];
  p0 = bs + (c - chunk_base[b]) * kChunk;
  p1 = min(be, p0 + kChunk);
}

// chunk bases per block (serial over blocks, tiny)
__global__ void k_mtf_chunks(const uint32_t *blk_start, const uint32_t *d_nb, uint32_t *chunk_base,
                             uint32_t *d_n_chunks, BlockCode *codes) {
  if (threadIdx.x != 0) return;
  const uint32_t nb = *d_nb;
  uint32_t acc = 0;
  for (uint32_t b = 0; b < nb; b++) {
    chunk_base[b] = acc;
    uint32_t m = blk_start[b + 1] - blk_start[b];
    uint32_t nc = (m + kChunk - 1) / kChunk;
    codes[b].chunk_start = acc;
    codes[b].n_chunks = nc;
    acc += nc;
  }
  chunk_base[nb] = acc;
  *d_n_chunks = acc;
}

// Used-byte bitmap of each chunk (8 words, plain stores; k_seq ORs a block's).
__global__ __launch_bounds__(256) void k_used(const uint8_t *L, const uint32_t *chunk_base, const uint32_t *d_n_chunks,
                                              const uint32_t *blk_start, const uint32_t *d_nb, uint32_t *used_chunk) {
  __shared__ uint32_t f[256];
  const uint32_t c = blockIdx.x;
  if (c >= *d_n_chunks) return;
  uint32_t b, p0, p1, bs, be;
  chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  f[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t p = p0 + threadIdx.x; p < p1; p += 256) f[L[p]] = 1;
  __syncthreads();
  const uint64_t bal = ballot64(f[threadIdx.x] != 0);
  if (lane_id() == 0) {
    const uint32_t wbase = threadIdx.x / 32;  // word index of this lane group
    used_chunk[(size_t)c * 8 + wbase] = (uint32_t)bal;
    used_chunk[(size_t)c * 8 + wbase + 1] = (uint32_t)(bal >> 32);
  }
  (void)b;
}

__global__ __launch_bounds__(256) void k_seq(const uint32_t *used_chunk, uint32_t *used, const uint32_t *d_nb,
                                             uint8_t *seq, BlockCode *codes) {
  __shared__ uint32_t u[8];
  const uint32_t b = blockIdx.x;
  if (b >= *d_nb) return;
  const uint32_t c = threadIdx.x;
  if (c < 8) u[c] = 0;
  __syncthreads();
  {
    // OR of the block's chunk bitmaps: thread t ORs word t % 8 of chunks t / 8, t / 8 + 32, ...
    const uint32_t k0 = codes[b].chunk_start, nc = codes[b].n_chunks, wd = c & 7u;
    uint32_t acc = 0;
    for (uint32_t k = c >> 3; k < nc; k += 32) acc |= used_chunk[(size_t)(k0 + k) * 8 + wd];
    if (acc) atomicOr(&u[wd], acc);
  }
  __syncthreads();
  if (c < 8) used[b * 8 + c] = u[c];
  uint32_t before = 0;
  for (uint32_t k = 0; k < c / 32; k++) before += __popc(u[k]);
  before += __popc(u[c / 32] & ((1u << (c % 32)) - 1u));
  seq[b * 256 + c] = (uint8_t)before;
  if (c == 255) {
    uint32_t nu = before + ((u[7] >> 31) & 1u);
    codes[b].n_in_use = nu;
    codes[b].alpha = nu + 2;
  }
}

__global__ __launch_bounds__(64) void k_mtf_partial(const uint8_t *L, const uint32_t *chunk_base,
                                                    const uint32_t *d_n_chunks, const uint32_t *blk_start,
                                                    const uint32_t *d_nb, const uint8_t *seq, uint8_t *plist,
                                                    uint32_t *plen) {
  __shared__ int lastpos[256];
  const uint32_t c = blockIdx.x;
  if (c >= *d_n_chunks) return;
  uint32_t b, p0, p1, bs, be;
  chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  for (int v = threadIdx.x; v < 256; v += 64) lastpos[v] = -1;
  __syncthreads();
  const uint8_t *sq = seq + b * 256;
  for (uint32_t p = p0 + threadIdx.x; p < p1; p += 64) atomicMax(&lastpos[sq[L[p]]], (int)(p - p0));
  __syncthreads();
  // the partial list orders the chunk's symbols by last occurrence, latest
  // first: walking the chunk backwards, it is the sequence of positions that
  // hold the last occurrence of their symbol.  Lane l takes the 16 positions
  // p1 - 1 - 16 l down to p1 - 16 (l + 1); a wavefront prefix count of the
  // flagged positions gives each its place in the list.
  constexpr uint32_t kPer = kChunk / 64;
  const uint32_t n = p1 - p0, lane = threadIdx.x;
  uint32_t flags = 0;
  uint8_t sy[kPer];
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const uint32_t q = lane * kPer + i;
    sy[i] = 0;
    if (q < n) {
      const uint32_t p = p1 - 1 - q;
      const uint8_t v = sq[L[p]];
      sy[i] = v;
      if (lastpos[v] == (int)(p - p0)) flags |= 1u << i;
    }
  }
  const uint32_t cnt = (uint32_t)__popc(flags);
  uint32_t incl = cnt;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d);
    if ((int)lane >= d) incl += t;
  }
  uint32_t r = incl - cnt;
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++)
    if ((flags >> i) & 1u) plist[(size_t)c * 256 + r++] = sy[i];
  if (lane == 63) plen[c] = incl;
}

// List chaining.  Folding a partial list P onto a list C gives P followed by
// C without P's symbols (order kept); folding is associative, so a block's
// chunks are chained in three shallow steps instead of one long one:
//   1. each of kMtfSegs segments of the block folds its chunks' partial lists
//      (from an empty list) into a segment partial list;
//   2. one workgroup per block folds the segment lists from the initial list
//      (ascending order), recording the list entering each segment;
//   3. each segment folds its chunks again from its entering list, recording
//      the list entering each chunk.
// A fold step runs on one workgroup of 256 threads, one list entry each.
struct FoldLds {
  uint8_t cur[256], nxt[256], mem[256];
  uint32_t len;
  uint32_t wcnt[4];
};

// cur/len := P ++ (cur - P) for units [0, n) of (lists, lens); before unit k
// the current list is written to out_in + k * 256 when out_in is set.
__device__ void fold_units(FoldLds &F, const uint8_t *lists, const uint32_t *lens, uint32_t n, uint8_t *out_in) {
  const uint32_t e = threadIdx.x;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint64_t lt = lanemask_lt();
  for (uint32_t k = 0; k < n; k++) {
    if (out_in) out_in[(size_t)k * 256 + e] = F.cur[e];
    F.mem[e] = 0;
    __syncthreads();
    const uint32_t pl = lens[k];
    if (e < pl) {
      const uint8_t v = lists[(size_t)k * 256 + e];
      F.mem[v] = 1;
      F.nxt[e] = v;
    }
    __syncthreads();
    const bool keep = e < F.len && !F.mem[F.cur[e]];
    const uint64_t bal = ballot64(keep);
    if (lane == 0) F.wcnt[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t off = (uint32_t)__popcll(bal & lt), tot = 0;
    for (int q = 0; q < 4; q++) {
      if (q < w) off += F.wcnt[q];
      tot += F.wcnt[q];
    }
    if (keep) F.nxt[pl + off] = F.cur[e];
    __syncthreads();
    F.cur[e] = F.nxt[e];
    if (e == 0) F.len = pl + tot;
    __syncthreads();
  }
}

__device__ __forceinline__ void seg_range(const BlockCode &C, uint32_t j, uint32_t &u0, uint32_t &u1) {
  const uint32_t per = (C.n_chunks + kMtfSegs - 1) / kMtfSegs;
  u0 = min(C.n_chunks, j * per);
  u1 = min(C.n_chunks, u0 + per);
}

// step 1: grid (kMtfSegs, blocks)
__global__ __launch_bounds__(256) void k_mtf_seg_fold(const uint32_t *d_nb, const BlockCode *codes,
                                                      const uint8_t *plist, const uint32_t *plen, uint8_t *seglist,
                                                      uint32_t *seglen) {
  __shared__ FoldLds F;
  const uint32_t b = blockIdx.y, j = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  uint32_t u0, u1;
  seg_range(C, j, u0, u1);
  if (threadIdx.x == 0) F.len = 0;
  __syncthreads();
  fold_units(F, plist + (size_t)(C.chunk_start + u0) * 256, plen + C.chunk_start + u0, u1 - u0, nullptr);
  seglist[((size_t)b * kMtfSegs + j) * 256 + threadIdx.x] = F.cur[threadIdx.x];
  if (threadIdx.x == 0) seglen[(size_t)b * kMtfSegs + j] = F.len;
}

// step 2: one workgroup per block; the segment lists are replaced by the
// lists entering the segments
__global__ __launch_bounds__(256) void k_mtf_seg_chain(const uint32_t *d_nb, uint8_t *seglist, const uint32_t *seglen) {
  __shared__ FoldLds F;
  __shared__ uint8_t parts[kMtfSegs * 256];
  const uint32_t b = blockIdx.x;
  if (b >= *d_nb) return;
  uint8_t *sl = seglist + (size_t)b * kMtfSegs * 256;
  for (uint32_t i = threadIdx.x; i < kMtfSegs * 256; i += 256) parts[i] = sl[i];
  F.cur[threadIdx.x] = (uint8_t)threadIdx.x;
  if (threadIdx.x == 0) F.len = 256;
  __syncthreads();
  fold_units(F, parts, seglen + (size_t)b * kMtfSegs, kMtfSegs, sl);
}

// step 3: grid (kMtfSegs, blocks)
__global__ __launch_bounds__(256) void k_mtf_chain(const uint32_t *d_nb, const BlockCode *codes, const uint8_t *plist,
                                                   const uint32_t *plen, const uint8_t *seglist, uint8_t *inlist) {
  __shared__ FoldLds F;
  const uint32_t b = blockIdx.y, j = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  uint32_t u0, u1;
  seg_range(C, j, u0, u1);
  if (u0 >= u1) return;
  F.cur[threadIdx.x] = seglist[((size_t)b * kMtfSegs + j) * 256 + threadIdx.x];
  if (threadIdx.x == 0) F.len = 256;
  __syncthreads();
  fold_units(F, plist + (size_t)(C.chunk_start + u0) * 256, plen + C.chunk_start + u0, u1 - u0,
             inlist + (size_t)(C.chunk_start + u0) * 256);
}

// Replay of one chunk by one wavefront.  The list is held as ranks (the
// position of each symbol), 16 bits per symbol, two symbols per register and
// two registers per lane: lane l holds the ranks of symbols l and l + 64
// (R0 low / high half) and l + 128 and l + 192 (R1).  A step reads the rank
// r of its symbol from the owning lane (uniform), then every lane updates
// both halves of both registers with packed 16-bit arithmetic: ranks below r
// grow by one, the rank equal to r (the symbol itself; ranks are distinct)
// becomes 0.  No lane diverges and no data moves between lanes.
// ranks x (two halves, each <= 255) after the symbol at rank r moves to front:
// t = x - r per half (wrapping below r), lt = t >> 15 (1 where x < r),
// ne = min(t, 1) (1 where x != r), result (x + lt) * ne.  Written as packed
// 16-bit instructions: the compiler otherwise splits the halves apart.  r is
// the low half of the scalar operand (both halves subtract it; its high
// half is ignored).
__device__ __forceinline__ uint32_t mtf_ranks(uint32_t x, uint32_t r) {
  uint32_t t, lt, y, ne, out;
  asm("v_pk_sub_u16 %0, %1, %2 op_sel_hi:[1,0]" : "=v"(t) : "v"(x), "s"(r));
  asm("v_pk_lshrrev_b16 %0, 15, %1 op_sel_hi:[0,1]" : "=v"(lt) : "v"(t));
  asm("v_pk_add_u16 %0, %1, %2" : "=v"(y) : "v"(x), "v"(lt));
  asm("v_pk_min_u16 %0, %1, 1 op_sel_hi:[1,0]" : "=v"(ne) : "v"(t));
  asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(out) : "v"(y), "v"(ne));
  return out;
}

constexpr int kRunWaves = 4;  // chunks per workgroup, one per wavefront

__global__ __launch_bounds__(64 * kRunWaves) void k_mtf_run(const uint8_t *L, const uint32_t *chunk_base,
                                                            const uint32_t *d_n_chunks, const uint32_t *blk_start,
                                                            const uint32_t *d_nb, const uint8_t *seq,
                                                            const uint8_t *inlist, uint8_t *idx) {
  __shared__ uint8_t rk_all[kRunWaves][256];
  __shared__ uint8_t smap_all[kRunWaves][256];
  __shared__ uint8_t ssym_all[kRunWaves][kChunk];
  const uint32_t wv = threadIdx.x / kWave;
  uint8_t *rk = rk_all[wv], *smap = smap_all[wv], *ssym = ssym_all[wv];
  const uint32_t c = blockIdx.x * kRunWaves + wv;
  const bool have = c < *d_n_chunks;  // every wavefront reaches the barriers below
  uint32_t b = 0, p0 = 0, p1 = 0, bs, be;
  if (have) chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t m = p1 - p0;
  if (have) {
    const uint8_t *il = inlist + (size_t)c * 256;
    for (uint32_t e = lane; e < 256; e += 64) {
      rk[il[e]] = (uint8_t)e;
      smap[e] = seq[b * 256 + e];
    }
    // the chunk's bytes, staged up front (many loads in flight) so that the
    // replay never waits on global memory
    for (uint32_t base = 0; base < m; base += 64 * 16) {
      uint8_t v[16];
#pragma unroll
      for (uint32_t k = 0; k < 16; k++) {
        const uint32_t i = base + k * 64 + lane;
        v[k] = i < m ? L[p0 + i] : (uint8_t)0;
      }
#pragma unroll
      for (uint32_t k = 0; k < 16; k++) {
        const uint32_t i = base + k * 64 + lane;
        if (i < m) ssym[i] = v[k];
      }
    }
  }
  __syncthreads();
  for (uint32_t i = lane; i < m; i += 64) ssym[i] = smap[ssym[i]];
  __syncthreads();
  if (!have) return;
  uint32_t R0 = (uint32_t)rk[lane] | ((uint32_t)rk[lane + 64] << 16);
  uint32_t R1 = (uint32_t)rk[lane + 128] | ((uint32_t)rk[lane + 192] << 16);
  // A symbol equal to the one before it has index 0 and leaves the list as
  // it is (about half the positions of a typical block): only the other
  // positions are replayed.  The chunk's first position is always replayed.
  uint32_t before = 0xFFFFFFFFu;  // symbol at the position before this batch
  for (uint32_t base = p0; base < p1; base += 64) {
    const uint32_t p = base + lane;
    const bool in = p < p1;
    const uint32_t vl = in ? (uint32_t)ssym[p - p0] : 0u;
    uint32_t pv = (uint32_t)__shfl_up((int)vl, 1);
    if (lane == 0) pv = before;
    uint64_t todo = ballot64(in && vl != pv);
    before = (uint32_t)__builtin_amdgcn_readlane((int)vl, 63);
    uint32_t mine = 0;
    while (todo) {
      const uint32_t k = (uint32_t)__builtin_ctzll(todo);
      todo &= todo - 1;
      const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)vl, (int)k);  // wave-uniform
      const uint32_t sl = v & 63u;
      const uint32_t a0 = (uint32_t)__builtin_amdgcn_readlane((int)R0, (int)sl);
      const uint32_t a1 = (uint32_t)__builtin_amdgcn_readlane((int)R1, (int)sl);
      const uint32_t word = (v & 128u) ? a1 : a0;
      // the move-to-front index in the low 16 bits (the high bits are never read:
      // the rank update takes the low half, the index is stored as a byte)
      const uint32_t r = (v & 64u) ? (word >> 16) : word;
      R0 = mtf_ranks(R0, r);
      R1 = mtf_ranks(R1, r);
      // lane k keeps its index (one SGPR operand per instruction: the lane goes through m0)
      asm("s_mov_b32 m0, %2\n\tv_writelane_b32 %0, %1, m0" : "+v"(mine) : "s"(r), "s"(k) : "m0");
    }
    if (in) idx[p] = (uint8_t)mine;
  }
}

// ---------------------------------------------------------------- zero runs
// Every position p of a block belongs to a segment that starts at zs[p]: the
// block start or the position after the last nonzero index.  Its symbol
// count is 1 for a nonzero index, the number of bijective base-2 digits of
// the run at the run's last zero, 0 elsewhere inside a run, plus 1 for the
// end-of-block symbol at the block's last position.  Three launches over
// tiles of 4096 positions (per-tile maxima of the segment-start marks;
// max-scan of the marks (zs) with per-tile symbol counts; exclusive scan of
// the counts), then the symbol output, one workgroup per chunk.

__device__ __forceinline__ uint32_t ndigits(uint32_t r) { return 31u - __clz(r + 1u); }



// A thread owns 16 consecutive positions of the tile (one 16-byte load of
// indices); the bytes just before and after them come from the neighbouring
// lanes.
struct ZBytes {
  uint8_t v[kTItems];
  uint32_t before, after;  // index at p0 - 1 and p0 + 16 (0 outside [0, N))
};

__device__ __forceinline__ ZBytes load_zbytes(const uint8_t *idx, uint32_t p0, uint32_t N) {
  ZBytes z;
  if (p0 + kTItems <= N) {
    const uint4 q = *(const uint4 *)(idx + p0);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < kTItems; i++) z.v[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
  } else {
#pragma unroll
    for (int i = 0; i < kTItems; i++) z.v[i] = p0 + i < N ? idx[p0 + i] : (uint8_t)0;
  }
  const int lane = lane_id();
  z.before = (uint32_t)__shfl_up((int)z.v[kTItems - 1], 1);
  z.after = (uint32_t)__shfl_down((int)z.v[0], 1);
  if (lane == 0) z.before = p0 > 0 && p0 - 1 < N ? idx[p0 - 1] : 0u;
  if (lane == kWave - 1) z.after = p0 + kTItems < N ? idx[p0 + kTItems] : 0u;
  return z;
}

// segment-start mark of position p0 + i (p0 + i < N)
__device__ __forceinline__ uint32_t zmark(const ZBytes &z, int i, uint32_t p, uint32_t bs) {
  const uint32_t prev = i == 0 ? z.before : z.v[i - 1];
  return p == bs || prev != 0 ? p : 0u;
}

// symbols of position p0 + i, whose segment starts at zsp
__device__ __forceinline__ uint32_t zlen(const ZBytes &z, int i, uint32_t p, uint32_t zsp, uint32_t be) {
  const uint32_t next = i == kTItems - 1 ? z.after : z.v[i + 1];
  uint32_t l;
  if (z.v[i] != 0)
    l = 1;
  else if (p + 1 == be || next != 0)
    l = ndigits(p - zsp + 1);
  else
    l = 0;
  return p + 1 == be ? l + 1 : l;  // end-of-block symbol
}

__global__ __launch_bounds__(kTThreads) void k_z_marks(const uint8_t *idx, const uint32_t *d_N,
                                                       const uint32_t *blk_start, const uint32_t *d_nb,
                                                       uint32_t *aggs) {
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t N = *d_N, nb = *d_nb;
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t base = tile * kTTile;
    const TileBlocks tb(blk_start, nb, base);
    const uint32_t p0 = base + threadIdx.x * kTItems;
    const ZBytes z = load_zbytes(idx, p0, N);
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t p = p0 + i;
      if (p < N) {
        uint32_t bs, be;
        tb.find(p, bs, be);
        m = max(m, zmark(z, i, p, bs));
      }
    }
    m = block_reduce<true>(m, sh);
    if (threadIdx.x == 0) aggs[tile] = m;
  }
}

__global__ __launch_bounds__(kTThreads) void k_z_runs(const uint8_t *idx, const uint32_t *d_N,
                                                      const uint32_t *blk_start, const uint32_t *d_nb,
                                                      const uint32_t *aggs_m, uint32_t *zs, uint32_t *aggs_l) {
  __shared__ uint32_t buf[kTPad];
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t N = *d_N, nb = *d_nb;
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  uint32_t carry = 0, counted = 0;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t base = tile * kTTile;
    const uint32_t p0 = base + threadIdx.x * kTItems;
    const ZBytes z = load_zbytes(idx, p0, N);  // issued before the carry's loads
    const TileBlocks tb(blk_start, nb, base);
    carry = tile_carry<true>(aggs_m, counted, tile, carry, sh);
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t p = p0 + i;
      uint32_t mk = 0;
      if (p < N) {
        uint32_t bs, be;
        tb.find(p, bs, be);
        mk = zmark(z, i, p, bs);
      }
      buf[tpad(threadIdx.x * kTItems + i)] = mk;
    }
    __syncthreads();
    tile_scan<true, true>(buf, carry, sh);
    uint32_t cnt = 0, zv[kTItems];
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t p = p0 + i;
      zv[i] = buf[tpad(threadIdx.x * kTItems + i)];
      if (p < N) {
        uint32_t bs, be;
        tb.find(p, bs, be);
        cnt += zlen(z, i, p, zv[i], be);
      }
    }
    if (p0 + kTItems <= N) {
      uint4 *o = (uint4 *)(zs + p0);
#pragma unroll
      for (int q = 0; q < kTItems / 4; q++) o[q] = make_uint4(zv[4 * q], zv[4 * q + 1], zv[4 * q + 2], zv[4 * q + 3]);
    } else {
#pragma unroll
      for (int i = 0; i < kTItems; i++)
        if (p0 + i < N) zs[p0 + i] = zv[i];
    }
    cnt = block_reduce<false>(cnt, sh);
    if (threadIdx.x == 0) aggs_l[tile] = cnt;
  }
}

// Exclusive scan of the symbol counts: off[p] = first symbol of position p;
// the total goes to *d_n_sym.
__global__ __launch_bounds__(kTThreads) void k_z_offs(const uint8_t *idx, const uint32_t *zs, const uint32_t *d_N,
                                                      const uint32_t *blk_start, const uint32_t *d_nb,
                                                      const uint32_t *aggs_l, uint32_t *off, uint32_t *d_n_sym) {
  __shared__ uint32_t buf[kTPad];
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t N = *d_N, nb = *d_nb;
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  if (blockIdx.x == 0 && threadIdx.x == 0 && nt == 0) *d_n_sym = 0;
  uint32_t carry = 0, counted = 0;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t base = tile * kTTile;
    const uint32_t p0 = base + threadIdx.x * kTItems;
    const ZBytes z = load_zbytes(idx, p0, N);  // issued before the carry's loads
    const TileBlocks tb(blk_start, nb, base);
    uint32_t zv[kTItems];
    if (p0 + kTItems <= N) {
      const uint4 *in = (const uint4 *)(zs + p0);
#pragma unroll
      for (int q = 0; q < kTItems / 4; q++) {
        const uint4 t = in[q];
        zv[4 * q] = t.x;
        zv[4 * q + 1] = t.y;
        zv[4 * q + 2] = t.z;
        zv[4 * q + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kTItems; i++) zv[i] = p0 + i < N ? zs[p0 + i] : 0u;
    }
    carry = tile_carry<false>(aggs_l, counted, tile, carry, sh);
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t p = p0 + i;
      uint32_t l = 0;
      if (p < N) {
        uint32_t bs, be;
        tb.find(p, bs, be);
        l = zlen(z, i, p, zv[i], be);
      }
      buf[tpad(threadIdx.x * kTItems + i)] = l;
    }
    __syncthreads();
    const uint32_t total = tile_scan<false, false>(buf, carry, sh);
#pragma unroll
    for (int i = 0; i < kTItems; i++) zv[i] = buf[tpad(threadIdx.x * kTItems + i)];
    if (p0 + kTItems <= N) {
      uint4 *o = (uint4 *)(off + p0);
#pragma unroll
      for (int q = 0; q < kTItems / 4; q++) o[q] = make_uint4(zv[4 * q], zv[4 * q + 1], zv[4 * q + 2], zv[4 * q + 3]);
    } else {
#pragma unroll
      for (int i = 0; i < kTItems; i++)
        if (p0 + i < N) off[p0 + i] = zv[i];
    }
    if (tile == nt - 1 && threadIdx.x == 0) *d_n_sym = carry + total;
    __syncthreads();
  }
}

// Symbol output, one workgroup per chunk: a nonzero index v becomes v + 1, a
// zero run of length r its bijective digits (RUNA = 0, RUNB = 1, least
// significant first), each block ends with n_in_use + 1; per-block symbol
// frequencies, first symbol and count.
__global__ __launch_bounds__(256) void k_rle2_write(const uint8_t *idx, const uint32_t *zs, const uint32_t *off,
                                                    const uint32_t *chunk_base, const uint32_t *d_n_chunks,
                                                    const uint32_t *blk_start, const uint32_t *d_nb,
                                                    BlockCode *codes, uint16_t *sym, uint32_t *freq) {
  __shared__ uint32_t f[kMaxAlpha];
  const uint32_t c = blockIdx.x;
  if (c >= *d_n_chunks) return;
  uint32_t b, p0, p1, bs, be;
  chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  for (int i = threadIdx.x; i < kMaxAlpha; i += 256) f[i] = 0;
  __syncthreads();
  const uint32_t nu = codes[b].n_in_use;
  for (uint32_t p = p0 + threadIdx.x; p < p1; p += 256) {
    uint32_t o = off[p];
    const uint32_t v = idx[p];
    if (v != 0) {
      sym[o++] = (uint16_t)(v + 1);
      atomicAdd(&f[v + 1], 1u);
    } else if (p + 1 == be || idx[p + 1] != 0) {
      uint32_t r = p - zs[p] + 1;
      while (r > 0) {
        const uint32_t d = (r & 1u) ? 0u : 1u;
        sym[o++] = (uint16_t)d;
        atomicAdd(&f[d], 1u);
        r = (r - 1u - d) >> 1;
      }
    }
    if (p + 1 == be) {
      sym[o] = (uint16_t)(nu + 1);
      atomicAdd(&f[nu + 1], 1u);
      codes[b].sym_start = off[bs];
      codes[b].n_mtf = o + 1 - off[bs];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kMaxAlpha; i += 256)
    if (f[i]) atomicAdd(&freq[b * kMaxAlpha + i], f[i]);
}

}  // namespace

void launch_mtf2(const uint8_t *L, const uint32_t *d_N, uint32_t N, const uint32_t *blk_start, const uint32_t *d_nb, uint32_t max_blocks,
                 uint32_t max_chunks, MtfWork w, BlockCode *codes, uint16_t *sym, uint32_t *freq,
                 uint32_t *d_n_sym, hipStream_t s) {
  PCBZ_LAUNCH(k_mtf_chunks, dim3(1), dim3(64), 0, s, blk_start, d_nb, w.chunk_block, w.d_n_chunks, codes);
  const uint32_t *cb = w.chunk_block;
  PCBZ_LAUNCH(k_used, dim3(max_chunks), dim3(256), 0, s, L, cb, w.d_n_chunks, blk_start, d_nb, w.used_chunk);
  PCBZ_LAUNCH(k_seq, dim3(max_blocks), dim3(256), 0, s, w.used_chunk, w.used, d_nb, w.seq, codes);
  PCBZ_LAUNCH(k_mtf_partial, dim3(max_chunks), dim3(64), 0, s, L, cb, w.d_n_chunks, blk_start, d_nb, w.seq,
                     w.plist, w.plen);
  PCBZ_LAUNCH(k_mtf_seg_fold, dim3(kMtfSegs, max_blocks), dim3(256), 0, s, d_nb, codes, w.plist, w.plen, w.seglist,
              w.seglen);
  PCBZ_LAUNCH(k_mtf_seg_chain, dim3(max_blocks), dim3(256), 0, s, d_nb, w.seglist, w.seglen);
  PCBZ_LAUNCH(k_mtf_chain, dim3(kMtfSegs, max_blocks), dim3(256), 0, s, d_nb, codes, w.plist, w.plen, w.seglist,
              w.inlist);
  PCBZ_LAUNCH(k_mtf_run, dim3((max_chunks + kRunWaves - 1) / kRunWaves), dim3(64 * kRunWaves), 0, s, L, cb,
              w.d_n_chunks, blk_start, d_nb, w.seq,
                     w.inlist, w.idx);
  const uint32_t gt = std::max<uint32_t>(1, std::min<uint32_t>(2048, (N + kTTile - 1) / kTTile));
  uint32_t *aggs_m = w.aggs, *aggs_l = w.aggs + (N / kTTile + 2);
  PCBZ_LAUNCH(k_z_marks, dim3(gt), dim3(kTThreads), 0, s, w.idx, d_N, blk_start, d_nb, aggs_m);
  PCBZ_LAUNCH(k_z_runs, dim3(gt), dim3(kTThreads), 0, s, w.idx, d_N, blk_start, d_nb, aggs_m, w.zs, aggs_l);
  PCBZ_LAUNCH(k_z_offs, dim3(gt), dim3(kTThreads), 0, s, w.idx, w.zs, d_N, blk_start, d_nb, aggs_l, w.off, d_n_sym);
  PCBZ_LAUNCH(k_rle2_write, dim3(max_chunks), dim3(256), 0, s, w.idx, w.zs, w.off, cb, w.d_n_chunks, blk_start, d_nb,
              codes, sym, freq);
}

}  // namespace pcbz
