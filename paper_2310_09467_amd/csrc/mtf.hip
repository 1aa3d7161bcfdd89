// mtf.hip -- move-to-front and the zero-run stage of bzip2.
//
// Move-to-front is sequential per block, so each block is cut into chunks of
// kMtfChunk positions.  The list after a chunk depends on the list before it only
// through a fixed rule: the chunk's distinct symbols in order of last
// occurrence (most recent first) move to the front, the rest keep their
// order.  So (1) every chunk computes that partial list, (2) the partial lists
// are chained (in three shallow steps) into each chunk's incoming list, and
// (3) every chunk replays move-to-front from its incoming list (k_mtf_run).
// Lists hold byte values.  A block's initial list is its used bytes in
// ascending order (the order of the format's symbol map, so a list position
// is the format's index), then the unused bytes, which never move.  Chunks
// are short (256 positions): the replay's cost per chunk varies with the
// data (runs are skipped, symbols deep in the list cost more), and short
// chunks keep the slowest wavefront close to the average.
//
// Zero runs: a run of r zero indices becomes the bijective base-2 digits of
// r, least significant first (RUNA = 0 for digit 1, RUNB = 1 for digit 2); a
// non-zero index v becomes v + 1; each block ends with nInUse + 1.
#include <algorithm>

#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr uint32_t kChunk = kMtfChunk;
static_assert(kChunk % 64 == 0 && kChunk <= 1024, "a chunk is replayed from registers, 64 positions a batch");

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

// The partial list of a chunk orders its bytes by last occurrence, latest
// first: walking the chunk backwards, it is the sequence of positions that
// hold the last occurrence of their byte.  Lane l takes the kPer positions
// p1 - 1 - kPer l down to p1 - kPer (l + 1); a wavefront prefix count of the
// flagged positions gives each its place in the list.
__global__ __launch_bounds__(64) void k_mtf_partial(const uint8_t *L, const uint32_t *chunk_base,
                                                    const uint32_t *d_n_chunks, const uint32_t *blk_start,
                                                    const uint32_t *d_nb, uint8_t *plist, uint32_t *plen) {
  __shared__ int lastpos[256];
  const uint32_t c = blockIdx.x;
  if (c >= *d_n_chunks) return;
  uint32_t b, p0, p1, bs, be;
  chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  for (int v = threadIdx.x; v < 256; v += 64) lastpos[v] = -1;
  __syncthreads();
  constexpr uint32_t kPer = kChunk / 64;
  const uint32_t n = p1 - p0, lane = threadIdx.x;
  uint8_t sy[kPer];
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const uint32_t q = lane * kPer + i;
    sy[i] = q < n ? L[p1 - 1 - q] : (uint8_t)0;
  }
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const uint32_t q = lane * kPer + i;
    if (q < n) atomicMax(&lastpos[sy[i]], (int)(n - 1 - q));
  }
  __syncthreads();
  uint32_t flags = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const uint32_t q = lane * kPer + i;
    if (q < n && lastpos[sy[i]] == (int)(n - 1 - q)) flags |= 1u << i;
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
  (void)b;
}

// List chaining.  Folding a partial list P onto a list C gives P followed by
// C without P's symbols (order kept); folding is associative, so a block's
// chunks are chained in three shallow steps instead of one long one:
//   1. each of kMtfSegs segments of the block folds its chunks' partial lists
//      (from an empty list) into a segment partial list;
//   2. one wavefront per block takes the block's used bytes from the segment
//      lists, builds the initial list and folds the segment lists onto it,
//      recording the list entering each segment;
//   3. each segment folds its chunks again from its entering list, recording
//      the list entering each chunk.
// Every step is one wavefront with its lists staged in LDS up front; a list
// of up to 256 bytes sits in four registers (lane l holds positions l,
// l + 64, l + 128, l + 192) and a fold step needs no workgroup barrier.

// cur/len := P ++ (cur - P), P given as pv (lane l: positions l + 64 k) of
// length pl.  mark[x] == stamp flags the bytes of P (stamps grow by one per
// step, so mark is never cleared); buf is the new list.  Branch-free: lanes
// with nothing to write write to their own slot past the 256 entries, so
// each group of LDS accesses goes out at once (three round trips a step).
constexpr uint32_t kFoldSlots = 256 + 64;

__device__ __forceinline__ void wave_fold(uint32_t (&cur)[4], uint32_t &len, const uint32_t (&pv)[4], uint32_t pl,
                                          uint32_t stamp, uint32_t *mark, uint8_t *buf) {
  const uint32_t lane = (uint32_t)lane_id();
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) mark[lane + 64 * k < pl ? pv[k] : 256 + lane] = stamp;
  __builtin_amdgcn_wave_barrier();
  uint32_t mk[4];
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) mk[k] = mark[cur[k]];  // cur holds bytes, also past len
  const uint64_t lt = lanemask_lt();
  uint32_t base = pl;
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) {
    const bool keep = lane + 64 * k < len && mk[k] != stamp;
    const uint64_t bal = ballot64(keep);
    buf[keep ? base + (uint32_t)__popcll(bal & lt) : 256 + lane] = (uint8_t)cur[k];
    base += (uint32_t)__popcll(bal);
  }
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) buf[lane + 64 * k < pl ? lane + 64 * k : 256 + lane] = (uint8_t)pv[k];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) cur[k] = buf[lane + 64 * k];
  len = base;
}

// list i of the LDS-staged lists, lane l taking positions l + 64 k
__device__ __forceinline__ void lds_list(uint32_t (&pv)[4], const uint8_t *lists, uint32_t i) {
  const uint32_t lane = (uint32_t)lane_id();
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) pv[k] = lists[i * 256 + lane + 64 * k];
}

// folds the staged lists [0, n) onto cur (stamps 1..n); before fold i the
// list is written to out + i * 256 when out is set.  The next list is read
// while the current fold runs.
__device__ __forceinline__ void fold_staged(uint32_t (&cur)[4], uint32_t &len, const uint8_t *lists,
                                            const uint32_t *lens, uint32_t n, uint32_t *mark, uint8_t *buf,
                                            uint8_t *out) {
  const uint32_t lane = (uint32_t)lane_id();
  if (n == 0) return;
  uint32_t pv[4];
  lds_list(pv, lists, 0);
  for (uint32_t i = 0; i < n; i++) {
    if (out) {
#pragma unroll
      for (uint32_t k = 0; k < 4; k++) out[(size_t)i * 256 + lane + 64 * k] = (uint8_t)cur[k];
    }
    uint32_t nx[4];
    lds_list(nx, lists, min(i + 1, n - 1));
    wave_fold(cur, len, pv, lens[i], i + 1, mark, buf);
#pragma unroll
    for (uint32_t k = 0; k < 4; k++) pv[k] = nx[k];
  }
}

__device__ __forceinline__ void seg_range(const BlockCode &C, uint32_t j, uint32_t &u0, uint32_t &u1) {
  const uint32_t per = (C.n_chunks + kMtfSegs - 1) / kMtfSegs;
  u0 = min(C.n_chunks, j * per);
  u1 = min(C.n_chunks, u0 + per);
}

// the partial lists of chunks [c0, c0 + n) into LDS
__device__ __forceinline__ void stage_lists(uint8_t *lists, uint32_t *lens, const uint8_t *plist,
                                            const uint32_t *plen, uint32_t c0, uint32_t n) {
  stage_to_lds((uint32_t *)lists, (const uint32_t *)(plist + (size_t)c0 * 256), n * 64);
  stage_to_lds(lens, plen + c0, n);
}

struct FoldLds {
  uint8_t lists[kMtfUnits * 256];
  uint32_t lens[kMtfUnits];
  uint32_t mark[kFoldSlots];
  uint8_t buf[kFoldSlots];
};

// step 1: grid (kMtfSegs, blocks), one wavefront each
__global__ __launch_bounds__(64) void k_mtf_seg_fold(const uint32_t *d_nb, const BlockCode *codes,
                                                     const uint8_t *plist, const uint32_t *plen, uint8_t *seglist,
                                                     uint32_t *seglen) {
  __shared__ FoldLds F;
  const uint32_t b = blockIdx.y, j = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  uint32_t u0, u1;
  seg_range(C, j, u0, u1);
  const uint32_t n = u1 - u0, lane = (uint32_t)lane_id();
  stage_lists(F.lists, F.lens, plist, plen, C.chunk_start + u0, n);
  for (uint32_t e = lane; e < kFoldSlots; e += 64) F.mark[e] = 0;
  __syncthreads();
  uint32_t cur[4] = {0, 0, 0, 0}, len = 0;
  fold_staged(cur, len, F.lists, F.lens, n, F.mark, F.buf, nullptr);
  uint8_t *o = seglist + ((size_t)b * kMtfSegs + j) * 256;
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) o[lane + 64 * k] = (uint8_t)cur[k];
  if (lane == 0) seglen[(size_t)b * kMtfSegs + j] = len;
}

// step 2: one wavefront per block; also writes the block's used-byte bitmap
// and symbol-map size.  The segment lists are replaced by the lists entering
// the segments.
__global__ __launch_bounds__(64) void k_mtf_seg_chain(const uint32_t *d_nb, uint8_t *seglist, const uint32_t *seglen,
                                                      uint32_t *used, BlockCode *codes) {
  __shared__ uint8_t lists[kMtfSegs * 256];
  __shared__ uint32_t lens[kMtfSegs];
  __shared__ uint32_t mark[kFoldSlots];
  __shared__ uint8_t buf[kFoldSlots];
  const uint32_t b = blockIdx.x;
  if (b >= *d_nb) return;
  const uint32_t lane = (uint32_t)lane_id();
  uint8_t *sl = seglist + (size_t)b * kMtfSegs * 256;
  stage_lists(lists, lens, sl, seglen + (size_t)b * kMtfSegs, 0, kMtfSegs);
  for (uint32_t e = lane; e < kFoldSlots; e += 64) mark[e] = 0;
  __syncthreads();
  // the block's used bytes: every byte of a segment list
  for (uint32_t i = 0; i < kMtfSegs; i++) {
    const uint32_t l = lens[i];
    for (uint32_t e = lane; e < l; e += 64) mark[lists[i * 256 + e]] = 1;
  }
  __syncthreads();
  uint64_t ub[4];
  uint32_t nu = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) {
    ub[k] = ballot64(mark[lane + 64 * k] != 0);
    nu += (uint32_t)__popcll(ub[k]);
  }
  if (lane == 0) {
#pragma unroll
    for (uint32_t w = 0; w < 8; w++) used[b * 8 + w] = (uint32_t)(ub[w / 2] >> (32 * (w % 2)));
    codes[b].n_in_use = nu;
    codes[b].alpha = nu + 2;
  }
  // initial list: used bytes ascending, then the unused ones
  const uint64_t lt = lanemask_lt();
  uint32_t nbu = 0, nbn = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) {
    const bool u = (ub[k] >> lane) & 1ull;
    const uint32_t pos = u ? nbu + (uint32_t)__popcll(ub[k] & lt) : nu + nbn + (uint32_t)__popcll(~ub[k] & lt);
    buf[pos] = (uint8_t)(lane + 64 * k);
    nbu += (uint32_t)__popcll(ub[k]);
    nbn += 64u - (uint32_t)__popcll(ub[k]);
  }
  __syncthreads();
  uint32_t cur[4], len = 256;
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) {
    cur[k] = buf[lane + 64 * k];
    mark[lane + 64 * k] = 0;
  }
  __syncthreads();
  // the last segment's fold is not needed (its result is the block's end)
  fold_staged(cur, len, lists, lens, kMtfSegs - 1, mark, buf, sl);
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) sl[(kMtfSegs - 1) * 256 + lane + 64 * k] = (uint8_t)cur[k];
}

// step 3: grid (kMtfSegs, blocks), one wavefront each
__global__ __launch_bounds__(64) void k_mtf_chain(const uint32_t *d_nb, const BlockCode *codes, const uint8_t *plist,
                                                  const uint32_t *plen, const uint8_t *seglist, uint8_t *inlist) {
  __shared__ FoldLds F;
  const uint32_t b = blockIdx.y, j = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  uint32_t u0, u1;
  seg_range(C, j, u0, u1);
  if (u0 >= u1) return;
  const uint32_t n = u1 - u0, lane = (uint32_t)lane_id();
  stage_lists(F.lists, F.lens, plist, plen, C.chunk_start + u0, n);
  const uint8_t *si = seglist + ((size_t)b * kMtfSegs + j) * 256;
  uint32_t cur[4], len = 256;
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) cur[k] = si[lane + 64 * k];
  for (uint32_t e = lane; e < kFoldSlots; e += 64) F.mark[e] = 0;
  __syncthreads();
  uint8_t *o = inlist + (size_t)(C.chunk_start + u0) * 256;
  fold_staged(cur, len, F.lists, F.lens, n - 1, F.mark, F.buf, o);
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) o[(size_t)(n - 1) * 256 + lane + 64 * k] = (uint8_t)cur[k];
}

// Replay of one chunk by one wavefront.  The list itself is held in four
// registers: lane l of Q[i] holds list position 64 i + l, as the byte value
// there.  A step finds its symbol by one compare with Q[0] (with
// Q[1..3] only when it is not among the first 64 entries), then moves it to
// the front: the entries in front of it shift back by one lane with a
// wavefront shift (DPP wave_shr:1), the symbol enters lane 0 of Q[0], and a
// register shifted whole passes its lane 63 on to lane 0 of the next one.
// For LFM data most non-zero indices are below 64.
//
// mtf_batch replays the positions of `todo` (lanes of the batch vl) in
// order; lane k of `mine` takes the index of position k.  A symbol among
// the first 64 entries (lane q of Q0) costs six vector and six scalar
// instructions: lanes 0..q of Q0 take Q0 shifted by one lane, lane 0 the
// symbol.  A deeper one (lane q of Q[j], j >= 1) shifts Q[0..j-1] whole
// (each passing its lane 63 on to lane 0 of the next) and lanes 0..q of
// Q[j].  The lane number lives in m0 (v_readlane / v_writelane select).
// All 64 lanes hold list entries, so the loop runs with the full exec mask
// (set here, five wait states before the first DPP, restored at the end);
// a DPP source needs two wait states after a vector write: the fast path's
// was written a dozen instructions earlier, the others get an s_nop.
__device__ __forceinline__ void mtf_batch(uint32_t &Q0, uint32_t &Q1, uint32_t &Q2, uint32_t &Q3, uint32_t &mine,
                                          uint64_t todo, uint32_t vl) {
  uint32_t v, q, c0, c1, c2, t;
  uint64_t mq, m1, m2, mk, ex;
  asm volatile(
      "s_mov_b64 %[ex], exec\n\t"
      "s_mov_b64 exec, -1\n\t"
      "s_nop 4\n"
      "1:\n\t"
      "s_cmp_eq_u64 %[todo], 0\n\t"
      "s_cbranch_scc1 9f\n\t"
      "s_ff1_i32_b64 m0, %[todo]\n\t"
      "s_bitset0_b64 %[todo], m0\n\t"
      "v_readlane_b32 %[v], %[vl], m0\n\t"
      "v_cmp_eq_u32_e64 %[mq], %[v], %[Q0]\n\t"
      "s_cmp_eq_u64 %[mq], 0\n\t"
      "s_cbranch_scc1 2f\n\t"
      // in Q0 at lane q
      "s_ff1_i32_b64 %[q], %[mq]\n\t"
      "s_lshl_b64 %[mk], -2, %[q]\n\t"
      "v_mov_b32 %[t], %[v]\n\t"
      "v_mov_b32_dpp %[t], %[Q0] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_cndmask_b32_e64 %[Q0], %[t], %[Q0], %[mk]\n\t"
      "v_writelane_b32 %[mine], %[q], m0\n\t"
      "s_branch 1b\n"
      // deeper: Q0 shifts whole
      "2:\n\t"
      "v_cmp_eq_u32_e64 %[m1], %[v], %[Q1]\n\t"
      "v_cmp_eq_u32_e64 %[m2], %[v], %[Q2]\n\t"
      "v_cmp_eq_u32_e64 %[mq], %[v], %[Q3]\n\t"
      "v_readlane_b32 %[c0], %[Q0], 63\n\t"
      "v_readlane_b32 %[c1], %[Q1], 63\n\t"
      "v_readlane_b32 %[c2], %[Q2], 63\n\t"
      "s_nop 1\n\t"
      "v_mov_b32_dpp %[Q0], %[Q0] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_writelane_b32 %[Q0], %[v], 0\n\t"
      "s_cmp_eq_u64 %[m1], 0\n\t"
      "s_cbranch_scc1 3f\n\t"
      // in Q1 at lane q
      "s_ff1_i32_b64 %[q], %[m1]\n\t"
      "s_lshl_b64 %[mk], -2, %[q]\n\t"
      "v_mov_b32 %[t], %[c0]\n\t"
      "s_nop 1\n\t"
      "v_mov_b32_dpp %[t], %[Q1] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_cndmask_b32_e64 %[Q1], %[t], %[Q1], %[mk]\n\t"
      "s_add_u32 %[q], %[q], 64\n\t"
      "v_writelane_b32 %[mine], %[q], m0\n\t"
      "s_branch 1b\n"
      // deeper: Q1 shifts whole
      "3:\n\t"
      "s_nop 1\n\t"
      "v_mov_b32_dpp %[Q1], %[Q1] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_writelane_b32 %[Q1], %[c0], 0\n\t"
      "s_cmp_eq_u64 %[m2], 0\n\t"
      "s_cbranch_scc1 4f\n\t"
      // in Q2 at lane q
      "s_ff1_i32_b64 %[q], %[m2]\n\t"
      "s_lshl_b64 %[mk], -2, %[q]\n\t"
      "v_mov_b32 %[t], %[c1]\n\t"
      "s_nop 1\n\t"
      "v_mov_b32_dpp %[t], %[Q2] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_cndmask_b32_e64 %[Q2], %[t], %[Q2], %[mk]\n\t"
      "s_add_u32 %[q], %[q], 128\n\t"
      "v_writelane_b32 %[mine], %[q], m0\n\t"
      "s_branch 1b\n"
      // in Q3 at lane q (every used byte is in the list): Q2 shifts whole
      "4:\n\t"
      "s_nop 1\n\t"
      "v_mov_b32_dpp %[Q2], %[Q2] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_writelane_b32 %[Q2], %[c1], 0\n\t"
      "s_ff1_i32_b64 %[q], %[mq]\n\t"
      "s_lshl_b64 %[mk], -2, %[q]\n\t"
      "v_mov_b32 %[t], %[c2]\n\t"
      "s_nop 1\n\t"
      "v_mov_b32_dpp %[t], %[Q3] wave_shr:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_cndmask_b32_e64 %[Q3], %[t], %[Q3], %[mk]\n\t"
      "s_add_u32 %[q], %[q], 192\n\t"
      "v_writelane_b32 %[mine], %[q], m0\n\t"
      "s_branch 1b\n"
      "9:\n\t"
      "s_mov_b64 exec, %[ex]"
      : [Q0] "+v"(Q0), [Q1] "+v"(Q1), [Q2] "+v"(Q2), [Q3] "+v"(Q3), [mine] "+v"(mine), [todo] "+s"(todo),
        [v] "=&s"(v), [q] "=&s"(q), [c0] "=&s"(c0), [c1] "=&s"(c1), [c2] "=&s"(c2), [mq] "=&s"(mq), [m1] "=&s"(m1),
        [m2] "=&s"(m2), [mk] "=&s"(mk), [t] "=&v"(t), [ex] "=&s"(ex)
      : [vl] "v"(vl)
      : "scc", "m0");
}

// wavefront shift right by one lane; lane 0 takes `in`
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x, uint32_t in) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)in, (int)x, 0x138, 0xf, 0xf, false);
}

constexpr int kRunWaves = 4;  // chunks per workgroup, one per wavefront

__global__ __launch_bounds__(64 * kRunWaves) void k_mtf_run(const uint8_t *L, const uint32_t *chunk_base,
                                                            const uint32_t *d_n_chunks, const uint32_t *blk_start,
                                                            const uint32_t *d_nb, const uint8_t *inlist,
                                                            uint8_t *idx) {
  const uint32_t c = blockIdx.x * kRunWaves + threadIdx.x / kWave;
  if (c >= *d_n_chunks) return;  // the wavefronts of a workgroup are independent
  uint32_t b, p0, p1, bs, be;
  chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t m = p1 - p0;
  // the chunk's bytes, lane l holding positions l, l + 64, ... (all loads in
  // flight at once, so that the replay never waits on global memory)
  uint32_t sy[kChunk / 64];
#pragma unroll
  for (uint32_t k = 0; k < kChunk / 64; k++) {
    const uint32_t i = k * 64 + lane;
    sy[k] = i < m ? (uint32_t)L[p0 + i] : 0x200u;
  }
  const uint8_t *il = inlist + (size_t)c * 256;
  uint32_t Q0 = il[lane], Q1 = il[lane + 64], Q2 = il[lane + 128], Q3 = il[lane + 192];
  // A symbol equal to the one before it has index 0 and leaves the list as
  // it is (about half the positions of a typical block): only the other
  // positions are replayed.  The chunk's first position is always replayed.
  uint32_t before = 0xFFFFFFFFu;  // symbol at the position before this batch
#pragma unroll
  for (uint32_t k = 0; k < kChunk / 64; k++) {
    if (k * 64 >= m) break;
    const uint32_t vl = sy[k];
    const bool in = k * 64 + lane < m;
    const uint32_t pv = wave_shr1(vl, before);
    uint64_t todo = ballot64(in && vl != pv);
    before = (uint32_t)__builtin_amdgcn_readlane((int)vl, 63);
    uint32_t mine = 0;
    mtf_batch(Q0, Q1, Q2, Q3, mine, todo, vl);
    if (in) idx[p0 + k * 64 + lane] = (uint8_t)mine;
  }
}

// ---------------------------------------------------------------- zero runs
// Every position p of a block belongs to a segment that starts at zs[p]: the
// block start or the position after the last nonzero index.  Its symbol
// count is 1 for a nonzero index, the number of bijective base-2 digits of
// the run at the run's last zero, 0 elsewhere inside a run, plus 1 for the
// end-of-block symbol at the block's last position.  Three launches over
// tiles of 4096 positions: per-tile maxima of the segment-start marks;
// max-scan of the marks (zs) with per-tile symbol counts; exclusive scan of
// the counts, which places the tile's symbols (staged in LDS, then written
// out in one coalesced run) and counts their frequencies per block.

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

// Exclusive scan of the symbol counts gives each position its first symbol;
// the symbols go out here.  A tile holds at most kTTile positions' symbols,
// plus the digits of a run that began in an earlier tile (< 32) and one
// end-of-block symbol per block that ends in it (<= kTTile).
constexpr uint32_t kZStage = 2 * kTTile + 64;

__device__ __forceinline__ void zcount(uint32_t *f, uint32_t *freq, uint32_t b, uint32_t b0, uint32_t s) {
  if (b == b0)
    atomicAdd(&f[s], 1u);
  else
    atomicAdd(&freq[b * kMaxAlpha + s], 1u);  // a block that starts inside the tile (rare)
}

__global__ __launch_bounds__(kTThreads) void k_z_write(const uint8_t *idx, const uint32_t *zs, const uint32_t *d_N,
                                                       const uint32_t *blk_start, const uint32_t *d_nb,
                                                       const uint32_t *aggs_l, BlockCode *codes, uint16_t *sym,
                                                       uint32_t *freq, uint32_t *d_n_sym) {
  __shared__ uint32_t buf[kTPad];
  __shared__ uint32_t sh[kTThreads / kWave];
  __shared__ uint32_t f[kMaxAlpha];
  __shared__ uint16_t stage[kZStage];
  const uint32_t N = *d_N, nb = *d_nb;
  const uint32_t nt = (N + kTTile - 1) / kTTile;
  if (blockIdx.x == 0 && threadIdx.x == 0 && nt == 0) *d_n_sym = 0;
  uint32_t carry = 0, counted = 0;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t base = tile * kTTile;
    const uint32_t p0 = base + threadIdx.x * kTItems;
    for (uint32_t i = threadIdx.x; i < kMaxAlpha; i += kTThreads) f[i] = 0;  // ordered by the reduction's barriers
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
    const uint32_t total = tile_scan<false, false>(buf, 0, sh);  // offsets inside the tile
#pragma unroll
    for (int i = 0; i < kTItems; i++) {
      const uint32_t p = p0 + i;
      if (p >= N) break;
      uint32_t bs, be;
      const uint32_t b = tb.find(p, bs, be);
      uint32_t o = buf[tpad(threadIdx.x * kTItems + i)];
      if (p == bs) codes[b].sym_start = carry + o;
      const uint32_t v = z.v[i];
      const uint32_t next = i == kTItems - 1 ? z.after : z.v[i + 1];
      if (v != 0) {
        stage[o++] = (uint16_t)(v + 1);
        zcount(f, freq, b, tb.b0, v + 1);
      } else if (p + 1 == be || next != 0) {
        uint32_t r = p - zv[i] + 1;
        while (r > 0) {
          const uint32_t d = (r & 1u) ? 0u : 1u;
          stage[o++] = (uint16_t)d;
          zcount(f, freq, b, tb.b0, d);
          r = (r - 1u - d) >> 1;
        }
      }
      if (p + 1 == be) {
        const uint32_t eob = codes[b].n_in_use + 1;
        stage[o] = (uint16_t)eob;
        zcount(f, freq, b, tb.b0, eob);
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < total; i += kTThreads) sym[carry + i] = stage[i];
    for (uint32_t i = threadIdx.x; i < kMaxAlpha; i += kTThreads)
      if (f[i]) atomicAdd(&freq[tb.b0 * kMaxAlpha + i], f[i]);
    if (tile == nt - 1 && threadIdx.x == 0) *d_n_sym = carry + total;
    __syncthreads();
  }
}

// symbols per block, from the block starts and the total
__global__ void k_mtf_ends(const uint32_t *d_nb, const uint32_t *d_n_sym, BlockCode *codes) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x, nb = *d_nb;
  if (b < nb) codes[b].n_mtf = (b + 1 < nb ? codes[b + 1].sym_start : *d_n_sym) - codes[b].sym_start;
}

}  // namespace

void launch_mtf2(const uint8_t *L, const uint32_t *d_N, uint32_t N, const uint32_t *blk_start, const uint32_t *d_nb, uint32_t max_blocks,
                 uint32_t max_chunks, MtfWork w, BlockCode *codes, uint16_t *sym, uint32_t *freq,
                 uint32_t *d_n_sym, hipStream_t s) {
  PCBZ_LAUNCH(k_mtf_chunks, dim3(1), dim3(64), 0, s, blk_start, d_nb, w.chunk_block, w.d_n_chunks, codes);
  const uint32_t *cb = w.chunk_block;
  PCBZ_LAUNCH(k_mtf_partial, dim3(max_chunks), dim3(64), 0, s, L, cb, w.d_n_chunks, blk_start, d_nb, w.plist, w.plen);
  PCBZ_LAUNCH(k_mtf_seg_fold, dim3(kMtfSegs, max_blocks), dim3(64), 0, s, d_nb, codes, w.plist, w.plen, w.seglist,
              w.seglen);
  PCBZ_LAUNCH(k_mtf_seg_chain, dim3(max_blocks), dim3(64), 0, s, d_nb, w.seglist, w.seglen, w.used, codes);
  PCBZ_LAUNCH(k_mtf_chain, dim3(kMtfSegs, max_blocks), dim3(64), 0, s, d_nb, codes, w.plist, w.plen, w.seglist,
              w.inlist);
  PCBZ_LAUNCH(k_mtf_run, dim3((max_chunks + kRunWaves - 1) / kRunWaves), dim3(64 * kRunWaves), 0, s, L, cb,
              w.d_n_chunks, blk_start, d_nb, w.inlist, w.idx);
  const uint32_t gt = std::max<uint32_t>(1, std::min<uint32_t>(2048, (N + kTTile - 1) / kTTile));
  uint32_t *aggs_m = w.aggs, *aggs_l = w.aggs + (N / kTTile + 2);
  PCBZ_LAUNCH(k_z_marks, dim3(gt), dim3(kTThreads), 0, s, w.idx, d_N, blk_start, d_nb, aggs_m);
  PCBZ_LAUNCH(k_z_runs, dim3(gt), dim3(kTThreads), 0, s, w.idx, d_N, blk_start, d_nb, aggs_m, w.zs, aggs_l);
  PCBZ_LAUNCH(k_z_write, dim3(gt), dim3(kTThreads), 0, s, w.idx, w.zs, d_N, blk_start, d_nb, aggs_l, codes, sym, freq,
              d_n_sym);
  PCBZ_LAUNCH(k_mtf_ends, dim3((max_blocks + 255) / 256), dim3(256), 0, s, d_nb, d_n_sym, codes);
}

}  // namespace pcbz
