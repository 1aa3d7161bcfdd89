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

// block and positions of chunk c (wave-uniform).  With fewer than 64 blocks
// lane l loads block l's first chunk and start (one round trip instead of a
// chain of dependent loads) and a ballot finds the block.
__device__ __forceinline__ void chunk_range(uint32_t c, const uint32_t *chunk_base, const uint32_t *blk_start,
                                            uint32_t nb, uint32_t &b, uint32_t &p0, uint32_t &p1, uint32_t &bs,
                                            uint32_t &be) {
  uint32_t cb;
  if (nb < (uint32_t)kWave) {
    const uint32_t lane = (uint32_t)lane_id();
    const uint32_t mc = lane <= nb ? chunk_base[lane] : 0xFFFFFFFFu;
    const uint32_t ms = lane <= nb ? blk_start[lane] : 0u;
    b = (uint32_t)__popcll(ballot64(lane < nb && mc <= c)) - 1u;
    cb = (uint32_t)__shfl((int)mc, (int)b);
    bs = (uint32_t)__shfl((int)ms, (int)b);
    be = (uint32_t)__shfl((int)ms, (int)b + 1);
  } else {
    b = upper_index(chunk_base, nb, c);
    cb = chunk_base[b];
    bs = blk_start[b];
    be = blk_start[b + 1];
  }
  p0 = bs + (c - cb) * kChunk;
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
constexpr uint32_t kPartWaves = 4;  // chunks per workgroup, one per wavefront

__global__ __launch_bounds__(64 * kPartWaves) void k_mtf_partial(const uint8_t *L, const uint32_t *chunk_base,
                                                                const uint32_t *d_n_chunks, const uint32_t *blk_start,
                                                                const uint32_t *d_nb, uint8_t *plist, uint32_t *plen) {
  __shared__ int lastpos_all[kPartWaves][256];
  const uint32_t c = blockIdx.x * kPartWaves + threadIdx.x / kWave;
  if (c >= *d_n_chunks) return;  // the wavefronts of a workgroup are independent
  int *lastpos = lastpos_all[threadIdx.x / kWave];
  uint32_t b, p0, p1, bs, be;
  chunk_range(c, chunk_base, blk_start, *d_nb, b, p0, p1, bs, be);
  constexpr uint32_t kPer = kChunk / 64;
  const uint32_t n = p1 - p0, lane = (uint32_t)lane_id();
  uint8_t sy[kPer];
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const uint32_t q = lane * kPer + i;
    sy[i] = q < n ? L[p1 - 1 - q] : (uint8_t)0;
  }
  for (uint32_t v = lane; v < 256; v += 64) lastpos[v] = -1;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (uint32_t i = 0; i < kPer; i++) {
    const uint32_t q = lane * kPer + i;
    if (q < n) atomicMax(&lastpos[sy[i]], (int)(n - 1 - q));
  }
  __builtin_amdgcn_wave_barrier();
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
// chunks are chained in three steps:
//   1. each of kMtfSegs segments of the block combines its chunks' partial
//      lists into a segment partial list;
//   2. one workgroup per block takes the block's used bytes from the segment
//      lists, builds the initial list and computes the list entering each
//      segment;
//   3. each segment computes the list entering each of its chunks from the
//      list entering the segment.
// Each step is a workgroup of W wavefronts with its lists staged in LDS.  A list of up to 256 bytes sits in four registers of a wavefront (lane
// l holds positions l, l + 64, l + 128, l + 192); one fold step needs no
// workgroup barrier.  Inside a step the n lists are split into W groups:
// each wavefront combines its group (n / W folds), a Hillis-Steele scan
// combines the group lists (log2 W folds), and
// each wavefront replays its group from the list entering it.

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

__device__ __forceinline__ void seg_range(const BlockCode &C, uint32_t j, uint32_t &u0, uint32_t &u1) {
  const uint32_t per = (C.n_chunks + kMtfSegs - 1) / kMtfSegs;
  u0 = min(C.n_chunks, j * per);
  u1 = min(C.n_chunks, u0 + per);
}

// wavefronts per workgroup: the per-block step has one workgroup per block
// and takes 16; the per-segment steps have one per segment (640 for ten
// blocks) and take 8, so that all of them fit on the chip at once
constexpr uint32_t kFoldMax = kMtfUnits > kMtfSegs ? kMtfUnits : kMtfSegs;  // lists a step holds

template <uint32_t W>
struct FoldLds {
  uint8_t lists[kFoldMax * 256];
  uint32_t lens[kFoldMax];
  uint8_t sl[2][W][256];  // scan buffers: group lists, then their prefixes
  uint32_t slen[2][W];
  uint8_t init[256];
  uint32_t mark[W][kFoldSlots];
  uint8_t buf[W][kFoldSlots];
};

// the n lists [c0, c0 + n) of (plist, plen) into LDS
template <uint32_t W>
__device__ __forceinline__ void stage_lists(FoldLds<W> &F, const uint8_t *plist, const uint32_t *plen, uint32_t c0,
                                            uint32_t n) {
  stage_to_lds((uint32_t *)F.lists, (const uint32_t *)(plist + (size_t)c0 * 256), n * 64);
  stage_to_lds(F.lens, plen + c0, n);
  for (uint32_t e = threadIdx.x; e < W * kFoldSlots; e += blockDim.x) (&F.mark[0][0])[e] = 0;
}

__device__ __forceinline__ void lds_get(uint32_t (&v)[4], const uint8_t *src) {
  const uint32_t lane = (uint32_t)lane_id();
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) v[k] = src[lane + 64 * k];
}
__device__ __forceinline__ void lds_put(uint8_t *dst, const uint32_t (&v)[4]) {
  const uint32_t lane = (uint32_t)lane_id();
#pragma unroll
  for (uint32_t k = 0; k < 4; k++) dst[lane + 64 * k] = (uint8_t)v[k];
}

// Each wavefront's group of the staged lists: [g0, g1).
template <uint32_t W>
__device__ __forceinline__ void fold_group(uint32_t n, uint32_t w, uint32_t &g0, uint32_t &g1) {
  const uint32_t g = (n + W - 1) / W;
  g0 = min(n, w * g);
  g1 = min(n, g0 + g);
}

// Phases 1 and 2: F.sl[r][w] / F.slen[r][w] (r returned) = lists [0, g1(w))
// combined (the newest first).  Wavefront w folds with F.mark[w], F.buf[w]
// and stamps from *stamp on.
template <uint32_t W>
__device__ uint32_t fold_scan(FoldLds<W> &F, uint32_t n, uint32_t &stamp) {
  const uint32_t w = threadIdx.x / kWave;
  uint32_t g0, g1;
  fold_group<W>(n, w, g0, g1);
  uint32_t cur[4] = {0, 0, 0, 0}, len = 0;
  for (uint32_t i = g0; i < g1; i++) {
    uint32_t pv[4];
    lds_get(pv, F.lists + i * 256);
    wave_fold(cur, len, pv, F.lens[i], ++stamp, F.mark[w], F.buf[w]);
  }
  lds_put(F.sl[0][w], cur);
  if (lane_id() == 0) F.slen[0][w] = len;
  uint32_t r = 0;
  for (uint32_t d = 1; d < W; d <<= 1) {
    __syncthreads();
    if (w >= d) {
      // the older lists combined, then this wavefront's (newer) on top
      uint32_t pv[4];
      lds_get(cur, F.sl[r][w - d]);
      lds_get(pv, F.sl[r][w]);
      len = F.slen[r][w - d];
      wave_fold(cur, len, pv, F.slen[r][w], ++stamp, F.mark[w], F.buf[w]);
    } else {
      lds_get(cur, F.sl[r][w]);
      len = F.slen[r][w];
    }
    lds_put(F.sl[r ^ 1][w], cur);
    if (lane_id() == 0) F.slen[r ^ 1][w] = len;
    r ^= 1;
  }
  __syncthreads();
  return r;
}

// Phase 3: the list entering each staged list i < n, written to
// out + i * 256, starting from the 256-entry list F.init.
template <uint32_t W>
__device__ void fold_replay(FoldLds<W> &F, uint32_t n, uint32_t r, uint32_t &stamp, uint8_t *out) {
  const uint32_t w = threadIdx.x / kWave;
  uint32_t g0, g1;
  fold_group<W>(n, w, g0, g1);
  if (g0 >= g1) return;
  uint32_t cur[4], len = 256;
  lds_get(cur, F.init);
  if (w > 0) {  // the groups before this one, combined, on top of the initial list
    uint32_t pv[4];
    lds_get(pv, F.sl[r][w - 1]);
    wave_fold(cur, len, pv, F.slen[r][w - 1], ++stamp, F.mark[w], F.buf[w]);
  }
  for (uint32_t i = g0; i < g1; i++) {
    lds_put(out + (size_t)i * 256, cur);  // global
    if (i + 1 < g1) {
      uint32_t pv[4];
      lds_get(pv, F.lists + i * 256);
      wave_fold(cur, len, pv, F.lens[i], ++stamp, F.mark[w], F.buf[w]);
    }
  }
}

constexpr uint32_t kSegWaves = 8, kBlkWaves = 16;

// step 1: grid (kMtfSegs, blocks)
__global__ __launch_bounds__(64 * kSegWaves) void k_mtf_seg_fold(const uint32_t *d_nb, const BlockCode *codes,
                                                                const uint8_t *plist, const uint32_t *plen,
                                                                uint8_t *seglist, uint32_t *seglen) {
  __shared__ FoldLds<kSegWaves> F;
  const uint32_t b = blockIdx.y, j = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  uint32_t u0, u1;
  seg_range(C, j, u0, u1);
  const uint32_t n = u1 - u0;
  stage_lists(F, plist, plen, C.chunk_start + u0, n);
  __syncthreads();
  uint32_t stamp = 0;
  const uint32_t r = fold_scan(F, n, stamp);
  // the last wavefront's prefix is the whole segment
  const uint32_t t = threadIdx.x;
  if (t < 256) seglist[((size_t)b * kMtfSegs + j) * 256 + t] = F.sl[r][kSegWaves - 1][t];
  if (t == 0) seglen[(size_t)b * kMtfSegs + j] = F.slen[r][kSegWaves - 1];
}

// step 2: one workgroup per block; also writes the block's used-byte bitmap
// and symbol-map size.  The segment lists are replaced by the lists entering
// the segments.
__global__ __launch_bounds__(64 * kBlkWaves) void k_mtf_seg_chain(const uint32_t *d_nb, uint8_t *seglist,
                                                                 const uint32_t *seglen, uint32_t *used,
                                                                 BlockCode *codes) {
  __shared__ FoldLds<kBlkWaves> F;
  __shared__ uint32_t seen[256];
  const uint32_t b = blockIdx.x;
  if (b >= *d_nb) return;
  const uint32_t t = threadIdx.x, lane = (uint32_t)lane_id();
  uint8_t *sl = seglist + (size_t)b * kMtfSegs * 256;
  stage_lists(F, sl, seglen + (size_t)b * kMtfSegs, 0, kMtfSegs);
  if (t < 256) seen[t] = 0;
  __syncthreads();
  // the block's used bytes: every byte of a segment list
  for (uint32_t e = t; e < kMtfSegs * 256; e += blockDim.x)
    if ((e & 255u) < F.lens[e >> 8]) seen[F.lists[e]] = 1;
  __syncthreads();
  if (t < kWave) {
    uint64_t ub[4];
    uint32_t nu = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; k++) {
      ub[k] = ballot64(seen[lane + 64 * k] != 0);
      nu += (uint32_t)__popcll(ub[k]);
    }
    if (lane == 0) {
#pragma unroll
      for (uint32_t q = 0; q < 8; q++) used[b * 8 + q] = (uint32_t)(ub[q / 2] >> (32 * (q % 2)));
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
      F.init[pos] = (uint8_t)(lane + 64 * k);
      nbu += (uint32_t)__popcll(ub[k]);
      nbn += 64u - (uint32_t)__popcll(ub[k]);
    }
  }
  __syncthreads();
  uint32_t stamp = 0;
  const uint32_t r = fold_scan(F, kMtfSegs, stamp);
  fold_replay(F, kMtfSegs, r, stamp, sl);
}

// step 3: grid (kMtfSegs, blocks)
__global__ __launch_bounds__(64 * kSegWaves) void k_mtf_chain(const uint32_t *d_nb, const BlockCode *codes,
                                                             const uint8_t *plist, const uint32_t *plen,
                                                             const uint8_t *seglist, uint8_t *inlist) {
  __shared__ FoldLds<kSegWaves> F;
  const uint32_t b = blockIdx.y, j = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  uint32_t u0, u1;
  seg_range(C, j, u0, u1);
  if (u0 >= u1) return;
  const uint32_t n = u1 - u0;
  stage_lists(F, plist, plen, C.chunk_start + u0, n);
  if (threadIdx.x < 256) F.init[threadIdx.x] = seglist[((size_t)b * kMtfSegs + j) * 256 + threadIdx.x];
  __syncthreads();
  uint32_t stamp = 0;
  const uint32_t r = fold_scan(F, n, stamp);
  fold_replay(F, n, r, stamp, inlist + (size_t)(C.chunk_start + u0) * 256);
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
// (set here, five wait states before the first DPP, restored at the end;
// m0 is saved and restored around the loop as well);
// a DPP source needs two wait states after a vector write: the fast path's
// was written a dozen instructions earlier, the others get an s_nop.
__device__ __forceinline__ void mtf_batch(uint32_t &Q0, uint32_t &Q1, uint32_t &Q2, uint32_t &Q3, uint32_t &mine,
                                          uint64_t todo, uint32_t vl) {
  uint32_t v, q, c0, c1, c2, t, m0s;
  uint64_t mq, m1, m2, mk, ex;
  asm volatile(
      "s_mov_b32 %[m0s], m0\n\t"
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
      "s_mov_b64 exec, %[ex]\n\t"
      "s_mov_b32 m0, %[m0s]\n\t"
      "s_nop 0"
      : [Q0] "+v"(Q0), [Q1] "+v"(Q1), [Q2] "+v"(Q2), [Q3] "+v"(Q3), [mine] "+v"(mine), [todo] "+s"(todo),
        [v] "=&s"(v), [q] "=&s"(q), [c0] "=&s"(c0), [c1] "=&s"(c1), [c2] "=&s"(c2), [mq] "=&s"(mq), [m1] "=&s"(m1),
        [m2] "=&s"(m2), [mk] "=&s"(mk), [t] "=&v"(t), [ex] "=&s"(ex), [m0s] "=&s"(m0s)
      : [vl] "v"(vl)
      : "scc");
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
    tile_store(buf, zs, base, N);
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
  PCBZ_LAUNCH(k_mtf_partial, dim3((max_chunks + kPartWaves - 1) / kPartWaves), dim3(64 * kPartWaves), 0, s, L, cb,
              w.d_n_chunks, blk_start, d_nb, w.plist, w.plen);
  PCBZ_LAUNCH(k_mtf_seg_fold, dim3(kMtfSegs, max_blocks), dim3(64 * kSegWaves), 0, s, d_nb, codes, w.plist, w.plen,
              w.seglist, w.seglen);
  PCBZ_LAUNCH(k_mtf_seg_chain, dim3(max_blocks), dim3(64 * kBlkWaves), 0, s, d_nb, w.seglist, w.seglen, w.used, codes);
  PCBZ_LAUNCH(k_mtf_chain, dim3(kMtfSegs, max_blocks), dim3(64 * kSegWaves), 0, s, d_nb, codes, w.plist, w.plen,
              w.seglist, w.inlist);
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
