// pack.hip -- bzip2 stream bit-packing and the PCBZ container.
//
// Each block becomes one complete stream (bits most significant first):
// "BZh" + level digit, block magic 0x314159265359, block CRC, randomised=0,
// origPtr (24), the two-level used-byte map, table count (3), selector count
// (15), move-to-front coded selectors in unary, delta-coded code lengths per
// table, the Huffman-coded symbols (table switched every 50 symbols), the
// end-of-stream magic 0x177245385090, the stream CRC (equal to the block CRC
// for a one-block stream) and zero padding to a byte.
//
// A workgroup per block builds the header bits in LDS.  Selector MTF indices
// come from per-table last-use scans over the workgroup's threads: a
// selector seen before sits behind every table used since its last use; one
// never seen sits behind all seen tables and the unseen tables with smaller
// index.  Symbol bit lengths
// are scanned into bit offsets, and a writer thread owns each 32-bit word of
// a stream, assembling it from the header bits, the symbols that overlap it
// (found by binary search) and the trailer.
//
// Container (all little-endian): "PCBZ", version 1, level, pitch (u16), H,
// W (u32), band count (u16), flags (bit 0: some band uses the temporal
// candidate), reserved; then per band (id u8, byte length u32); then the
// streams in band order.
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

__device__ __forceinline__ void put_bits(uint32_t *w, uint32_t o, uint32_t nbits, uint32_t val) {
  // nbits in 1..32, MSB-first at bit offset o
  const uint64_t v = (uint64_t)(nbits == 32 ? val : (val & ((1u << nbits) - 1u))) << (64 - nbits - (o & 31));
  const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
  if (hi) atomicOr(&w[o >> 5], hi);
  if (lo) atomicOr(&w[(o >> 5) + 1], lo);
}

// Exclusive scans over a workgroup (any multiple of 64 threads): a shuffle
// scan inside each wavefront, then every thread combines the totals of the
// wavefronts before its own (sh holds one entry per wavefront).
template <typename T, typename Op>
__device__ T wg_excl_scan(T v, T ident, Op op, T *sh, T &total) {
  const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  T incl = v;
  for (int d = 1; d < kWave; d <<= 1) {
    const T t = __shfl_up(incl, d);
    if (lane >= d) incl = op(incl, t);
  }
  if (lane == kWave - 1) sh[w] = incl;
  __syncthreads();
  T before = ident, tot = ident;
  for (int k = 0; k < nw; k++) {
    const T x = sh[k];
    if (k < w) before = op(before, x);
    tot = op(tot, x);
  }
  __syncthreads();  // sh may be reused after this
  T prev = __shfl_up(incl, 1);
  if (lane == 0) prev = ident;
  total = tot;
  return op(before, prev);
}

__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *sh, uint32_t &total) {
  return wg_excl_scan<uint32_t>(v, 0u, [](uint32_t a, uint32_t b) { return a + b; }, sh, total);
}

__device__ __forceinline__ int block_excl_max(int v, int *sh) {  // identity -1
  int total;
  return wg_excl_scan<int>(v, -1, [](int a, int b) { return max(a, b); }, sh, total);
}

constexpr int kPfxThreads = 1024;

__global__ __launch_bounds__(kPfxThreads) void k_prefix(const uint32_t *d_nb, const BlockDesc *blocks, BlockCode *codes,
                                                const uint32_t *used, const uint8_t *sel, const uint8_t *lens,
                                                uint32_t *prefix) {
  __shared__ uint32_t w[kPrefixWords];
  __shared__ uint32_t shu[kPfxThreads / kWave];
  __shared__ int shi[kPfxThreads / kWave];
  const uint32_t b = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockDesc B = blocks[b];
  const BlockCode C = codes[b];
  const uint32_t G = C.n_groups, nsel = C.n_sel, alpha = C.alpha;
  for (int i = threadIdx.x; i < (int)kPrefixWords; i += kPfxThreads) w[i] = 0;
  __syncthreads();
  const uint32_t *u = used + b * 8;
  uint32_t nranges = 0;
  for (int r = 0; r < 16; r++) nranges += ((u[r >> 1] >> ((r & 1) * 16)) & 0xFFFFu) ? 1u : 0u;
  uint32_t o = 0;
  if (threadIdx.x == 0) {
    put_bits(w, 0, 32, 0x425A6800u | (uint32_t)('0' + B.level));
    put_bits(w, 32, 24, 0x314159u);
    put_bits(w, 56, 24, 0x265359u);
    put_bits(w, 80, 32, B.crc);
    put_bits(w, 112, 1, 0);
    put_bits(w, 113, 24, C.orig_ptr);
    uint32_t q = 137;
    uint32_t top = 0;
    for (int r = 0; r < 16; r++) top = (top << 1) | (((u[r >> 1] >> ((r & 1) * 16)) & 0xFFFFu) ? 1u : 0u);
    put_bits(w, q, 16, top);
    q += 16;
    for (int r = 0; r < 16; r++) {
      uint32_t bits16 = (u[r >> 1] >> ((r & 1) * 16)) & 0xFFFFu;
      if (!bits16) continue;
      // byte 16r + j is bit j of the word; the stream lists j = 0 first
      put_bits(w, q, 16, __brev(bits16) >> 16);
      q += 16;
    }
    put_bits(w, q, 3, G);
    put_bits(w, q + 3, 15, nsel);
  }
  o = 137 + 16 + 16 * nranges + 18;
  __syncthreads();
  // selectors: staged in LDS; each thread takes a contiguous slice.  The
  // last use of every table before a slice is an exclusive max-scan of the
  // slices' own last uses; with it each thread computes its selectors' MTF
  // indices, the bit offset of its slice is a scan of the slices' bit
  // counts, and each thread writes its slice's unary codes.
  __shared__ uint8_t ssel[kMaxSelectors];
  stage_to_lds(ssel, sel + C.sel_start, min(nsel, kMaxSelectors));
  __syncthreads();
  {
    const uint32_t K = (nsel + kPfxThreads - 1u) / kPfxThreads;
    const uint32_t j0 = min(nsel, threadIdx.x * K), j1 = min(nsel, j0 + K);
    int ll[kMaxGroups];
#pragma unroll
    for (int g = 0; g < kMaxGroups; g++) ll[g] = -1;
    for (uint32_t j = j0; j < j1; j++) {
      const int sj = ssel[j];
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) ll[g] = sj == g ? (int)j : ll[g];
    }
    int carry[kMaxGroups];
#pragma unroll
    for (int g = 0; g < kMaxGroups; g++) carry[g] = block_excl_max(ll[g], shi);
    // MTF index of selector value sv given the last uses before it
    auto mtf_index = [&](const int *last, int sv) {
      uint32_t idx = 0;
      const int ls = last[sv];
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) {
        if (g == sv || g >= (int)G) continue;
        if (ls >= 0)
          idx += last[g] > ls ? 1u : 0u;
        else
          idx += (last[g] >= 0 || g < sv) ? 1u : 0u;
      }
      return idx;
    };
    int last[kMaxGroups];
#pragma unroll
    for (int g = 0; g < kMaxGroups; g++) last[g] = carry[g];
    uint32_t bits = 0;
    for (uint32_t j = j0; j < j1; j++) {
      const int sj = ssel[j];
      int lcopy[kMaxGroups];
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) lcopy[g] = last[g];
      bits += mtf_index(lcopy, sj) + 1u;
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) last[g] = sj == g ? (int)j : last[g];
    }
    uint32_t tot;
    const uint32_t base = block_excl_sum(bits, shu, tot);
    uint32_t pos = o + base;
#pragma unroll
    for (int g = 0; g < kMaxGroups; g++) last[g] = carry[g];
    for (uint32_t j = j0; j < j1; j++) {
      const int sj = ssel[j];
      int lcopy[kMaxGroups];
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) lcopy[g] = last[g];
      const uint32_t idx = mtf_index(lcopy, sj);
      if (idx > 0) put_bits(w, pos, idx, (1u << idx) - 1u);  // idx ones; the zero is already there
      pos += idx + 1u;
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) last[g] = sj == g ? (int)j : last[g];
    }
    o += tot;
  }
  __syncthreads();
  // code lengths, per table: 5-bit start, then per symbol +1 ("10") / -1 ("11") steps and "0"
  for (uint32_t g = 0; g < G; g++) {
    const uint8_t *L = lens + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
    if (threadIdx.x == 0) put_bits(w, o, 5, L[0]);
    o += 5;
    for (uint32_t t0 = 0; t0 < alpha; t0 += kPfxThreads) {
      const uint32_t sidx = t0 + threadIdx.x;
      int d = 0;
      uint32_t nb = 0;
      if (sidx < alpha) {
        d = (int)L[sidx] - (int)L[sidx == 0 ? 0 : sidx - 1];
        nb = 2u * (uint32_t)abs(d) + 1u;
      }
      uint32_t tot;
      const uint32_t off = block_excl_sum(nb, shu, tot);
      if (sidx < alpha) {
        uint32_t q = o + off;
        const uint32_t pat = d > 0 ? 2u : 3u;
        for (int k = 0; k < abs(d); k++, q += 2) put_bits(w, q, 2, pat);
      }
      o += tot;
    }
  }
  __syncthreads();
  uint32_t *dst = prefix + (size_t)b * kPrefixWords;
  const uint32_t nw = (o + 31) / 32;
  for (uint32_t i = threadIdx.x; i < nw; i += kPfxThreads) dst[i] = w[i];
  if (threadIdx.x == 0) codes[b].prefix_bits = o;
}

__global__ void k_blk_sym_start(const uint32_t *d_nb, const BlockCode *codes, uint32_t *blk_sym_start) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nb = *d_nb;
  if (b < nb) blk_sym_start[b] = codes[b].sym_start;
  if (b == nb && nb > 0) blk_sym_start[nb] = codes[nb - 1].sym_start + codes[nb - 1].n_mtf;
  if (b == 0 && nb == 0) blk_sym_start[0] = 0;
}

// Bit offsets of the coded symbols: the code length of every symbol (its
// block's table for its group of 50), exclusively scanned over all blocks.
// Two launches over tiles of 4096 symbols (256 threads x 16 consecutive): the
// tile sums, then the scan from a carry summed from the sums in front of the
// tile; sym_off[n_sym] receives the total.
__device__ __forceinline__ void sym_lens16(const uint16_t *sym, uint32_t nsym, uint32_t k0, TileBlocks tb,
                                           const BlockCode *codes, const uint8_t *sel, const uint8_t *lens,
                                           uint32_t *bits) {
  uint16_t sy[kTItems];
  if (k0 + kTItems <= nsym) {
    const uint4 *q = (const uint4 *)(sym + k0);
#pragma unroll
    for (int j = 0; j < kTItems / 8; j++) {
      const uint4 t = q[j];
      sy[8 * j + 0] = (uint16_t)(t.x & 0xFFFFu);
      sy[8 * j + 1] = (uint16_t)(t.x >> 16);
      sy[8 * j + 2] = (uint16_t)(t.y & 0xFFFFu);
      sy[8 * j + 3] = (uint16_t)(t.y >> 16);
      sy[8 * j + 4] = (uint16_t)(t.z & 0xFFFFu);
      sy[8 * j + 5] = (uint16_t)(t.z >> 16);
      sy[8 * j + 6] = (uint16_t)(t.w & 0xFFFFu);
      sy[8 * j + 7] = (uint16_t)(t.w >> 16);
    }
  } else {
#pragma unroll
    for (int i = 0; i < kTItems; i++) sy[i] = k0 + i < nsym ? sym[k0 + i] : (uint16_t)0;
  }
  uint32_t cb = 0xFFFFFFFFu, ss = 0, sstart = 0;
#pragma unroll
  for (int i = 0; i < kTItems; i++) {
    const uint32_t k = k0 + i;
    uint32_t v = 0;
    if (k < nsym) {
      uint32_t s0, e0;
      const uint32_t b = tb.find(k, s0, e0);
      if (b != cb) {
        cb = b;
        ss = codes[b].sel_start;
        sstart = s0;
      }
      const uint32_t t = sel[ss + (k - sstart) / kGroupSize];
      v = lens[((size_t)b * kMaxGroups + t) * kMaxAlpha + sy[i]];
    }
    bits[i] = v;
  }
}

__global__ __launch_bounds__(kTThreads) void k_sym_sums(const uint16_t *sym, const uint32_t *d_n_sym,
                                                        const uint32_t *d_nb, const uint32_t *blk_sym_start,
                                                        const BlockCode *codes, const uint8_t *sel,
                                                        const uint8_t *lens, uint32_t *aggs) {
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t nsym = *d_n_sym, nb = *d_nb;
  const uint32_t nt = (nsym + kTTile - 1) / kTTile;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const TileBlocks tb(blk_sym_start, nb, tile * kTTile);
    uint32_t bits[kTItems], cnt = 0;
    sym_lens16(sym, nsym, tile * kTTile + threadIdx.x * kTItems, tb, codes, sel, lens, bits);
#pragma unroll
    for (int i = 0; i < kTItems; i++) cnt += bits[i];
    cnt = block_reduce<false>(cnt, sh);
    if (threadIdx.x == 0) aggs[tile] = cnt;
  }
}

__global__ __launch_bounds__(kTThreads) void k_sym_offs(const uint16_t *sym, const uint32_t *d_n_sym,
                                                        const uint32_t *d_nb, const uint32_t *blk_sym_start,
                                                        const BlockCode *codes, const uint8_t *sel,
                                                        const uint8_t *lens, const uint32_t *aggs,
                                                        uint32_t *sym_off) {
  __shared__ uint32_t buf[kTPad];
  __shared__ uint32_t sh[kTThreads / kWave];
  const uint32_t nsym = *d_n_sym, nb = *d_nb;
  const uint32_t nt = (nsym + kTTile - 1) / kTTile;
  if (nt == 0 && blockIdx.x == 0 && threadIdx.x == 0) sym_off[0] = 0;
  uint32_t carry = 0, counted = 0;
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint32_t k0 = tile * kTTile + threadIdx.x * kTItems;
    const TileBlocks tb(blk_sym_start, nb, tile * kTTile);
    uint32_t bits[kTItems];
    sym_lens16(sym, nsym, k0, tb, codes, sel, lens, bits);
    carry = tile_carry<false>(aggs, counted, tile, carry, sh);
#pragma unroll
    for (int i = 0; i < kTItems; i++) buf[tpad(threadIdx.x * kTItems + i)] = bits[i];
    __syncthreads();
    const uint32_t total = tile_scan<false, false>(buf, carry, sh);
    tile_store(buf, sym_off, tile * kTTile, nsym);
    if (tile == nt - 1 && threadIdx.x == 0) sym_off[nsym] = carry + total;
    __syncthreads();
  }
}

// Stream sizes, offsets inside each frame's container, band lengths and the
// writer's word index space.  One thread; blocks are few.
__global__ void k_layout(const uint32_t *d_nb, const BlockDesc *blocks, BlockCode *codes, const uint32_t *sym_off,
                         const uint32_t *blk_sym_start, const FrameOut *frames, uint32_t n_frames,
                         const BandDesc * /*bands*/, uint32_t *band_len, uint64_t *frame_len, uint32_t *word_start,
                         uint32_t *d_words) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t nb = *d_nb;
  for (uint32_t f = 0; f < n_frames; f++) {
    frame_len[f] = 20u + 5u * frames[f].n_bands;
    for (uint32_t k = 0; k < frames[f].n_bands; k++) band_len[frames[f].band_base + k] = 0;
  }
  uint32_t words = 0;
  for (uint32_t b = 0; b < nb; b++) {
    const BlockDesc B = blocks[b];
    const uint32_t data = sym_off[blk_sym_start[b + 1]] - sym_off[blk_sym_start[b]];
    const uint32_t bits = codes[b].prefix_bits + data + 80u;
    const uint32_t bytes = (bits + 7u) / 8u;
    codes[b].data_bits = data;
    codes[b].stream_bytes = bytes;
    codes[b].stream_off = (uint32_t)frame_len[B.frame_id];
    codes[b].word_start = words;
    frame_len[B.frame_id] += bytes;
    band_len[B.band] += bytes;
    words += (bytes + 3u) / 4u;
  }
  word_start[nb] = words;
  for (uint32_t b = 0; b < nb; b++) word_start[b] = codes[b].word_start;
  *d_words = words;
}

__device__ __forceinline__ uint32_t trailer_bits(uint32_t crc, uint32_t from, uint32_t n) {
  // bits [from, from+n) of the 80-bit trailer 0x177245385090 . crc, MSB-first (n <= 32)
  const uint64_t hi48 = 0x177245385090ull;
  uint32_t r = 0;
  for (uint32_t i = 0; i < n; i++) {
    const uint32_t p = from + i;
    const uint32_t bit = p < 48 ? (uint32_t)((hi48 >> (47 - p)) & 1u) : ((crc >> (79 - p)) & 1u);
    r = (r << 1) | bit;
  }
  return r;
}

__global__ __launch_bounds__(256) void k_write(const uint32_t *d_words, const uint32_t *word_start,
                                               const uint32_t *d_nb, const BlockDesc *blocks, const BlockCode *codes,
                                               const uint32_t *prefix, const uint16_t *sym, const uint32_t *sym_off,
                                               const uint32_t *blk_sym_start, const uint8_t *sel,
                                               const uint8_t *lens, const uint32_t *code_words,
                                               const FrameOut *frames, const uint64_t *frame_len) {
  const uint32_t nwords = *d_words, nb = *d_nb;
  for (uint32_t wi = blockIdx.x * blockDim.x + threadIdx.x; wi < nwords; wi += gridDim.x * blockDim.x) {
    const uint32_t b = upper_index(word_start, nb, wi);
    const BlockDesc B = blocks[b];
    const FrameOut F = frames[B.frame_id];
    if (frame_len[B.frame_id] > F.cap) continue;
    const BlockCode C = codes[b];
    const uint32_t lw = wi - word_start[b];
    const uint32_t w0 = lw * 32u, w1 = w0 + 32u;
    const uint32_t P = C.prefix_bits, D = C.data_bits;
    uint32_t word = 0;
    // header bits
    if (w0 < P) {
      uint32_t pw = prefix[(size_t)b * kPrefixWords + lw];
      if (P < w1) pw &= ~(0xFFFFFFFFu >> (P - w0));
      word |= pw;
    }
    // symbols overlapping [max(w0,P), min(w1,P+D))
    const uint32_t d0 = max(w0, P), d1 = min(w1, P + D);
    if (d0 < d1) {
      const uint32_t s0 = blk_sym_start[b], s1 = blk_sym_start[b + 1];
      const uint32_t base = sym_off[s0];
      const uint32_t rel0 = d0 - P;
      // last symbol whose start <= rel0
      uint32_t lo = s0, hi = s1 - 1;
      while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (sym_off[mid] - base <= rel0) lo = mid; else hi = mid - 1;
      }
      for (uint32_t k = lo; k < s1; k++) {
        const uint32_t st = P + (sym_off[k] - base);
        if (st >= d1) break;
        const uint32_t local = k - s0;
        const uint32_t t = sel[C.sel_start + local / kGroupSize];
        const size_t ti = ((size_t)b * kMaxGroups + t) * kMaxAlpha + sym[k];
        const uint32_t len = lens[ti], code = code_words[ti];
        // place bits [st, st+len) into [w0, w0+32)
        const int64_t shift = (int64_t)(w0 + 32) - (int64_t)(st + len);  // left shift of the code inside the word
        uint64_t v = (uint64_t)code;
        uint32_t part;
        if (shift >= 0)
          part = (uint32_t)(v << shift);
        else
          part = (uint32_t)(v >> (-shift));
        // keep only bits inside [d0, d1) (the code cannot reach before st >= P region start)
        word |= part;
      }
    }
    // trailer
    const uint32_t t0 = P + D, t1 = t0 + 80u;
    const uint32_t a0 = max(w0, t0), a1 = min(w1, t1);
    if (a0 < a1) {
      const uint32_t n = a1 - a0;
      const uint32_t bitsv = trailer_bits(B.crc, a0 - t0, n);
      word |= bitsv << (w1 - a1);
    }
    // write big-endian bytes
    uint8_t *dst = F.out + C.stream_off + 4u * lw;
    const uint32_t rem = C.stream_bytes - 4u * lw;
    for (uint32_t i = 0; i < 4u && i < rem; i++) dst[i] = (uint8_t)(word >> (24 - 8 * i));
  }
}

__global__ __launch_bounds__(256) void k_header(const FrameOut *frames, const uint64_t *frame_len,
                                                const BandDesc * /*bands*/, const uint8_t *choice,
                                                const uint32_t *band_len) {
  const FrameOut F = frames[blockIdx.x];
  if (frame_len[blockIdx.x] > F.cap) return;
  uint8_t *o = F.out;
  __shared__ int any_dt;
  if (threadIdx.x == 0) any_dt = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < F.n_bands; k += 256) {
    const uint32_t bi = F.band_base + k;
    const uint8_t id = choice[bi];
    const uint32_t ln = band_len[bi];
    uint8_t *e = o + 20 + 5 * k;
    e[0] = id;
    e[1] = (uint8_t)ln;
    e[2] = (uint8_t)(ln >> 8);
    e[3] = (uint8_t)(ln >> 16);
    e[4] = (uint8_t)(ln >> 24);
    if (id == 3) atomicOr(&any_dt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    o[0] = 'P';
    o[1] = 'C';
    o[2] = 'B';
    o[3] = 'Z';
    o[4] = 1;
    o[5] = (uint8_t)F.level;
    o[6] = (uint8_t)F.pitch;
    o[7] = (uint8_t)(F.pitch >> 8);
    for (int i = 0; i < 4; i++) {
      o[8 + i] = (uint8_t)(F.h >> (8 * i));
      o[12 + i] = (uint8_t)(F.w >> (8 * i));
    }
    o[16] = (uint8_t)F.n_bands;
    o[17] = (uint8_t)(F.n_bands >> 8);
    o[18] = (uint8_t)(any_dt ? 1 : 0);
    o[19] = 0;
  }
}

}  // namespace

void launch_pack_prefix(const uint32_t *d_nb, uint32_t max_blocks, const BlockDesc *blocks, BlockCode *codes,
                        const uint32_t *used, const uint8_t *sel, const uint8_t *lens, uint32_t *prefix,
                        hipStream_t s) {
  PCBZ_LAUNCH(k_prefix, dim3(max_blocks), dim3(kPfxThreads), 0, s, d_nb, blocks, codes, used, sel, lens, prefix);
}

void launch_pack2(const uint32_t *d_nb, uint32_t max_blocks, const BlockDesc *blocks, BlockCode *codes,
                  const uint8_t *sel, const uint8_t *lens, const uint32_t *code_words, const uint16_t *sym,
                  const uint32_t *d_n_sym, uint32_t max_sym, const uint32_t *prefix, uint32_t *sym_bits,
                  uint32_t *sym_off, uint32_t *blk_sym_start, const FrameOut *frames,
                  uint32_t n_frames, const BandDesc *bands, const uint8_t *choice, uint32_t *band_len,
                  uint64_t *frame_len, uint32_t *word_start, uint32_t *d_words, uint32_t max_words,
                  hipEvent_t prefix_ready, hipStream_t s) {
  PCBZ_LAUNCH(k_blk_sym_start, dim3((max_blocks + 256) / 256), dim3(256), 0, s, d_nb, codes, blk_sym_start);
  // sym_bits holds the tile sums (tiles + 1 <= max_sym + 1 words)
  const uint32_t gt = std::max<uint32_t>(1, std::min<uint32_t>(2048, (max_sym + kTTile - 1) / kTTile));
  PCBZ_LAUNCH(k_sym_sums, dim3(gt), dim3(kTThreads), 0, s, sym, d_n_sym, d_nb, blk_sym_start, codes, sel, lens,
              sym_bits);
  PCBZ_LAUNCH(k_sym_offs, dim3(gt), dim3(kTThreads), 0, s, sym, d_n_sym, d_nb, blk_sym_start, codes, sel, lens,
              sym_bits, sym_off);
  if (prefix_ready) (void)hipStreamWaitEvent(s, prefix_ready, 0);
  PCBZ_LAUNCH(k_layout, dim3(1), dim3(64), 0, s, d_nb, blocks, codes, sym_off, blk_sym_start, frames, n_frames,
                     bands, band_len, frame_len, word_start, d_words);
  const uint32_t gw = std::min<uint32_t>((max_words + 255) / 256 + 1, 16384);
  PCBZ_LAUNCH(k_write, dim3(gw), dim3(256), 0, s, d_words, word_start, d_nb, blocks, codes, prefix, sym,
                     sym_off, blk_sym_start, sel, lens, code_words, frames, frame_len);
  PCBZ_LAUNCH(k_header, dim3(n_frames), dim3(256), 0, s, frames, frame_len, bands, choice, band_len);
}

}  // namespace pcbz
