// decode.hip -- the decompression path on the GPU (paper Fig. 1c and Fig. 2b:
// read the header and the per-band arrangement ids, decode each band's bzip2
// data, then invert the arrangement).
//
// Every band of every container of a call is decoded at once, block by block:
//   1. stream header, tables and Huffman data of each block (one wavefront
//      per block; the streams of a band follow each other, so the k-th
//      streams of all bands are decoded in the k-th pass);
//   2. the zero runs and move-to-front (chunks of 1024 symbols replayed
//      against a placeholder list, then one chain per block that turns the
//      chunks' final lists into each chunk's incoming list);
//   3. the inverse BWT: a stable sort of each block's positions by byte gives
//      each row's successor, and the successor cycle is ranked from sampled
//      splitters (walks between splitters, pointer jumping over the
//      splitters in LDS, walks again to write the bytes);
//   4. the first run-length stage is undone with a scan over the five states
//      of its decoder, and each block's CRC is checked;
//   5. the arrangement is inverted into the frame (cumulative sums for the
//      lens-neighbour delta, the previous frame for the temporal delta, the
//      inverse of the sub-aperture-view index map).
// The format is the public bzip2 layout; the container holds one stream per
// block, as the encoder writes it.
#include "pcbz.h"
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr int kLutBits = 12;
constexpr uint32_t kLutSize = 1u << kLutBits;
constexpr uint32_t kWinWords = 1024;  // 4 KB window of Huffman data bits in LDS
constexpr uint32_t kInvalid = 0x1FFu;
constexpr uint32_t kMaxLen = 20;      // the format's longest code
constexpr uint32_t kOutBuf = 1024;    // symbols gathered in LDS before a store

__device__ __forceinline__ void set_err(uint32_t *ctr, uint32_t bit, uint32_t band) {
  atomicOr(&ctr[0], bit);
  atomicMin(&ctr[1], band);
}

// Words [w0, w0 + n) of the big-endian word view of src[0, len) into dst
// (bytes past len read as zero), by the whole wavefront; every load is in
// bounds and unconditional, so that a lane's sixteen loads are in flight
// together (len >= 1).
__device__ __forceinline__ void stage_be_words(uint32_t *dst, const uint8_t *src, uint32_t len, uint32_t w0,
                                               uint32_t n) {
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t k0 = 0; k0 < n; k0 += 4 * kWave) {
    uint32_t b[16];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const uint32_t i = 4 * (w0 + k0 + q * kWave + lane) + j;
        b[q * 4 + j] = src[min(i, len - 1)];
      }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const uint32_t k = k0 + q * kWave + lane;
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < 4; j++) v = (v << 8) | (4 * (w0 + k) + j < len ? b[q * 4 + j] : 0u);
      if (k < n) dst[k] = v;
    }
  }
}

// 32 bits starting at bit q of a word array (MSB first).
__device__ __forceinline__ uint32_t bits32(const uint32_t *wds, uint32_t q) {
  const uint32_t i = q >> 5, s = q & 31u;
  const uint64_t v = ((uint64_t)wds[i] << 32) | wds[i + 1];
  return (uint32_t)((v << s) >> 32);
}

struct HeadLds {
  uint32_t words[kDecHeadBytes / 4 + 2];
};
struct DecodeLds {
  uint16_t lut[kMaxGroups][kLutSize];  // symbol | length << 9 (length 0: longer than kLutBits)
  uint32_t win[kWinWords + 4];
  uint32_t first[kMaxGroups][kMaxLen + 2], count[kMaxGroups][kMaxLen + 2], base[kMaxGroups][kMaxLen + 2];
  uint16_t perm[kMaxGroups][kMaxAlpha];
};
union BlockLds {
  HeadLds head;
  DecodeLds dec;
};

// Follows code boundaries across the lanes: nx holds, per lane, the bit
// where the next code starts if a code starts at that lane's bit (lane plus
// the code's length; 128 plus the lane when the first-level entry has no
// length).  From lane p it marks each start in `starts` and steps to its
// successor until the successor is 64 or more (past the window, or 128 + a
// lane to decode by the canonical search), and returns that successor.
// Scalar registers and branches only, unrolled four codes deep: a lane read
// whose select was written by a vector instruction (another lane read, or
// the caller's first-lane read of p) needs four instructions between them,
// and a taken branch costs more than the exits it replaces.
__device__ __forceinline__ uint32_t chain_run(uint32_t nx, uint64_t &starts, uint32_t p) {
  uint32_t q;
  asm volatile(
      "s_nop 3\n\t"
      "s_cmp_ge_u32 %[p], 64\n\t"
      "s_cbranch_scc1 9f\n"
      "1:\n\t"
      "v_readlane_b32 %[q], %[nx], %[p]\n\t"
      "s_bitset1_b64 %[st], %[p]\n\t"
      "s_cmp_ge_u32 %[q], 64\n\t"
      "s_cbranch_scc1 8f\n\t"
      "s_nop 0\n\t"
      "v_readlane_b32 %[p], %[nx], %[q]\n\t"
      "s_bitset1_b64 %[st], %[q]\n\t"
      "s_cmp_ge_u32 %[p], 64\n\t"
      "s_cbranch_scc1 9f\n\t"
      "s_nop 0\n\t"
      "v_readlane_b32 %[q], %[nx], %[p]\n\t"
      "s_bitset1_b64 %[st], %[p]\n\t"
      "s_cmp_ge_u32 %[q], 64\n\t"
      "s_cbranch_scc1 8f\n\t"
      "s_nop 0\n\t"
      "v_readlane_b32 %[p], %[nx], %[q]\n\t"
      "s_bitset1_b64 %[st], %[q]\n\t"
      "s_cmp_ge_u32 %[p], 64\n\t"
      "s_cbranch_scc1 9f\n\t"
      "s_nop 0\n\t"
      "s_branch 1b\n"
      "8:\n\t"
      "s_mov_b32 %[p], %[q]\n"
      "9:"
      : [st] "+s"(starts), [p] "+s"(p), [q] "=&s"(q)
      : [nx] "v"(nx)
      : "scc");
  return p;
}

// The same walk four codes per lane read: j holds, per lane, where the walk
// from that lane stands after four codes (or where it left the window or met
// an entry without length), and (mlo, mhi) the code starts it passes on the
// way (the lane's own bit included, the landing excluded).
__device__ __forceinline__ uint32_t chain_jump(uint32_t j, uint32_t mlo, uint32_t mhi, uint64_t &starts) {
  uint32_t p = 0, q, a, b, lo = 0, hi = 0;
  asm volatile(
      "1:\n\t"
      "v_readlane_b32 %[q], %[j], %[p]\n\t"
      "v_readlane_b32 %[a], %[ml], %[p]\n\t"
      "v_readlane_b32 %[b], %[mh], %[p]\n\t"
      "s_or_b32 %[lo], %[lo], %[a]\n\t"
      "s_or_b32 %[hi], %[hi], %[b]\n\t"
      "s_cmp_ge_u32 %[q], 64\n\t"
      "s_cbranch_scc1 8f\n\t"
      "v_readlane_b32 %[p], %[j], %[q]\n\t"
      "v_readlane_b32 %[a], %[ml], %[q]\n\t"
      "v_readlane_b32 %[b], %[mh], %[q]\n\t"
      "s_or_b32 %[lo], %[lo], %[a]\n\t"
      "s_or_b32 %[hi], %[hi], %[b]\n\t"
      "s_cmp_ge_u32 %[p], 64\n\t"
      "s_cbranch_scc0 1b\n\t"
      "s_branch 9f\n"
      "8:\n\t"
      "s_mov_b32 %[p], %[q]\n"
      "9:"
      : [p] "+s"(p), [q] "=&s"(q), [a] "=&s"(a), [b] "=&s"(b), [lo] "+s"(lo), [hi] "+s"(hi)
      : [j] "v"(j), [ml] "v"(mlo), [mh] "v"(mhi)
      : "scc");
  starts = (uint64_t)hi << 32 | lo;
  return p;
}

// Four steps of the walk for every lane at once (two rounds of lane
// permutes: the successor's successor, then the successor of that and its
// own successor's successor); positions of 64 and more stay where they are.
__device__ __forceinline__ void walk4(uint32_t nx, int lane, uint32_t &j, uint32_t &mlo, uint32_t &mhi) {
  const uint32_t n1 = nx;
  const uint32_t t2 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(n1 << 2), (int)nx);
  const uint32_t n2 = n1 < 64 ? t2 : n1;
  const uint32_t t3 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(n2 << 2), (int)nx);
  const uint32_t t4 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(n2 << 2), (int)n2);
  const uint32_t n3 = n2 < 64 ? t3 : n2;
  j = n2 < 64 ? t4 : n2;
  uint64_t m = 1ull << lane;
  if (n1 < 64) m |= 1ull << n1;
  if (n2 < 64) m |= 1ull << n2;
  if (n3 < 64) m |= 1ull << n3;
  mlo = (uint32_t)m;
  mhi = (uint32_t)(m >> 32);
}

// Canonical decode of a 32-bit window with table g (codes assigned in
// (length, symbol) order): symbol | length << 9, or kInvalid.
__device__ __forceinline__ uint32_t canon_decode(const DecodeLds &L, int g, uint32_t w) {
  for (uint32_t l = 1; l <= kMaxLen; l++) {
    const uint32_t c = w >> (32 - l);
    const uint32_t d = c - L.first[g][l];
    if (d < L.count[g][l]) return (uint32_t)L.perm[g][L.base[g][l] + d] | (l << 9);
  }
  return kInvalid;
}

// One wavefront per band: parses the stream in the band's slot `pass` (it
// starts where the previous slot's stream ended), builds its decode tables
// and decodes its Huffman data into symbols.
__global__ __launch_bounds__(64) void k_dec_block(const DecBand *bands, DecSlot *slots, uint8_t *seq_all,
                                                  uint16_t *sym_all, uint32_t pass, uint32_t *ctr) {
  __shared__ BlockLds S;
  __shared__ uint8_t sel_lds[kMaxSelectors];
  __shared__ uint8_t lens_lds[kMaxGroups][kMaxAlpha];
  __shared__ uint8_t seq_lds[256];
  __shared__ uint32_t over_lds;
  // decoded symbols gather here and go to global memory a thousand at a time
  // (a store per step made every step wait for the last one's data register)
  __shared__ uint16_t obuf[kOutBuf + 64];  // 64 spare entries for lanes with nothing to store
  const uint32_t b = blockIdx.x;
  const DecBand B = bands[b];
  const int lane = threadIdx.x;
  if (pass >= B.nslots) return;
  const uint32_t slot = B.slot0 + pass;
  uint32_t start, sym0;
  if (pass == 0) {
    start = 0;
    sym0 = B.sym_base;
  } else {
    const DecSlot &pv = slots[slot - 1];
    if (!pv.valid || pv.end_byte >= B.src_len) {
      if (lane == 0) slots[slot].valid = 0;
      return;
    }
    start = pv.end_byte;
    sym0 = pv.sym_off + pv.n_sym;
  }
  const uint32_t sym_cap = (uint32_t)__builtin_amdgcn_readfirstlane((int)(B.sym_end > sym0 ? B.sym_end - sym0 : 0u));
  const uint8_t *src = B.src + start;
  const uint32_t len = B.src_len - start;  // bytes left in the band
  auto fail = [&](void) {
    if (lane == 0) {
      slots[slot].valid = 0;
      set_err(ctr, kDecErrStream, b);
    }
  };
  // ---- stage the header bytes (big-endian words) into LDS
  const uint32_t head_bytes = min(len, kDecHeadBytes);
  if (head_bytes > 0) stage_be_words(S.head.words, src, head_bytes, 0, kDecHeadBytes / 4 + 2);
  __syncthreads();
  // ---- header fields (every lane parses the same uniform values)
  const uint32_t *hw = S.head.words;
  const uint32_t hbits = head_bytes * 8;
  uint32_t q = 0;
  // the two header words around q stay in registers while q moves inside them
  uint32_t hci = 0xFFFFFFFFu;
  uint64_t hw64 = 0;
  auto peek = [&](uint32_t at) -> uint32_t {
    const uint32_t i = at >> 5;
    if (i != hci) {  // scalar registers: every lane parses the same header
      hci = i;
      hw64 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)hw[i]) << 32) |
             (uint32_t)__builtin_amdgcn_readfirstlane((int)hw[i + 1]);
    }
    return (uint32_t)((hw64 << (at & 31u)) >> 32);
  };
  auto get = [&](uint32_t k) -> uint32_t {  // k <= 24 bits
    const uint32_t v = peek(q) >> (32 - k);
    q += k;
    return v;
  };
  bool bad = head_bytes < 10;
  if (!bad) {
    const uint32_t magic = get(24);
    const uint32_t digit = get(8);
    const uint32_t m_hi = get(24), m_lo = get(24);
    bad = magic != 0x425A68u || digit < '1' || digit > '9' || digit - '0' != B.level || m_hi != 0x314159u ||
          m_lo != 0x265359u;
  }
  if (bad) {
    fail();
    return;
  }
  const uint32_t crc_hi = get(16);
  const uint32_t crc = (crc_hi << 16) | get(16);
  const uint32_t randomised = get(1);
  const uint32_t orig_ptr = get(24);
  const uint32_t used16 = get(16);
  // symbol map: used byte values in ascending order
  uint32_t n_in_use = 0;
  for (int r = 0; r < 16; r++) {
    if (!((used16 >> (15 - r)) & 1u)) continue;
    const uint32_t bitsr = get(16);
    // lanes 0..15 place the bytes of this range
    const uint32_t mine = lane < 16 ? (bitsr >> (15 - lane)) & 1u : 0u;
    const uint64_t bal = ballot64(mine != 0u);
    if (mine) seq_lds[n_in_use + __popcll(bal & lanemask_lt())] = (uint8_t)(16 * r + lane);
    n_in_use += (uint32_t)__popcll(bal);
  }
  const uint32_t G = get(3);
  const uint32_t nsel = get(15);
  if (randomised || n_in_use == 0 || G < 2 || G > kMaxGroups || nsel < 1 || nsel > kMaxSelectors || q > hbits) {
    fail();
    return;
  }
  const uint32_t alpha = n_in_use + 2;
  // selectors: unary codes (j ones, then a zero) of move-to-front indices
  {
    uint32_t list = 0x543210u;  // 4 bits per entry, front in the low bits
    for (uint32_t k = 0; k < nsel; k++) {
      if (q > hbits) break;  // reported below
      const uint32_t w = peek(q);
      const uint32_t j = __clz(~w);  // leading ones
      if (j >= G) {
        fail();
        return;
      }
      q += j + 1;
      const uint32_t v = (list >> (4 * j)) & 15u;
      const uint32_t below = (1u << (4 * j)) - 1u;
      list = (list & ~((below << 4) | 15u)) | ((list & below) << 4) | v;
      sel_lds[k] = (uint8_t)v;  // every lane writes the same value (no divergent branch)
    }
  }
  if (q > hbits) {
    fail();
    return;
  }
  // code lengths: a 5-bit start, then per symbol "1x" steps (10: +1, 11: -1) ended by "0"
  for (uint32_t g = 0; g < G; g++) {
    int cur = (int)get(5);
    for (uint32_t sy = 0; sy < alpha; sy++) {
      for (;;) {
        if (cur < 1 || cur > (int)kMaxLen || q > hbits) {
          fail();
          return;
        }
        const uint32_t w = peek(q);
        if (!(w >> 31)) {
          q += 1;
          break;
        }
        cur += (w >> 30) & 1u ? -1 : 1;
        q += 2;
      }
      lens_lds[g][sy] = (uint8_t)cur;
    }
  }
  if (q > hbits) {
    fail();
    return;
  }
  const uint32_t data_bit = q;  // relative to `src`
  __syncthreads();
  // ---- decode tables (the header area is reused)
  DecodeLds &D = S.dec;
  for (uint32_t g = 0; g < G; g++) {
    if (lane <= (int)kMaxLen) D.count[g][lane] = 0;
  }
  __syncthreads();
  if (lane == 0) {
    bool over = false;
    for (uint32_t g = 0; g < G; g++) {
      for (uint32_t sy = 0; sy < alpha; sy++) D.count[g][lens_lds[g][sy]]++;
      uint32_t code = 0, idx = 0;
      for (uint32_t l = 1; l <= kMaxLen; l++) {
        D.first[g][l] = code;
        D.base[g][l] = idx;
        idx += D.count[g][l];
        code = (code + D.count[g][l]) << 1;
        if (code > (2u << l)) over = true;  // more codes of length <= l than fit
      }
      uint32_t fill[kMaxLen + 1];
      for (uint32_t l = 0; l <= kMaxLen; l++) fill[l] = 0;
      for (uint32_t sy = 0; sy < alpha; sy++) {
        const uint32_t l = lens_lds[g][sy];
        D.perm[g][D.base[g][l] + fill[l]++] = (uint16_t)sy;
      }
    }
    over_lds = over ? 1u : 0u;
  }
  __syncthreads();
  if (over_lds) {  // more codes than the code space holds
    fail();
    return;
  }
  // first-level table: a prefix of kLutBits bits resolves when a code of at
  // most kLutBits bits matches it; other prefixes (0) take the canonical
  // search.  Each symbol with a short code fills the entries of its code
  // (its code is first[l] plus its place among the codes of length l).
  for (uint32_t g = 0; g < G; g++)
    for (uint32_t e = lane; e < kLutSize; e += 64) D.lut[g][e] = 0;
  __syncthreads();
  for (uint32_t g = 0; g < G; g++)
    for (uint32_t i = lane; i < alpha; i += 64) {
      const uint32_t sy = D.perm[g][i];
      const uint32_t l = lens_lds[g][sy];
      if (l > (uint32_t)kLutBits) continue;
      const uint32_t c = D.first[g][l] + (i - D.base[g][l]);
      const uint32_t e0 = c << (kLutBits - l), e1 = (c + 1) << (kLutBits - l);
      for (uint32_t e = e0; e < e1 && e < kLutSize; e++) D.lut[g][e] = (uint16_t)(sy | (l << 9));
    }
  // the symbol map goes to global memory for the move-to-front stage
  for (uint32_t i = lane; i < 256; i += 64) seq_all[(size_t)slot * 256 + i] = i < n_in_use ? seq_lds[i] : 0;
  __syncthreads();
  // ---- Huffman data: 64 lanes decode one code each at 64 consecutive bit
  // positions; the true code boundaries are then followed from the first
  uint16_t *out = sym_all + sym0;
  const uint32_t eob = alpha - 1;
  uint32_t o = data_bit;         // bit position relative to src
  uint32_t wbase = 0xFFFFFFFFu;  // first bit held by the window
  uint32_t g = 0, in_grp = 0, nsym = 0, nbuf = 0;
  uint32_t t = sel_lds[0];
  auto flush = [&]() {
    for (uint32_t i = lane; i < nbuf; i += 64) out[nsym - nbuf + i] = obuf[i];
    nbuf = 0;
  };
  bool done = false, ok = true;
  const uint32_t total_bits = len * 8;
  while (!done) {
    if (o > total_bits || g >= nsel) {  // ran past the band, or past the last group
      ok = false;
      break;
    }
    if (wbase == 0xFFFFFFFFu || o + 64 + 32 > wbase + kWinWords * 32) {
      __syncthreads();
      wbase = o & ~31u;
      stage_be_words(D.win, src, len, wbase >> 5, kWinWords + 4);
      __syncthreads();
    }
    // the next group's table, read ahead (the last group's own when none follows)
    const uint32_t t_next = sel_lds[g + 1 < nsel ? g + 1 : g];
    const uint32_t w = bits32(D.win, o - wbase + lane);
    // first-level table only: most lanes sit at positions that are no code
    // boundary, and a longer code is decoded below when the chain reaches it
    uint32_t e = D.lut[t][w >> (32 - kLutBits)];
    // follow the true code boundaries from the first lane to the end of the
    // window, marking them; codes past the group's end (read with this
    // group's table) and past the block's end are cut off after
    const uint32_t room = (uint32_t)__builtin_amdgcn_readfirstlane((int)(kGroupSize - in_grp));
    const uint32_t len0 = e >> 9;
    uint32_t nx = len0 ? (uint32_t)lane + len0 : 128u + (uint32_t)lane;
    uint32_t j, mlo, mhi;
    walk4(nx, lane, j, mlo, mhi);
    uint64_t starts;
    uint32_t p = chain_jump(j, mlo, mhi, starts);
    bool stuck = false;
    // after a stop the lanes' four-code jumps no longer hold: one code a read
    while (p >= 128) {
      // a start whose first-level entry has no length: a code longer than
      // the first-level table (decoded here and put into that lane), or none.
      // Not needed when the group or the block ends before it.
      const uint32_t s = p - 128;
      if ((uint32_t)__popcll(starts) - 1u >= room) break;
      if (ballot64(((starts >> lane) & 1ull) && lane != (int)s && (e & 0x1FFu) == eob)) break;
      const uint32_t r = canon_decode(D, (int)t, (uint32_t)__builtin_amdgcn_readlane((int)w, (int)s));
      if ((r >> 9) == 0u) {
        stuck = true;
        break;
      }
      e = lane == (int)s ? r : e;
      p = (uint32_t)__builtin_amdgcn_readfirstlane((int)(s + (r >> 9)));
      nx = lane == (int)s ? p : nx;
      p = chain_run(nx, starts, p);
    }
    // the cuts: the group ends after its room-th code, the block after its
    // end-of-block code, whichever comes first (both masks from one pair of
    // compares; a lane that is no start takes a rank no cut matches)
    const uint32_t sy = e & 0x1FFu;
    const uint32_t rank = (uint32_t)__popcll(starts & lanemask_lt());
    const uint32_t key = (starts >> lane) & 1ull ? rank : 0xFFFFu;
    const uint64_t over = ballot64(key == room);
    const uint64_t ends = ballot64((sy == eob ? key : 0xFFFFu) < room);
    uint32_t adv = p;  // bits consumed
    if (ends) {  // the block ends: drop whatever was followed past its last symbol
      const uint32_t f = (uint32_t)__builtin_ctzll(ends);
      starts &= f == 63 ? ~0ull : (2ull << f) - 1ull;
      adv = f + ((uint32_t)__builtin_amdgcn_readlane((int)e, (int)f) >> 9);
      done = true;
    } else if (over) {  // the rest is the next group's
      adv = (uint32_t)__builtin_ctzll(over);
      starts &= (1ull << adv) - 1ull;
    } else if (stuck) {
      ok = false;
      break;
    }
    const uint32_t cnt = (uint32_t)__popcll(starts);
    if (nsym + cnt > sym_cap) {
      ok = false;
      break;
    }
    // every lane stores: the cut starts in order (the cuts keep the lower
    // ranks), the others into the spare entries past the buffer
    obuf[(starts >> lane) & 1ull ? nbuf + rank : kOutBuf + (uint32_t)lane] = (uint16_t)sy;
    nsym += cnt;
    nbuf += cnt;
    if (nbuf > kOutBuf - 64 || done) flush();
    o += adv;
    in_grp += cnt;
    const bool next_group = in_grp == kGroupSize;
    in_grp = next_group ? 0u : in_grp;
    g += next_group ? 1u : 0u;
    t = next_group ? t_next : t;
  }
  // end of stream: magic 0x177245385090, the combined CRC (= the block CRC
  // for a one-block stream), padding to a byte
  if (ok) {
    if (o + 80 > total_bits) {
      ok = false;
    } else {
      __syncthreads();
      stage_be_words(D.win, src, len, o >> 5, 8);
      __syncthreads();
      const uint32_t r = o & 31u;
      const uint32_t a = bits32(D.win, r), c = bits32(D.win, r + 32), d = bits32(D.win, r + 64);
      const uint32_t magic_hi = a, magic_lo = c >> 16;
      const uint32_t stored = (c << 16) | (d >> 16);
      ok = magic_hi == 0x17724538u && magic_lo == 0x5090u && stored == crc && nsym >= 1;
    }
  }
  if (!ok) {
    fail();
    return;
  }
  if (lane == 0) {
    DecSlot &D2 = slots[slot];
    D2.valid = 1;
    D2.band = b;
    D2.start_byte = start;
    D2.end_byte = start + (o + 80 + 7) / 8;
    D2.crc = crc;
    D2.orig_ptr = orig_ptr;
    D2.n_in_use = n_in_use;
    D2.n_sym = nsym;
    D2.sym_off = sym0;
  }
}


// ---------------------------------------------------------------- block layout scans
// Exclusive scan of one value per thread over a 1024-thread workgroup; the
// total goes to *total (every thread).
__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
  const int lane = lane_id(), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t x = v;
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)x, d);
    if (lane >= d) x += o;
  }
  __syncthreads();
  if (lane == kWave - 1) sh[wave] = x;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (int k = 0; k < nw; k++) {
    if (k < wave) before += sh[k];
    tot += sh[k];
  }
  total = tot;
  return before + x - v;
}

// Checks that every band's streams were all read, then lays out the
// move-to-front chunks and segments of the valid slots.
__global__ __launch_bounds__(1024) void k_dec_layout1(const DecBand *bands, uint32_t n_bands, DecSlot *slots,
                                                      uint32_t n_slots, uint32_t *chunk_slot, uint32_t *seg_slot,
                                                      uint32_t *ctr) {
  __shared__ uint32_t sh[32];
  for (uint32_t b = threadIdx.x; b < n_bands; b += blockDim.x) {
    const DecBand B = bands[b];
    uint32_t last = 0xFFFFFFFFu;
    for (uint32_t k = 0; k < B.nslots; k++)
      if (slots[B.slot0 + k].valid) last = B.slot0 + k;
    if (last == 0xFFFFFFFFu || slots[last].end_byte != B.src_len) set_err(ctr, kDecErrSlots, b);
  }
  uint32_t carry_c = 0, carry_s = 0;
  for (uint32_t base = 0; base < n_slots; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t nc = 0;
    if (i < n_slots && slots[i].valid) nc = (slots[i].n_sym + kDecChunk - 1) / kDecChunk;
    const uint32_t ns = (nc + kDecSeg - 1) / kDecSeg;
    uint32_t tc, ts;
    const uint32_t c0 = carry_c + wg_excl_scan(nc, sh, tc);
    const uint32_t s0 = carry_s + wg_excl_scan(ns, sh, ts);
    if (i < n_slots) {
      slots[i].chunk0 = c0;
      slots[i].n_chunks = nc;
      slots[i].seg0 = s0;
      slots[i].n_segs = ns;
      for (uint32_t k = 0; k < nc; k++) chunk_slot[c0 + k] = i;
      for (uint32_t k = 0; k < ns; k++) seg_slot[s0 + k] = i;
    }
    carry_c += tc;
    carry_s += ts;
  }
  if (threadIdx.x == 0) {
    ctr[kDcChunks] = carry_c;
    ctr[kDcSegs] = carry_s;
  }
}

// ---------------------------------------------------------------- zero runs and move-to-front
// Run position of each zero-run symbol (RUNA = 0, RUNB = 1) in a batch of 64
// symbols, one per lane: how many run symbols directly precede it (`carry`
// counts those before the batch).  Returns the bytes the symbol stands for
// (run digit d at position r: d << r; other symbols 1; end of block 0) and
// updates carry.  Runs of more than 24 digits are errors (flag).
__device__ __forceinline__ uint32_t run_bytes(uint32_t sy, bool valid, uint32_t eob, uint32_t &carry, bool &bad) {
  const int lane = lane_id();
  const bool run = valid && sy <= 1u;
  const uint64_t runs = ballot64(run);
  const uint64_t nonrun_below = ~runs & lanemask_lt();
  const uint32_t r =
      nonrun_below == 0 ? (uint32_t)lane + carry : (uint32_t)(lane - (63 - __clzll((long long)nonrun_below)) - 1);
  uint32_t c = 0;
  if (run) {
    if (r >= 24)
      bad = true;
    else
      c = (sy + 1u) << r;
  } else if (valid && sy != eob) {
    c = 1;
  }
  // run symbols at the top of a full batch continue into the next one
  carry = runs == ~0ull ? carry + 64u : (uint32_t)__clzll((long long)~runs);
  return c;
}

// Run symbols directly before position i0 of a block whose symbols start at s0.
__device__ __forceinline__ uint32_t run_carry_before(const uint16_t *sym, uint32_t s0, uint32_t i0, bool &bad) {
  if (i0 == s0) return 0;
  const int lane = lane_id();
  const int64_t j = (int64_t)i0 - 64 + lane;
  const bool in = j >= (int64_t)s0;
  const bool run = in && sym[j] <= 1u;
  const uint64_t runs = ballot64(run);
  if (~runs == 0ull) {
    bad = true;  // more than 64 run digits in a row
    return 0;
  }
  return (uint32_t)__clzll((long long)~runs);
}

// One wavefront per chunk of 1024 symbols: the move-to-front replay against
// a placeholder list (entry i stands for entry i of the list the chunk
// starts with).  Writes each symbol's placeholder token, the chunk's final
// placeholder list and the bytes it expands to.
__global__ __launch_bounds__(64) void k_imtf_chunk(const DecSlot *slots, const uint16_t *sym, uint8_t *tok,
                                                   const uint32_t *chunk_slot, uint8_t *chunk_fin, uint32_t *chunk_tot,
                                                   uint32_t *ctr) {
  const uint32_t n_chunks = ctr[kDcChunks];
  const int lane = lane_id();
  for (uint32_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    const uint32_t slot = chunk_slot[c];
    const DecSlot S = slots[slot];
    const uint32_t i0 = S.sym_off + (c - S.chunk0) * kDecChunk;
    const uint32_t i1 = min(S.sym_off + S.n_sym, i0 + kDecChunk);
    const uint32_t eob = S.n_in_use + 1, niu = S.n_in_use;
    bool bad = false;
    uint32_t carry = run_carry_before(sym, S.sym_off, i0, bad);
    uint32_t word = (uint32_t)(4 * lane) | (uint32_t)(4 * lane + 1) << 8 | (uint32_t)(4 * lane + 2) << 16 |
                    (uint32_t)(4 * lane + 3) << 24;
    uint64_t total = 0;
    for (uint32_t b0 = i0; b0 < i1; b0 += 64) {
      const uint32_t i = b0 + lane;
      const bool valid = i < i1;
      const uint32_t sy = valid ? sym[i] : 0u;
      uint32_t cb = run_bytes(sy, valid, eob, carry, bad);
      for (int d = 32; d > 0; d >>= 1) cb += (uint32_t)__shfl_xor((int)cb, d);
      total += cb;
      const uint32_t cnt = min(64u, i1 - b0);
      uint32_t tokv = 0;
      for (uint32_t q = 0; q < cnt; q++) {
        const uint32_t s1 = wave_read(sy, (int)q);
        uint32_t token = 0;
        if (s1 <= 1u) {
          token = wave_read(word, 0) & 255u;
        } else if (s1 != eob) {
          const uint32_t j = s1 - 1u;
          if (j >= niu) {
            bad = true;
            break;
          }
          token = (wave_read(word, (int)(j >> 2)) >> (8 * (j & 3u))) & 255u;
          // entries 0..j-1 move up one place, entry j goes to the front
          const uint32_t prevb = (uint32_t)__shfl_up((int)word, 1) >> 24;
          const uint32_t shifted = (word << 8) | (lane ? prevb : 0u);
          const int keep = (int)(j + 1) - 4 * lane;
          const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
          word = (shifted & m) | (word & ~m);
          if (lane == 0) word = (word & ~255u) | token;
        }
        tokv = lane == (int)q ? token : tokv;
      }
      if (valid) tok[i] = (uint8_t)tokv;
      if (bad) break;
    }
    ((uint32_t *)(chunk_fin + (size_t)c * 256))[lane] = word;
    if (lane == 0) {
      if (bad || total >= (1ull << 31)) {
        set_err(ctr, kDecErrMtf, S.band);
        total = 0;
      }
      chunk_tot[c] = (uint32_t)total;
    }
  }
}

// Segment of up to 32 chunks: the composed placeholder permutation (entry i
// of the list after the segment is entry P[i] of the list before it) and
// the bytes the segment expands to.
__global__ __launch_bounds__(256) void k_imtf_seg(const DecSlot *slots, const uint32_t *seg_slot,
                                                  const uint8_t *chunk_fin, const uint32_t *chunk_tot,
                                                  uint8_t *seg_perm, uint32_t *seg_tot, const uint32_t *ctr) {
  __shared__ uint8_t P[256];
  const uint32_t n_segs = ctr[kDcSegs];
  const uint32_t i = threadIdx.x;
  for (uint32_t sg = blockIdx.x; sg < n_segs; sg += gridDim.x) {
    const DecSlot S = slots[seg_slot[sg]];
    const uint32_t c0 = S.chunk0 + (sg - S.seg0) * kDecSeg;
    const uint32_t c1 = min(S.chunk0 + S.n_chunks, c0 + kDecSeg);
    P[i] = (uint8_t)i;
    uint32_t tot = 0;
    __syncthreads();
    for (uint32_t c = c0; c < c1; c++) {
      const uint8_t nv = P[chunk_fin[(size_t)c * 256 + i]];
      tot += chunk_tot[c];
      __syncthreads();
      P[i] = nv;
      __syncthreads();
    }
    seg_perm[(size_t)sg * 256 + i] = P[i];
    if (i == 0) seg_tot[sg] = tot;
    __syncthreads();
  }
}

// One workgroup per slot: the list entering each segment (entries are ranks
// in the symbol map) and the segments' first bytes; the block length m.
__global__ __launch_bounds__(256) void k_imtf_segchain(const DecBand *bands, DecSlot *slots, uint32_t n_slots,
                                                       const uint8_t *seg_perm, const uint32_t *seg_tot,
                                                       uint8_t *seg_in, uint32_t *seg_off, uint32_t *ctr) {
  __shared__ uint8_t X[256];
  const uint32_t slot = blockIdx.x;
  if (slot >= n_slots) return;
  const DecSlot S = slots[slot];
  if (!S.valid) return;
  const uint32_t i = threadIdx.x;
  X[i] = (uint8_t)i;
  __syncthreads();
  uint64_t run = 0;
  for (uint32_t sg = S.seg0; sg < S.seg0 + S.n_segs; sg++) {
    const uint8_t cur = X[i];
    seg_in[(size_t)sg * 256 + i] = cur;
    const uint8_t nv = X[seg_perm[(size_t)sg * 256 + i]];
    if (i == 0) seg_off[sg] = (uint32_t)run;
    run += seg_tot[sg];
    __syncthreads();
    X[i] = nv;
    __syncthreads();
  }
  if (i == 0) {
    const uint32_t limit = 100000u * bands[S.band].level;
    const bool ok = run >= 1 && run <= limit && S.orig_ptr < run;
    slots[slot].m = ok ? (uint32_t)run : 0u;
    if (!ok) set_err(ctr, kDecErrMtf, S.band);
  }
}

// The list entering each chunk of a segment and the chunk's first byte.
__global__ __launch_bounds__(256) void k_imtf_chunkin(const DecSlot *slots, const uint32_t *seg_slot,
                                                      const uint8_t *seg_in, const uint32_t *seg_off,
                                                      const uint8_t *chunk_fin, const uint32_t *chunk_tot,
                                                      uint8_t *chunk_in, uint32_t *chunk_off, const uint32_t *ctr) {
  __shared__ uint8_t X[256];
  const uint32_t n_segs = ctr[kDcSegs];
  const uint32_t i = threadIdx.x;
  for (uint32_t sg = blockIdx.x; sg < n_segs; sg += gridDim.x) {
    const DecSlot S = slots[seg_slot[sg]];
    const uint32_t c0 = S.chunk0 + (sg - S.seg0) * kDecSeg;
    const uint32_t c1 = min(S.chunk0 + S.n_chunks, c0 + kDecSeg);
    X[i] = seg_in[(size_t)sg * 256 + i];
    uint32_t run = seg_off[sg];
    __syncthreads();
    for (uint32_t c = c0; c < c1; c++) {
      chunk_in[(size_t)c * 256 + i] = X[i];
      if (i == 0) chunk_off[c] = run;
      run += chunk_tot[c];
      const uint8_t nv = X[chunk_fin[(size_t)c * 256 + i]];
      __syncthreads();
      X[i] = nv;
      __syncthreads();
    }
  }
}

// Dense blocks: the valid slots in band order, laid out in the block space,
// with their splitters and run-length tiles.
__global__ __launch_bounds__(1024) void k_dec_layout2(const DecBand *bands, uint32_t n_bands, DecSlot *slots,
                                                      uint32_t n_slots, uint32_t *blk_start, uint32_t *blk_slot,
                                                      uint32_t *blk_spl0, uint32_t *blk_tile0, uint32_t *ctr) {
  __shared__ uint32_t sh[32];
  for (uint32_t b = threadIdx.x; b < n_bands; b += blockDim.x) {
    const DecBand B = bands[b];
    uint64_t tot = 0;
    for (uint32_t k = 0; k < B.nslots; k++)
      if (slots[B.slot0 + k].valid) tot += slots[B.slot0 + k].m;
    if (tot > B.blk_cap) {
      set_err(ctr, kDecErrMtf, b);
      for (uint32_t k = 0; k < B.nslots; k++) slots[B.slot0 + k].m = 0;
    }
  }
  __syncthreads();
  uint32_t cb = 0, cl = 0, cs = 0, ct = 0;
  for (uint32_t base = 0; base < n_slots; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool v = i < n_slots && slots[i].valid && slots[i].m > 0;
    const uint32_t m = v ? slots[i].m : 0u;
    const uint32_t nspl = v ? (m + kDecSplit - 1) / kDecSplit + 1 : 0u;
    const uint32_t ntl = v ? (m + kDecTile - 1) / kDecTile : 0u;
    uint32_t tb, tl, ts, tt;
    const uint32_t kb = cb + wg_excl_scan(v ? 1u : 0u, sh, tb);
    const uint32_t kl = cl + wg_excl_scan(m, sh, tl);
    const uint32_t ks = cs + wg_excl_scan(nspl, sh, ts);
    const uint32_t kt = ct + wg_excl_scan(ntl, sh, tt);
    if (i < n_slots) {
      slots[i].blk = v ? kb : 0xFFFFFFFFu;
      slots[i].l_off = kl;
      if (!v) slots[i].valid = 0;
    }
    if (v) {
      blk_start[kb] = kl;
      blk_slot[kb] = i;
      blk_spl0[kb] = ks;
      blk_tile0[kb] = kt;
    }
    cb += tb;
    cl += tl;
    cs += ts;
    ct += tt;
  }
  if (threadIdx.x == 0) {
    blk_start[cb] = cl;
    blk_spl0[cb] = cs;
    blk_tile0[cb] = ct;
    ctr[kDcBlocks] = cb;
    ctr[kDcN] = cl;
    ctr[kDcSpl] = cs;
    ctr[kDcTiles] = ct;
  }
}

// One wavefront per chunk: the bytes of the block (zero runs repeat the
// list's front entry).  Long runs are written by the whole wavefront.
__global__ __launch_bounds__(64) void k_imtf_write(const DecSlot *slots, const uint16_t *sym, const uint8_t *tok,
                                                   const uint32_t *chunk_slot, const uint8_t *chunk_in,
                                                   const uint32_t *chunk_off, const uint8_t *seq_all, uint8_t *L,
                                                   uint32_t n_chunks) {
  __shared__ uint8_t lst[256];
  const int lane = lane_id();
  for (uint32_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    const uint32_t slot = chunk_slot[c];
    const DecSlot S = slots[slot];
    if (!S.valid) continue;
    __syncthreads();
    for (int k = lane; k < 256; k += 64) lst[k] = seq_all[(size_t)slot * 256 + chunk_in[(size_t)c * 256 + k]];
    __syncthreads();
    const uint32_t i0 = S.sym_off + (c - S.chunk0) * kDecChunk;
    const uint32_t i1 = min(S.sym_off + S.n_sym, i0 + kDecChunk);
    const uint32_t eob = S.n_in_use + 1;
    bool bad = false;
    uint32_t carry = run_carry_before(sym, S.sym_off, i0, bad);
    uint8_t *dst = L + S.l_off;
    const uint32_t m = S.m;
    uint32_t run = chunk_off[c];
    for (uint32_t b0 = i0; b0 < i1; b0 += 64) {
      const uint32_t i = b0 + lane;
      const bool valid = i < i1;
      const uint32_t sy = valid ? sym[i] : 0u;
      const uint32_t cb = run_bytes(sy, valid, eob, carry, bad);
      uint32_t x = cb;
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)x, d);
        if (lane >= d) x += o;
      }
      const uint32_t off = run + x - cb;
      const uint32_t tot = wave_read(x, 63);
      const uint8_t byte = lst[valid ? tok[i] : 0];
      const bool big = cb > 32;
      if (!big) {
        for (uint32_t k = 0; k < cb; k++)
          if (off + k < m) dst[off + k] = byte;
      }
      uint64_t bigs = ballot64(big);
      while (bigs) {
        const int l = __ffsll((long long)bigs) - 1;
        bigs &= bigs - 1;
        const uint32_t o2 = wave_read(off, l), n2 = wave_read(cb, l), v2 = wave_read(byte, l);
        for (uint32_t k = lane; k < n2; k += 64)
          if (o2 + k < m) dst[o2 + k] = (uint8_t)v2;
      }
      run += tot;
    }
  }
}

// ---------------------------------------------------------------- inverse BWT
__global__ void k_ibwt_keys(const uint8_t *L, uint32_t N, uint64_t *key) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) key[i] = L[i];
}

// After the stable sort of each block's positions by byte: row i's successor
// (the row of the rotation one further) and its first byte, packed.
__global__ void k_ibwt_pack(const uint64_t *key, const uint32_t *val, const uint32_t *blk_start, uint32_t nb,
                            uint32_t N, uint32_t *E) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint32_t b = upper_index(blk_start, nb, i);
    E[i] = ((val[i] - blk_start[b]) << 8) | (uint32_t)(key[i] & 255u);
  }
}

struct SplitterAt {
  uint32_t b, l0, m, o, nreg, k, pos;
  bool active;
};
__device__ __forceinline__ SplitterAt splitter_at(uint32_t g, const uint32_t *blk_spl0, const uint32_t *blk_start,
                                                  const uint32_t *blk_slot, const DecSlot *slots, uint32_t nb) {
  SplitterAt s;
  s.b = upper_index(blk_spl0, nb, g);
  const DecSlot &S = slots[blk_slot[s.b]];
  s.l0 = blk_start[s.b];
  s.m = S.m;
  s.o = S.orig_ptr;
  s.nreg = (s.m + kDecSplit - 1) / kDecSplit;
  s.k = g - blk_spl0[s.b];
  if (s.k < s.nreg) {
    s.pos = s.k * kDecSplit;
    s.active = true;
  } else {
    s.pos = s.o;
    s.active = (s.o % kDecSplit) != 0;
  }
  return s;
}

// Rows i with i % 64 == 0 and the row of the original string are splitters;
// each walks the successor cycle to the next splitter.
__global__ void k_ibwt_walk1(const uint32_t *E, const DecSlot *slots, const uint32_t *blk_spl0,
                             const uint32_t *blk_start, const uint32_t *blk_slot, uint32_t nb, uint32_t n_spl,
                             uint32_t *spl_nxt, uint32_t *spl_len) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_spl) return;
  const SplitterAt s = splitter_at(g, blk_spl0, blk_start, blk_slot, slots, nb);
  if (!s.active) {
    spl_nxt[g] = 0xFFFFFFFFu;
    spl_len[g] = 0;
    return;
  }
  const uint32_t *e = E + s.l0;
  uint32_t i = s.pos, steps = 0;
  for (;;) {
    i = e[i] >> 8;
    steps++;
    if ((i % kDecSplit) == 0 || i == s.o || steps > s.m) break;
  }
  spl_nxt[g] = (i % kDecSplit) == 0 ? i / kDecSplit : s.nreg;
  spl_len[g] = steps;
}

// One workgroup per block: pointer jumping over the splitters (in LDS) gives
// each splitter's distance to the end of the cycle that starts at the row of
// the original string.  The bytes are that cycle walked from the origin
// again and again until the block is full (what a sequential decoder does):
// a block that repeats a shorter string has one such cycle per repetition,
// any other block one cycle through every row.  The cycle's length must
// therefore divide the block; splitters off the origin's cycle write nothing.
__global__ __launch_bounds__(1024) void k_ibwt_rank(DecSlot *slots, const uint32_t *blk_spl0,
                                                    const uint32_t *blk_slot, const uint32_t *spl_nxt,
                                                    const uint32_t *spl_len, uint32_t *spl_pos, uint32_t *ctr) {
  constexpr uint32_t kPer = (kDecMaxSpl + 1023) / 1024;
  constexpr uint16_t kNil = 0xFFFFu;
  __shared__ uint16_t nx[kDecMaxSpl];
  __shared__ uint32_t d[kDecMaxSpl];
  const uint32_t b = blockIdx.x;
  DecSlot &S = slots[blk_slot[b]];
  const uint32_t s0 = blk_spl0[b], ns = blk_spl0[b + 1] - s0;
  const uint32_t m = S.m, o = S.orig_ptr;
  const uint32_t oi = (o % kDecSplit) == 0 ? o / kDecSplit : ns - 1;
  for (uint32_t e = threadIdx.x; e < ns; e += blockDim.x) {
    const uint32_t t = spl_nxt[s0 + e];
    nx[e] = (t == 0xFFFFFFFFu || t == oi) ? kNil : (uint16_t)t;
    d[e] = spl_len[s0 + e];
  }
  __syncthreads();
  uint32_t rounds = 1;
  while ((1u << rounds) < ns + 1) rounds++;
  for (uint32_t r = 0; r <= rounds; r++) {
    uint32_t nd[kPer], nn[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
      const uint32_t e = threadIdx.x + k * 1024;
      nd[k] = 0;
      nn[k] = kNil;
      if (e < ns && nx[e] != kNil) {
        const uint32_t t = nx[e];
        nd[k] = min(d[e] + d[t], 0x7FFFFFFFu);
        nn[k] = nx[t];
      }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
      const uint32_t e = threadIdx.x + k * 1024;
      if (e < ns && nx[e] != kNil) {
        d[e] = nd[k];
        nx[e] = (uint16_t)nn[k];
      }
    }
    __syncthreads();
  }
  const uint32_t c = d[oi];  // the origin's cycle
  const bool ok = c >= 1 && c <= m && m % c == 0;
  for (uint32_t e = threadIdx.x; e < ns; e += blockDim.x) {
    const bool act = !(e == ns - 1 && (o % kDecSplit) == 0);
    const bool on = e == oi || nx[e] == kNil;  // reached the end: on the origin's cycle
    spl_pos[s0 + e] = (ok && act && on) ? (e == oi ? 0u : c - d[e]) : 0xFFFFFFFFu;
  }
  if (threadIdx.x == 0) {
    S.cyc = ok ? c : 0u;
    if (!ok) set_err(ctr, kDecErrBwt, S.band);
  }
}

// A block that repeats a shorter string: the rest of it copies the cycle.
__global__ __launch_bounds__(256) void k_ibwt_repeat(const DecSlot *slots, const uint32_t *blk_slot,
                                                     const uint32_t *blk_start, uint8_t *T) {
  const DecSlot &S = slots[blk_slot[blockIdx.x]];
  const uint32_t c = S.cyc, m = S.m;
  if (c == 0 || c >= m) return;
  uint8_t *t = T + blk_start[blockIdx.x];
  for (uint32_t k = c + blockIdx.y * blockDim.x + threadIdx.x; k < m; k += gridDim.y * blockDim.x) t[k] = t[k % c];
}

// Each splitter walks again and writes the bytes of its stretch.
__global__ void k_ibwt_walk2(const uint32_t *E, const DecSlot *slots, const uint32_t *blk_spl0,
                             const uint32_t *blk_start, const uint32_t *blk_slot, uint32_t nb, uint32_t n_spl,
                             const uint32_t *spl_len, const uint32_t *spl_pos, uint8_t *T) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_spl) return;
  const uint32_t p = spl_pos[g];
  if (p == 0xFFFFFFFFu) return;
  const SplitterAt s = splitter_at(g, blk_spl0, blk_start, blk_slot, slots, nb);
  if (!s.active) return;
  const uint32_t *e = E + s.l0;
  uint8_t *t = T + s.l0;
  const uint32_t n = spl_len[g];
  if (p + n > s.m) return;
  uint32_t i = s.pos;
  for (uint32_t k = 0; k < n; k++) {
    const uint32_t v = e[i];
    t[p + k] = (uint8_t)v;
    i = v >> 8;
  }
}

// ---------------------------------------------------------------- first run-length stage, inverted
// The stage's decoder has five states (bytes seen of the current run, 1..4,
// or 0 after a count byte): in state 4 a byte is a count (it stands for that
// many copies of the previous byte, then state 0); in state 0 a byte starts
// a run (state 1); otherwise a byte equal to its predecessor extends the run
// and any other byte starts a new one.  A stretch of positions maps each
// entry state to an exit state and to the bytes it produces: those maps
// compose, so tiles and threads are scanned like sums.
struct ML {
  uint32_t map;  // 3 bits per entry state
  uint32_t l0, l1, l2, l3, l4;
};
constexpr uint32_t kMlIdentity = (4u << 12) | (3u << 9) | (2u << 6) | (1u << 3);

__device__ __forceinline__ uint32_t ml_st(uint32_t map, uint32_t j) { return (map >> (3 * j)) & 7u; }
__device__ __forceinline__ uint32_t ml_len(const ML &a, uint32_t j) {
  return j == 0 ? a.l0 : j == 1 ? a.l1 : j == 2 ? a.l2 : j == 3 ? a.l3 : a.l4;
}
// a, then b
__device__ __forceinline__ ML ml_then(const ML &a, const ML &b) {
  ML r;
  const uint32_t s0 = ml_st(a.map, 0), s1 = ml_st(a.map, 1), s2 = ml_st(a.map, 2), s3 = ml_st(a.map, 3),
                 s4 = ml_st(a.map, 4);
  r.map = ml_st(b.map, s0) | ml_st(b.map, s1) << 3 | ml_st(b.map, s2) << 6 | ml_st(b.map, s3) << 9 |
          ml_st(b.map, s4) << 12;
  r.l0 = a.l0 + ml_len(b, s0);
  r.l1 = a.l1 + ml_len(b, s1);
  r.l2 = a.l2 + ml_len(b, s2);
  r.l3 = a.l3 + ml_len(b, s3);
  r.l4 = a.l4 + ml_len(b, s4);
  return r;
}
__device__ __forceinline__ uint32_t st_step(uint32_t st, bool eq) { return st == 4 ? 0u : st == 0 ? 1u : eq ? st + 1 : 1u; }
__device__ __forceinline__ uint32_t st_out(uint32_t st, uint32_t c) { return st == 4 ? c : 1u; }
// one position (byte c, equal to its predecessor or not) applied to every track
__device__ __forceinline__ void ml_push(ML &a, uint32_t c, bool eq) {
  uint32_t s;
  uint32_t map = 0;
  s = ml_st(a.map, 0); a.l0 += st_out(s, c); map |= st_step(s, eq);
  s = ml_st(a.map, 1); a.l1 += st_out(s, c); map |= st_step(s, eq) << 3;
  s = ml_st(a.map, 2); a.l2 += st_out(s, c); map |= st_step(s, eq) << 6;
  s = ml_st(a.map, 3); a.l3 += st_out(s, c); map |= st_step(s, eq) << 9;
  s = ml_st(a.map, 4); a.l4 += st_out(s, c); map |= st_step(s, eq) << 12;
  a.map = map;
}
__device__ __forceinline__ ML ml_shfl_up(const ML &a, int d) {
  ML r;
  r.map = (uint32_t)__shfl_up((int)a.map, d);
  r.l0 = (uint32_t)__shfl_up((int)a.l0, d);
  r.l1 = (uint32_t)__shfl_up((int)a.l1, d);
  r.l2 = (uint32_t)__shfl_up((int)a.l2, d);
  r.l3 = (uint32_t)__shfl_up((int)a.l3, d);
  r.l4 = (uint32_t)__shfl_up((int)a.l4, d);
  return r;
}

// The tile a thread's 16 positions are in, and the thread's map.
struct R1Tile {
  uint32_t b, slot, l0, m, p0, p1;  // block, slot, block start, length, the tile's positions [p0, p1)
};
__device__ __forceinline__ R1Tile r1_tile(uint32_t t, const uint32_t *blk_tile0, const uint32_t *blk_start,
                                          const uint32_t *blk_slot, const DecSlot *slots, uint32_t nb) {
  R1Tile r;
  r.b = upper_index(blk_tile0, nb, t);
  r.slot = blk_slot[r.b];
  r.l0 = blk_start[r.b];
  r.m = slots[r.slot].m;
  r.p0 = (t - blk_tile0[r.b]) * kDecTile;
  r.p1 = min(r.m, r.p0 + kDecTile);
  return r;
}
__device__ __forceinline__ ML r1_thread_map(const uint8_t *T, const R1Tile &r, uint32_t q0) {
  ML a{kMlIdentity, 0, 0, 0, 0, 0};
  uint32_t prevc = q0 > 0 && q0 < r.m ? T[r.l0 + q0 - 1] : 0x100u;
  for (uint32_t k = 0; k < 16; k++) {
    const uint32_t q = q0 + k;
    if (q >= r.p1) break;
    const uint32_t c = T[r.l0 + q];
    ml_push(a, c, c == prevc);
    prevc = c;
  }
  return a;
}
// Exclusive scan of the 256 threads' maps; *tot receives the tile's map.
__device__ __forceinline__ ML ml_wg_excl(const ML &v, ML *sh, ML *tot) {
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  ML x = v;
  for (int d = 1; d < kWave; d <<= 1) {
    const ML o = ml_shfl_up(x, d);
    if (lane >= d) x = ml_then(o, x);
  }
  ML xe = ml_shfl_up(x, 1);
  if (lane == 0) xe = ML{kMlIdentity, 0, 0, 0, 0, 0};
  __syncthreads();
  if (lane == kWave - 1) sh[wave] = x;
  __syncthreads();
  ML before{kMlIdentity, 0, 0, 0, 0, 0};
  for (int k = 0; k < wave; k++) before = ml_then(before, sh[k]);
  if (tot) {
    ML t{kMlIdentity, 0, 0, 0, 0, 0};
    for (int k = 0; k < (int)(blockDim.x / kWave); k++) t = ml_then(t, sh[k]);
    *tot = t;
  }
  return ml_then(before, xe);
}

__global__ __launch_bounds__(256) void k_ir1_tiles(const uint8_t *T, const DecSlot *slots, const uint32_t *blk_tile0,
                                                   const uint32_t *blk_start, const uint32_t *blk_slot, uint32_t nb,
                                                   uint32_t n_tiles, uint32_t *tile_agg) {
  __shared__ ML sh[4];
  const uint32_t t = blockIdx.x;
  if (t >= n_tiles) return;
  const R1Tile r = r1_tile(t, blk_tile0, blk_start, blk_slot, slots, nb);
  const ML a = r1_thread_map(T, r, r.p0 + 16 * threadIdx.x);
  ML tot;
  ml_wg_excl(a, sh, &tot);
  if (threadIdx.x == 0) {
    uint32_t *o = tile_agg + (size_t)t * 6;
    o[0] = tot.map;
    o[1] = tot.l0;
    o[2] = tot.l1;
    o[3] = tot.l2;
    o[4] = tot.l3;
    o[5] = tot.l4;
  }
}

// One wavefront per block: each tile's entry state and first output byte,
// and the block's raw length.
__global__ __launch_bounds__(64) void k_ir1_chain(DecSlot *slots, const uint32_t *blk_tile0, const uint32_t *blk_slot,
                                                  const uint32_t *tile_agg, uint32_t *tile_in) {
  const uint32_t b = blockIdx.x;
  const int lane = lane_id();
  const uint32_t t0 = blk_tile0[b], t1 = blk_tile0[b + 1];
  uint32_t st = 0;
  uint64_t off = 0;
  for (uint32_t base = t0; base < t1; base += 64) {
    const uint32_t t = base + lane;
    uint32_t v[6] = {0, 0, 0, 0, 0, 0};
    if (t < t1)
      for (int k = 0; k < 6; k++) v[k] = tile_agg[(size_t)t * 6 + k];
    const uint32_t cnt = min(64u, t1 - base);
    uint32_t in_st = 0, in_off = 0;
    for (uint32_t q = 0; q < cnt; q++) {
      if (lane == (int)q) {
        in_st = st;
        in_off = (uint32_t)off;
      }
      const uint32_t map = wave_read(v[0], (int)q);
      const uint32_t l = wave_read(st == 0 ? v[1] : st == 1 ? v[2] : st == 2 ? v[3] : st == 3 ? v[4] : v[5], (int)q);
      off += l;
      st = ml_st(map, st);
    }
    if (t < t1) {
      tile_in[(size_t)t * 2] = in_st;
      tile_in[(size_t)t * 2 + 1] = in_off;
    }
  }
  if (lane == 0) slots[blk_slot[b]].raw_len = off > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)off;
}

// Per band: the blocks' raw ranges must add up to the band; they are laid
// out from the band's first raw byte (clamped to the band, so that the
// ranges always tile the raw space).
__global__ __launch_bounds__(1024) void k_dec_layout3(const DecBand *bands, uint32_t n_bands, DecSlot *slots,
                                                      BlockDesc *blocks, uint32_t *blk_raw_start, uint32_t nb,
                                                      uint32_t raw_total, uint32_t *ctr) {
  for (uint32_t b = threadIdx.x; b < n_bands; b += blockDim.x) {
    const DecBand B = bands[b];
    uint64_t tot = 0;
    uint32_t last = 0xFFFFFFFFu;
    for (uint32_t k = 0; k < B.nslots; k++) {
      const DecSlot &S = slots[B.slot0 + k];
      if (S.valid) {
        tot += S.raw_len;
        last = B.slot0 + k;
      }
    }
    const bool ok = tot == B.n && last != 0xFFFFFFFFu;
    if (!ok) set_err(ctr, kDecErrLen, b);
    const uint32_t end = B.raw_off + B.n;
    uint32_t at = B.raw_off;
    for (uint32_t k = 0; k < B.nslots; k++) {
      DecSlot &S = slots[B.slot0 + k];
      if (!S.valid) continue;
      const uint32_t lo = at, hi = (B.slot0 + k == last) ? end : (uint32_t)min<uint64_t>(end, (uint64_t)at + S.raw_len);
      S.raw_off = ok ? lo : 0xFFFFFFFFu;
      blocks[S.blk].raw_start = lo;
      blocks[S.blk].raw_end = hi;
      blk_raw_start[S.blk] = lo;
      at = hi;
    }
  }
  if (threadIdx.x == 0) blk_raw_start[nb] = raw_total;
}

__global__ __launch_bounds__(256) void k_ir1_write(const uint8_t *T, const DecSlot *slots, const uint32_t *blk_tile0,
                                                   const uint32_t *blk_start, const uint32_t *blk_slot, uint32_t nb,
                                                   uint32_t n_tiles, const uint32_t *tile_in, uint8_t *raw) {
  __shared__ ML sh[4];
  const uint32_t t = blockIdx.x;
  if (t >= n_tiles) return;
  const R1Tile r = r1_tile(t, blk_tile0, blk_start, blk_slot, slots, nb);
  const DecSlot &S = slots[r.slot];
  const uint32_t q0 = r.p0 + 16 * threadIdx.x;
  const ML a = r1_thread_map(T, r, q0);
  const ML ex = ml_wg_excl(a, sh, nullptr);
  const uint32_t raw_off = S.raw_off;
  if (raw_off == 0xFFFFFFFFu) return;
  const uint32_t tst = tile_in[(size_t)t * 2], toff = tile_in[(size_t)t * 2 + 1];
  uint32_t st = ml_st(ex.map, tst);
  uint32_t off = toff + ml_len(ex, tst);
  const uint32_t lim = S.raw_len;
  uint8_t *dst = raw + raw_off;
  uint32_t prevc = q0 > 0 && q0 < r.m ? T[r.l0 + q0 - 1] : 0x100u;
  for (uint32_t k = 0; k < 16; k++) {
    const uint32_t q = q0 + k;
    if (q >= r.p1) break;
    const uint32_t c = T[r.l0 + q];
    if (st == 4) {
      for (uint32_t j = 0; j < c; j++)
        if (off + j < lim) dst[off + j] = (uint8_t)prevc;
      off += c;
    } else {
      if (off < lim) dst[off] = (uint8_t)c;
      off += 1;
    }
    st = st_step(st, c == prevc);
    prevc = c;
  }
}

__global__ void k_dec_crc_check(const BlockDesc *blocks, const DecSlot *slots, const uint32_t *blk_slot, uint32_t nb,
                                uint32_t *ctr) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const DecSlot &S = slots[blk_slot[b]];
  if (blocks[b].crc != S.crc) set_err(ctr, kDecErrCrc, S.band);
}

// ---------------------------------------------------------------- arrangement, inverted
// Lens-neighbour delta: the first lens column of every view is a running sum
// down the lens rows (mod 2^16), kept apart from the band bytes.
__global__ __launch_bounds__(256) void k_udx_col0(const DecBand *bands, const uint8_t *raw, uint16_t *col0,
                                                  const uint32_t *ctr) {
  const DecBand B = bands[blockIdx.x];
  if (B.id != PCBZ_VIEW_DX || ctr[kDcErr]) return;
  const uint16_t *a = (const uint16_t *)(raw + B.raw_off);
  uint16_t *c = col0 + B.col0_off;
  const uint32_t views = B.pitch * B.pitch;
  for (uint32_t k = threadIdx.x; k < views; k += blockDim.x) {
    uint16_t acc = 0;
    for (uint32_t s = 0; s < B.Rb; s++) {
      acc = (uint16_t)(acc + a[((size_t)k * B.Rb + s) * B.Nt]);
      c[(size_t)k * B.Rb + s] = acc;
    }
  }
}

// One workgroup per (band, lens row): the row's pixels from the arranged
// band (raster copy, inverse view map, view map plus the previous frame, or
// view rows summed along the lens columns).
__global__ __launch_bounds__(256) void k_unarrange(const DecBand *bands, const RowItem *rows, const uint8_t *raw,
                                                   const uint16_t *col0, const uint32_t *ctr) {
  if (ctr[kDcErr]) return;
  const RowItem R = rows[blockIdx.x];
  const DecBand B = bands[R.band];
  if (B.id >= 4) return;  // the predictor family has kernels of its own
  const uint32_t p = B.pitch, W = B.W, s = R.s;
  const uint16_t *a = (const uint16_t *)(raw + B.raw_off);
  uint16_t *out = B.out + (size_t)(B.y0 + s * p) * W;
  const uint32_t npx = p * W;
  if (B.id == PCBZ_VIEW_DX) {
    for (uint32_t k = threadIdx.x; k < p * p; k += blockDim.x) {
      const uint32_t u = k / p, v = k % p;
      const uint16_t *row = a + ((size_t)k * B.Rb + s) * B.Nt;
      uint16_t acc = col0[B.col0_off + (size_t)k * B.Rb + s];
      out[(size_t)u * W + v] = acc;
      for (uint32_t t = 1; t < B.Nt; t++) {
        acc = (uint16_t)(acc + row[t]);
        out[(size_t)u * W + t * p + v] = acc;
      }
    }
    return;
  }
  const uint16_t *prev = B.id == PCBZ_VIEW_DT ? B.prev + (size_t)(B.y0 + s * p) * W : nullptr;
  for (uint32_t i = threadIdx.x; i < npx; i += blockDim.x) {
    const uint32_t u = i / W, x = i % W;
    uint16_t v;
    if (B.id == PCBZ_RASTER) {
      v = a[(size_t)s * npx + i];
    } else {
      const uint32_t t = x / p, vv = x % p;
      v = a[((size_t)(u * p + vv) * B.Rb + s) * B.Nt + t];
      if (prev) v = (uint16_t)(v + prev[i]);
    }
    out[i] = v;
  }
}

// ---------------------------------------------------------------- predictor family, inverted
// Ids 4..15: X = prediction + residual (mod 2^16), the prediction taken from
// already reconstructed neighbours (see the encoder: A left, B above, C
// above-left over pixels, lenses or phase space; four lossless-JPEG
// functions; band-local edges).  The residual comes back from its map
// 0, 1, 2, 3, ... -> 0, -1, 1, -2, ...
__device__ __forceinline__ int32_t dpred_fn(uint32_t f, int32_t A, int32_t B, int32_t C) {
  return f == 0 ? A + B - C : f == 1 ? A + ((B - C) >> 1) : f == 2 ? B + ((A - C) >> 1) : (A + B) >> 1;
}
__device__ __forceinline__ int32_t unzigzag16(uint32_t z) { return (int32_t)(z >> 1) ^ -(int32_t)(z & 1u); }
__device__ __forceinline__ uint16_t predict_inv(uint32_t f, bool hasA, bool hasB, int32_t A, int32_t B, int32_t C,
                                                uint32_t z) {
  const int32_t pred = (hasA && hasB) ? dpred_fn(f, A, B, C) : hasA ? A : hasB ? B : 0;
  return (uint16_t)(pred + unzigzag16(z));
}

// Pixel neighbours (domain 0): one workgroup per band; rows go to threads 256
// at a time and run as a skewed wavefront (at step k thread i takes column
// k - i), the value above coming from the previous thread through LDS.
__global__ __launch_bounds__(256) void k_upred_pixel(const DecBand *bands, const uint8_t *raw, const uint32_t *ctr) {
  __shared__ uint16_t lastv[2][256];
  if (ctr[kDcErr]) return;
  const DecBand B = bands[blockIdx.x];
  if (B.id < 4 || ((B.id - 4) >> 2) != 0) return;
  const uint32_t f = (B.id - 4) & 3, W = B.W, rows = B.Rb * B.pitch;
  const uint16_t *res = (const uint16_t *)(raw + B.raw_off);
  uint16_t *out = B.out + (size_t)B.y0 * W;
  const uint32_t i = threadIdx.x;
  for (uint32_t base = 0; base < rows; base += 256) {
    const uint32_t row = base + i, nr = min(256u, rows - base);
    const bool active = i < nr;
    int32_t a = 0, cB = 0;  // X one to the left, and the value above it
    for (uint32_t k = 0; k < W + nr - 1; k++) {
      const int32_t j = (int32_t)k - (int32_t)i;
      if (active && j >= 0 && j < (int32_t)W) {
        int32_t bv = 0;
        if (row >= 1) bv = i == 0 ? out[(size_t)(row - 1) * W + j] : lastv[(k - 1) & 1][i - 1];
        const uint16_t x = predict_inv(f, j >= 1, row >= 1, a, bv, cB, res[(size_t)row * W + j]);
        out[(size_t)row * W + j] = x;
        lastv[k & 1][i] = x;
        a = x;
        cB = bv;
      }
      __syncthreads();
    }
  }
}

// Lens neighbours (domain 1) and phase space (domain 2): independent lines of
// a 2D recurrence.  Domain 1: one line set per view (u, v), rows are lens rows,
// columns lens columns.  Domain 2: one per (lens row, v), rows are the pixel
// rows u inside the lens, columns lens columns.  A thread walks its set row
// by row and keeps the previous row in LDS.
__global__ void k_upred_lines(const DecBand *bands, const uint8_t *raw, const uint32_t *ctr, uint32_t tpw) {
  extern __shared__ uint16_t rowbuf[];
  if (ctr[kDcErr]) return;
  const DecBand B = bands[blockIdx.x];
  if (B.id < 4) return;
  const uint32_t domain = (B.id - 4) >> 2, f = (B.id - 4) & 3;
  if (domain == 0) return;
  const uint32_t p = B.pitch, W = B.W, Nt = B.Nt;
  const uint32_t nsets = domain == 1 ? p * p : B.Rb * p;
  const uint32_t q = blockIdx.y * tpw + threadIdx.x;
  if (q >= nsets || threadIdx.x >= tpw) return;
  uint16_t *rb = rowbuf + (size_t)threadIdx.x * Nt;
  const uint16_t *res = (const uint16_t *)(raw + B.raw_off);
  uint16_t *out = B.out + (size_t)B.y0 * W;
  const uint32_t nrows = domain == 1 ? B.Rb : p;
  const uint32_t v = q % p, hi = q / p;  // domain 1: u = hi; domain 2: lens row = hi
  for (uint32_t r = 0; r < nrows; r++) {
    const uint32_t yy = domain == 1 ? r * p + hi : hi * p + r;
    const uint16_t *rres = res + (size_t)yy * W;
    uint16_t *rout = out + (size_t)yy * W;
    int32_t a = 0, cB = 0;
    for (uint32_t t = 0; t < Nt; t++) {
      const int32_t bv = r >= 1 ? rb[t] : 0;
      const uint16_t x = predict_inv(f, t >= 1, r >= 1, a, bv, cB, rres[t * p + v]);
      rout[t * p + v] = x;
      rb[t] = x;
      a = x;
      cB = bv;
    }
  }
}

}  // namespace

void launch_dec_front(const DecWork &w, hipStream_t s) {
  trace_stage("dec_huffman");
  for (uint32_t pass = 0; pass < w.max_nslots; pass++)
    PCBZ_LAUNCH(k_dec_block, dim3(w.n_bands), dim3(64), 0, s, w.bands, w.slots, w.seq, w.sym, pass, w.ctr);
  trace_stage("dec_mtf");
  PCBZ_LAUNCH(k_dec_layout1, dim3(1), dim3(1024), 0, s, w.bands, w.n_bands, w.slots, w.n_slots, w.chunk_slot,
              w.seg_slot, w.ctr);
  PCBZ_LAUNCH(k_imtf_chunk, dim3(std::max<uint32_t>(1, std::min<uint32_t>(w.max_chunks, 16384))), dim3(64), 0, s,
              w.slots, w.sym, w.tok, w.chunk_slot, w.chunk_fin, w.chunk_tot, w.ctr);
  const uint32_t gs = std::max<uint32_t>(1, std::min<uint32_t>(w.max_segs, 4096));
  PCBZ_LAUNCH(k_imtf_seg, dim3(gs), dim3(256), 0, s, w.slots, w.seg_slot, w.chunk_fin, w.chunk_tot, w.seg_perm,
              w.seg_tot, w.ctr);
  PCBZ_LAUNCH(k_imtf_segchain, dim3(w.n_slots), dim3(256), 0, s, w.bands, w.slots, w.n_slots, w.seg_perm, w.seg_tot,
              w.seg_in, w.seg_off, w.ctr);
  PCBZ_LAUNCH(k_imtf_chunkin, dim3(gs), dim3(256), 0, s, w.slots, w.seg_slot, w.seg_in, w.seg_off, w.chunk_fin,
              w.chunk_tot, w.chunk_in, w.chunk_off, w.ctr);
  PCBZ_LAUNCH(k_dec_layout2, dim3(1), dim3(1024), 0, s, w.bands, w.n_bands, w.slots, w.n_slots, w.blk_start, w.blk_slot,
              w.blk_spl0, w.blk_tile0, w.ctr);
}

void launch_dec_back(const DecWork &w, const uint32_t *hc, int radix_items, const uint32_t *xpow_chunk,
                     const uint32_t *xpow_byte, const uint32_t *xpow2, hipStream_t s) {
  const uint32_t nb = hc[kDcBlocks], N = hc[kDcN], n_spl = hc[kDcSpl], n_tiles = hc[kDcTiles], nc = hc[kDcChunks];
  if (nb == 0 || N == 0) return;
  trace_stage("dec_mtf");
  PCBZ_LAUNCH(k_imtf_write, dim3(std::max<uint32_t>(1, std::min<uint32_t>(nc, 16384))), dim3(64), 0, s, w.slots, w.sym,
              w.tok, w.chunk_slot, w.chunk_in, w.chunk_off, w.seq, w.L, nc);
  const uint32_t g = std::min<uint32_t>((N + 255) / 256, 8192);
  trace_stage("dec_bwt");
  PCBZ_LAUNCH(k_ibwt_keys, dim3(g), dim3(256), 0, s, w.L, N, w.key[0]);
  uint64_t *keys[2] = {w.key[0], w.key[1]};
  uint32_t *vals[2] = {w.val[0], w.val[1]};
  const int cur = radix_sort(keys, vals, w.ctr + kDcN, N, 8, radix_items, true, w.blk_start, w.ctr + kDcBlocks, nb,
                             w.counts, w.ctr + kDcCountN, s);
  PCBZ_LAUNCH(k_ibwt_pack, dim3(g), dim3(256), 0, s, keys[cur], vals[cur], w.blk_start, nb, N, w.E);
  PCBZ_LAUNCH(k_ibwt_walk1, dim3((n_spl + 255) / 256), dim3(256), 0, s, w.E, w.slots, w.blk_spl0, w.blk_start,
              w.blk_slot, nb, n_spl, w.spl_nxt, w.spl_len);
  PCBZ_LAUNCH(k_ibwt_rank, dim3(nb), dim3(1024), 0, s, w.slots, w.blk_spl0, w.blk_slot, w.spl_nxt, w.spl_len,
              w.spl_pos, w.ctr);
  PCBZ_LAUNCH(k_ibwt_walk2, dim3((n_spl + 255) / 256), dim3(256), 0, s, w.E, w.slots, w.blk_spl0, w.blk_start,
              w.blk_slot, nb, n_spl, w.spl_len, w.spl_pos, w.T);
  PCBZ_LAUNCH(k_ibwt_repeat, dim3(nb, 16), dim3(256), 0, s, w.slots, w.blk_slot, w.blk_start, w.T);
  trace_stage("dec_rle1");
  PCBZ_LAUNCH(k_ir1_tiles, dim3(n_tiles), dim3(256), 0, s, w.T, w.slots, w.blk_tile0, w.blk_start, w.blk_slot, nb,
              n_tiles, w.tile_agg);
  PCBZ_LAUNCH(k_ir1_chain, dim3(nb), dim3(64), 0, s, w.slots, w.blk_tile0, w.blk_slot, w.tile_agg, w.tile_in);
  PCBZ_LAUNCH(k_dec_layout3, dim3(1), dim3(1024), 0, s, w.bands, w.n_bands, w.slots, w.blocks, w.blk_raw_start, nb,
              w.raw_total, w.ctr);
  PCBZ_LAUNCH(k_ir1_write, dim3(n_tiles), dim3(256), 0, s, w.T, w.slots, w.blk_tile0, w.blk_start, w.blk_slot, nb,
              n_tiles, w.tile_in, w.raw);
  launch_crc2(w.raw, w.raw_total, w.blocks, w.ctr + kDcBlocks, nb, w.blk_raw_start, xpow_chunk, xpow_byte, xpow2,
              w.crc_acc, s);
  PCBZ_LAUNCH(k_dec_crc_check, dim3((nb + 255) / 256), dim3(256), 0, s, w.blocks, w.slots, w.blk_slot, nb, w.ctr);
  trace_stage("dec_arrange");
  PCBZ_LAUNCH(k_udx_col0, dim3(w.n_bands), dim3(256), 0, s, w.bands, w.raw, w.col0, w.ctr);
  PCBZ_LAUNCH(k_unarrange, dim3(w.n_rows), dim3(256), 0, s, w.bands, w.rows, w.raw, w.col0, w.ctr);
  if (w.pred_pixel) PCBZ_LAUNCH(k_upred_pixel, dim3(w.n_bands), dim3(256), 0, s, w.bands, w.raw, w.ctr);
  if (w.pred_lines) {
    const uint32_t tpw = std::max<uint32_t>(1, std::min<uint32_t>(64, 32768u / std::max<uint32_t>(1, w.nt_max)));
    PCBZ_LAUNCH(k_upred_lines, dim3(w.n_bands, (w.pred_sets + tpw - 1) / tpw), dim3(tpw), (size_t)tpw * w.nt_max * 2,
                s, w.bands, w.raw, w.ctr, tpw);
  }
}

}  // namespace pcbz
