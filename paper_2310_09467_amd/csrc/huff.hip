// huff.hip -- Huffman table construction for every block.
//
// Table count from the symbol count (<200: 2, <800: 3, <2400: 4, <6000: 5,
// else 6, and at most the alphabet size); initial tables cover contiguous
// symbol ranges of roughly equal total frequency (cost 0 inside the range,
// 1 outside); then four rounds of: each 50-symbol group picks the table of
// least total cost (ties to the lowest table), per-table frequencies are
// counted, and each table's code lengths are rebuilt by package-merge with
// weights max(freq, 1) over the whole alphabet and a 17-bit limit.
//
// Package-merge runs on one wavefront per (block, table): leaves sorted by
// (weight, symbol); each level merges the leaves with the pairwise packages
// of the level below, leaves first on equal weight, by computing every
// item's merged position with a binary search in the other list.  Selecting
// the first 2(n-1) items of the top list selects prefixes all the way down,
// so a leaf's length is the number of levels whose selected prefix holds it.
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

constexpr int kLevels = kMaxCodeLen;
constexpr int kMaxItems = 2 * kMaxAlpha + 4;

// One workgroup per block: the frequencies are staged in LDS, one thread cuts
// the alphabet into G contiguous ranges of about equal remaining frequency,
// and the workgroup writes the 0/1 cost tables.
__global__ __launch_bounds__(256) void k_tab_init(const uint32_t *d_nb, BlockCode *codes, const uint32_t *freq,
                                                  uint8_t *cost) {
  __shared__ uint32_t f[kMaxAlpha];
  __shared__ uint64_t P[kMaxAlpha];  // running sums of f
  __shared__ uint32_t lo[kMaxGroups], hi[kMaxGroups];
  const uint32_t b = blockIdx.x;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  const uint32_t nmtf = C.n_mtf, alpha = C.alpha;
  uint32_t G = nmtf < 200 ? 2 : nmtf < 800 ? 3 : nmtf < 2400 ? 4 : nmtf < 6000 ? 5 : 6;
  if (G > alpha) G = alpha;
  for (uint32_t s = threadIdx.x; s < alpha; s += blockDim.x) f[s] = freq[(size_t)b * kMaxAlpha + s];
  __syncthreads();
  if (threadIdx.x == 0) {
    codes[b].n_groups = G;
    codes[b].n_sel = (nmtf + kGroupSize - 1) / kGroupSize;
    // group g takes symbols from `start` until its count times the groups
    // left reaches the remaining count, keeping one symbol for each later
    // group.  With the running sums P (non-decreasing) that end is found by
    // binary search instead of a symbol-by-symbol walk.
    uint64_t run = 0;
#pragma unroll 8
    for (uint32_t s = 0; s < alpha; s++) {
      run += f[s];
      P[s] = run;
    }
    uint64_t remaining = nmtf;
    uint32_t start = 0;
    for (uint32_t g = 0; g < G; g++) {
      const uint32_t left = G - g;
      const uint64_t before = start > 0 ? P[start - 1] : 0ull;
      uint32_t end;
      if (g == G - 1) {
        end = alpha - 1;
      } else {
        uint32_t a = start, z = alpha - 1;  // first s in [start, alpha - 1] with (P[s] - before) * left >= remaining
        while (a < z) {
          const uint32_t mid = (a + z) >> 1;
          if ((P[mid] - before) * left >= remaining) z = mid; else a = mid + 1;
        }
        end = min(a, alpha - left);
      }
      lo[g] = start;
      hi[g] = end;
      remaining -= P[end] - before;
      start = end + 1;
    }
  }
  __syncthreads();
  uint8_t *cst = cost + (size_t)b * kMaxGroups * kMaxAlpha;
  for (uint32_t i = threadIdx.x; i < G * alpha; i += blockDim.x) {
    const uint32_t g = i / alpha, sy = i % alpha;
    cst[g * kMaxAlpha + sy] = (sy >= lo[g] && sy <= hi[g]) ? 0 : 1;
  }
}

// Selector bases per block (serial over blocks).
__global__ void k_sel_bases(const uint32_t *d_nb, BlockCode *codes, uint32_t *group_base, uint32_t *d_n_groups) {
  if (threadIdx.x != 0) return;
  const uint32_t nb = *d_nb;
  uint32_t acc = 0;
  for (uint32_t b = 0; b < nb; b++) {
    group_base[b] = acc;
    codes[b].sel_start = acc;
    acc += codes[b].n_sel;
  }
  group_base[nb] = acc;
  *d_n_groups = acc;
}

// One workgroup per 64 selector groups, four lanes per group (each sums
// the costs of every fourth symbol; the lanes then combine their sums).
constexpr int kSelLanes = 4;
constexpr int kSelGroups = 64;
constexpr int kSelThreads = kSelGroups * kSelLanes;

__global__ __launch_bounds__(kSelThreads) void k_tab_select(const uint16_t *sym, const uint32_t *d_nb,
                                                            const BlockCode *codes, const uint32_t *group_base,
                                                            const uint32_t *d_n_groups, const uint8_t *cost,
                                                            uint8_t *sel, uint32_t *tfreq) {
  __shared__ uint32_t tf[kMaxGroups * kMaxAlpha];
  __shared__ uint64_t c03[kMaxAlpha];  // costs of tables 0..3 in 16-bit lanes (a group sums to <= 50*17)
  __shared__ uint32_t c45[kMaxAlpha];  // tables 4..5
  __shared__ uint16_t ssym[kSelGroups * kGroupSize];
  const uint32_t ngroups = *d_n_groups, nb = *d_nb;
  const uint32_t g0 = blockIdx.x * kSelGroups;
  if (g0 >= ngroups) return;
  for (int i = threadIdx.x; i < kMaxGroups * kMaxAlpha; i += kSelThreads) tf[i] = 0;
  // block of a group: the number of blocks b in [1, nb) with
  // group_base[b] <= group; with fewer than 64 blocks every lane holds one
  // group base and a ballot counts them (one load instead of a search)
  const bool lane_tab = nb < (uint32_t)kWave;
  const int lane = lane_id();
  const uint32_t gbl = lane_tab && lane >= 1 && (uint32_t)lane < nb ? group_base[lane] : 0xFFFFFFFFu;
  auto block_of_group = [&](uint32_t grp) -> uint32_t {
    return lane_tab ? (uint32_t)__popcll(ballot64(gbl <= grp)) : upper_index(group_base, nb, grp);
  };
  const uint32_t b0 = block_of_group(g0);
  const BlockCode C0 = codes[b0];
  {
    const uint8_t *cst = cost + (size_t)b0 * kMaxGroups * kMaxAlpha;
    for (uint32_t s = threadIdx.x; s < C0.alpha; s += kSelThreads) {
      c03[s] = (uint64_t)cst[s] | ((uint64_t)cst[kMaxAlpha + s] << 16) | ((uint64_t)cst[2 * kMaxAlpha + s] << 32) |
               ((uint64_t)cst[3 * kMaxAlpha + s] << 48);
      c45[s] = (uint32_t)cst[4 * kMaxAlpha + s] | ((uint32_t)cst[5 * kMaxAlpha + s] << 16);
    }
  }
  // this workgroup's symbols, staged with coalesced loads
  const uint32_t first_sym = C0.sym_start + (g0 - group_base[b0]) * kGroupSize;
  uint32_t end_sym;
  {
    const uint32_t gl = min(g0 + (uint32_t)kSelGroups, ngroups) - 1u;
    const uint32_t bl = block_of_group(gl);
    const BlockCode CL = codes[bl];
    end_sym = min(CL.sym_start + (gl - group_base[bl]) * kGroupSize + kGroupSize, CL.sym_start + CL.n_mtf);
  }
  stage_to_lds(ssym, sym + first_sym, end_sym - first_sym);
  __syncthreads();
  const uint32_t gi = g0 + threadIdx.x / kSelLanes, sub = threadIdx.x % kSelLanes;
  const uint32_t b0_end = group_base[b0 + 1];
  // every lane of a group takes the same branches (the group index decides them)
  const bool valid = gi < ngroups;
  uint32_t b = b0;
  if (valid && gi >= b0_end) {  // a group past the workgroup's first block (per lane)
    if (lane_tab) {
      b = 0;
      for (uint32_t j = 1; j < nb; j++) b += gi >= (uint32_t)__builtin_amdgcn_readlane((int)gbl, (int)j) ? 1u : 0u;
    } else {
      b = upper_index(group_base, nb, gi);
    }
  }
  BlockCode C = C0;
  if (b != b0) C = codes[b];
  const uint32_t j = valid ? gi - group_base[b] : 0u;
  const uint32_t lo = C.sym_start + j * kGroupSize;
  const uint32_t hi = valid ? min(C.sym_start + C.n_mtf, lo + kGroupSize) : lo;
  uint64_t a03 = 0;
  uint32_t a45 = 0;
  if (b == b0) {
    for (uint32_t k = lo + sub; k < hi; k += kSelLanes) {
      const uint32_t s = ssym[k - first_sym];
      a03 += c03[s];
      a45 += c45[s];
    }
  } else {
    const uint8_t *cst = cost + (size_t)b * kMaxGroups * kMaxAlpha;
    for (uint32_t k = lo + sub; k < hi; k += kSelLanes) {
      const uint32_t s = ssym[k - first_sym];
      a03 += (uint64_t)cst[s] | ((uint64_t)cst[kMaxAlpha + s] << 16) | ((uint64_t)cst[2 * kMaxAlpha + s] << 32) |
             ((uint64_t)cst[3 * kMaxAlpha + s] << 48);
      a45 += (uint32_t)cst[4 * kMaxAlpha + s] | ((uint32_t)cst[5 * kMaxAlpha + s] << 16);
    }
  }
  // combine the four lanes of the group (16-bit fields cannot carry over: <= 50 * 17)
  for (int d = 1; d < kSelLanes; d <<= 1) {
    const uint32_t lo32 = (uint32_t)__shfl_xor((int)(uint32_t)a03, d);
    const uint32_t hi32 = (uint32_t)__shfl_xor((int)(uint32_t)(a03 >> 32), d);
    a03 += ((uint64_t)hi32 << 32) | lo32;
    a45 += (uint32_t)__shfl_xor((int)a45, d);
  }
  if (valid) {
    const uint32_t c[kMaxGroups] = {(uint32_t)(a03 & 0xFFFFu), (uint32_t)((a03 >> 16) & 0xFFFFu),
                                    (uint32_t)((a03 >> 32) & 0xFFFFu), (uint32_t)(a03 >> 48), a45 & 0xFFFFu,
                                    a45 >> 16};
    uint32_t best = 0, bc = c[0];
    for (uint32_t g = 1; g < C.n_groups; g++)
      if (c[g] < bc) {
        bc = c[g];
        best = g;
      }
    if (sub == 0) sel[C.sel_start + j] = (uint8_t)best;
    // separate loops keep the LDS counters on LDS atomics (a pointer that may
    // point to either memory would make every update a flat atomic)
    if (b == b0) {
      uint32_t *t = tf + best * kMaxAlpha;
      for (uint32_t k = lo + sub; k < hi; k += kSelLanes) atomicAdd(&t[ssym[k - first_sym]], 1u);
    } else {
      uint32_t *t = tfreq + ((size_t)b * kMaxGroups + best) * kMaxAlpha;
      for (uint32_t k = lo + sub; k < hi; k += kSelLanes) atomicAdd(&t[ssym[k - first_sym]], 1u);
    }
  }
  __syncthreads();
  uint32_t *t0 = tfreq + (size_t)b0 * kMaxGroups * kMaxAlpha;
  for (int i = threadIdx.x; i < kMaxGroups * kMaxAlpha; i += kSelThreads)
    if (tf[i]) atomicAdd(&t0[i], tf[i]);
}

// Number of elements of the sorted LDS array a[0, n) below x (kLE: at most
// x) by an 8-way search: a step reads seven pivots at once (one LDS round
// trip instead of three for a binary search) and keeps the part of the range
// they bracket; the predicate is true on a prefix of the pivots, so the last
// true pivot and the first false one bound the count.  Three steps for
// n <= 258 (the levels of package-merge are a chain of these searches).
template <bool kLE>
__device__ __forceinline__ uint32_t count_sorted(const uint32_t *a, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;  // the count lies in [lo, hi]
  while (hi > lo) {
    const uint32_t w = hi - lo;
    uint32_t pv[7];
    bool pr[7];
#pragma unroll
    for (int i = 0; i < 7; i++) pv[i] = lo + (w * (uint32_t)(i + 1) >> 3);  // in [lo, hi), non-decreasing
#pragma unroll
    for (int i = 0; i < 7; i++) {
      const uint32_t v = a[pv[i]];
      pr[i] = kLE ? v <= x : v < x;
    }
    uint32_t nlo = lo, nhi = hi;
#pragma unroll
    for (int i = 0; i < 7; i++)
      if (pr[i]) nlo = pv[i] + 1;
#pragma unroll
    for (int i = 6; i >= 0; i--)
      if (!pr[i]) nhi = pv[i];
    lo = nlo;
    hi = nhi;
  }
  return lo;
}

// One workgroup of 512 threads per (block, table): each leaf and each
// package of a level has its own thread, so a level costs one binary search.
constexpr int kPmThreads = 512;

__global__ __launch_bounds__(kPmThreads) void k_tab_lengths(const uint32_t *d_nb, const BlockCode *codes,
                                                            uint32_t *tfreq, uint8_t *cost, uint8_t *lens,
                                                            uint32_t *code_words, int last) {
  constexpr int kPadAlpha = (kMaxAlpha + 3) / 4 * 4;
  __shared__ __align__(16) uint32_t key_s[kPadAlpha];  // padded with keys above every real one
  __shared__ uint32_t lw[kMaxAlpha];
  __shared__ uint16_t lsym[kMaxAlpha];
  __shared__ uint32_t wt[2][kMaxItems];
  __shared__ uint32_t pw[kMaxItems / 2 + 2];
  __shared__ uint8_t pk[kLevels + 1][kMaxItems];
  __shared__ __align__(4) uint8_t ln[kPadAlpha];
  __shared__ uint32_t nlen[kMaxCodeLen + 2], base[kMaxCodeLen + 2];
  __shared__ uint64_t pkw[kLevels + 1][2 * kPmThreads / kWave];  // package flags of each level as bit words
  __shared__ uint32_t leaves_sel[kLevels + 1];                      // leaves among each level's selected prefix
  const uint32_t b = blockIdx.x / kMaxGroups, g = blockIdx.x % kMaxGroups;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  if (g >= C.n_groups) return;
  const uint32_t n = C.alpha, t = threadIdx.x;
  uint32_t *tfr = tfreq + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  // leaves sorted by (weight, symbol): rank = number of smaller keys,
  // counted four keys per 16-byte LDS read (all lanes read the same words)
  if (t < (uint32_t)kPadAlpha) key_s[t] = t < n ? (max(tfr[t], 1u) << 9) | t : 0xFFFFFFFFu;
  if (t < kMaxCodeLen + 2) nlen[t] = 0;
  __syncthreads();
  if (t < n) {
    const uint32_t key = key_s[t];
    const uint4 *k4 = (const uint4 *)key_s;
    uint32_t r = 0;
#pragma unroll 4
    for (uint32_t u = 0; u < (n + 3) / 4; u++) {
      const uint4 q = k4[u];
      r += (q.x < key ? 1u : 0u) + (q.y < key ? 1u : 0u) + (q.z < key ? 1u : 0u) + (q.w < key ? 1u : 0u);
    }
    lw[r] = key >> 9;
    lsym[r] = (uint16_t)t;
  }
  __syncthreads();
  if (t < n) {
    wt[0][t] = lw[t];
    pk[kLevels][t] = 0;
  }
  int cur = 0;
  uint32_t size = n;
  __syncthreads();
  for (int j = kLevels - 1; j >= 1; j--) {
    const uint32_t np = size / 2;
    if (t < np) pw[t] = wt[cur][2 * t] + wt[cur][2 * t + 1];
    __syncthreads();
    if (t < n) {
      const uint32_t pos = t + count_sorted<false>(pw, np, lw[t]);
      wt[cur ^ 1][pos] = lw[t];
      pk[j][pos] = 0;
    }
    if (t < np) {
      const uint32_t pos = t + count_sorted<true>(lw, n, pw[t]);
      wt[cur ^ 1][pos] = pw[t];
      pk[j][pos] = 1;
    }
    size = n + np;
    cur ^= 1;
    __syncthreads();
    // this level's package flags as bit words (positions t and t + kPmThreads)
    const uint64_t w0 = ballot64(t < size && pk[j][t]);
    const uint64_t w1 = ballot64(t + kPmThreads < size && pk[j][t + kPmThreads]);
    if (lane_id() == 0) {
      pkw[j][t / kWave] = w0;
      pkw[j][kPmThreads / kWave + t / kWave] = w1;
    }
  }
  __syncthreads();
  // select the first 2(n-1) items at the top and follow the packages down:
  // at each level p = packages among the selected prefix, its leaves are the
  // first selc - p leaves, and the level below selects 2p items
  // (one wavefront: lane q counts the packages in bit word q of the prefix)
  if (t < (uint32_t)kWave) {
    uint32_t selc = 2 * (n - 1);
    for (int j = 1; j <= kLevels; j++) {
      uint32_t p = 0;
      if (j < kLevels && t < 2 * kPmThreads / kWave) {
        const uint32_t full = selc / kWave, rest = selc % kWave;
        const uint64_t word = pkw[j][t];
        if (t < full) p = (uint32_t)__popcll(word);
        else if (t == full && rest) p = (uint32_t)__popcll(word & ((1ull << rest) - 1ull));
      }
      // only lanes 0..15 hold words: a prefix sum along the first row of 16
      // lanes with DPP row shifts, the total in lane 15
      p += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)p, 0x111, 0xf, 0xf, false);  // row_shr:1
      p += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)p, 0x112, 0xf, 0xf, false);  // row_shr:2
      p += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)p, 0x114, 0xf, 0xf, false);  // row_shr:4
      p += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)p, 0x118, 0xf, 0xf, false);  // row_shr:8
      p = (uint32_t)__builtin_amdgcn_readlane((int)p, 15);
      if (t == 0) leaves_sel[j] = selc - p;
      selc = 2 * p;
    }
  }
  __syncthreads();
  uint32_t cnt = 0;
  for (int j = 1; j <= kLevels; j++) cnt += t < n && t < leaves_sel[j] ? 1u : 0u;
  if (t < n) {
    ln[lsym[t]] = (uint8_t)cnt;
    atomicAdd(&nlen[cnt], 1u);
  }
  __syncthreads();
  uint8_t *L = lens + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  uint8_t *cst = cost + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  if (t < n) {
    L[t] = ln[t];
    cst[t] = ln[t];
  }
  if (t < (uint32_t)kMaxAlpha) tfr[t] = 0;
  if (last) {
    // canonical codes in (length, symbol) order: first code of each length,
    // plus the symbol's rank among the symbols of that length
    if (t == 0) {
      uint32_t c = 0;
      for (uint32_t l = 1; l <= (uint32_t)kMaxCodeLen; l++) {
        base[l] = c;
        c = (c + nlen[l]) << 1;
      }
    }
    __syncthreads();
    if (t < n) {
      // symbols before t with the same length, four lengths per LDS read
      const uint32_t l = ln[t];
      const uint32_t *l4 = (const uint32_t *)ln;
      uint32_t r = 0;
#pragma unroll 4
      for (uint32_t u = 0; u < t / 4; u++) {
        const uint32_t x = l4[u];
        r += ((x & 255u) == l ? 1u : 0u) + (((x >> 8) & 255u) == l ? 1u : 0u) + (((x >> 16) & 255u) == l ? 1u : 0u) +
             ((x >> 24) == l ? 1u : 0u);
      }
      for (uint32_t u = t & ~3u; u < t; u++) r += ln[u] == l ? 1u : 0u;
      code_words[((size_t)b * kMaxGroups + g) * kMaxAlpha + t] = base[l] + r;
    }
  }
}

}  // namespace

void launch_huff2(const uint16_t *sym, const uint32_t *d_nb, uint32_t max_blocks, uint32_t max_groups,
                  BlockCode *codes, const uint32_t *freq, uint8_t *cost, uint32_t *tfreq, uint32_t *group_base,
                  uint32_t *d_n_groups, uint8_t *sel, uint8_t *lens, uint32_t *code_words, hipStream_t s) {
  PCBZ_LAUNCH(k_tab_init, dim3(max_blocks), dim3(256), 0, s, d_nb, codes, freq, cost);
  PCBZ_LAUNCH(k_sel_bases, dim3(1), dim3(64), 0, s, d_nb, codes, group_base, d_n_groups);
  for (int it = 0; it < 4; it++) {
    PCBZ_LAUNCH(k_tab_select, dim3((max_groups + kSelGroups - 1) / kSelGroups), dim3(kSelThreads), 0, s, sym, d_nb,
                codes, group_base, d_n_groups, cost, sel, tfreq);
    PCBZ_LAUNCH(k_tab_lengths, dim3(max_blocks * kMaxGroups), dim3(kPmThreads), 0, s, d_nb, codes, tfreq, cost, lens,
                       code_words, it == 3 ? 1 : 0);
  }
}

}  // namespace pcbz
