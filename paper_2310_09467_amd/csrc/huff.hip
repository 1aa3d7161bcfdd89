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
    uint64_t remaining = nmtf;
    uint32_t start = 0;
    for (uint32_t g = 0; g < G; g++) {
      const uint32_t left = G - g;
      uint64_t acc = 0;
      uint32_t end;
      if (g == G - 1) {
        end = alpha - 1;
        for (uint32_t s = start; s <= end; s++) acc += f[s];
      } else {
        uint32_t s = start;
        for (;;) {
          acc += f[s];
          if (acc * left >= remaining) break;
          if (alpha - 1 - s == left - 1) break;
          s++;
        }
        end = s;
      }
      lo[g] = start;
      hi[g] = end;
      remaining -= acc;
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

__global__ __launch_bounds__(256) void k_tab_select(const uint16_t *sym, const uint32_t *d_nb,
                                                    const BlockCode *codes, const uint32_t *group_base,
                                                    const uint32_t *d_n_groups, const uint8_t *cost, uint8_t *sel,
                                                    uint32_t *tfreq) {
  __shared__ uint32_t tf[kMaxGroups * kMaxAlpha];
  __shared__ uint64_t c03[kMaxAlpha];  // costs of tables 0..3 in 16-bit lanes (a group sums to <= 50*17)
  __shared__ uint32_t c45[kMaxAlpha];  // tables 4..5
  __shared__ uint16_t ssym[256 * kGroupSize];
  const uint32_t ngroups = *d_n_groups, nb = *d_nb;
  const uint32_t g0 = blockIdx.x * blockDim.x;
  if (g0 >= ngroups) return;
  for (int i = threadIdx.x; i < kMaxGroups * kMaxAlpha; i += 256) tf[i] = 0;
  const uint32_t b0 = upper_index(group_base, nb, g0);
  const BlockCode C0 = codes[b0];
  {
    const uint8_t *cst = cost + (size_t)b0 * kMaxGroups * kMaxAlpha;
    for (uint32_t s = threadIdx.x; s < C0.alpha; s += 256) {
      c03[s] = (uint64_t)cst[s] | ((uint64_t)cst[kMaxAlpha + s] << 16) | ((uint64_t)cst[2 * kMaxAlpha + s] << 32) |
               ((uint64_t)cst[3 * kMaxAlpha + s] << 48);
      c45[s] = (uint32_t)cst[4 * kMaxAlpha + s] | ((uint32_t)cst[5 * kMaxAlpha + s] << 16);
    }
  }
  // this workgroup's symbols, staged with coalesced loads
  const uint32_t first_sym = C0.sym_start + (g0 - group_base[b0]) * kGroupSize;
  uint32_t end_sym;
  {
    const uint32_t gl = min(g0 + 256u, ngroups) - 1u;
    const uint32_t bl = upper_index(group_base, nb, gl);
    const BlockCode CL = codes[bl];
    end_sym = min(CL.sym_start + (gl - group_base[bl]) * kGroupSize + kGroupSize, CL.sym_start + CL.n_mtf);
  }
  stage_to_lds(ssym, sym + first_sym, end_sym - first_sym);
  __syncthreads();
  const uint32_t gi = g0 + threadIdx.x;
  const uint32_t b0_end = group_base[b0 + 1];
  if (gi < ngroups) {
    const uint32_t b = gi < b0_end ? b0 : upper_index(group_base, nb, gi);
    const BlockCode C = codes[b];
    const uint32_t j = gi - group_base[b];
    const uint32_t lo = C.sym_start + j * kGroupSize;
    const uint32_t hi = min(C.sym_start + C.n_mtf, lo + kGroupSize);
    uint32_t c[kMaxGroups] = {0, 0, 0, 0, 0, 0};
    if (b == b0) {
      uint64_t a03 = 0;
      uint32_t a45 = 0;
      for (uint32_t k = lo; k < hi; k++) {
        const uint32_t s = ssym[k - first_sym];
        a03 += c03[s];
        a45 += c45[s];
      }
      c[0] = (uint32_t)(a03 & 0xFFFFu);
      c[1] = (uint32_t)((a03 >> 16) & 0xFFFFu);
      c[2] = (uint32_t)((a03 >> 32) & 0xFFFFu);
      c[3] = (uint32_t)(a03 >> 48);
      c[4] = a45 & 0xFFFFu;
      c[5] = a45 >> 16;
    } else {
      const uint8_t *cst = cost + (size_t)b * kMaxGroups * kMaxAlpha;
      for (uint32_t k = lo; k < hi; k++) {
        const uint32_t s = ssym[k - first_sym];
#pragma unroll
        for (int g = 0; g < kMaxGroups; g++) c[g] += cst[g * kMaxAlpha + s];
      }
    }
    uint32_t best = 0, bc = c[0];
    for (uint32_t g = 1; g < C.n_groups; g++)
      if (c[g] < bc) {
        bc = c[g];
        best = g;
      }
    sel[C.sel_start + j] = (uint8_t)best;
    if (b == b0) {
      for (uint32_t k = lo; k < hi; k++) atomicAdd(&tf[best * kMaxAlpha + ssym[k - first_sym]], 1u);
    } else {
      uint32_t *t = tfreq + ((size_t)b * kMaxGroups + best) * kMaxAlpha;
      for (uint32_t k = lo; k < hi; k++) atomicAdd(&t[ssym[k - first_sym]], 1u);
    }
  }
  __syncthreads();
  uint32_t *t0 = tfreq + (size_t)b0 * kMaxGroups * kMaxAlpha;
  for (int i = threadIdx.x; i < kMaxGroups * kMaxAlpha; i += 256)
    if (tf[i]) atomicAdd(&t0[i], tf[i]);
}

__device__ __forceinline__ uint32_t count_less(const uint32_t *a, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;  // first index with a[i] >= x
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint32_t count_le(const uint32_t *a, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;  // first index with a[i] > x
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One workgroup of 512 threads per (block, table): each leaf and each
// package of a level has its own thread, so a level costs one binary search.
constexpr int kPmThreads = 512;

__global__ __launch_bounds__(kPmThreads) void k_tab_lengths(const uint32_t *d_nb, const BlockCode *codes,
                                                            uint32_t *tfreq, uint8_t *cost, uint8_t *lens,
                                                            uint32_t *code_words, int last) {
  __shared__ uint32_t key_s[kMaxAlpha];
  __shared__ uint32_t lw[kMaxAlpha];
  __shared__ uint16_t lsym[kMaxAlpha];
  __shared__ uint32_t wt[2][kMaxItems];
  __shared__ uint32_t pw[kMaxItems / 2 + 2];
  __shared__ uint8_t pk[kLevels + 1][kMaxItems];
  __shared__ uint8_t ln[kMaxAlpha];
  __shared__ uint32_t nlen[kMaxCodeLen + 2], base[kMaxCodeLen + 2];
  const uint32_t b = blockIdx.x / kMaxGroups, g = blockIdx.x % kMaxGroups;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  if (g >= C.n_groups) return;
  const uint32_t n = C.alpha, t = threadIdx.x;
  uint32_t *tfr = tfreq + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  // leaves sorted by (weight, symbol): rank = number of smaller keys
  if (t < n) key_s[t] = (max(tfr[t], 1u) << 9) | t;
  if (t < kMaxCodeLen + 2) nlen[t] = 0;
  __syncthreads();
  if (t < n) {
    const uint32_t key = key_s[t];
    uint32_t r = 0;
    for (uint32_t u = 0; u < n; u++) r += key_s[u] < key ? 1u : 0u;
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
      const uint32_t pos = t + count_less(pw, np, lw[t]);
      wt[cur ^ 1][pos] = lw[t];
      pk[j][pos] = 0;
    }
    if (t < np) {
      const uint32_t pos = t + count_le(lw, n, pw[t]);
      wt[cur ^ 1][pos] = pw[t];
      pk[j][pos] = 1;
    }
    size = n + np;
    cur ^= 1;
    __syncthreads();
  }
  // select the first 2(n-1) items at the top and follow the packages down
  uint32_t cnt = 0;
  uint32_t selc = 2 * (n - 1);
  for (int j = 1; j <= kLevels; j++) {
    const uint32_t p = (uint32_t)__syncthreads_count(t < selc && pk[j][t]) +
                       (uint32_t)__syncthreads_count(t + kPmThreads < selc && pk[j][t + kPmThreads]);
    if (t < n && t < selc - p) cnt++;
    selc = 2 * p;
  }
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
      const uint32_t l = ln[t];
      uint32_t r = 0;
      for (uint32_t u = 0; u < t; u++) r += ln[u] == l ? 1u : 0u;
      code_words[((size_t)b * kMaxGroups + g) * kMaxAlpha + t] = base[l] + r;
    }
  }
}

}  // namespace

void launch_huff2(const uint16_t *sym, const uint32_t *d_nb, uint32_t max_blocks, uint32_t max_groups,
                  BlockCode *codes, const uint32_t *freq, uint8_t *cost, uint32_t *tfreq, uint32_t *group_base,
                  uint32_t *d_n_groups, uint8_t *sel, uint8_t *lens, uint32_t *code_words, hipStream_t s) {
  fill_u32(tfreq, 0, (size_t)max_blocks * kMaxGroups * kMaxAlpha, s);
  PCBZ_LAUNCH(k_tab_init, dim3(max_blocks), dim3(256), 0, s, d_nb, codes, freq, cost);
  PCBZ_LAUNCH(k_sel_bases, dim3(1), dim3(64), 0, s, d_nb, codes, group_base, d_n_groups);
  for (int it = 0; it < 4; it++) {
    PCBZ_LAUNCH(k_tab_select, dim3((max_groups + 255) / 256), dim3(256), 0, s, sym, d_nb, codes, group_base,
                       d_n_groups, cost, sel, tfreq);
    PCBZ_LAUNCH(k_tab_lengths, dim3(max_blocks * kMaxGroups), dim3(kPmThreads), 0, s, d_nb, codes, tfreq, cost, lens,
                       code_words, it == 3 ? 1 : 0);
  }
}

}  // namespace pcbz
