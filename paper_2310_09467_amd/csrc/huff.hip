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

__global__ void k_tab_init(const uint32_t *d_nb, BlockCode *codes, const uint32_t *freq, uint8_t *cost) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= *d_nb) return;
  BlockCode C = codes[b];
  const uint32_t nmtf = C.n_mtf, alpha = C.alpha;
  uint32_t G = nmtf < 200 ? 2 : nmtf < 800 ? 3 : nmtf < 2400 ? 4 : nmtf < 6000 ? 5 : 6;
  if (G > alpha) G = alpha;
  codes[b].n_groups = G;
  codes[b].n_sel = (nmtf + kGroupSize - 1) / kGroupSize;
  const uint32_t *f = freq + (size_t)b * kMaxAlpha;
  uint8_t *cst = cost + (size_t)b * kMaxGroups * kMaxAlpha;
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
    for (uint32_t s = 0; s < alpha; s++) cst[g * kMaxAlpha + s] = (s >= start && s <= end) ? 0 : 1;
    remaining -= acc;
    start = end + 1;
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
  const uint32_t ngroups = *d_n_groups, nb = *d_nb;
  const uint32_t g0 = blockIdx.x * blockDim.x;
  if (g0 >= ngroups) return;
  for (int i = threadIdx.x; i < kMaxGroups * kMaxAlpha; i += 256) tf[i] = 0;
  const uint32_t b0 = upper_index(group_base, nb, g0);
  __syncthreads();
  const uint32_t gi = g0 + threadIdx.x;
  if (gi < ngroups) {
    const uint32_t b = upper_index(group_base, nb, gi);
    const BlockCode C = codes[b];
    const uint32_t j = gi - group_base[b];
    const uint32_t lo = C.sym_start + j * kGroupSize;
    const uint32_t hi = min(C.sym_start + C.n_mtf, lo + kGroupSize);
    const uint8_t *cst = cost + (size_t)b * kMaxGroups * kMaxAlpha;
    uint32_t c[kMaxGroups] = {0, 0, 0, 0, 0, 0};
    for (uint32_t k = lo; k < hi; k++) {
      const uint32_t s = sym[k];
#pragma unroll
      for (int g = 0; g < kMaxGroups; g++) c[g] += cst[g * kMaxAlpha + s];
    }
    uint32_t best = 0, bc = c[0];
    for (uint32_t g = 1; g < C.n_groups; g++)
      if (c[g] < bc) {
        bc = c[g];
        best = g;
      }
    sel[C.sel_start + j] = (uint8_t)best;
    if (b == b0) {
      for (uint32_t k = lo; k < hi; k++) atomicAdd(&tf[best * kMaxAlpha + sym[k]], 1u);
    } else {
      uint32_t *t = tfreq + ((size_t)b * kMaxGroups + best) * kMaxAlpha;
      for (uint32_t k = lo; k < hi; k++) atomicAdd(&t[sym[k]], 1u);
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

// One wavefront per (block, table).
__global__ __launch_bounds__(64) void k_tab_lengths(const uint32_t *d_nb, const BlockCode *codes, uint32_t *tfreq,
                                                    uint8_t *cost, uint8_t *lens, uint32_t *code_words, int last) {
  __shared__ uint32_t lw[kMaxAlpha];
  __shared__ uint16_t lsym[kMaxAlpha];
  __shared__ uint32_t wt[2][kMaxItems];
  __shared__ uint32_t pw[kMaxItems / 2 + 2];
  __shared__ uint8_t pk[kLevels + 1][kMaxItems];
  __shared__ uint8_t ln[kMaxAlpha];
  const uint32_t b = blockIdx.x / kMaxGroups, g = blockIdx.x % kMaxGroups;
  if (b >= *d_nb) return;
  const BlockCode C = codes[b];
  if (g >= C.n_groups) return;
  const uint32_t n = C.alpha;
  const int lane = lane_id();
  uint32_t *tfr = tfreq + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  // leaves sorted by (weight, symbol)
  for (uint32_t s = lane; s < n; s += 64) {
    const uint32_t ws = max(tfr[s], 1u);
    const uint32_t key = (ws << 9) | s;
    uint32_t r = 0;
    for (uint32_t t = 0; t < n; t++) {
      const uint32_t wt2 = max(tfr[t], 1u);
      r += ((wt2 << 9) | t) < key ? 1u : 0u;
    }
    lw[r] = ws;
    lsym[r] = (uint16_t)s;
  }
  __syncthreads();
  int cur = 0;
  uint32_t size = n;
  for (uint32_t i = lane; i < n; i += 64) {
    wt[0][i] = lw[i];
    pk[kLevels][i] = 0;
  }
  __syncthreads();
  for (int j = kLevels - 1; j >= 1; j--) {
    const uint32_t np = size / 2;
    for (uint32_t k = lane; k < np; k += 64) pw[k] = wt[cur][2 * k] + wt[cur][2 * k + 1];
    __syncthreads();
    for (uint32_t i = lane; i < n; i += 64) {
      const uint32_t pos = i + count_less(pw, np, lw[i]);
      wt[cur ^ 1][pos] = lw[i];
      pk[j][pos] = 0;
    }
    for (uint32_t k = lane; k < np; k += 64) {
      const uint32_t pos = k + count_le(lw, n, pw[k]);
      wt[cur ^ 1][pos] = pw[k];
      pk[j][pos] = 1;
    }
    size = n + np;
    cur ^= 1;
    __syncthreads();
  }
  // select the first 2(n-1) items at the top and follow the packages down
  uint32_t cnt[(kMaxAlpha + 63) / 64] = {0, 0, 0, 0, 0};
  uint32_t selc = 2 * (n - 1);
  for (int j = 1; j <= kLevels; j++) {
    uint32_t p = 0;
    for (uint32_t i = lane; i < selc; i += 64) p += pk[j][i];
    for (int d = 32; d > 0; d >>= 1) p += __shfl_xor(p, d);
    const uint32_t q = selc - p;
#pragma unroll
    for (int r = 0; r < (kMaxAlpha + 63) / 64; r++) {
      const uint32_t i = r * 64 + lane;
      if (i < n && i < q) cnt[r]++;
    }
    selc = 2 * p;
  }
#pragma unroll
  for (int r = 0; r < (kMaxAlpha + 63) / 64; r++) {
    const uint32_t i = r * 64 + lane;
    if (i < n) ln[lsym[i]] = (uint8_t)cnt[r];
  }
  __syncthreads();
  uint8_t *L = lens + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  uint8_t *cst = cost + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
  for (uint32_t s = lane; s < n; s += 64) {
    L[s] = ln[s];
    cst[s] = ln[s];
  }
  for (uint32_t s = lane; s < kMaxAlpha; s += 64) tfr[s] = 0;
  if (last && lane == 0) {
    // canonical codes in (length, symbol) order
    uint32_t *cw = code_words + ((size_t)b * kMaxGroups + g) * kMaxAlpha;
    uint32_t c = 0;
    for (uint32_t l = 1; l <= kMaxCodeLen; l++) {
      for (uint32_t s = 0; s < n; s++)
        if (ln[s] == l) cw[s] = c++;
      c <<= 1;
    }
  }
}

}  // namespace

void launch_huff2(const uint16_t *sym, const uint32_t *d_nb, uint32_t max_blocks, uint32_t max_groups,
                  BlockCode *codes, const uint32_t *freq, uint8_t *cost, uint32_t *tfreq, uint32_t *group_base,
                  uint32_t *d_n_groups, uint8_t *sel, uint8_t *lens, uint32_t *code_words, hipStream_t s) {
  fill_u32(tfreq, 0, (size_t)max_blocks * kMaxGroups * kMaxAlpha, s);
  hipLaunchKernelGGL(k_tab_init, dim3((max_blocks + 63) / 64), dim3(64), 0, s, d_nb, codes, freq, cost);
  hipLaunchKernelGGL(k_sel_bases, dim3(1), dim3(64), 0, s, d_nb, codes, group_base, d_n_groups);
  for (int it = 0; it < 4; it++) {
    hipLaunchKernelGGL(k_tab_select, dim3((max_groups + 255) / 256), dim3(256), 0, s, sym, d_nb, codes, group_base,
                       d_n_groups, cost, sel, tfreq);
    hipLaunchKernelGGL(k_tab_lengths, dim3(max_blocks * kMaxGroups), dim3(64), 0, s, d_nb, codes, tfreq, cost, lens,
                       code_words, it == 3 ? 1 : 0);
  }
}

}  // namespace pcbz
