// judge.hip -- phase-space rearrangement and the 2D-entropy judgement.
//
// Rearrangement (paper Sec. 2.1.1, Fig. 3a/3c): each workgroup stages a lens
// row of the band (pitch pixel rows, a run of lens columns plus the lens to
// their left) in LDS with coalesced reads, then writes every requested
// arrangement with coalesced runs: RASTER (the band as stored), VIEW
// (sub-aperture views (u,v), each an Rb x Nt image over lenses), VIEW_DX
// (lens-neighbour delta inside each view, mod 2^16: left lens, else the lens
// above in the first column, else zero) and VIEW_DT (delta against the
// previous frame, then VIEW order).  Bytes are little-endian (Fig. 2c).
//
// Judgement (Sec. 2.1.2, Eq. 1, Fig. 2c): the rotation sort on the first byte
// only, with ties in generation order, lists rotations bucket by bucket; the
// last column of rotation i is x[i-1].  Adjacent entries of that column are
// therefore (a) x[i-1], x[i'-1] for consecutive occurrences i < i' of the same
// byte, and (b) at each boundary between consecutive non-empty buckets, the
// last entry of one and the first of the next.  The kernel counts (a) with
// one wavefront per 4096-byte segment (ballot match on the byte value finds
// the previous occurrence inside the 64-byte step; a per-wave LDS table
// carries the last one across steps) into a 65536-bin 16-bit LDS histogram
// per workgroup of 16 segments; the workgroup links each byte's chain across
// its segments, and a fix-up pass links workgroup tiles and adds (b).  The score
// S = sum_t Tq(P[t]) with Tq(c) = round(c*log2(c)*2^20) is an exact integer,
// so the lowest-entropy choice (largest S, ties to the lowest id) does not
// depend on summation order.
#include "pcbz_internal.hpp"

namespace pcbz {

namespace {

constexpr int kSeg = 4096;
constexpr int kJWaves = 16;
constexpr int kJTile = kSeg * kJWaves;  // positions per workgroup tile

// ---------------------------------------------------------------- rearrangement
__global__ __launch_bounds__(256) void k_remap(const BandDesc *bands, const RowItem *rows, CandBufs cb,
                                               const uint8_t *forced, uint32_t write_mask, uint32_t lens_per_wg) {
  extern __shared__ uint16_t sm[];
  const RowItem ri = rows[blockIdx.x];
  const BandDesc B = bands[ri.band];
  const uint32_t p = B.pitch, W = B.W, Nt = B.Nt, Rb = B.Rb, s = ri.s;
  const uint32_t t0 = blockIdx.y * lens_per_wg;
  if (t0 >= Nt) return;
  const uint32_t t1 = min(Nt, t0 + lens_per_wg);
  const uint32_t nl = t1 - t0;
  const uint32_t fc = forced ? forced[ri.band] : 0xFFu;
  uint32_t wm = (fc != 0xFFu ? (1u << fc) : B.cand_mask) & write_mask;
  if (!wm) return;
  const bool need_dt = (wm >> 3) & 1;
  const bool need_dx = (wm >> 2) & 1;
  const uint32_t left = (need_dx && t0 > 0) ? 1 : 0;  // stage the lens to the left
  const uint32_t tw = (nl + left) * p;                 // staged tile width in pixels
  const uint32_t x_lo = (t0 - left) * p;
  uint16_t *cur = sm;                   // [p][tw]
  uint16_t *prv = sm + p * tw;          // [p][nl*p] (VIEW_DT only)
  uint16_t *up = prv + (need_dt ? p * nl * p : 0);  // [p][p]: lens above the first lens column
  const size_t row0 = (size_t)B.y0 + (size_t)s * p;
  for (uint32_t e = threadIdx.x; e < p * tw; e += blockDim.x) {
    uint32_t u = e / tw, xx = e % tw;
    cur[e] = B.frame[(row0 + u) * W + x_lo + xx];
  }
  if (need_dt) {
    const uint32_t pw = nl * p;
    for (uint32_t e = threadIdx.x; e < p * pw; e += blockDim.x) {
      uint32_t u = e / pw, xx = e % pw;
      prv[e] = B.prev[(row0 + u) * W + (size_t)t0 * p + xx];
    }
  }
  const bool have_up = need_dx && t0 == 0 && s > 0;
  if (have_up) {
    for (uint32_t e = threadIdx.x; e < p * p; e += blockDim.x) {
      uint32_t u = e / p, v = e % p;
      up[e] = B.frame[(row0 - p + u) * W + v];
    }
  }
  __syncthreads();
  const size_t vstride = (size_t)Rb * Nt;  // elements per view image
  // RASTER: the band rows as stored
  if (wm & 1u) {
    uint16_t *out = (uint16_t *)(cb.p[0] + B.off);
    const uint32_t pw = nl * p;
    for (uint32_t e = threadIdx.x; e < p * pw; e += blockDim.x) {
      uint32_t u = e / pw, xx = e % pw;
      out[((size_t)s * p + u) * W + (size_t)t0 * p + xx] = cur[u * tw + left * p + xx];
    }
  }
  // view-ordered candidates
  const uint32_t nv = p * p * nl;
  for (uint32_t e = threadIdx.x; e < nv; e += blockDim.x) {
    uint32_t uv = e / nl, tt = e % nl;
    uint32_t u = uv / p, v = uv % p;
    uint32_t t = t0 + tt;
    size_t idx = (size_t)uv * vstride + (size_t)s * Nt + t;
    uint16_t a = cur[u * tw + (left + tt) * p + v];
    if (wm & 2u) ((uint16_t *)(cb.p[1] + B.off))[idx] = a;
    if (wm & 4u) {
      uint16_t pred;
      if (t > 0)
        pred = cur[u * tw + (left + tt - 1) * p + v];
      else if (s > 0)
        pred = up[u * p + v];
      else
        pred = 0;
      ((uint16_t *)(cb.p[2] + B.off))[idx] = (uint16_t)(a - pred);
    }
    if (wm & 8u) ((uint16_t *)(cb.p[3] + B.off))[idx] = (uint16_t)(a - prv[u * (nl * p) + tt * p + v]);
  }
}

// ---------------------------------------------------------------- predictor family
// Arrangement ids 4..15 (Sec. 2.1.1, Fig. 1b, Fig. 3b/3c): id = 4 + 4 * domain
// + function.  Each pixel X is predicted from three causal neighbours A
// (left), B (above), C (above-left) taken over neighbouring pixels (domain
// 0), neighbouring lenses (domain 1: the same pixel one lens over) or phase
// space (domain 2: A one lens to the left, B the pixel above inside the
// lens, C the pixel above inside the lens to the left), with the four
// multi-neighbour lossless-JPEG functions A+B-C, A+floor((B-C)/2),
// B+floor((A-C)/2), floor((A+B)/2).  Neighbours must lie in the band: only
// A -> A, only B -> B, neither -> 0.  The residual mod 2^16, read as a signed
// 16-bit value, is mapped 0, -1, 1, -2, ... -> 0, 1, 2, 3, ... and written in
// the band's raster order.  A workgroup stages its lens row and the one
// above (when the band has it), with the lens to the left of its run.
__device__ __forceinline__ int32_t pred_fn(uint32_t f, int32_t A, int32_t B, int32_t C) {
  return f == 0 ? A + B - C : f == 1 ? A + ((B - C) >> 1) : f == 2 ? B + ((A - C) >> 1) : (A + B) >> 1;
}
__device__ __forceinline__ uint16_t zigzag16(int32_t r) {
  const int32_t v = (int16_t)(uint16_t)r;
  return (uint16_t)((v << 1) ^ (v >> 15));
}

__global__ __launch_bounds__(256) void k_predict(const BandDesc *bands, const RowItem *rows, CandBufs cb,
                                                 const uint8_t *forced, uint32_t lens_per_wg) {
  extern __shared__ uint16_t sm[];
  const RowItem ri = rows[blockIdx.x];
  const BandDesc B = bands[ri.band];
  const uint32_t p = B.pitch, W = B.W, Nt = B.Nt, s = ri.s;
  const uint32_t t0 = blockIdx.y * lens_per_wg;
  if (t0 >= Nt) return;
  const uint32_t t1 = min(Nt, t0 + lens_per_wg), nl = t1 - t0;
  const uint32_t fc = forced ? forced[ri.band] : 0xFFu;
  const uint32_t wm = (fc != 0xFFu ? (1u << fc) : B.cand_mask) & 0xFFF0u;
  if (!wm) return;
  const uint32_t left = t0 > 0 ? 1u : 0u, up = s > 0 ? 1u : 0u;
  const uint32_t tw = (nl + left) * p, th = (1 + up) * p;
  const uint32_t x_lo = (t0 - left) * p;
  const size_t row_lo = (size_t)B.y0 + (size_t)(s - up) * p;
  for (uint32_t e = threadIdx.x; e < th * tw; e += blockDim.x) {
    const uint32_t r = e / tw, c = e % tw;
    sm[e] = B.frame[(row_lo + r) * W + x_lo + c];
  }
  __syncthreads();
  const uint32_t pw = nl * p;
  for (uint32_t bits = wm; bits; bits &= bits - 1) {
    const uint32_t id = __ffs(bits) - 1, k = id - 4, domain = k >> 2, f = k & 3;
    uint16_t *out = (uint16_t *)(cb.p[id] + B.off);
    // A one step left along x, B one step up; the step lengths per domain
    const uint32_t ax = domain == 0 ? 1u : p, by = domain == 1 ? p : 1u;
    for (uint32_t e = threadIdx.x; e < p * pw; e += blockDim.x) {
      const uint32_t u = e / pw, xx = e % pw;
      const uint32_t yy = s * p + u, x = t0 * p + xx;
      const uint32_t sr = up * p + u, sc = left * p + xx;
      const int32_t X = sm[sr * tw + sc];
      const bool hasA = x >= ax;
      const bool hasB = domain == 0 ? yy >= 1 : domain == 1 ? s >= 1 : u >= 1;
      int32_t pred = 0;
      if (hasA && hasB)
        pred = pred_fn(f, sm[sr * tw + sc - ax], sm[(sr - by) * tw + sc], sm[(sr - by) * tw + sc - ax]);
      else if (hasA)
        pred = sm[sr * tw + sc - ax];
      else if (hasB)
        pred = sm[(sr - by) * tw + sc];
      out[(size_t)yy * W + x] = zigzag16(X - pred);
    }
  }
}

// ---------------------------------------------------------------- pair histogram
__global__ __launch_bounds__(1024) void k_judge_pairs(const JudgeTask *tasks, const uint32_t *tile_task,
                                                      const uint32_t *tile_local, CandBufs cb, uint16_t *seg_first,
                                                      uint16_t *seg_last, uint32_t *hist_g, const uint8_t *forced) {
  __shared__ uint32_t hist[32768];  // 65536 16-bit bins
  __shared__ uint16_t lastp[kJWaves][256];
  __shared__ uint16_t firstp[kJWaves][256];
  const uint32_t ti = tile_task[blockIdx.x];
  const JudgeTask T = tasks[ti];
  if (forced && forced[T.band] != 0xFFu) return;  // band already decided (uniform per workgroup)
  const uint8_t *x = cb.p[T.cand] + T.x_off;
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < 32768; i += 1024) hist[i] = 0;
  for (int c = lane; c < 256; c += kWave) {
    lastp[w][c] = (uint16_t)kNone16;
    firstp[w][c] = (uint16_t)kNone16;
  }
  __syncthreads();
  const uint32_t seg = tile_local[blockIdx.x] * kJWaves + w;
  const uint64_t p0 = (uint64_t)seg * kSeg;
  const uint32_t n = T.n;
  if (p0 < n) {
    const uint32_t pend = (uint32_t)min<uint64_t>(p0 + kSeg, n);
    uint32_t carry = x[(p0 + n - 1) % n];
    const uint64_t lt = lanemask_lt();
    for (uint32_t base = (uint32_t)p0; base < pend; base += kWave) {
      const uint32_t pos = base + lane;
      const bool valid = pos < pend;
      const uint32_t c = valid ? x[pos] : 0u;
      uint32_t pr = __shfl_up(c, 1);
      if (lane == 0) pr = carry;
      carry = wave_read(c, kWave - 1);
      const uint64_t act = ballot64(valid);
      const uint64_t peers = match_any8(c, act);
      const uint64_t earlier = peers & lt;
      const int j = earlier ? 63 - __clzll(earlier) : lane;
      const uint32_t prj = __shfl(pr, j);
      if (valid) {
        uint32_t q = 0;
        bool have = true;
        if (earlier) {
          q = (prj << 8) | pr;
        } else {
          uint32_t lp = lastp[w][c];
          if (lp != kNone16)
            q = (lp << 8) | pr;
          else {
            firstp[w][c] = (uint16_t)pr;
            have = false;
          }
        }
        if (have) atomicAdd(&hist[q >> 1], 1u << ((q & 1u) * 16u));
        const uint64_t later = peers & ~(lt | (1ull << lane));
        if (!later) lastp[w][c] = (uint16_t)pr;
      }
    }
  }
  __syncthreads();
  // link each byte's occurrence chain across the waves of this tile; the
  // tile's first and last predecessor per byte go to the tile tables
  if (threadIdx.x < 256) {
    const uint32_t c = threadIdx.x;
    uint32_t last = kNone16, first = kNone16;
    for (int wv = 0; wv < kJWaves; wv++) {
      const uint32_t f = firstp[wv][c];
      if (f == kNone16) continue;
      if (last != kNone16) {
        const uint32_t q = (last << 8) | f;
        atomicAdd(&hist[q >> 1], 1u << ((q & 1u) * 16u));
      } else {
        first = f;
      }
      last = lastp[wv][c];
    }
    const size_t tb = (size_t)(T.seg_base + tile_local[blockIdx.x]) * 256 + c;
    seg_first[tb] = (uint16_t)first;
    seg_last[tb] = (uint16_t)last;
  }
  __syncthreads();
  uint32_t *H = hist_g + (size_t)ti * 65536;
  for (int i = threadIdx.x; i < 32768; i += 1024) {
    uint32_t v = hist[i];
    if (v & 0xFFFFu) atomicAdd(&H[2 * i], v & 0xFFFFu);
    if (v >> 16) atomicAdd(&H[2 * i + 1], v >> 16);
  }
}

// Links each byte's occurrence chain across the tiles of a task and adds the
// pairs at bucket boundaries.  One workgroup per task, one thread per byte
// value; pairs are counted in a 16-bit LDS histogram (at most 256 per tile
// boundary plus 255 bucket boundaries per bin) and flushed once.
constexpr int kFixThreads = 1024;

__global__ __launch_bounds__(kFixThreads) void k_judge_fixup(const JudgeTask *tasks, const uint16_t *tile_first,
                                                     const uint16_t *tile_last, uint32_t *hist_g,
                                                     const uint8_t *forced) {
  __shared__ uint32_t lh[32768];
  __shared__ uint16_t fe[256], le[256];
  const JudgeTask T = tasks[blockIdx.x];
  if (forced && forced[T.band] != 0xFFu) return;
  const uint32_t c = threadIdx.x;
  const uint32_t ntile = (T.n + kJTile - 1) / kJTile;
  uint32_t *H = hist_g + (size_t)blockIdx.x * 65536;
  const bool use_lds = ntile <= 200;  // keeps every 16-bit LDS bin below 65536
  for (int i = threadIdx.x; i < 32768; i += kFixThreads) lh[i] = 0;
  __syncthreads();
  auto add = [&](uint32_t q) {
    if (use_lds)
      atomicAdd(&lh[q >> 1], 1u << ((q & 1u) * 16u));
    else
      atomicAdd(&H[q], 1u);
  };
  uint32_t last = kNone16, first_ever = kNone16;
  constexpr uint32_t kBatch = 16;  // independent loads in flight per step
  // threads 0..255 follow the chain of byte c = thread; all threads clear
  // and flush the histogram
  for (uint32_t s0 = 0; c < 256 && s0 < ntile; s0 += kBatch) {
    uint32_t f[kBatch], l[kBatch];
#pragma unroll
    for (uint32_t k = 0; k < kBatch; k++) {
      const size_t sb = (size_t)(T.seg_base + s0 + k) * 256 + c;
      f[k] = s0 + k < ntile ? tile_first[sb] : kNone16;
      l[k] = s0 + k < ntile ? tile_last[sb] : kNone16;
    }
#pragma unroll
    for (uint32_t k = 0; k < kBatch; k++) {
      if (f[k] == kNone16) continue;
      if (last != kNone16)
        add((last << 8) | f[k]);
      else
        first_ever = f[k];
      last = l[k];
    }
  }
  if (c < 256) {
    fe[c] = (uint16_t)first_ever;
    le[c] = (uint16_t)last;
  }
  __syncthreads();
  if (c < 256 && last != kNone16) {
    for (uint32_t c2 = c + 1; c2 < 256; c2++) {
      if (fe[c2] != kNone16) {
        add((last << 8) | fe[c2]);
        break;
      }
    }
  }
  __syncthreads();
  if (use_lds) {
    for (int i = threadIdx.x; i < 32768; i += kFixThreads) {
      const uint32_t v = lh[i];
      if (v & 0xFFFFu) atomicAdd(&H[2 * i], v & 0xFFFFu);
      if (v >> 16) atomicAdd(&H[2 * i + 1], v >> 16);
    }
  }
}

// S[task] += sum Tq(P[t]) over 1024 bins per workgroup; clears the bins.
__global__ __launch_bounds__(256) void k_judge_score(uint32_t *hist_g, const int64_t *tq,
                                                     unsigned long long *score, const JudgeTask *tasks,
                                                     const uint8_t *forced) {
  __shared__ unsigned long long part[256 / kWave];
  if (forced && forced[tasks[blockIdx.y].band] != 0xFFu) return;  // its bins were never touched
  uint32_t *H = hist_g + (size_t)blockIdx.y * 65536 + (size_t)blockIdx.x * 1024;
  unsigned long long acc = 0;
  for (int i = threadIdx.x; i < 1024; i += 256) {
    uint32_t c = H[i];
    if (c) {
      acc += (unsigned long long)tq[c];
      H[i] = 0;
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_down(acc, d);
  if (lane_id() == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < 256 / kWave; i++) t += part[i];
    if (t) atomicAdd(&score[blockIdx.y], t);
  }
}

__global__ void k_choose(const BandDesc * /*bands*/, uint32_t n_bands, const int32_t *task_of,
                         const unsigned long long *score, const JudgeTask *tasks, const uint8_t *forced,
                         uint8_t *choice, double *entropy, int64_t *score_out) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bands) return;
  if (forced && forced[b] != 0xFFu) {
    choice[b] = forced[b];
    return;
  }
  int best = -1;
  int64_t bestS = 0;
  for (int id = 0; id < kNumCand; id++) {
    int32_t t = task_of[b * kNumCand + id];
    if (t < 0) {
      if (entropy) entropy[b * kNumCand + id] = __longlong_as_double(0x7FF8000000000000ll);
      if (score_out) score_out[b * kNumCand + id] = (int64_t)0x8000000000000000ull;
      continue;
    }
    int64_t S = (int64_t)score[t];
    if (score_out) score_out[b * kNumCand + id] = S;
    if (entropy) {
      uint32_t n = tasks[t].n;
      double H = 0.0;
      if (n >= 2) {
        double N = (double)(n - 1);
        H = log2(N) - (double)S / (1048576.0 * N);
      }
      entropy[b * kNumCand + id] = H;
    }
    if (best < 0 || S > bestS) {
      best = id;
      bestS = S;
    }
  }
  choice[b] = (uint8_t)(best < 0 ? 0 : best);
}

// Forced ids: 0xFF = judge this band; ids above 3 are EINVAL, the temporal
// id without a previous frame is ENEEDPREV.  Bad entries are replaced by 0 so
// that later kernels stay in bounds; the host reports the error.
__global__ void k_validate_forced(const BandDesc *bands, uint32_t n_bands, uint8_t *forced, uint32_t *err) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bands) return;
  const uint32_t f = forced[b];
  if (f == 0xFFu) return;
  if (f >= (uint32_t)kNumCand) {
    atomicOr(err, 1u);
    forced[b] = 0;
  } else if (f == 3u && bands[b].prev == nullptr) {
    atomicOr(err, 2u);
    forced[b] = 0;
  }
}

// chosen[g] = candidate region of the band's choice at the same position.
__global__ void k_gather_chosen(const uint32_t *band_start, uint32_t n_bands, CandBufs cb, const uint8_t *choice,
                                uint8_t *chosen, uint64_t total) {
  const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  if (i0 >= total) return;
  const uint64_t i1 = min<uint64_t>(i0 + 16, total);
  uint32_t b0 = upper_index(band_start, n_bands, (uint32_t)i0);
  uint32_t b1 = upper_index(band_start, n_bands, (uint32_t)(i1 - 1));
  if (b0 == b1 && i1 - i0 == 16) {
    const uint4 *src = (const uint4 *)(cb.p[choice[b0]] + i0);
    *(uint4 *)(chosen + i0) = *src;
  } else {
    for (uint64_t i = i0; i < i1; i++) {
      uint32_t b = upper_index(band_start, n_bands, (uint32_t)i);
      chosen[i] = cb.p[choice[b]][i];
    }
  }
}

}  // namespace

size_t remap_lds_bytes(uint32_t pitch, uint32_t lens_per_wg) {
  size_t p = pitch, nl = lens_per_wg;
  return ((nl + 1) * p * p + nl * p * p + p * p) * sizeof(uint16_t);
}

void launch_remap2(const BandDesc *bands, const RowItem *rows, uint32_t n_rows, uint32_t max_chunks,
                   uint32_t lens_per_wg, uint32_t pitch_max, CandBufs cb, const uint8_t *forced,
                   uint32_t write_mask, hipStream_t s) {
  if (!n_rows) return;
  size_t lds = remap_lds_bytes(pitch_max, lens_per_wg);
  PCBZ_LAUNCH(k_remap, dim3(n_rows, max_chunks), dim3(256), lds, s, bands, rows, cb, forced, write_mask,
                     lens_per_wg);
}

size_t predict_lds_bytes(uint32_t pitch, uint32_t lens_per_wg) {
  return (size_t)2 * pitch * (lens_per_wg + 1) * pitch * sizeof(uint16_t);
}

void launch_predict(const BandDesc *bands, const RowItem *rows, uint32_t n_rows, uint32_t max_chunks,
                    uint32_t lens_per_wg, uint32_t pitch_max, CandBufs cb, const uint8_t *forced, hipStream_t s) {
  if (!n_rows) return;
  PCBZ_LAUNCH(k_predict, dim3(n_rows, max_chunks), dim3(256), predict_lds_bytes(pitch_max, lens_per_wg), s, bands,
              rows, cb, forced, lens_per_wg);
}

void launch_judge2(const JudgeTask *tasks, uint32_t n_tasks, const uint32_t *tile_task, const uint32_t *tile_local,
                   uint32_t n_tiles, CandBufs cb, uint16_t *seg_first, uint16_t *seg_last, uint32_t *hist,
                   const int64_t *tq, unsigned long long *score, const uint8_t *forced, hipStream_t s) {
  if (!n_tasks) return;
  PCBZ_LAUNCH(k_judge_pairs, dim3(n_tiles), dim3(1024), 0, s, tasks, tile_task, tile_local, cb, seg_first,
                     seg_last, hist, forced);
  PCBZ_LAUNCH(k_judge_fixup, dim3(n_tasks), dim3(kFixThreads), 0, s, tasks, seg_first, seg_last, hist, forced);
  PCBZ_LAUNCH(k_judge_score, dim3(64, n_tasks), dim3(256), 0, s, hist, tq, score, tasks, forced);
}

void launch_choose2(const BandDesc *bands, uint32_t n_bands, const int32_t *task_of,
                    const unsigned long long *score, const JudgeTask *tasks, const uint8_t *forced, uint8_t *choice,
                    double *entropy, int64_t *score_out, hipStream_t s) {
  if (!n_bands) return;
  PCBZ_LAUNCH(k_choose, dim3((n_bands + 127) / 128), dim3(128), 0, s, bands, n_bands, task_of, score, tasks,
                     forced, choice, entropy, score_out);
}

namespace {
// Per-band forced ids from each frame's caller array (0xFF: judge the band).
__global__ void k_gather_forced(const FrameOut *frames, uint8_t *forced) {
  const FrameOut F = frames[blockIdx.x];
  for (uint32_t k = threadIdx.x; k < F.n_bands; k += blockDim.x)
    forced[F.band_base + k] = F.forced ? F.forced[k] : (uint8_t)0xFFu;
}
}  // namespace

void launch_gather_forced(const FrameOut *frames, uint32_t n_frames, uint8_t *forced, hipStream_t s) {
  if (!n_frames) return;
  PCBZ_LAUNCH(k_gather_forced, dim3(n_frames), dim3(256), 0, s, frames, forced);
}

void launch_validate_forced(const BandDesc *bands, uint32_t n_bands, uint8_t *forced, uint32_t *err,
                            hipStream_t s) {
  if (!n_bands) return;
  PCBZ_LAUNCH(k_validate_forced, dim3((n_bands + 127) / 128), dim3(128), 0, s, bands, n_bands, forced, err);
}

void launch_gather2(const uint32_t *band_start, uint32_t n_bands, CandBufs cb, const uint8_t *choice,
                    uint8_t *chosen, uint64_t total, hipStream_t s) {
  if (!total) return;
  uint64_t threads = (total + 15) / 16;
  PCBZ_LAUNCH(k_gather_chosen, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, band_start, n_bands,
                     cb, choice, chosen, total);
}

}  // namespace pcbz
