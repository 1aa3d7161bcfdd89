/*
 * pcbz_oracle.c -- CPU oracle for the PC-bzip2 hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the GPU library.  Plain sequential
 * code in the order the method states its steps; speed is not a goal.
 *
 * Paper map (arXiv 2310.09467):
 *   - lenslet layout, lens-neighbour ("angular"/"spatial") prediction:
 *     Sec. 2.1 and 2.1.1, Fig. 1a/1b, Fig. 3a/3c;
 *   - residual -> non-negative "symbol image": Fig. 2a, Fig. 3b;
 *   - 16-bit image read as an 8-bit string, rotation sort on the first byte
 *     only with ties in generation order, last column, adjacent-byte pairs,
 *     2D entropy of the pair histogram: Sec. 2.1.2, Eq. (1), Fig. 2c;
 *   - bzip2 coding of independent blocks, written out in turn: Sec. 2.1.3;
 *   - an 8-bit predictor id in the header: Sec. 2.1.4.
 * The bzip2 stream layout follows the public bzip2 format; every free encoder
 * choice is pinned by the PCBZ-1 profile rules E1..E20 noted below.
 */
#include "pcbz_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Band plan                                                                 */
/* ------------------------------------------------------------------------ */

/* E1: a block holds at most 100000*level - 19 bytes after the first
 * run-length stage, a little under the bound the level digit declares. */
uint32_t orc_block_limit(uint32_t level) { return 100000u * level - 19u; }

static void plan_raw(const orc_params *p, uint32_t *R, uint32_t *nb) {
  uint64_t lens_row_bytes = 2ull * p->pitch * p->w;
  uint64_t r = orc_block_limit(p->level) / lens_row_bytes;
  uint32_t ns = p->h / p->pitch;
  if (r < 1) r = 1;
  *R = (uint32_t)r;
  *nb = (uint32_t)((ns + r - 1) / r);
}

int orc_check_params(const orc_params *p) {
  uint32_t R, nb;
  if (!p) return ORC_EINVAL;
  if (p->pitch == 0 || p->pitch > 65535 || p->h == 0 || p->w == 0) return ORC_EINVAL;
  if (p->h % p->pitch || p->w % p->pitch) return ORC_EINVAL;
  if (p->level < 1 || p->level > 9) return ORC_EINVAL;
  if (p->cand_mask == 0 || (p->cand_mask & ~0xFFFFu)) return ORC_EINVAL;
  plan_raw(p, &R, &nb);
  if (nb > 65535) return ORC_EINVAL;
  return ORC_OK;
}

/* Bands are runs of whole lens rows: R = max(1, floor(limit / (2*pitch*W)))
 * lens rows each, the last band taking what is left.  A band's raw bytes
 * then never exceed one block unless a single lens row already does. */
int orc_plan(const orc_params *p, uint32_t *rows_per_band, uint32_t *n_bands) {
  int st = orc_check_params(p);
  if (st) return st;
  plan_raw(p, rows_per_band, n_bands);
  return ORC_OK;
}

int orc_band_geometry(const orc_params *p, uint32_t band, uint32_t *first_lens_row, uint32_t *lens_rows) {
  uint32_t R, nb, ns;
  int st = orc_plan(p, &R, &nb);
  if (st) return st;
  if (band >= nb) return ORC_EINVAL;
  ns = p->h / p->pitch;
  *first_lens_row = band * R;
  *lens_rows = (ns - band * R) < R ? (ns - band * R) : R;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Arrangements (Sec. 2.1.1; Fig. 2a "symbol images"; Fig. 3)               */
/* ------------------------------------------------------------------------ */

/* Position of raw band pixel (yy, x) in sub-aperture-view order: the p*p
 * views (u, v) one after another, each an Rb x Nt image over lenses (s, t). */
static size_t view_index(uint32_t yy, uint32_t x, uint32_t p, uint32_t Rb, uint32_t Nt) {
  uint32_t s = yy / p, u = yy % p, t = x / p, v = x % p;
  return ((size_t)(u * p + v) * Rb + s) * Nt + t;
}

/* Lens-neighbour predictor inside one view image: the same (u, v) in the
 * left lens; in the first lens column the lens above; zero at the corner.
 * Residuals wrap mod 2^16, which maps them onto the non-negative range. */
static uint16_t dx_pred(const uint16_t *img, uint32_t s, uint32_t t, uint32_t Nt) {
  if (t > 0) return img[(size_t)s * Nt + t - 1];
  if (s > 0) return img[(size_t)(s - 1) * Nt];
  return 0;
}

/* The predictor family of Sec. 2.1.1 and Fig. 3b/3c.  X is predicted from
 * three causal neighbours A, B, C; the paper's Fig. 1b names three choices of
 * them (the figure itself is missing, the text describes them):
 *   domain 0, neighbouring pixels (the paper's spatial continuity): A the
 *     pixel to the left, B the pixel above, C the pixel above-left;
 *   domain 1, neighbouring microlenses (angular continuity): A, B, C the
 *     same pixel in the lens to the left, above, above-left;
 *   domain 2, phase space (both): A the same pixel in the lens to the left,
 *     B the pixel above inside the same lens, C the pixel above inside the
 *     lens to the left.
 * The functions are the four multi-neighbour predictors of lossless JPEG:
 * A + B - C, A + floor((B - C) / 2), B + floor((A - C) / 2),
 * floor((A + B) / 2), in exact integers.  Neighbours must lie in the band:
 * with only A the prediction is A, with only B it is B, with neither 0.  The
 * residual X - prediction is taken mod 2^16 as a signed 16-bit value and
 * mapped onto 0..65535 as 0, -1, 1, -2, 2, ... -> 0, 1, 2, 3, 4, ... (the
 * "positive interval" map of Fig. 3b).  The residual image keeps the band's
 * raster order (the predicted image of Sec. 2.1.2). */
static int32_t pred_fn(int f, int32_t A, int32_t B, int32_t C) {
  int32_t d;
  switch (f) {
    case 0: return A + B - C;
    case 1: d = B - C; return A + (d >= 0 ? d / 2 : -((-d + 1) / 2));
    case 2: d = A - C; return B + (d >= 0 ? d / 2 : -((-d + 1) / 2));
    default: return (A + B) / 2;
  }
}

/* Neighbours of band pixel (yy, x) for a domain; *has receives bit 0 for A,
 * bit 1 for B (C exists when both do). */
static void pred_neighbours(const uint16_t *band, uint32_t W, uint32_t pitch, int domain, uint32_t yy, uint32_t x,
                            int32_t *A, int32_t *B, int32_t *C, int *has) {
  uint32_t dxa, dyb;  /* offsets of A (left) and B (up) */
  int ha, hb;
  if (domain == 0) {
    dxa = 1;
    dyb = 1;
    ha = x >= 1;
    hb = yy >= 1;
  } else if (domain == 1) {
    dxa = pitch;
    dyb = pitch;
    ha = x >= pitch;
    hb = yy >= pitch;
  } else {
    dxa = pitch;
    dyb = 1;
    ha = x >= pitch;
    hb = (yy % pitch) >= 1;
  }
  *has = (ha ? 1 : 0) | (hb ? 2 : 0);
  *A = ha ? band[(size_t)yy * W + x - dxa] : 0;
  *B = hb ? band[(size_t)(yy - dyb) * W + x] : 0;
  *C = (ha && hb) ? band[(size_t)(yy - dyb) * W + x - dxa] : 0;
}

static int32_t predict(const uint16_t *band, uint32_t W, uint32_t pitch, int id, uint32_t yy, uint32_t x) {
  const int k = id - ORC_PRED_FIRST, domain = k / 4, f = k % 4;
  int32_t A, B, C;
  int has;
  pred_neighbours(band, W, pitch, domain, yy, x, &A, &B, &C, &has);
  if (has == 3) return pred_fn(f, A, B, C);
  if (has == 1) return A;
  if (has == 2) return B;
  return 0;
}

/* 16-bit residual -> 0..65535: 0, -1, 1, -2, ... -> 0, 1, 2, 3, ... */
uint16_t orc_zigzag16(uint16_t r) {
  int32_t v = (int16_t)r;
  return (uint16_t)(v >= 0 ? 2 * v : -2 * v - 1);
}
uint16_t orc_unzigzag16(uint16_t z) {
  int32_t v = (z & 1u) ? -(int32_t)((z + 1u) / 2u) : (int32_t)(z / 2u);
  return (uint16_t)v;
}

int orc_arrange(const orc_params *p, uint32_t band, int id, const uint16_t *frame, const uint16_t *prev,
                uint16_t *out) {
  uint32_t y0l, Rb, pitch = p->pitch, W = p->w, Nt, yy, x;
  size_t npix;
  int st = orc_band_geometry(p, band, &y0l, &Rb);
  if (st) return st;
  if (id < 0 || id >= ORC_NCAND) return ORC_EINVAL;
  if (id == ORC_VIEW_DT && !prev) return ORC_ENEEDPREV;
  Nt = W / pitch;
  npix = (size_t)Rb * pitch * W;
  if (id >= ORC_PRED_FIRST) {
    const uint16_t *bandpx = frame + (size_t)y0l * pitch * W;
    for (yy = 0; yy < Rb * pitch; yy++)
      for (x = 0; x < W; x++) {
        int32_t pr = predict(bandpx, W, pitch, id, yy, x);
        out[(size_t)yy * W + x] = orc_zigzag16((uint16_t)((int32_t)bandpx[(size_t)yy * W + x] - pr));
      }
    return ORC_OK;
  }
  for (yy = 0; yy < Rb * pitch; yy++) {
    size_t y = (size_t)y0l * pitch + yy;
    for (x = 0; x < W; x++) {
      uint16_t a = frame[y * W + x];
      size_t idx;
      if (id == ORC_VIEW_DT) a = (uint16_t)(a - prev[y * W + x]);
      idx = (id == ORC_RASTER) ? (size_t)yy * W + x : view_index(yy, x, pitch, Rb, Nt);
      out[idx] = a;
    }
  }
  if (id == ORC_VIEW_DX) {
    uint16_t *view = (uint16_t *)malloc(npix * sizeof(uint16_t));
    size_t k, vsz = (size_t)Rb * Nt;
    uint32_t s, t;
    if (!view) return ORC_ENOMEM;
    memcpy(view, out, npix * sizeof(uint16_t));
    for (k = 0; k < (size_t)pitch * pitch; k++) {
      const uint16_t *img = view + k * vsz;
      for (s = 0; s < Rb; s++)
        for (t = 0; t < Nt; t++)
          out[k * vsz + (size_t)s * Nt + t] = (uint16_t)(img[(size_t)s * Nt + t] - dx_pred(img, s, t, Nt));
    }
    free(view);
  }
  return ORC_OK;
}

int orc_unarrange(const orc_params *p, uint32_t band, int id, const uint16_t *arranged, const uint16_t *prev,
                  uint16_t *frame) {
  uint32_t y0l, Rb, pitch = p->pitch, W = p->w, Nt, yy, x;
  size_t npix;
  uint16_t *a;
  int st = orc_band_geometry(p, band, &y0l, &Rb);
  if (st) return st;
  if (id < 0 || id >= ORC_NCAND) return ORC_EINVAL;
  if (id == ORC_VIEW_DT && !prev) return ORC_ENEEDPREV;
  Nt = W / pitch;
  npix = (size_t)Rb * pitch * W;
  if (id >= ORC_PRED_FIRST) {
    /* raster scan: every neighbour of (yy, x) precedes it */
    uint16_t *bandpx = frame + (size_t)y0l * pitch * W;
    for (yy = 0; yy < Rb * pitch; yy++)
      for (x = 0; x < W; x++) {
        int32_t pr = predict(bandpx, W, pitch, id, yy, x);
        bandpx[(size_t)yy * W + x] = (uint16_t)(pr + (int16_t)orc_unzigzag16(arranged[(size_t)yy * W + x]));
      }
    return ORC_OK;
  }
  a = (uint16_t *)malloc(npix * sizeof(uint16_t));
  if (!a) return ORC_ENOMEM;
  memcpy(a, arranged, npix * sizeof(uint16_t));
  if (id == ORC_VIEW_DX) {
    /* Undo the delta in the same scan order, so every predictor value is
     * already reconstructed when it is needed. */
    size_t k, vsz = (size_t)Rb * Nt;
    uint32_t s, t;
    for (k = 0; k < (size_t)pitch * pitch; k++) {
      uint16_t *img = a + k * vsz;
      for (s = 0; s < Rb; s++)
        for (t = 0; t < Nt; t++) img[(size_t)s * Nt + t] = (uint16_t)(img[(size_t)s * Nt + t] + dx_pred(img, s, t, Nt));
    }
  }
  for (yy = 0; yy < Rb * pitch; yy++) {
    size_t y = (size_t)y0l * pitch + yy;
    for (x = 0; x < W; x++) {
      size_t idx = (id == ORC_RASTER) ? (size_t)yy * W + x : view_index(yy, x, pitch, Rb, Nt);
      uint16_t v = a[idx];
      if (id == ORC_VIEW_DT) v = (uint16_t)(v + prev[y * W + x]);
      frame[y * W + x] = v;
    }
  }
  free(a);
  return ORC_OK;
}

/* Fig. 2c: the 16-bit image is read as a string of bytes, low byte first. */
void orc_to_bytes(const uint16_t *v, size_t count, uint8_t *out) {
  size_t i;
  for (i = 0; i < count; i++) {
    out[2 * i] = (uint8_t)(v[i] & 0xFF);
    out[2 * i + 1] = (uint8_t)(v[i] >> 8);
  }
}

/* ------------------------------------------------------------------------ */
/* Entropy judgement (Sec. 2.1.2, Eq. 1, Fig. 2c)                           */
/* ------------------------------------------------------------------------ */

/* The judge's rotation sort compares only the first byte of each rotation
 * and keeps rotations with equal first bytes in generation order, i.e. it is
 * a stable sort of positions by x[i]; counting sort is such a stable sort.
 * The last column of rotation i is its cyclic predecessor x[i-1]. */
void orc_order1_lastcol(const uint8_t *x, size_t n, uint8_t *T) {
  size_t count[256], next[256], i, run = 0;
  int c;
  if (n == 0) return;
  memset(count, 0, sizeof(count));
  for (i = 0; i < n; i++) count[x[i]]++;
  for (c = 0; c < 256; c++) {
    next[c] = run;
    run += count[c];
  }
  for (i = 0; i < n; i++) T[next[x[i]]++] = x[(i + n - 1) % n];
}

/* Adjacent bytes of the transformed string form n-1 16-bit values (first
 * byte high); P counts each value. */
void orc_pair_hist(const uint8_t *T, size_t n, uint32_t *P) {
  size_t j;
  memset(P, 0, 65536 * sizeof(uint32_t));
  for (j = 0; j + 1 < n; j++) P[((uint32_t)T[j] << 8) | T[j + 1]]++;
}

/* Fixed-point c*log2(c), scaled by 2^20 and rounded to the nearest integer,
 * so that the per-band comparison is an exact integer comparison. */
int64_t orc_tq(uint64_t c) {
  if (c < 2) return 0;
  return (int64_t)llround((double)c * log2((double)c) * 1048576.0);
}

int64_t orc_score(const uint32_t *P) {
  int64_t S = 0;
  int t;
  for (t = 0; t < 65536; t++) S += orc_tq(P[t]);
  return S;
}

/* Shannon entropy in bits of the pair distribution, with N = n-1 pairs:
 * H = -sum (P/N) log2(P/N) = log2 N - (sum P log2 P) / N. */
double orc_entropy_bits(int64_t S, size_t n) {
  double N;
  if (n < 2) return 0.0;
  N = (double)(n - 1);
  return log2(N) - (double)S / (1048576.0 * N);
}

int64_t orc_band_score(const uint8_t *x, size_t n) {
  uint8_t *T = (uint8_t *)malloc(n ? n : 1);
  uint32_t *P = (uint32_t *)malloc(65536 * sizeof(uint32_t));
  int64_t S;
  orc_order1_lastcol(x, n, T);
  orc_pair_hist(T, n, P);
  S = orc_score(P);
  free(T);
  free(P);
  return S;
}

/* Per band, every candidate in the mask is scored; the lowest entropy
 * (largest S, since n is the same for all candidates of a band) wins, ties
 * going to the lowest id.  S[b*4+id] = INT64_MIN and H = NaN for candidates
 * outside the mask. */
int orc_judge(const orc_params *p, const uint16_t *frame, const uint16_t *prev, uint8_t *choice, int64_t *S,
              double *H) {
  uint32_t R, nb, b, y0l, Rb;
  int st = orc_plan(p, &R, &nb), id;
  if (st) return st;
  if ((p->cand_mask & (1u << ORC_VIEW_DT)) && !prev) return ORC_ENEEDPREV;
  for (b = 0; b < nb; b++) {
    size_t npix, n;
    uint16_t *arr;
    uint8_t *bytes;
    int best = -1;
    int64_t bestS = 0;
    orc_band_geometry(p, b, &y0l, &Rb);
    npix = (size_t)Rb * p->pitch * p->w;
    n = 2 * npix;
    arr = (uint16_t *)malloc(npix * sizeof(uint16_t));
    bytes = (uint8_t *)malloc(n);
    if (!arr || !bytes) return ORC_ENOMEM;
    for (id = 0; id < ORC_NCAND; id++) {
      int64_t s;
      if (!(p->cand_mask & (1u << id))) {
        if (S) S[b * ORC_NCAND + id] = INT64_MIN;
        if (H) H[b * ORC_NCAND + id] = NAN;
        continue;
      }
      orc_arrange(p, b, id, frame, prev, arr);
      orc_to_bytes(arr, npix, bytes);
      s = orc_band_score(bytes, n);
      if (S) S[b * ORC_NCAND + id] = s;
      if (H) H[b * ORC_NCAND + id] = orc_entropy_bits(s, n);
      if (best < 0 || s > bestS) {
        best = id;
        bestS = s;
      }
    }
    choice[b] = (uint8_t)best;
    free(arr);
    free(bytes);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* bzip2 block coding, PCBZ-1 profile (Sec. 2.1.3)                          */
/* ------------------------------------------------------------------------ */

/* E4: CRC-32/BZIP2 from its definition: polynomial 0x04C11DB7, bits taken
 * most significant first, initial value and final xor 0xFFFFFFFF. */
uint32_t orc_crc32_bzip2(const uint8_t *data, size_t n) {
  uint32_t crc = 0xFFFFFFFFu;
  size_t i;
  int k;
  for (i = 0; i < n; i++) {
    crc ^= (uint32_t)data[i] << 24;
    for (k = 0; k < 8; k++) crc = (crc & 0x80000000u) ? (crc << 1) ^ 0x04C11DB7u : (crc << 1);
  }
  return crc ^ 0xFFFFFFFFu;
}

/* E2 + E3: the first run-length stage.  Each maximal run of one byte is cut
 * greedily into pieces of at most 255; a piece of length L < 4 is written as
 * L bytes, 4 <= L <= 255 as four copies followed by the count L-4.  Pieces
 * are appended to the current block while it stays within `limit` bytes;
 * otherwise a new block starts with that piece.  Returns the number of
 * output bytes; raw_start[k] / rle_start[k] are where block k starts in the
 * input and the output. */
size_t orc_rle1_blocks(const uint8_t *in, size_t n, uint32_t limit, uint8_t *out, size_t *raw_start,
                       size_t *rle_start, size_t max_blocks, size_t *n_blocks) {
  size_t i = 0, o = 0, cur = 0, nb = 0;
  if (n > 0 && max_blocks > 0) {
    raw_start[0] = 0;
    rle_start[0] = 0;
    nb = 1;
  }
  while (i < n) {
    uint8_t c = in[i];
    size_t r = 1, done = 0;
    while (i + r < n && in[i + r] == c) r++;
    while (done < r) {
      size_t L = (r - done) < 255 ? (r - done) : 255, olen = L < 4 ? L : 5, k;
      if (cur + olen > limit) {
        if (nb < max_blocks) {
          raw_start[nb] = i + done;
          rle_start[nb] = o;
        }
        nb++;
        cur = 0;
      }
      if (L < 4) {
        for (k = 0; k < L; k++) out[o++] = c;
      } else {
        for (k = 0; k < 4; k++) out[o++] = c;
        out[o++] = (uint8_t)(L - 4);
      }
      cur += olen;
      done += L;
    }
    i += r;
  }
  *n_blocks = nb;
  return o;
}

/* E5: Burrows-Wheeler transform over cyclic rotations, ordered by
 * (rotation string, start index).  Prefix doubling: rank_h orders
 * rotations by their first h bytes; sorting (rank_h[i], rank_h[i+h mod m], i)
 * gives rank_2h.  Once 2h >= m, rotations with equal rank are identical and
 * the index key already orders them. */
typedef struct {
  uint32_t a, b, i;
} orc_trip;

static int trip_cmp(const void *x, const void *y) {
  const orc_trip *p = (const orc_trip *)x, *q = (const orc_trip *)y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  return 0;
}

void orc_bwt(const uint8_t *blk, size_t m, uint32_t *sa, uint8_t *L, uint32_t *orig_ptr) {
  uint32_t *rank, *nrank;
  orc_trip *t;
  size_t h = 1, j;
  if (m == 0) {
    *orig_ptr = 0;
    return;
  }
  rank = (uint32_t *)malloc(m * sizeof(uint32_t));
  nrank = (uint32_t *)malloc(m * sizeof(uint32_t));
  t = (orc_trip *)malloc(m * sizeof(orc_trip));
  for (j = 0; j < m; j++) rank[j] = blk[j];
  for (;;) {
    size_t groups = 0;
    uint32_t r = 0;
    for (j = 0; j < m; j++) {
      t[j].a = rank[j];
      t[j].b = rank[(j + h) % m];
      t[j].i = (uint32_t)j;
    }
    qsort(t, m, sizeof(orc_trip), trip_cmp);
    for (j = 0; j < m; j++) {
      if (j == 0 || t[j].a != t[j - 1].a || t[j].b != t[j - 1].b) {
        r = (uint32_t)j;
        groups++;
      }
      nrank[t[j].i] = r;
    }
    memcpy(rank, nrank, m * sizeof(uint32_t));
    if (groups == m || 2 * h >= m) break;
    h *= 2;
  }
  for (j = 0; j < m; j++) {
    sa[j] = t[j].i;
    L[j] = blk[(t[j].i + m - 1) % m];
    if (t[j].i == 0) *orig_ptr = (uint32_t)j;
  }
  free(rank);
  free(nrank);
  free(t);
}

/* E6..E8: the symbol map is exactly the set of byte values in the block;
 * move-to-front runs over their ranks, starting from the ascending list.  A
 * run of r zero outputs becomes the bijective base-2 digits of r, least
 * significant first (digit 1 -> RUNA = 0, digit 2 -> RUNB = 1); a non-zero
 * index v becomes v+1; the end-of-block symbol nInUse+1 closes the block.
 * Returns the symbol count including the end-of-block symbol. */
size_t orc_mtf_rle2(const uint8_t *L, size_t m, uint16_t *sym, uint32_t *freq, uint32_t *n_in_use) {
  int used[256], seq[256], list[256], c, nu = 0;
  size_t i, o = 0, zrun = 0;
  memset(used, 0, sizeof(used));
  for (i = 0; i < m; i++) used[L[i]] = 1;
  for (c = 0; c < 256; c++)
    if (used[c]) {
      seq[c] = nu;
      list[nu] = nu;
      nu++;
    }
  memset(freq, 0, 258 * sizeof(uint32_t));
  for (i = 0; i <= m; i++) {
    int j = -1;
    if (i < m) {
      int v = seq[L[i]], k;
      for (j = 0; list[j] != v; j++) {
      }
      for (k = j; k > 0; k--) list[k] = list[k - 1];
      list[0] = v;
      if (j == 0) {
        zrun++;
        continue;
      }
    }
    while (zrun > 0) {
      uint16_t d = (zrun & 1) ? 0 : 1;
      sym[o++] = d;
      freq[d]++;
      zrun = (zrun - 1 - d) / 2;
    }
    if (i < m) {
      sym[o++] = (uint16_t)(j + 1);
      freq[j + 1]++;
    }
  }
  sym[o++] = (uint16_t)(nu + 1);
  freq[nu + 1]++;
  *n_in_use = (uint32_t)nu;
  return o;
}

/* E13: package-merge (Larmore-Hirschberg) code lengths limited to `limit`.
 * Level lists run from the deepest level up: each level merges the sorted
 * leaves with the packages (consecutive pairs) of the level below, leaves
 * first on equal weight.  The first 2(n-1) items of the top list are
 * selected; a symbol's length is the number of times it occurs in them. */
typedef struct {
  uint64_t w;
  int leaf;  /* 1: leaf with symbol `ref`; 0: package of items 2*ref, 2*ref+1 one level deeper */
  int ref;
} orc_pm_item;

static void pm_count(orc_pm_item **lv, int level, int limit, int idx, uint8_t *len) {
  const orc_pm_item *it = &lv[level][idx];
  if (it->leaf) {
    len[it->ref]++;
    return;
  }
  pm_count(lv, level + 1, limit, 2 * it->ref, len);
  pm_count(lv, level + 1, limit, 2 * it->ref + 1, len);
}

void orc_package_merge(const uint32_t *w, int n, int limit, uint8_t *len) {
  orc_pm_item **lv = (orc_pm_item **)calloc((size_t)limit + 2, sizeof(orc_pm_item *));
  int *size = (int *)calloc((size_t)limit + 2, sizeof(int));
  int *order = (int *)malloc((size_t)n * sizeof(int));
  int i, j, k;
  /* leaves sorted by (weight, symbol): insertion sort keeps it plain */
  for (i = 0; i < n; i++) {
    int s = i;
    for (j = i; j > 0 && (w[order[j - 1]] > w[s] || (w[order[j - 1]] == w[s] && order[j - 1] > s)); j--)
      order[j] = order[j - 1];
    order[j] = s;
  }
  for (j = 1; j <= limit; j++) lv[j] = (orc_pm_item *)malloc((size_t)(2 * n + 2) * sizeof(orc_pm_item));
  for (i = 0; i < n; i++) {
    lv[limit][i].w = w[order[i]];
    lv[limit][i].leaf = 1;
    lv[limit][i].ref = order[i];
  }
  size[limit] = n;
  for (j = limit - 1; j >= 1; j--) {
    int npk = size[j + 1] / 2, li = 0, pi = 0, o = 0;
    while (li < n || pi < npk) {
      uint64_t pw = pi < npk ? lv[j + 1][2 * pi].w + lv[j + 1][2 * pi + 1].w : 0;
      if (li < n && (pi >= npk || (uint64_t)w[order[li]] <= pw)) {
        lv[j][o].w = w[order[li]];
        lv[j][o].leaf = 1;
        lv[j][o].ref = order[li];
        li++;
      } else {
        lv[j][o].w = pw;
        lv[j][o].leaf = 0;
        lv[j][o].ref = pi;
        pi++;
      }
      o++;
    }
    size[j] = o;
  }
  memset(len, 0, (size_t)n);
  for (k = 0; k < 2 * (n - 1); k++) pm_count(lv, 1, limit, k, len);
  for (j = 1; j <= limit; j++) free(lv[j]);
  free(lv);
  free(size);
  free(order);
}

/* E14: canonical codes in (length, symbol) order. */
void orc_canonical_codes(const uint8_t *len, int n, uint32_t *code) {
  uint32_t c = 0;
  int L, s;
  for (L = 1; L <= 20; L++) {
    for (s = 0; s < n; s++)
      if (len[s] == L) code[s] = c++;
    c <<= 1;
  }
}

/* E11: the initial partition of the alphabet 0..alpha-1 into G contiguous
 * ranges.  Range g takes symbols from where range g-1 stopped and closes at
 * the first symbol where its running count reaches the remaining total
 * divided by the ranges left (acc * left >= remaining, in integers), or
 * earlier if every later range still needs one symbol of its own; the last
 * range takes the rest.  end[g] receives the last symbol of range g. */
void orc_huff_init_ranges(const uint32_t *freq, int alpha, int G, uint64_t total, int *end) {
  uint64_t remaining = total;
  int g, s, start = 0;
  for (g = 0; g < G; g++) {
    int left = G - g;
    uint64_t acc = 0;
    if (g == G - 1) {
      end[g] = alpha - 1;
      for (s = start; s <= alpha - 1; s++) acc += freq[s];
    } else {
      s = start;
      for (;;) {
        acc += freq[s];
        if (acc * (uint64_t)left >= remaining) break;
        if (alpha - 1 - s == left - 1) break;
        s++;
      }
      end[g] = s;
    }
    remaining -= acc;
    start = end[g] + 1;
  }
}

/* E12 (a): for each group of 50 symbols (the last one shorter) the table
 * with the smallest summed cost; equal sums go to the lowest table. */
void orc_huff_select(const uint16_t *sym, size_t n_mtf, const uint32_t *cost /* [G][258] */, int G,
                     uint8_t *sel) {
  size_t i, g_i, nsel = (n_mtf + 49) / 50;
  int g;
  for (g_i = 0; g_i < nsel; g_i++) {
    size_t lo = g_i * 50, hi = lo + 50 < n_mtf ? lo + 50 : n_mtf;
    uint64_t best_c = 0;
    int best = 0;
    for (g = 0; g < G; g++) {
      uint64_t c = 0;
      for (i = lo; i < hi; i++) c += cost[g * 258 + sym[i]];
      if (g == 0 || c < best_c) {
        best_c = c;
        best = g;
      }
    }
    sel[g_i] = (uint8_t)best;
  }
}

/* E9..E12: table count by symbol count, initial tables from contiguous
 * ranges of equal cumulative frequency, then four rounds of (choose the
 * cheapest table per group of 50 symbols, count, rebuild lengths). */
int orc_huff_tables(const uint16_t *sym, size_t n_mtf, int alpha, int *n_groups, uint32_t *n_sel, uint8_t *sel,
                    uint8_t *len) {
  uint32_t freq[258], cost[6 * 258], tf[6][258], w[258];
  size_t i, nsel = (n_mtf + 49) / 50;
  int G, g, s, it, end[6], start;
  G = n_mtf < 200 ? 2 : n_mtf < 800 ? 3 : n_mtf < 2400 ? 4 : n_mtf < 6000 ? 5 : 6;
  if (G > alpha) G = alpha;
  memset(freq, 0, sizeof(freq));
  for (i = 0; i < n_mtf; i++) freq[sym[i]]++;
  /* E11: cost 0 inside a table's initial range, 1 outside */
  orc_huff_init_ranges(freq, alpha, G, n_mtf, end);
  for (g = 0, start = 0; g < G; start = end[g] + 1, g++)
    for (s = 0; s < 258; s++) cost[g * 258 + s] = (s >= start && s <= end[g]) ? 0 : 1;
  /* E12 */
  for (it = 0; it < 4; it++) {
    orc_huff_select(sym, n_mtf, cost, G, sel);
    memset(tf, 0, sizeof(tf));
    for (i = 0; i < n_mtf; i++) tf[sel[i / 50]][sym[i]]++;
    for (g = 0; g < G; g++) {
      for (s = 0; s < alpha; s++) w[s] = tf[g][s] > 0 ? tf[g][s] : 1;
      orc_package_merge(w, alpha, 17, len + g * 258);
      for (s = 0; s < alpha; s++) cost[g * 258 + s] = len[g * 258 + s];
    }
  }
  *n_groups = G;
  *n_sel = (uint32_t)nsel;
  return ORC_OK;
}

/* E17: bits go out most significant first. */
typedef struct {
  uint8_t *buf;
  size_t cap;
  uint64_t nbits;
} orc_bw;

static void bw_put(orc_bw *b, int nbits, uint64_t v) {
  int k;
  for (k = nbits - 1; k >= 0; k--) {
    uint64_t pos = b->nbits++;
    if (pos / 8 < b->cap) {
      if ((v >> k) & 1) b->buf[pos / 8] |= (uint8_t)(0x80u >> (pos % 8));
    }
  }
}

/* E18 + E19: one block of first-stage output (m bytes) as one complete
 * stream: "BZh"+level, block header, symbol map, tables, selectors, coded
 * symbols, end-of-stream marker, stream CRC, zero pad to a byte. */
int orc_block_stream(const uint8_t *rle, size_t m, uint32_t block_crc, uint32_t level, uint8_t *out, size_t cap,
                     size_t *len) {
  uint32_t *sa = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
  uint8_t *L = (uint8_t *)malloc(m ? m : 1);
  uint16_t *sym = (uint16_t *)malloc((m + 2) * sizeof(uint16_t));
  uint8_t *sel = (uint8_t *)malloc((m + 2) / 50 + 2);
  uint8_t lens[6 * 258];
  uint32_t codes[6][258], freq[258], orig = 0, nu, nsel;
  int used[256], G, alpha, g, s, i, list[6];
  size_t nmtf, k;
  orc_bw b;
  if (!sa || !L || !sym || !sel) return ORC_ENOMEM;
  orc_bwt(rle, m, sa, L, &orig);
  nmtf = orc_mtf_rle2(L, m, sym, freq, &nu);
  alpha = (int)nu + 2;
  orc_huff_tables(sym, nmtf, alpha, &G, &nsel, sel, lens);
  for (g = 0; g < G; g++) orc_canonical_codes(lens + g * 258, alpha, codes[g]);
  memset(used, 0, sizeof(used));
  for (k = 0; k < m; k++) used[rle[k]] = 1;

  if (cap) memset(out, 0, cap);
  b.buf = out;
  b.cap = cap;
  b.nbits = 0;
  bw_put(&b, 8, 'B');
  bw_put(&b, 8, 'Z');
  bw_put(&b, 8, 'h');
  bw_put(&b, 8, '0' + level);
  bw_put(&b, 24, 0x314159);
  bw_put(&b, 24, 0x265359);
  bw_put(&b, 32, block_crc);
  bw_put(&b, 1, 0);
  bw_put(&b, 24, orig);
  for (i = 0; i < 16; i++) {
    int any = 0;
    for (s = 0; s < 16; s++) any |= used[16 * i + s];
    bw_put(&b, 1, (uint64_t)any);
  }
  for (i = 0; i < 16; i++) {
    int any = 0;
    for (s = 0; s < 16; s++) any |= used[16 * i + s];
    if (any)
      for (s = 0; s < 16; s++) bw_put(&b, 1, (uint64_t)used[16 * i + s]);
  }
  bw_put(&b, 3, (uint64_t)G);
  bw_put(&b, 15, nsel);
  /* E15 */
  for (g = 0; g < G; g++) list[g] = g;
  for (k = 0; k < nsel; k++) {
    int j = 0, q;
    while (list[j] != sel[k]) j++;
    for (q = 0; q < j; q++) bw_put(&b, 1, 1);
    bw_put(&b, 1, 0);
    for (q = j; q > 0; q--) list[q] = list[q - 1];
    list[0] = sel[k];
  }
  /* E16 */
  for (g = 0; g < G; g++) {
    int cur = lens[g * 258];
    bw_put(&b, 5, (uint64_t)cur);
    for (s = 0; s < alpha; s++) {
      int target = lens[g * 258 + s];
      while (cur < target) {
        bw_put(&b, 2, 2);
        cur++;
      }
      while (cur > target) {
        bw_put(&b, 2, 3);
        cur--;
      }
      bw_put(&b, 1, 0);
    }
  }
  for (k = 0; k < nmtf; k++) {
    int t = sel[k / 50];
    bw_put(&b, lens[t * 258 + sym[k]], codes[t][sym[k]]);
  }
  bw_put(&b, 24, 0x177245);
  bw_put(&b, 24, 0x385090);
  bw_put(&b, 32, block_crc); /* one block: the stream CRC is rotl(0,1) ^ block CRC */
  while (b.nbits % 8) bw_put(&b, 1, 0);
  *len = (size_t)(b.nbits / 8);
  free(sa);
  free(L);
  free(sym);
  free(sel);
  return *len <= cap ? ORC_OK : ORC_ENOSPC;
}

/* One band: first-stage run-length coding with greedy block cuts, then one
 * stream per block, concatenated. */
int orc_band_streams(const uint8_t *raw, size_t n, uint32_t level, uint8_t *out, size_t cap, size_t *len,
                     size_t *n_blocks) {
  size_t maxb = n / 4 + 4, nb, total = 0, k, rlen;
  uint8_t *rle = (uint8_t *)malloc(n + n / 4 + 8);
  size_t *rs = (size_t *)malloc(maxb * sizeof(size_t)), *os = (size_t *)malloc(maxb * sizeof(size_t));
  int st = ORC_OK;
  if (!rle || !rs || !os) return ORC_ENOMEM;
  rlen = orc_rle1_blocks(raw, n, orc_block_limit(level), rle, rs, os, maxb, &nb);
  for (k = 0; k < nb; k++) {
    size_t r0 = rs[k], r1 = k + 1 < nb ? rs[k + 1] : n;
    size_t o0 = os[k], o1 = k + 1 < nb ? os[k + 1] : rlen;
    uint32_t crc = orc_crc32_bzip2(raw + r0, r1 - r0);
    size_t sl = 0, room = total < cap ? cap - total : 0;
    int s = orc_block_stream(rle + o0, o1 - o0, crc, level, out + (room ? total : 0), room, &sl);
    if (s == ORC_ENOMEM) {
      st = s;
      break;
    }
    if (s == ORC_ENOSPC) st = ORC_ENOSPC;
    total += sl;
  }
  *len = total;
  *n_blocks = nb;
  free(rle);
  free(rs);
  free(os);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Container: "PCBZ" header, (id, length) per band, then the band streams   */
/* ------------------------------------------------------------------------ */

static void put_le(uint8_t *p, uint64_t v, int nbytes) {
  int i;
  for (i = 0; i < nbytes; i++) p[i] = (uint8_t)(v >> (8 * i));
}

static uint64_t get_le(const uint8_t *p, int nbytes) {
  uint64_t v = 0;
  int i;
  for (i = 0; i < nbytes; i++) v |= (uint64_t)p[i] << (8 * i);
  return v;
}

size_t orc_container_header_bytes(uint32_t n_bands) { return 20 + 5 * (size_t)n_bands; }

int orc_compress(const orc_params *p, const uint16_t *frame, const uint16_t *prev, const uint8_t *forced_choice,
                 uint8_t *out, size_t cap, size_t *len, uint8_t *choice_out) {
  uint32_t R, nb, b, y0l, Rb;
  uint8_t *choice, *buf, *hdr;
  size_t bufcap, pos, hlen, npix_max;
  int st = orc_plan(p, &R, &nb), any_dt = 0;
  uint16_t *arr;
  uint8_t *bytes;
  if (st) return st;
  choice = (uint8_t *)malloc(nb);
  if (forced_choice) {
    for (b = 0; b < nb; b++) {
      if (forced_choice[b] >= ORC_NCAND) {
        free(choice);
        return ORC_EINVAL;
      }
      if (forced_choice[b] == ORC_VIEW_DT && !prev) {
        free(choice);
        return ORC_ENEEDPREV;
      }
      choice[b] = forced_choice[b];
    }
  } else {
    st = orc_judge(p, frame, prev, choice, NULL, NULL);
    if (st) {
      free(choice);
      return st;
    }
  }
  hlen = orc_container_header_bytes(nb);
  npix_max = (size_t)R * p->pitch * p->w;
  if (npix_max > (size_t)p->h * p->w) npix_max = (size_t)p->h * p->w;
  bufcap = hlen + (size_t)p->h * p->w * 3 + 4096 * (size_t)nb;
  buf = (uint8_t *)calloc(bufcap, 1);
  arr = (uint16_t *)malloc(npix_max * sizeof(uint16_t));
  bytes = (uint8_t *)malloc(2 * npix_max);
  hdr = buf;
  pos = hlen;
  for (b = 0; b < nb; b++) {
    size_t npix, sl = 0, nblk = 0;
    orc_band_geometry(p, b, &y0l, &Rb);
    npix = (size_t)Rb * p->pitch * p->w;
    orc_arrange(p, b, choice[b], frame, prev, arr);
    orc_to_bytes(arr, npix, bytes);
    st = orc_band_streams(bytes, 2 * npix, p->level, buf + pos, bufcap - pos, &sl, &nblk);
    if (st) break;
    hdr[20 + 5 * b] = choice[b];
    put_le(hdr + 20 + 5 * b + 1, sl, 4);
    if (choice[b] == ORC_VIEW_DT) any_dt = 1;
    pos += sl;
  }
  if (!st) {
    memcpy(hdr, "PCBZ", 4);
    hdr[4] = 1;
    hdr[5] = (uint8_t)p->level;
    put_le(hdr + 6, p->pitch, 2);
    put_le(hdr + 8, p->h, 4);
    put_le(hdr + 12, p->w, 4);
    put_le(hdr + 16, nb, 2);
    hdr[18] = (uint8_t)(any_dt ? 1 : 0);
    hdr[19] = 0;
    *len = pos;
    if (pos > cap)
      st = ORC_ENOSPC;
    else
      memcpy(out, buf, pos);
    if (choice_out) memcpy(choice_out, choice, nb);
  }
  free(choice);
  free(buf);
  free(arr);
  free(bytes);
  return st;
}

int orc_peek(const uint8_t *in, size_t in_len, orc_params *out, uint32_t *n_bands, uint8_t *ids,
             uint64_t *band_len) {
  uint32_t nb, b;
  uint64_t total;
  if (in_len < 20 || memcmp(in, "PCBZ", 4) != 0 || in[4] != 1) return ORC_EDATA;
  out->level = in[5];
  out->pitch = (uint32_t)get_le(in + 6, 2);
  out->h = (uint32_t)get_le(in + 8, 4);
  out->w = (uint32_t)get_le(in + 12, 4);
  nb = (uint32_t)get_le(in + 16, 2);
  out->cand_mask = 0;
  if (in_len < orc_container_header_bytes(nb)) return ORC_EDATA;
  total = orc_container_header_bytes(nb);
  for (b = 0; b < nb; b++) {
    uint8_t id = in[20 + 5 * b];
    uint64_t l = get_le(in + 20 + 5 * b + 1, 4);
    if (id >= ORC_NCAND) return ORC_EDATA;
    out->cand_mask |= 1u << id;
    if (ids) ids[b] = id;
    if (band_len) band_len[b] = l;
    total += l;
  }
  if (total != in_len) return ORC_EDATA;
  *n_bands = nb;
  return ORC_OK;
}
