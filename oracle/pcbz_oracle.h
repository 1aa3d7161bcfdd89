/*
 * pcbz_oracle.h -- CPU oracle for the PC-bzip2 hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential C
 * implementation of what the GPU library computes: the band plan, the
 * lenslet -> sub-aperture-view rearrangements with their mod 2^16 deltas
 * (paper Sec. 2.1.1, Fig. 3), the order-1 rotation sort and 2D pair entropy
 * judgement (Sec. 2.1.2, Eq. 1, Fig. 2c), and the bzip2 block coding of each
 * band (Sec. 2.1.3) packed with an 8-bit arrangement id per band
 * (Sec. 2.1.4).  Only the tests, the smoke check and the CPU baseline leg of
 * the benchmark may load it.  It shares no source with the GPU library.
 *
 * Every bzip2 encoder choice that the format leaves free is fixed here as the
 * "PCBZ-1 profile" so that two independent implementations emit identical
 * bytes; see the comments at each stage.
 */
#ifndef PCBZ_ORACLE_H
#define PCBZ_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOSPC = -2, ORC_EDATA = -3, ORC_ENEEDPREV = -4, ORC_ENOMEM = -5 };
enum { ORC_RASTER = 0, ORC_VIEW = 1, ORC_VIEW_DX = 2, ORC_VIEW_DT = 3, ORC_NCAND = 16 };
/* ids 4..15: the multi-neighbour predictor family, id = 4 + 4 * domain + function
 * (domain 0 pixel neighbours, 1 lens neighbours, 2 phase space; function 0
 * A+B-C, 1 A+floor((B-C)/2), 2 B+floor((A-C)/2), 3 floor((A+B)/2)). */
enum { ORC_PRED_FIRST = 4 };

typedef struct {
  uint32_t h, w, pitch, level, cand_mask;
} orc_params;

/* ---- band plan and arrangements ---- */
uint32_t orc_block_limit(uint32_t level);
int orc_check_params(const orc_params *p);
int orc_plan(const orc_params *p, uint32_t *rows_per_band, uint32_t *n_bands);
int orc_band_geometry(const orc_params *p, uint32_t band, uint32_t *first_lens_row, uint32_t *lens_rows);
int orc_arrange(const orc_params *p, uint32_t band, int id, const uint16_t *frame, const uint16_t *prev,
                uint16_t *out);
/* The map of 16-bit residuals onto 0..65535 used by the predictor family
 * (0, -1, 1, -2, ... -> 0, 1, 2, 3, ...) and its inverse. */
uint16_t orc_zigzag16(uint16_t r);
uint16_t orc_unzigzag16(uint16_t z);
int orc_unarrange(const orc_params *p, uint32_t band, int id, const uint16_t *arranged, const uint16_t *prev,
                  uint16_t *frame);
void orc_to_bytes(const uint16_t *v, size_t count, uint8_t *out);

/* ---- entropy judgement ---- */
void orc_order1_lastcol(const uint8_t *x, size_t n, uint8_t *T);
void orc_pair_hist(const uint8_t *T, size_t n, uint32_t *P);
int64_t orc_tq(uint64_t c);
int64_t orc_score(const uint32_t *P);
double orc_entropy_bits(int64_t S, size_t n);
int64_t orc_band_score(const uint8_t *x, size_t n);
int orc_judge(const orc_params *p, const uint16_t *frame, const uint16_t *prev, uint8_t *choice, int64_t *S,
              double *H);

/* ---- bzip2 block coding (PCBZ-1 profile) ---- */
uint32_t orc_crc32_bzip2(const uint8_t *data, size_t n);
size_t orc_rle1_blocks(const uint8_t *in, size_t n, uint32_t limit, uint8_t *out, size_t *raw_start,
                       size_t *rle_start, size_t max_blocks, size_t *n_blocks);
void orc_bwt(const uint8_t *blk, size_t m, uint32_t *sa, uint8_t *L, uint32_t *orig_ptr);
size_t orc_mtf_rle2(const uint8_t *L, size_t m, uint16_t *sym, uint32_t *freq, uint32_t *n_in_use);
void orc_package_merge(const uint32_t *w, int n, int limit, uint8_t *len);
void orc_canonical_codes(const uint8_t *len, int n, uint32_t *code);
void orc_huff_init_ranges(const uint32_t *freq, int alpha, int G, uint64_t total, int *end /* [G] */);
void orc_huff_select(const uint16_t *sym, size_t n_mtf, const uint32_t *cost /* [G*258] */, int G, uint8_t *sel);
int orc_huff_tables(const uint16_t *sym, size_t n_mtf, int alpha, int *n_groups, uint32_t *n_sel, uint8_t *sel,
                    uint8_t *len /* [6*258] */);
int orc_block_stream(const uint8_t *rle, size_t m, uint32_t block_crc, uint32_t level, uint8_t *out, size_t cap,
                     size_t *len);
int orc_band_streams(const uint8_t *raw, size_t n, uint32_t level, uint8_t *out, size_t cap, size_t *len,
                     size_t *n_blocks);

/* ---- whole frame ---- */
size_t orc_container_header_bytes(uint32_t n_bands);
int orc_compress(const orc_params *p, const uint16_t *frame, const uint16_t *prev, const uint8_t *forced_choice,
                 uint8_t *out, size_t cap, size_t *len, uint8_t *choice_out);
int orc_peek(const uint8_t *in, size_t in_len, orc_params *out, uint32_t *n_bands, uint8_t *ids,
             uint64_t *band_len);

#ifdef __cplusplus
}
#endif
#endif
