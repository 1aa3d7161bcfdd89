/*
 * pcbz.h -- C ABI of libpcbz, a GPU (MI355X / gfx950) implementation of the
 * PC-bzip2 hot path for light-field microscopy frames (arXiv 2310.09467).
 *
 * A frame is H x W uint16 pixels, row-major, little-endian, made of
 * pitch x pitch microlens images (paper Sec. 2.1, Fig. 1a).  It is cut into
 * bands of whole lens rows, each within one bzip2 block.  For every band the
 * library builds candidate arrangements (Sec. 2.1.1, Fig. 2a, Fig. 3):
 *   PCBZ_RASTER   the band as stored (the paper's "no predictor" option),
 *   PCBZ_VIEW     sub-aperture-view (phase-space) order,
 *   PCBZ_VIEW_DX  view order with the lens-neighbour delta mod 2^16,
 *   PCBZ_VIEW_DT  view order of the delta to the previous frame mod 2^16,
 *   ids 4..15     the paper's predictor family (Sec. 2.1.1, Fig. 1b, Fig. 3b/3c):
 *                 id = 4 + 4 * domain + function; each pixel X predicted from
 *                 three causal neighbours A (left), B (above), C (above-left)
 *                 over neighbouring pixels (domain 0), the same pixel in
 *                 neighbouring lenses (domain 1) or phase space (domain 2: A
 *                 one lens to the left, B the pixel above inside the lens, C
 *                 the pixel above inside the lens to the left), with the
 *                 lossless-JPEG functions A+B-C, A+floor((B-C)/2),
 *                 B+floor((A-C)/2), floor((A+B)/2) (function 0..3); band-local
 *                 edges (only A: A, only B: B, neither: 0); the residual mod
 *                 2^16 as a signed value mapped 0,-1,1,-2,... -> 0,1,2,3,...;
 *                 raster order,
 * scores them with the 2D image entropy criterion (Sec. 2.1.2, Eq. 1:
 * first-byte-only rotation sort, last column, adjacent-byte pair entropy),
 * codes the chosen arrangement with bzip2 (Sec. 2.1.3), and stores an 8-bit
 * arrangement id per band in the container header (Sec. 2.1.4).
 *
 * Every compute step runs as HIP kernels on the GPU.  Pointers named d_* are
 * device pointers owned by the caller; nothing is retained after a call
 * returns.  `stream` is a hipStream_t (NULL = the null stream); work is
 * stream-ordered, and calls that report a length synchronise that stream.
 * A context is not thread-safe: use one per host thread.
 *
 * Errors are returned as pcbz_status codes; no exception or abort crosses the
 * ABI.  pcbz_last_error() describes the last failure of a context.  Entry
 * points declare an int result holding a pcbz_status value: C leaves the
 * width of an enum to the compiler, an int keeps the ABI fixed.
 */
#ifndef PCBZ_H
#define PCBZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PCBZ_OK = 0,
  PCBZ_EINVAL = -1,    /* bad parameters: h or w zero or not a multiple of pitch, pitch outside 1..90,
                          level outside 1..9, cand_mask empty or with bits above 15, sizes too large */
  PCBZ_ENOSPC = -2,    /* out_cap below the container size; *out_len receives the required size */
  PCBZ_EDATA = -3,     /* corrupt container: bad magic, lengths or a CRC mismatch */
  PCBZ_ENEEDPREV = -4, /* the temporal candidate is requested or stored but d_prev is NULL */
  PCBZ_ENOMEM = -5,    /* workspace above the context's HBM budget, or allocation failed */
  PCBZ_EDEVICE = -6    /* HIP runtime error (see pcbz_last_error) */
} pcbz_status;

enum { PCBZ_RASTER = 0, PCBZ_VIEW = 1, PCBZ_VIEW_DX = 2, PCBZ_VIEW_DT = 3, PCBZ_PRED_FIRST = 4, PCBZ_NCAND = 16 };

/* Frame geometry and coding parameters.  level 1..9 sets the bzip2 block
 * limit 100000*level-19 bytes; cand_mask bit i enables arrangement id i
 * (i = 0..15). */
typedef struct {
  uint32_t h, w, pitch, level, cand_mask;
} pcbz_params;

typedef struct pcbz_ctx pcbz_ctx;
typedef struct pcbz_selector pcbz_selector; /* learned arrangement selector (below) */

/* Creates a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * device workspace (0 = no cap).  Returns PCBZ_EDEVICE if the device cannot
 * be used. */
int pcbz_create(pcbz_ctx **out, int hip_device, size_t hbm_budget_bytes);
void pcbz_destroy(pcbz_ctx *ctx);
const char *pcbz_last_error(const pcbz_ctx *ctx);

/* Band plan: the frame is cut into blocks before bzip2 coding (Sec. 2.1.3,
 * where the paper's blocks follow the thread count); here a band is
 * R = max(1, floor((100000*level-19)/(2*pitch*W))) whole lens rows, so that
 * every arrangement of a band holds the same pixels and fits one bzip2 block.
 * Host only: writes the band count and an upper bound on the container size
 * (either pointer may be NULL).  PCBZ_EINVAL for invalid parameters. */
int pcbz_plan(const pcbz_params *prm, uint32_t *n_bands, size_t *compress_bound);

/* Entropy judgement only (Sec. 2.1.2, Eq. 1).  Writes d_choice[n_bands] (the
 * lowest-entropy enabled arrangement per band, ties to the lowest id) and,
 * when non-NULL, d_entropy[n_bands*16] (bits per pair; NaN for disabled ids)
 * and d_score[n_bands*16] (the exact fixed-point sum of P*log2(P)*2^20 that
 * decides the choice; INT64_MIN for disabled ids), 16 entries per band, one
 * per arrangement id. */
int pcbz_judge(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
               uint8_t *d_choice, double *d_entropy, int64_t *d_score, void *stream);

/* pcbz_judge for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same outputs as pcbz_judge, but the workspace (plan
 * tables, candidate bytes, pair histograms, scores) is a fixed 48 MiB device
 * array and the Tq table a fixed 900,002-entry array, each held once per
 * device from the first pcbz_create on that device until the process ends.
 * The call allocates nothing (no hipMalloc, hipHostMalloc or hipFree): the
 * caller passes the frame and the outputs.  A frame whose workspace exceeds
 * 48 MiB (about one 2040 x 2040 frame with four candidates) gets
 * PCBZ_ENOMEM and nothing is written.  The plan tables are copied from
 * pageable host memory and the call synchronises `stream` once, after that
 * copy.  Every call on a device shares its one workspace, which keeps the last
 * call's contents (the accumulators are cleared by each call): calls that can
 * overlap on one device, from any context, stream or thread, race and must be
 * serialised by the caller. */
int pcbz_judge_noalloc(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
                       uint8_t *d_choice, double *d_entropy, int64_t *d_score, void *stream);

/* The compression pipeline of Fig. 1c and Fig. 2a: arrangements (Sec. 2.1.1),
 * entropy judgement per band (Sec. 2.1.2), bzip2 coding of the chosen
 * arrangement (Sec. 2.1.3) and the header with one 8-bit arrangement id per
 * band (Sec. 2.1.4).  Compresses one frame into a PCBZ container in d_out
 * (device, out_cap bytes, written only when the container fits: otherwise
 * PCBZ_ENOSPC with the required size in *out_len).  With d_forced_choice
 * (device, n_bands ids) the judgement is skipped.  When a selector is set on
 * the context (pcbz_set_selector) confident bands skip the judgement.  The call
 * synchronises `stream` and writes the container length to *out_len (host).
 * d_choice_out (device, may be NULL) receives the per-band ids used.
 * Container: "PCBZ", u8 version 1, u8 level, u16 pitch, u32 H, u32 W,
 * u16 n_bands, u8 flags (bit 0: a band uses PCBZ_VIEW_DT), u8 0; then
 * n_bands x (u8 id, u32 byte length); then each band's bzip2 streams (one
 * stream per block) in band order.  All integers little-endian. */
int pcbz_compress(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
                  const uint8_t *d_forced_choice, uint8_t *d_out, size_t out_cap, size_t *out_len,
                  uint8_t *d_choice_out, void *stream);

/* The pipeline of pcbz_compress for n frames of possibly different shapes in
 * one pass over all of their blocks (the paper codes blocks in parallel,
 * Sec. 2.1.3).  Arrays are host arrays of n entries; d_prevs and d_forced
 * may be NULL or hold NULL entries.  sel (NULL: every band is judged) and
 * min_conf apply to this call only, in place of any selector set on the
 * context; a band whose predicted probability reaches min_conf (>= 0) skips
 * the judgement.  lens (host) receives each container length; each frame's
 * bytes equal pcbz_compress of that frame alone with the same selector.
 * Returns the first error; frames whose container exceeds caps[i] get
 * PCBZ_ENOSPC with lens[i] set to the required size. */
int pcbz_compress_batch(pcbz_ctx *ctx, uint32_t n, const pcbz_params *prm, const uint16_t *const *d_frames,
                        const uint16_t *const *d_prevs, const uint8_t *const *d_forced,
                        const pcbz_selector *sel, float min_conf, uint8_t *const *d_outs, const size_t *caps,
                        size_t *lens, void *stream);

/* Unpacks the header of a container in host memory (Sec. 2.1.4: the 8-bit
 * arrangement id is stored in the header; Fig. 2b: decompression starts by
 * reading it): frame geometry, level and candidate flags into *out, band
 * count into *n_bands (may be NULL).  PCBZ_EDATA for a bad magic, version
 * or length. */
int pcbz_peek(const uint8_t *in, size_t in_len, pcbz_params *out, uint32_t *n_bands);

/* The decompression pipeline of Fig. 1c and Fig. 2b: unpack the header,
 * decode each band's bzip2 streams, invert the arrangement named by the
 * band's id (Sec. 2.1, last paragraph before 2.1.1), all on the device.
 * Decompresses a container held in device memory (d_in, in_len bytes) into
 * d_out (device, out_elems >= H*W pixels, else PCBZ_ENOSPC).  d_prev is
 * required when a band uses PCBZ_VIEW_DT (PCBZ_ENEEDPREV).  Every block CRC
 * is checked; a malformed field, a CRC mismatch or a band that decodes to the
 * wrong size gives PCBZ_EDATA (d_out may then be partly written).  Reads the
 * container header back to the host, synchronises `stream`. */
int pcbz_decompress(pcbz_ctx *ctx, const uint8_t *d_in, size_t in_len, const uint16_t *d_prev, uint16_t *d_out,
                    size_t out_elems, void *stream);

/* pcbz_decompress for n containers at once (every block of every container
 * is decoded in one pass).  Arrays are host arrays of n entries; d_prevs may
 * be NULL or hold NULL entries.  Returns the first error. */
int pcbz_decompress_batch(pcbz_ctx *ctx, uint32_t n, const uint8_t *const *d_ins, const size_t *in_lens,
                          const uint16_t *const *d_prevs, uint16_t *const *d_outs, const size_t *out_elems,
                          void *stream);

/* Copies the first `bytes` of one intermediate array of the last
 * decompression call on `ctx` to host memory, so that its stages can be
 * checked one by one (valid until the next call on the context):
 *   which 0  per-slot block records (header fields, symbol counts, lengths),
 *         1  Huffman-decoded symbols (uint16, band after band),
 *         2  the blocks after the zero runs and move-to-front (the BWT output),
 *         3  the blocks after the inverse BWT (the first run-length stage),
 *         4  the raw band bytes (arranged), 5 the call's counters.
 * PCBZ_EINVAL for an unknown `which`, too many bytes or no call yet. */
int pcbz_decompress_inspect(const pcbz_ctx *ctx, int which, void *host, size_t bytes);

/* Statistics of the last compress call on this context (for profiling):
 * raw bytes, first-stage bytes, blocks, doubling rounds of the suffix sort. */
int pcbz_last_stats(const pcbz_ctx *ctx, uint64_t *raw_bytes, uint64_t *rle_bytes, uint32_t *n_blocks,
                    uint32_t *bwt_rounds);

/* Kernel tracing for profiling (process-wide).  When enabled, every kernel
 * launch whose name equals `filter` (all launches when filter is NULL) is
 * bracketed by HIP events on the launch stream.  pcbz_trace_read waits for
 * the recorded events and returns, per kernel name, the summed milliseconds,
 * the launch count and the summed algorithmic bytes (what the step itself
 * must read and write, as counted by the launcher; 0 where not counted).
 * Names are written into rows of `name_stride` bytes.  *n receives the number
 * of traced names (which may exceed `max`).  Any output array may be NULL. */
int pcbz_trace_enable(pcbz_ctx *ctx, int on, const char *filter);
int pcbz_trace_read(pcbz_ctx *ctx, char *names, size_t name_stride, double *ms, uint64_t *calls, uint64_t *bytes,
                    uint32_t max, uint32_t *n, int reset);

/* ------------------------------------------------------------------------
 * Learned arrangement selector.  The paper judges every candidate of every
 * band (Sec. 2.1.2) and names a cheaper decision criterion as future work
 * (Sec. 4).  The selector is a small network that predicts, from per-band
 * features, the arrangement the judgement would choose; bands whose
 * predicted probability reaches min_conf skip the judgement and build only
 * the predicted arrangement, the rest are judged as usual.  Output stays a
 * valid container whose ids may differ from the exhaustive choice.  The
 * network predicts among ids 0..3: a band whose cand_mask enables any of the
 * predictor family (ids 4..15) is always judged.
 *
 * Features (pcbz_features): per band, the band's pixels are split into
 * 64 x 64 cells (cell (i, j) covers rows [i*Hb/64, (i+1)*Hb/64) and columns
 * [j*W/64, (j+1)*W/64), Hb = band rows); each cell gives log1p(mean),
 * log1p(population variance), log1p(mean |x - x one lens to the left|)
 * (pixels of the first lens column excluded from the sum, divided by all
 * pixels) and log1p(mean |x - prev|) (0 without d_prev); empty cells are 0.
 * Layout: FP32 [n_bands][64][64][4].
 *
 * Network (151,076 FP32 parameters, in this order): conv 3x3 stride 2 pad 1
 * 4->32 (W1 [32][3][3][4], b1 [32]), ReLU; conv 32->32 (W2 [32][3][3][32],
 * b2), ReLU; conv 32->32 (W3, b3), ReLU; FC 2048->64 (W4 [64][2048] over the
 * 8x8x32 map flattened (y, x, c), b4), ReLU; FC 64->4 (W5 [4][64], b5).  The
 * input is (feature - mean[c]) / std[c] (norm8 = mean[4], std[4]).  Every
 * layer input is rounded to bfloat16 (round to nearest even) and products
 * accumulate in FP32 on the matrix cores.
 *
 * A selector lives on its context's device; it may be shared by contexts on
 * that device but not used by two calls at once.  Unset it from every
 * context (pcbz_set_selector(ctx, NULL, 0)) before pcbz_selector_free.
 * ------------------------------------------------------------------------ */

size_t pcbz_selector_num_params(void);
/* params: host FP32 array of pcbz_selector_num_params() values or NULL
 * (zeros); norm8: host mean[4], std[4] or NULL (0 and 1). */
int pcbz_selector_create(pcbz_ctx *ctx, const float *params, const float *norm8, pcbz_selector **out);
void pcbz_selector_free(pcbz_selector *sel);
int pcbz_selector_get_params(const pcbz_selector *sel, float *params, float *norm8);
int pcbz_selector_set_params(pcbz_selector *sel, const float *params, const float *norm8);
/* File: "PCBZSEL1", u32 parameter count, norm8, parameters (FP32 LE).
 * Load returns PCBZ_EDATA for a bad file. */
int pcbz_selector_save(const pcbz_selector *sel, const char *path);
int pcbz_selector_load(pcbz_ctx *ctx, const char *path, pcbz_selector **out);

/* Features of every band of one frame into d_feat (device, n_bands*16384
 * floats).  Synchronises `stream`. */
int pcbz_features(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
                  float *d_feat, void *stream);
/* Logits d_logits[n][4] (device) for n feature maps (device). */
int pcbz_selector_forward(pcbz_selector *sel, const float *d_feat, uint32_t n, float *d_logits, void *stream);
/* Softmax cross-entropy with per-class weights (class_w4, host, NULL =
 * ones), averaged as sum w[y_i] * loss_i / sum w[y_i], over n <= 4096
 * samples with labels d_label[n] (device, 0..3).  Writes the parameter
 * gradient (device, num_params floats, may be NULL) and the loss (host, may
 * be NULL). */
int pcbz_selector_gradients(pcbz_selector *sel, const float *d_feat, const uint8_t *d_label, uint32_t n,
                            const float *class_w4, float *d_grad, float *loss, void *stream);
/* Copies one tensor of the last pcbz_selector_gradients (or train_step) call
 * on `sel` to host memory, so that the kernels can be checked layer by layer.
 * n = that call's sample count; bytes must equal the tensor's size.
 *   which 0..4  bf16 bits, layer inputs as rounded for the products: 0 the
 *               normalised features [n][64][64][4], 1 conv1 output
 *               [n][32][32][32], 2 conv2 output [n][16][16][32], 3 conv3
 *               output [n][2048] (= FC4 input, flattened (y, x, c)), 4 FC4
 *               output [n][64];
 *   which 5..8  FP32 pre-activations (products plus bias, before ReLU):
 *               5 conv1 [n*1024][32], 6 conv2 [n*256][32], 7 conv3
 *               [n*64][32], 8 FC4 [n][64];
 *   which 9, 10 FP32 logits [n][4] and dloss/dlogits [n][4];
 *   which 11..15 bf16 bits of dloss/dpre after the ReLU mask, as fed to the
 *               gradient products: 11 FC5 [n][4], 12 FC4 [n][64], 13 conv3
 *               [n*64][32], 14 conv2 [n*256][32], 15 conv1 [n*1024][32].
 * PCBZ_EINVAL for an unknown `which`, a wrong size or no call yet. */
int pcbz_selector_inspect(const pcbz_selector *sel, int which, void *host, size_t bytes);
/* One AdamW step (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay)
 * on the gradient of the batch. */
int pcbz_selector_train_step(pcbz_selector *sel, const float *d_feat, const uint8_t *d_label, uint32_t n,
                             const float *class_w4, float lr, float weight_decay, float *loss, void *stream);
/* Plain GEMM on the selector's matrix-core kernel, for checking it:
 * C[M][N] (FP32) = A[M][K] x B[K][N], A and B row-major bfloat16 bits. */
int pcbz_gemm_bf16(int M, int N, int K, const uint16_t *d_a, const uint16_t *d_b, float *d_c, void *stream);

/* Makes pcbz_compress consult `sel` (NULL: judge every band); the
 * single-frame call has no selector argument, so the context carries it
 * (pcbz_compress_batch takes its selector as an argument instead).
 * min_conf > 1 judges every band; 0 trusts every prediction.  Bands of
 * frames with a caller-forced array keep the caller's ids. */
int pcbz_set_selector(pcbz_ctx *ctx, pcbz_selector *sel, float min_conf);
/* Bands seen by the selector in the last compress call and how many of
 * them were judged (fell below min_conf). */
int pcbz_selector_stats(const pcbz_ctx *ctx, uint32_t *n_bands, uint32_t *n_judged);

/* Batch execution mode: on = 1 (the default) lets the autotuner compare, on
 * a shape's first call, an eager call with a replay of a captured graph per
 * candidate schedule and keep the fastest; on = 2 always replays graphs;
 * on = 0 always runs eagerly (useful when shapes rarely repeat).  Output
 * bytes are the same in every mode; other values give PCBZ_EINVAL. */
int pcbz_set_graphs(pcbz_ctx *ctx, int on);

/* ------------------------------------------------------------------------
 * Serving loop.  Frames arrive from cameras over time (pcbz_server_submit,
 * host memory that must stay valid until the frame's result is polled).
 * Admission, first in first out, gives a frame its device blocks (frame and
 * output) from a pool holding an eighth of hbm_budget; a frame waits on the
 * host while the pool is full.  n_workers worker threads, each with its own
 * context and stream (and its own copy of `sel`, if given, used with
 * min_conf), repeatedly take every admitted frame (up to max_batch_bytes of
 * input; 0 = derived from the budget) and compress them in one
 * pcbz_compress_batch call, so batches of different workers overlap on the
 * device and frames that arrive meanwhile join the next batch.  The rest of
 * the budget is split between the workers' workspaces; a batch that does not
 * fit is split.  hbm_budget must be at least 64 MiB.
 *
 * Temporal candidate: when a frame's cand_mask has bit 3, the previous frame
 * of the same camera and shape (kept on the device as camera state) is its
 * previous frame; the first frame of a camera and shape is coded without the
 * temporal candidate.  The result names the previous frame's tag.
 *
 * Each container equals what pcbz_compress gives for that frame alone with
 * the same previous frame (and the same selector and min_conf).
 * ------------------------------------------------------------------------ */
typedef struct pcbz_server pcbz_server;

typedef struct {
  uint64_t tag;        /* the submit tag */
  uint64_t prev_tag;   /* tag of the previous frame used, UINT64_MAX if none */
  uint32_t camera;
  int32_t status;      /* pcbz_status of the frame */
  const uint8_t *data; /* container bytes, valid until the next pcbz_server_poll */
  size_t len;
  double latency_ms;   /* submit -> container in host memory */
  double submit_ms;    /* submit time on the server's steady clock */
} pcbz_server_result;

typedef struct {
  uint64_t submitted, completed, pending, admitted, in_flight;
  uint64_t batches, batched_frames;
  uint64_t pool_bytes, pool_used, pool_peak; /* device pool for frames, outputs and camera state */
  double busy_ms;    /* time with at least one batch running */
  double overlap_ms; /* time with two or more batches running at once */
} pcbz_server_info;

int pcbz_server_create(int hip_device, size_t hbm_budget, uint32_t n_workers, size_t max_batch_bytes,
                       const pcbz_selector *sel, float min_conf, pcbz_server **out);
/* Returns PCBZ_ENOMEM if the frame can never fit the pool, PCBZ_ENEEDPREV if
 * the temporal arrangement is its only candidate and its camera has sent no
 * earlier frame of this shape.  A frame that fails once batched (a device
 * error, say) gets its own status in its result; the others complete. */
int pcbz_server_submit(pcbz_server *srv, const pcbz_params *prm, const uint16_t *host_frame, uint32_t camera,
                       uint64_t tag);
/* Up to max finished results; waits up to timeout_ms (-1: until one is
 * ready, 0: no wait).  *n receives the count. */
int pcbz_server_poll(pcbz_server *srv, pcbz_server_result *res, uint32_t max, uint32_t *n, int timeout_ms);
int pcbz_server_stats(const pcbz_server *srv, pcbz_server_info *st);
/* Finishes admitted work, drops frames never admitted, frees everything. */
void pcbz_server_destroy(pcbz_server *srv);

#ifdef __cplusplus
}
#endif
#endif
