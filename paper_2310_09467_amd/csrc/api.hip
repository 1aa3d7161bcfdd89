// api.hip -- C ABI of libpcbz: context, workspace arena, band planning and the
// launch sequence of the compression path (all compute in HIP kernels).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pcbz.h"
#include "pcbz_internal.hpp"

using namespace pcbz;

namespace pcbz {

// ---------------------------------------------------------------- tracing
bool g_trace_on = false;
thread_local const char *g_trace_stage = nullptr;

namespace {
struct TraceRec {
  const char *name;
  const char *stage;
  hipEvent_t a, b;
};
std::string trace_key(const char *stage, const char *name) {
  return stage ? std::string(stage) + "|" + name : std::string(name);
}
struct Tracer {
  std::string filter;
  std::vector<TraceRec> open, done;
  std::vector<hipEvent_t> pool;
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<uint64_t> calls;
  std::vector<uint64_t> bytes;
  struct Pending {
    size_t slot;
    uint64_t per_elem;
  };
  // byte counts waiting for their element counts, which a one-thread kernel
  // copied at launch time into snap[i] (device)
  std::vector<Pending> pending;
  uint32_t *snap = nullptr;
  static constexpr size_t kSnap = 4096;
  size_t slot(const std::string &name) {
    size_t i = 0;
    while (i < names.size() && names[i] != name) i++;
    if (i == names.size()) {
      names.push_back(name);
      ms.push_back(0.0);
      calls.push_back(0);
      bytes.push_back(0);
    }
    return i;
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // folds finished records into the per-name totals (waits for their events)
  void collect() {
    for (TraceRec &r : done) {
      float t = 0.f;
      (void)hipEventSynchronize(r.b);
      (void)hipEventElapsedTime(&t, r.a, r.b);
      const size_t i = slot(trace_key(r.stage, r.name));
      ms[i] += t;
      calls[i]++;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    done.clear();
  }
};
Tracer g_tracer;
}  // namespace

void trace_begin_impl(const char *name, hipStream_t s) {
  if (!g_tracer.filter.empty() && g_tracer.filter != name) return;
  TraceRec r{name, g_trace_stage, g_tracer.ev(), g_tracer.ev()};
  (void)hipEventRecord(r.a, s);
  g_tracer.open.push_back(r);
}

void trace_bytes_impl(const char *name, uint64_t bytes) {
  if (!g_tracer.filter.empty() && g_tracer.filter != name) return;
  g_tracer.bytes[g_tracer.slot(trace_key(g_trace_stage, name))] += bytes;
}

__global__ void k_trace_snap(const uint32_t *d_count, uint32_t *snap) { *snap = *d_count; }

void trace_bytes_count_impl(const char *name, uint64_t per_elem, const uint32_t *d_count, hipStream_t s) {
  if (!g_tracer.filter.empty() && g_tracer.filter != name) return;
  if (!g_tracer.snap && hipMalloc((void **)&g_tracer.snap, Tracer::kSnap * sizeof(uint32_t)) != hipSuccess) {
    g_tracer.snap = nullptr;
    return;
  }
  if (g_tracer.pending.size() >= Tracer::kSnap) return;
  hipLaunchKernelGGL(k_trace_snap, dim3(1), dim3(1), 0, s, d_count, g_tracer.snap + g_tracer.pending.size());
  g_tracer.pending.push_back({g_tracer.slot(trace_key(g_trace_stage, name)), per_elem});
}

void trace_settle_impl(hipStream_t s) {
  if (g_tracer.pending.empty()) return;
  std::vector<uint32_t> n(g_tracer.pending.size());
  if (hipMemcpyAsync(n.data(), g_tracer.snap, n.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s) == hipSuccess &&
      hipStreamSynchronize(s) == hipSuccess)
    for (size_t i = 0; i < n.size(); i++) g_tracer.bytes[g_tracer.pending[i].slot] += g_tracer.pending[i].per_elem * n[i];
  g_tracer.pending.clear();
}

void trace_end_impl(const char *name, hipStream_t s) {
  for (size_t i = g_tracer.open.size(); i-- > 0;) {
    if (g_tracer.open[i].name == name || strcmp(g_tracer.open[i].name, name) == 0) {
      (void)hipEventRecord(g_tracer.open[i].b, s);
      g_tracer.done.push_back(g_tracer.open[i]);
      g_tracer.open.erase(g_tracer.open.begin() + i);
      break;
    }
  }
  if (g_tracer.done.size() > 4096) g_tracer.collect();
}


// A captured compression graph for one batch shape and schedule.
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
  uint64_t gen = 0;
  int items = 16, rounds = 0;
  uint64_t seg_mask = 0;
};

// Autotuner record: the schedule chosen for a batch shape.
struct TuneRec {
  std::string key;
  int items = 16;   // radix tile elements per thread
  int rounds = 0;   // doubling rounds enqueued in the graph
  uint64_t seg_mask = 0;  // rounds sorted group by group in the graph
  double ms = 0.0;  // timed graph replay of the winner
};
int peek_container(const uint8_t *in, size_t in_len, pcbz_params *out, uint32_t *n_bands,
                   std::vector<uint8_t> *ids, std::vector<uint32_t> *lens);
}  // namespace pcbz

struct pcbz_ctx {
  int device = 0;
  size_t budget = 0;
  std::string err;
  uint8_t *arena = nullptr;
  size_t arena_size = 0;
  int64_t *d_tq = nullptr;
  size_t tq_n = 0;
  uint32_t *d_xpow2 = nullptr;
  uint32_t *d_xbyte = nullptr;  // x^(8r) mod P, r < 256
  uint32_t *d_xchunk = nullptr;
  size_t xchunk_n = 0;
  uint8_t *h_stage = nullptr;
  size_t h_stage_size = 0;
  uint32_t *h_small = nullptr;  // pinned read-back area (4 KB)
  uint64_t last_raw = 0, last_rle = 0;
  uint32_t last_blocks = 0, last_rounds = 0, last_graph = 0;
  uint64_t last_seg_mask = 0;  // rounds the last eager call sorted group by group
  // captured graphs and the autotuner's per-shape choices
  uint64_t gen = 1;  // bumped whenever a buffer a graph refers to is reallocated
  hipStream_t gstream = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  // a second stream for work off the critical path (block CRCs during the
  // suffix sort, header bits during the symbol-length scan), joined by events
  hipStream_t side = nullptr;
  hipEvent_t fev[3] = {nullptr, nullptr, nullptr};
  std::vector<pcbz::GraphEntry> graphs;
  std::vector<pcbz::TuneRec> tune;
  // pcbz_compress: per-shape round count and in-group-sort rounds of the last
  // call that read its counts back (the later calls enqueue that schedule)
  std::vector<pcbz::TuneRec> fixed;
  std::string tune_path;
  int eager_items = 8;
  int tune_rounds = 0;          // round budget the tuner gives graphs (0: the eager call's rounds + 1)
  int tune_failed_replays = 0;  // the last tuning saw a replay that did not reproduce the eager bytes
  // learned arrangement selector (optional): confident bands skip the judge
  pcbz_selector *sel = nullptr;
  float min_conf = 1.f;
  int use_graphs = 1;  // pcbz_compress_batch: 0 eager, 1 graphs where faster, 2 graphs
  int use_fixed = 1;   // pcbz_compress: enqueue a known shape's schedule without read-backs
  uint32_t last_sel_bands = 0, last_sel_fallback = 0;
  std::string fixed_err;  // why the fixed workspace could not be set up (empty: it is)
  // decompression: pinned header read-back area and the last call's workspace
  uint8_t *h_dec = nullptr;
  size_t h_dec_size = 0;
  pcbz::DecWork last_dec{};
  bool last_dec_valid = false;
};

namespace {

constexpr uint32_t kPoly = 0x04C11DB7u;
constexpr uint32_t kMaxPitch = 90;

int fail(pcbz_ctx *c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(ctx, PCBZ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

uint32_t h_mulmod(uint32_t a, uint32_t b) {
  uint32_t r = 0;
  for (int i = 31; i >= 0; i--) {
    r = (r & 0x80000000u) ? (r << 1) ^ kPoly : (r << 1);
    if ((b >> i) & 1u) r ^= a;
  }
  return r;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over the arena; with base == nullptr it only measures.
struct Arena {
  uint8_t *base;
  size_t off = 0;
  template <typename T>
  T *get(size_t count) {
    off = align_up(off, 256);
    T *p = base ? (T *)(base + off) : nullptr;
    off += count * sizeof(T) + 16;
    return p;
  }
};

int check_params(const pcbz_params *p) {
  if (!p) return PCBZ_EINVAL;
  if (p->pitch == 0 || p->pitch > kMaxPitch || p->h == 0 || p->w == 0) return PCBZ_EINVAL;
  if (p->h % p->pitch || p->w % p->pitch) return PCBZ_EINVAL;
  if (p->level < 1 || p->level > 9) return PCBZ_EINVAL;
  if (p->cand_mask == 0 || (p->cand_mask & ~0xFFFFu)) return PCBZ_EINVAL;
  uint64_t lens_row = 2ull * p->pitch * p->w;
  uint64_t r = (100000ull * p->level - 19) / lens_row;
  if (r < 1) r = 1;
  uint64_t ns = p->h / p->pitch;
  if ((ns + r - 1) / r > 65535) return PCBZ_EINVAL;
  if (2ull * p->h * p->w >= (1ull << 31)) return PCBZ_EINVAL;
  return PCBZ_OK;
}

void plan_rows(const pcbz_params *p, uint32_t *R, uint32_t *nb) {
  uint64_t lens_row = 2ull * p->pitch * p->w;
  uint64_t r = (100000ull * p->level - 19) / lens_row;
  if (r < 1) r = 1;
  uint32_t ns = p->h / p->pitch;
  *R = (uint32_t)r;
  *nb = (uint32_t)((ns + r - 1) / r);
}

struct FrameIn {
  pcbz_params p;
  const uint16_t *frame, *prev;
  const uint8_t *forced;
  uint8_t *out;
  size_t cap;
};

struct Plan {
  std::vector<BandDesc> bands;
  std::vector<RowItem> rows;
  std::vector<JudgeTask> tasks;
  std::vector<uint32_t> tile_task, tile_local;
  std::vector<int32_t> task_of;
  std::vector<uint32_t> band_start;
  std::vector<FrameOut> frames;
  uint64_t ntot = 0;
  uint32_t slots = 0, segs = 0, pitch_max = 1, nt_max = 1, band_n_max = 0, lens_per_wg = 1, remap_chunks = 1;
  bool any_forced = false;
  bool selector = false;  // the selector decides bands before the judge
  uint32_t used_ids = 0;  // arrangement ids some band may need (all of them for forced frames)
  bool use_forced() const { return any_forced || selector; }
};

int build_plan(pcbz_ctx *ctx, const std::vector<FrameIn> &fin, bool judge_only, Plan &P) {
  for (size_t f = 0; f < fin.size(); f++) {
    const FrameIn &F = fin[f];
    int st = check_params(&F.p);
    if (st) return fail(ctx, st, "frame %zu: invalid parameters", f);
    if (!F.frame) return fail(ctx, PCBZ_EINVAL, "frame %zu: null frame", f);
    if (!F.forced && (F.p.cand_mask & 8u) && !F.prev)
      return fail(ctx, PCBZ_ENEEDPREV, "frame %zu: temporal candidate without a previous frame", f);
    if (F.forced) P.any_forced = true;
    P.used_ids |= F.forced ? 0xFFFFu : F.p.cand_mask;
    uint32_t R, nb;
    plan_rows(&F.p, &R, &nb);
    const uint32_t p = F.p.pitch, W = F.p.w, ns = F.p.h / p;
    const uint32_t lim = 100000u * F.p.level - 19u;
    FrameOut fo;
    fo.out = F.out;
    fo.cap = F.cap;
    fo.h = F.p.h;
    fo.w = W;
    fo.pitch = p;
    fo.level = F.p.level;
    fo.n_bands = nb;
    fo.band_base = (uint32_t)P.bands.size();
    fo.forced = F.forced;
    P.frames.push_back(fo);
    P.pitch_max = std::max(P.pitch_max, p);
    P.nt_max = std::max(P.nt_max, W / p);
    for (uint32_t k = 0; k < nb; k++) {
      BandDesc B;
      B.frame = F.frame;
      B.prev = F.prev;
      B.W = W;
      B.pitch = p;
      B.Nt = W / p;
      B.Rb = std::min(R, ns - k * R);
      B.y0 = k * R * p;
      B.frame_id = (uint32_t)f;
      B.band_in_frame = k;
      B.cand_mask = F.p.cand_mask;
      B.level = F.p.level;
      B.n = 2u * B.Rb * p * W;
      B.off = P.ntot;
      uint64_t rle_max = (uint64_t)B.n + B.n / 4 + 8;
      B.blk_slots = (uint32_t)((rle_max + (lim - 4) - 1) / (lim - 4) + 1);
      B.blk_slot = P.slots;
      P.slots += B.blk_slots;
      const uint32_t bi = (uint32_t)P.bands.size();
      P.band_start.push_back((uint32_t)P.ntot);
      P.ntot += B.n;
      P.band_n_max = std::max(P.band_n_max, B.n);
      for (uint32_t s = 0; s < B.Rb; s++) P.rows.push_back(RowItem{bi, s});
      for (int id = 0; id < kNumCand; id++) {
        int32_t t = -1;
        if (!F.forced && (F.p.cand_mask >> id) & 1u) {
          JudgeTask T;
          T.band = bi;
          T.cand = id;
          T.n = B.n;
          const uint32_t tiles = (B.n + 65535) / 65536;  // 16 segments of 4096 bytes per workgroup
          T.seg_base = P.segs;
          T.x_off = B.off;
          P.segs += tiles;
          t = (int32_t)P.tasks.size();
          for (uint32_t q = 0; q < tiles; q++) {
            P.tile_task.push_back((uint32_t)t);
            P.tile_local.push_back(q);
          }
          P.tasks.push_back(T);
        }
        P.task_of.push_back(t);
      }
      P.bands.push_back(B);
    }
  }
  if (P.ntot >= (1ull << 31)) return fail(ctx, PCBZ_EINVAL, "batch too large (%llu bytes)", (unsigned long long)P.ntot);
  P.band_start.push_back((uint32_t)P.ntot);
  const uint32_t pm = P.pitch_max;
  // lenses per rearrangement workgroup: 16 gives a 2040x2040 frame about
  // 1200 workgroups (32 lenses per workgroup: 33 us, 16: 24 us, 8: 23 us)
  uint32_t tl = 16384u / (pm * pm);
  tl = tl > 1 ? tl - 1 : 0;
  if (tl > 16) tl = 16;
  if (tl < 1) return fail(ctx, PCBZ_EINVAL, "pitch %u too large", pm);
  P.lens_per_wg = tl;
  P.remap_chunks = (P.nt_max + tl - 1) / tl;
  P.selector = !judge_only && ctx->sel != nullptr && !P.bands.empty();
  return PCBZ_OK;
}

// Device pointers of one call's workspace.
struct Work {
  BandDesc *bands;
  RowItem *rows;
  JudgeTask *tasks;
  uint32_t *tile_task, *tile_local;
  int32_t *task_of;
  uint32_t *band_start;
  FrameOut *frames;
  uint8_t *forced;
  uint32_t *ctr;  // [0] err flags, [1] n_blocks, [2] crc chunks, [3] bwt u, [4] n_chunks, [5] n_sym, [6] n_groups, [7] words, [8] cut err
  uint8_t *choice;
  CandBufs cb;
  uint8_t *chosen;
  uint32_t *hist;
  uint16_t *seg_first, *seg_last;
  unsigned long long *score;
  // compression
  uint32_t *runstart, *r1len, *r1off;
  uint8_t *rle;
  BlockDesc *slots, *blocks;
  uint32_t *slot_count, *blk_raw_start, *blk_rle_start, *crc_chunk_base, *crc_acc;
  BwtWork bw;
  uint32_t *sa;
  uint8_t *L;
  BlockCode *codes;
  MtfWork mw;
  uint16_t *sym;
  uint32_t *freq;
  uint8_t *cost, *lens, *sel;
  uint32_t *tfreq, *code_words, *group_base;
  uint32_t *prefix, *sym_bits, *sym_off, *blk_sym_start, *word_start, *band_len;
  uint64_t *frame_len;
  float *feat, *logits;  // selector features [band][64][64][4] and logits [band][4]
  // sizes
  uint32_t max_blocks, n_rle_max, max_chunks, max_sym, max_groups, max_words;
};

size_t layout(Arena &A, const Plan &P, bool compress, Work &w) {
  const uint32_t nbands = (uint32_t)P.bands.size();
  w.bands = A.get<BandDesc>(nbands);
  w.rows = A.get<RowItem>(P.rows.size());
  w.tasks = A.get<JudgeTask>(P.tasks.size());
  w.tile_task = A.get<uint32_t>(P.tile_task.size());
  w.tile_local = A.get<uint32_t>(P.tile_local.size());
  w.task_of = A.get<int32_t>(P.task_of.size());
  w.band_start = A.get<uint32_t>(P.band_start.size());
  w.frames = A.get<FrameOut>(P.frames.size());
  w.forced = A.get<uint8_t>(nbands + 4);
  w.ctr = A.get<uint32_t>(64);
  w.choice = A.get<uint8_t>(nbands + 4);
  // a candidate buffer per arrangement id that some band of the call can use
  for (int id = 0; id < kNumCand; id++) w.cb.p[id] = ((P.used_ids >> id) & 1u) ? A.get<uint8_t>(P.ntot + 16) : nullptr;
  w.hist = A.get<uint32_t>((size_t)P.tasks.size() * 65536);
  w.seg_first = A.get<uint16_t>((size_t)P.segs * 256);
  w.seg_last = A.get<uint16_t>((size_t)P.segs * 256);
  w.score = A.get<unsigned long long>(P.tasks.size() + 1);
  w.feat = P.selector ? A.get<float>((size_t)nbands * kFeatCells * kFeatChan) : nullptr;
  w.logits = P.selector ? A.get<float>((size_t)nbands * 4) : nullptr;
  if (!compress) return A.off;
  const uint64_t N = P.ntot;
  w.chosen = A.get<uint8_t>(N + 16);
  w.runstart = A.get<uint32_t>(N + 1);
  w.r1len = A.get<uint32_t>(N + 1);
  w.r1off = A.get<uint32_t>(N + 1);
  const uint64_t nr = N + N / 4 + 8ull * nbands + 64;
  w.n_rle_max = (uint32_t)nr;
  w.rle = A.get<uint8_t>(nr + 16);
  const uint32_t S = P.slots;
  w.max_blocks = S;
  w.slots = A.get<BlockDesc>(S);
  w.blocks = A.get<BlockDesc>(S + 1);
  w.slot_count = A.get<uint32_t>(nbands);
  w.blk_raw_start = A.get<uint32_t>(S + 1);
  w.blk_rle_start = A.get<uint32_t>(S + 1);
  w.crc_chunk_base = A.get<uint32_t>(S + 1);
  w.crc_acc = A.get<uint32_t>(S + 1);
  w.bw.key[0] = A.get<uint64_t>(nr + 1);
  w.bw.key[1] = A.get<uint64_t>(nr + 1);
  w.bw.val[0] = A.get<uint32_t>(nr + 1);
  w.bw.val[1] = A.get<uint32_t>(nr + 1);
  w.bw.slot = A.get<uint32_t>(nr + 1);
  w.bw.slot2 = A.get<uint32_t>(nr + 1);
  w.bw.rank = A.get<uint32_t>(nr + 1);
  w.bw.counts = A.get<uint32_t>(radix_counts_words((uint32_t)nr, S));
  w.bw.seg_bound = A.get<uint32_t>(seg_bound_words((uint32_t)nr));
  w.bw.gstart = A.get<uint32_t>(nr + 1);
  w.bw.aggs = A.get<uint32_t>(rnd_aggs_words((uint32_t)nr));
  w.bw.d_u = w.ctr ? w.ctr + 10 : nullptr;        // [10], [11]
  w.bw.d_count_n = w.ctr ? w.ctr + 12 : nullptr;
  w.bw.d_min_m = w.ctr ? w.ctr + 13 : nullptr;
  w.bw.d_maxg = w.ctr ? w.ctr + 16 : nullptr;  // d_u + 6: read back with the counts
  w.bw.d_fail = w.ctr ? w.ctr + 17 : nullptr;
  w.sa = A.get<uint32_t>(nr + 1);
  w.L = A.get<uint8_t>(nr + 16);
  w.codes = A.get<BlockCode>(S + 1);
  w.max_chunks = (uint32_t)(nr / kMtfChunk + S + 2);
  w.mw.used = A.get<uint32_t>((size_t)S * 8);
  w.mw.chunk_block = A.get<uint32_t>(w.max_chunks + 1);
  w.mw.plist = A.get<uint8_t>((size_t)w.max_chunks * 256);
  w.mw.plen = A.get<uint32_t>(w.max_chunks);
  w.mw.inlist = A.get<uint8_t>((size_t)w.max_chunks * 256);
  w.mw.seglist = A.get<uint8_t>((size_t)S * kMtfSegs * 256);
  w.mw.seglen = A.get<uint32_t>((size_t)S * kMtfSegs);
  w.mw.idx = A.get<uint8_t>(nr + 16);
  // the MTF stage runs after the suffix sort: reuse the sort's key buffers
  w.mw.zs = w.bw.key[0] ? (uint32_t *)w.bw.key[0] : nullptr;
  w.mw.aggs = w.bw.aggs;  // free once the suffix sort is done
  w.mw.d_n_chunks = w.ctr ? w.ctr + 4 : nullptr;
  w.max_sym = (uint32_t)(nr + S + 1);
  w.sym = A.get<uint16_t>(w.max_sym + 16);
  w.freq = A.get<uint32_t>((size_t)S * kMaxAlpha);
  const size_t tab = (size_t)S * kMaxGroups * kMaxAlpha;
  w.cost = A.get<uint8_t>(tab);
  w.lens = A.get<uint8_t>(tab);
  w.tfreq = A.get<uint32_t>(tab);
  w.code_words = A.get<uint32_t>(tab);
  w.group_base = A.get<uint32_t>(S + 1);
  w.max_groups = w.max_sym / kGroupSize + S + 1;
  w.sel = A.get<uint8_t>(w.max_groups + 16);
  w.prefix = A.get<uint32_t>((size_t)S * kPrefixWords);
  w.sym_bits = A.get<uint32_t>(w.max_sym + 1);
  w.sym_off = A.get<uint32_t>(w.max_sym + 1);
  w.blk_sym_start = A.get<uint32_t>(S + 1);
  w.word_start = A.get<uint32_t>(S + 1);
  w.band_len = A.get<uint32_t>(nbands);
  w.frame_len = A.get<uint64_t>(P.frames.size());
  // data bits <= 9 per symbol (a 9-bit code is always feasible), header < 20 KB
  w.max_words = (uint32_t)std::min<uint64_t>(0xFFFFFFF0ull, ((uint64_t)w.max_sym * 9 / 8 + (uint64_t)S * 20600) / 4 + S);
  return A.off;
}

int ensure_arena(pcbz_ctx *ctx, size_t need) {
  if (ctx->budget && need > ctx->budget)
    return fail(ctx, PCBZ_ENOMEM, "workspace %zu bytes exceeds the HBM budget %zu", need, ctx->budget);
  if (need <= ctx->arena_size) return PCBZ_OK;
  HIPCHK(ctx, hipDeviceSynchronize());
  if (ctx->arena) HIPCHK(ctx, hipFree(ctx->arena));
  ctx->arena = nullptr;
  ctx->arena_size = 0;
  size_t sz = align_up(need + need / 8, 1 << 20);
  if (hipMalloc((void **)&ctx->arena, sz) != hipSuccess) {
    (void)hipGetLastError();
    ctx->arena = nullptr;
    return fail(ctx, PCBZ_ENOMEM, "hipMalloc(%zu) failed", sz);
  }
  ctx->arena_size = sz;
  ctx->gen++;
  return PCBZ_OK;
}

// The judge's fixed-point table Tq(c) = round(c * log2(c) * 2^20), Tq(0) =
// Tq(1) = 0 (the summand of the pair entropy, Sec. 2.1.2, Eq. 1), computed
// on the host in double so that the decision never depends on device math.
void fill_tq(int64_t *t, size_t n) {
  for (size_t c = 0; c < n; c++) t[c] = c < 2 ? 0 : (int64_t)llround((double)c * log2((double)c) * 1048576.0);
}

int ensure_tables(pcbz_ctx *ctx, uint32_t band_n_max) {
  if (!ctx->d_xpow2) {
    uint32_t x[64];
    x[0] = 2u;  // x^1
    for (int k = 1; k < 64; k++) x[k] = h_mulmod(x[k - 1], x[k - 1]);
    HIPCHK(ctx, hipMalloc((void **)&ctx->d_xpow2, sizeof x));
    HIPCHK(ctx, hipMemcpy(ctx->d_xpow2, x, sizeof x, hipMemcpyHostToDevice));
    uint32_t xb[256];
    xb[0] = 1u;
    for (int r = 1; r < 256; r++) xb[r] = h_mulmod(xb[r - 1], 0x100u);  // times x^8
    HIPCHK(ctx, hipMalloc((void **)&ctx->d_xbyte, sizeof xb));
    HIPCHK(ctx, hipMemcpy(ctx->d_xbyte, xb, sizeof xb, hipMemcpyHostToDevice));
  }
  const size_t need_chunks = (size_t)band_n_max / 256 + 4;
  if (need_chunks > ctx->xchunk_n) {
    const size_t n = std::max<size_t>(need_chunks, 4096);
    std::vector<uint32_t> t(n);
    uint32_t x2048 = 2u;
    for (int k = 0; k < 11; k++) x2048 = h_mulmod(x2048, x2048);
    t[0] = 1u;
    for (size_t j = 1; j < n; j++) t[j] = h_mulmod(t[j - 1], x2048);
    if (ctx->d_xchunk) HIPCHK(ctx, hipFree(ctx->d_xchunk));
    HIPCHK(ctx, hipMalloc((void **)&ctx->d_xchunk, n * sizeof(uint32_t)));
    HIPCHK(ctx, hipMemcpy(ctx->d_xchunk, t.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice));
    ctx->xchunk_n = n;
    ctx->gen++;
  }
  const size_t need_tq = (size_t)band_n_max + 2;
  if (need_tq > ctx->tq_n) {
    const size_t n = std::max<size_t>(need_tq, 900002);
    std::vector<int64_t> t(n);
    fill_tq(t.data(), n);
    if (ctx->d_tq) HIPCHK(ctx, hipFree(ctx->d_tq));
    HIPCHK(ctx, hipMalloc((void **)&ctx->d_tq, n * sizeof(int64_t)));
    HIPCHK(ctx, hipMemcpy(ctx->d_tq, t.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
    ctx->tq_n = n;
    ctx->gen++;
  }
  return PCBZ_OK;
}

// Autotuner cache: one JSON object per line,
// {"key": ..., "items": ..., "rounds": ..., "seg": ..., "ms": ...}.
void save_tuning(pcbz_ctx *ctx) {
  if (ctx->tune_path.empty()) return;
  FILE *f = fopen(ctx->tune_path.c_str(), "w");
  if (!f) return;
  for (const TuneRec &r : ctx->tune)
    fprintf(f, "{\"key\": \"%s\", \"items\": %d, \"rounds\": %d, \"seg\": %llu, \"ms\": %.4f}\n", r.key.c_str(),
            r.items, r.rounds, (unsigned long long)r.seg_mask, r.ms);
  fclose(f);
}

void load_tuning(pcbz_ctx *ctx) {
  if (ctx->tune_path.empty()) return;
  FILE *f = fopen(ctx->tune_path.c_str(), "r");
  if (!f) return;
  char line[4096], key[3072];
  while (fgets(line, sizeof line, f)) {
    TuneRec r;
    double ms = 0.0;
    unsigned long long seg = 0;
    if (sscanf(line, "{\"key\": \"%3071[^\"]\", \"items\": %d, \"rounds\": %d, \"seg\": %llu, \"ms\": %lf}", key,
               &r.items, &r.rounds, &seg, &ms) == 5) {
      r.key = key;
      r.ms = ms;
      r.seg_mask = seg;
      if ((r.items == 0 || r.items == 8 || r.items == 16) && r.rounds > 0 && r.rounds < 64) ctx->tune.push_back(r);
    }
  }
  fclose(f);
}

// The plan tables go host -> device through a pinned staging area: the host
// writes the staging buffer (after the previous copies finished), then the
// copies are enqueued (and may be captured into a graph).
struct UploadItem {
  size_t off, bytes;
  void *dst;
};

int stage_plan(pcbz_ctx *ctx, const Plan &P, const Work &w, hipStream_t s, std::vector<UploadItem> &items) {
  std::vector<uint8_t> buf;
  items.clear();
  // each array at the offset the arena gives it (256-byte aligned, 16 bytes
  // of slack after it, also after an empty one), so that the arrays usually
  // reach the device in one copy
  auto add = [&](const void *src, size_t bytes, void *dst) {
    size_t off = align_up(buf.size(), 256);
    buf.resize(off + bytes + 16);
    if (!bytes || !dst) return;
    memcpy(buf.data() + off, src, bytes);
    items.push_back({off, bytes, dst});
  };
  add(P.bands.data(), P.bands.size() * sizeof(BandDesc), w.bands);
  add(P.rows.data(), P.rows.size() * sizeof(RowItem), w.rows);
  add(P.tasks.data(), P.tasks.size() * sizeof(JudgeTask), w.tasks);
  add(P.tile_task.data(), P.tile_task.size() * sizeof(uint32_t), w.tile_task);
  add(P.tile_local.data(), P.tile_local.size() * sizeof(uint32_t), w.tile_local);
  add(P.task_of.data(), P.task_of.size() * sizeof(int32_t), w.task_of);
  add(P.band_start.data(), P.band_start.size() * sizeof(uint32_t), w.band_start);
  add(P.frames.data(), P.frames.size() * sizeof(FrameOut), w.frames);
  // the previous call's copies from the staging area must be finished
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (buf.size() > ctx->h_stage_size) {
    if (ctx->h_stage) HIPCHK(ctx, hipHostFree(ctx->h_stage));
    ctx->h_stage = nullptr;
    size_t sz = align_up(buf.size() * 2, 1 << 16);
    HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_stage, sz, hipHostMallocDefault));
    ctx->h_stage_size = sz;
    ctx->gen++;  // graphs hold the old staging address
  }
  memcpy(ctx->h_stage, buf.data(), buf.size());
  return PCBZ_OK;
}

int enqueue_upload(pcbz_ctx *ctx, const std::vector<UploadItem> &items, hipStream_t s) {
  if (items.empty()) return PCBZ_OK;
  // one copy of the whole span when every destination sits at its staging
  // offset (the gaps between the arrays are the arena's unused slack)
  bool one = true;
  const uint8_t *d0 = (const uint8_t *)items[0].dst;
  for (const UploadItem &it : items)
    if ((const uint8_t *)it.dst < d0 || (size_t)((const uint8_t *)it.dst - d0) != it.off - items[0].off) one = false;
  if (one) {
    const size_t span = items.back().off + items.back().bytes - items[0].off;
    HIPCHK(ctx, hipMemcpyAsync(items[0].dst, ctx->h_stage + items[0].off, span, hipMemcpyHostToDevice, s));
    return PCBZ_OK;
  }
  for (const UploadItem &it : items)
    HIPCHK(ctx, hipMemcpyAsync(it.dst, ctx->h_stage + it.off, it.bytes, hipMemcpyHostToDevice, s));
  return PCBZ_OK;
}

int ensure_small(pcbz_ctx *ctx) {
  if (!ctx->h_small) HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_small, 4096, hipHostMallocDefault));
  return PCBZ_OK;
}

// Judge stages shared by pcbz_judge and the compress path.
void enqueue_judge(const int64_t *tq, const Plan &P, Work &w, hipStream_t s) {
  const uint8_t *forced = P.use_forced() ? w.forced : nullptr;
  trace_stage("arrange");
  if (P.used_ids & 0xFu)
    launch_remap2(w.bands, w.rows, (uint32_t)P.rows.size(), P.remap_chunks, P.lens_per_wg, P.pitch_max, w.cb, forced,
                  0xFu, s);
  if (P.used_ids & 0xFFF0u)
    launch_predict(w.bands, w.rows, (uint32_t)P.rows.size(), P.remap_chunks, P.lens_per_wg, P.pitch_max, w.cb, forced,
                   s);
  trace_stage("judge");
  if (!P.tasks.empty()) {
    // the caller has cleared w.hist and w.score
    launch_judge2(w.tasks, (uint32_t)P.tasks.size(), w.tile_task, w.tile_local, (uint32_t)P.tile_task.size(), w.cb,
                  w.seg_first, w.seg_last, w.hist, tq, w.score, forced, s);
  }
}

// Schedule choices that do not change the output bytes.
struct Tuning {
  int radix_items = 16;  // elements per thread of a radix tile (8 or 16)
  int rounds = 0;        // doubling rounds to enqueue; 0 = read the count back and stop early
  uint64_t seg_mask = 0;  // rounds sorted group by group (bit r - 1: the sort after round r)
};

// Enqueues the whole compression of a plan.  With tu.rounds == 0 the host
// reads the block count, the first-stage length and each round's unresolved
// count back (tight launches); otherwise nothing is read back and every
// launch is sized by its bound, so the sequence can be captured.
int enqueue_compress(pcbz_ctx *ctx, const Plan &P, Work &w, const Tuning &tu, hipStream_t s, int *rounds_out) {
  const uint32_t nbands = (uint32_t)P.bands.size();
  const uint32_t N = (uint32_t)P.ntot;
  const bool eager = tu.rounds == 0;
  trace_stage("arrange");
  {
    // every buffer the call accumulates into, cleared by one launch: the
    // counters, the judge's pair histograms and scores, the block CRC
    // accumulators and the symbol and table counts
    ZeroSpans z;
    z.add(w.ctr, 64);
    z.add(w.hist, P.tasks.size() * 65536);
    z.add(w.score, P.tasks.size() * 2);
    z.add(w.crc_acc, w.max_blocks);
    z.add(w.freq, (size_t)w.max_blocks * kMaxAlpha);
    z.add(w.tfreq, (size_t)w.max_blocks * kMaxGroups * kMaxAlpha);
    zero_spans(z, s);
  }
  if (P.use_forced()) {
    launch_gather_forced(w.frames, (uint32_t)P.frames.size(), w.forced, s);
    launch_validate_forced(w.bands, nbands, w.forced, w.ctr, s);
  }
  if (P.selector) {
    // learned selector: confident bands get their id here and skip the judge
    trace_stage("select");
    launch_features(w.bands, nbands, w.feat, s);
    int st = selector_forward(ctx->sel, w.feat, nbands, w.logits, s);
    if (st) return fail(ctx, st, "selector forward failed");
    launch_select(w.logits, nbands, w.bands, ctx->min_conf, w.forced, w.ctr + 14, s);
  }
  enqueue_judge(ctx->d_tq, P, w, s);
  launch_choose2(w.bands, nbands, w.task_of, w.score, w.tasks, P.use_forced() ? w.forced : nullptr, w.choice, nullptr,
                 nullptr, s);
  trace_stage("gather");
  launch_gather2(w.band_start, nbands, w.cb, w.choice, w.chosen, P.ntot, s);
  trace_stage("rle1");
  // first run-length stage, block cuts, CRCs
  launch_rle1_2(w.band_start, nbands, w.chosen, N, w.runstart, w.r1len, w.r1off, w.rle, w.ctr + 3, s);
  launch_cut2(w.bands, nbands, w.band_start, N, w.runstart, w.r1off, w.slots, w.slot_count, w.ctr + 8, w.blocks,
              w.blk_raw_start, w.blk_rle_start, w.crc_chunk_base, w.ctr + 1, w.ctr + 2, s);
  // the block CRCs run beside the suffix sort (only the header bits need them)
  hipStream_t cs = ctx->side ? ctx->side : s;
  if (ctx->side) {
    HIPCHK(ctx, hipEventRecord(ctx->fev[0], s));
    HIPCHK(ctx, hipStreamWaitEvent(cs, ctx->fev[0], 0));
  }
  launch_crc2(w.chosen, N, w.blocks, w.ctr + 1, w.max_blocks, w.blk_raw_start, ctx->d_xchunk, ctx->d_xbyte,
              ctx->d_xpow2, w.crc_acc, cs);
  uint32_t nb = w.max_blocks, nrle = w.n_rle_max;
  const uint32_t *d_nrle = w.r1off + N;
  if (eager) {
    // counters: [1] blocks, [3] run-length output bytes, [8] slot overflow
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_small, w.ctr, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (ctx->h_small[8]) return fail(ctx, PCBZ_EDEVICE, "block slot overflow");
    nb = ctx->h_small[1];
    nrle = ctx->h_small[3];
  }
  // suffix sort of every block
  trace_stage("bwt");
  uint64_t seg_mask = eager ? 0ull : tu.seg_mask;
  const int rounds = run_bwt(w.rle, d_nrle, nrle, w.ctr + 1, nb, w.blk_rle_start, w.bw, w.sa, w.L, w.codes,
                             eager ? 40 : tu.rounds, tu.radix_items, eager ? ctx->h_small + 32 : nullptr, &seg_mask,
                             w.ctr + 9, s);
  if (eager) ctx->last_seg_mask = seg_mask;
  if (rounds_out) *rounds_out = rounds;
  // move-to-front, zero runs, tables, bit-packing
  trace_stage("mtf");
  launch_mtf2(w.L, d_nrle, nrle, w.blk_rle_start, w.ctr + 1, nb, nrle / kMtfChunk + nb + 1, w.mw, w.codes, w.sym, w.freq,
              w.ctr + 5, s);
  const uint32_t max_sym = nrle + nb;
  trace_stage("tables");
  launch_huff2(w.sym, w.ctr + 1, nb, max_sym / kGroupSize + nb + 1, w.codes, w.freq, w.cost, w.tfreq, w.group_base,
               w.ctr + 6, w.sel, w.lens, w.code_words, s);
  const uint32_t max_words =
      (uint32_t)std::min<uint64_t>(0xFFFFFFF0ull, ((uint64_t)max_sym * 9 / 8 + (uint64_t)nb * 20600) / 4 + nb);
  trace_stage("pack");
  // header bits on the side stream (after the CRCs), beside the symbol lengths
  if (ctx->side) {
    HIPCHK(ctx, hipEventRecord(ctx->fev[1], s));
    HIPCHK(ctx, hipStreamWaitEvent(cs, ctx->fev[1], 0));
  }
  launch_pack_prefix(w.ctr + 1, nb, w.blocks, w.codes, w.mw.used, w.sel, w.lens, w.prefix, cs);
  if (ctx->side) HIPCHK(ctx, hipEventRecord(ctx->fev[2], cs));
  launch_pack2(w.ctr + 1, nb, w.blocks, w.codes, w.sel, w.lens, w.code_words, w.sym, w.ctr + 5, max_sym, w.prefix,
               w.sym_bits, w.sym_off, w.blk_sym_start, w.frames, (uint32_t)P.frames.size(), w.bands,
               w.choice, w.band_len, w.frame_len, w.word_start, w.ctr + 7, max_words, ctx->side ? ctx->fev[2] : nullptr,
               s);
  trace_stage(nullptr);
  return PCBZ_OK;
}

// Reads the per-frame lengths and the error words back (synchronises s).
int read_results(pcbz_ctx *ctx, const Plan &P, const Work &w, hipStream_t s, std::vector<size_t> &lens,
                 uint32_t *ctr_out) {
  const size_t nf = P.frames.size();
  std::vector<uint64_t> tmp(nf);
  uint64_t *hl = (uint64_t *)(ctx->h_small + 64);
  const bool fits = nf <= (4096 - 256) / 8;
  HIPCHK(ctx, hipMemcpyAsync(fits ? (void *)hl : (void *)tmp.data(), w.frame_len, nf * sizeof(uint64_t),
                             hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_small, w.ctr, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  HIPCHK(ctx, hipGetLastError());
  if (fits)
    lens.assign(hl, hl + nf);
  else
    lens.assign(tmp.begin(), tmp.end());
  memcpy(ctr_out, ctx->h_small, 16 * sizeof(uint32_t));
  return PCBZ_OK;
}

int check_results(pcbz_ctx *ctx, const std::vector<FrameIn> &fin, const std::vector<size_t> &lens,
                  const uint32_t *ctr) {
  if (ctr[8]) return fail(ctx, PCBZ_EDEVICE, "block slot overflow");
  if (ctr[0] & 1u) return fail(ctx, PCBZ_EINVAL, "forced arrangement id above 3");
  if (ctr[0] & 2u) return fail(ctx, PCBZ_ENEEDPREV, "forced temporal arrangement without a previous frame");
  for (size_t f = 0; f < lens.size(); f++)
    if (lens[f] > fin[f].cap) return fail(ctx, PCBZ_ENOSPC, "frame %zu needs %zu bytes", f, lens[f]);
  return PCBZ_OK;
}

int prepare(pcbz_ctx *ctx, const std::vector<FrameIn> &fin, Plan &P, Work &w) {
  int st = build_plan(ctx, fin, false, P);
  if (st) return st;
  Arena meas{nullptr};
  size_t need = layout(meas, P, true, w);
  if ((st = ensure_arena(ctx, need))) return st;
  if ((st = ensure_tables(ctx, P.band_n_max))) return st;
  if ((st = ensure_small(ctx))) return st;
  Arena A{ctx->arena};
  layout(A, P, true, w);
  return PCBZ_OK;
}

void copy_choices(pcbz_ctx *ctx, const Plan &P, const Work &w, const std::vector<uint8_t *> &choice_out,
                  hipStream_t s) {
  for (size_t f = 0; f < P.frames.size() && f < choice_out.size(); f++)
    if (choice_out[f])
      (void)hipMemcpyAsync(choice_out[f], w.choice + P.frames[f].band_base, P.frames[f].n_bands,
                           hipMemcpyDeviceToDevice, s);
  (void)ctx;
}

// Compression with host read-backs (fixed null: the block count, the
// first-stage size and each round's unresolved count are read back and size
// every launch tightly) or with a fixed schedule (no read-back until the
// results).  A fixed schedule that leaves rotations unresolved, or meets a
// group too large for the in-group sort, returns kRedo: the outputs then
// hold no valid result and the caller runs the call again with read-backs.
constexpr int kRedo = -1000;

int run_compress(pcbz_ctx *ctx, const std::vector<FrameIn> &fin, hipStream_t s, std::vector<size_t> &lens,
                 std::vector<uint8_t *> choice_out, const Tuning *fixed = nullptr) {
  Plan P;
  Work w{};
  int st = prepare(ctx, fin, P, w);
  if (st) return st;
  std::vector<UploadItem> items;
  if ((st = stage_plan(ctx, P, w, s, items))) return st;
  if ((st = enqueue_upload(ctx, items, s))) return st;
  Tuning tu;
  tu.radix_items = ctx->eager_items;
  if (fixed) tu = *fixed;
  int rounds = 0;
  if ((st = enqueue_compress(ctx, P, w, tu, s, &rounds))) return st;
  copy_choices(ctx, P, w, choice_out, s);
  uint32_t ctr[16];
  if ((st = read_results(ctx, P, w, s, lens, ctr))) return st;
  trace_settle(s);
  if (fixed && ctr[9] != 0) return kRedo;
  ctx->last_raw = P.ntot;
  ctx->last_rle = ctr[3];
  ctx->last_blocks = ctr[1];
  ctx->last_rounds = (uint32_t)rounds;
  ctx->last_graph = 0;
  ctx->last_sel_bands = P.selector ? (uint32_t)P.bands.size() : 0;
  ctx->last_sel_fallback = P.selector ? ctr[14] : 0;
  return check_results(ctx, fin, lens, ctr);
}

// Shape signature of a batch: everything that fixes the captured launch
// sequence (geometry, level, candidates, and which frames have prev/forced).
std::string shape_key(pcbz_ctx *ctx, const std::vector<FrameIn> &fin) {
  std::string k;
  char buf[96];
  for (const FrameIn &F : fin) {
    snprintf(buf, sizeof buf, "%ux%u/%u/%u/%x/%d%d;", F.p.h, F.p.w, F.p.pitch, F.p.level, F.p.cand_mask,
             F.prev ? 1 : 0, F.forced ? 1 : 0);
    k += buf;
  }
  if (ctx->sel) {
    snprintf(buf, sizeof buf, "sel%p/%a/%llu", (void *)ctx->sel, (double)ctx->min_conf,
             (unsigned long long)selector_gen(ctx->sel));
    k += buf;
  }
  return k;
}

// Rounds a graph sorts group by group, from the last eager call: the rounds
// it sorted that way, and every round after its last (normally empty).
uint64_t seg_schedule(const pcbz_ctx *ctx) {
  const uint32_t r = ctx->last_rounds;
  const uint64_t later = r >= 1 && r <= 64 ? ~0ull << (r - 1) : (r == 0 ? ~0ull : 0ull);
  return ctx->last_seg_mask | later;
}

GraphEntry *find_graph(pcbz_ctx *ctx, const std::string &key, const Tuning &tu) {
  for (GraphEntry &g : ctx->graphs)
    if (g.key == key && g.items == tu.radix_items && g.rounds == tu.rounds && g.seg_mask == tu.seg_mask &&
        g.gen == ctx->gen)
      return &g;
  return nullptr;
}

// Captures enqueue_compress for this plan into a graph (uploads included).
int capture(pcbz_ctx *ctx, const Plan &P, Work &w, const std::vector<UploadItem> &items, const std::string &key,
            const Tuning &tu, GraphEntry **out) {
  hipStream_t gs = ctx->gstream;
  hipGraph_t graph = nullptr;
  if (ctx->graphs.size() >= 16) {  // bounded cache: drop the oldest graph
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  const bool trace_was_on = g_trace_on;  // event tracing applies to eager calls only
  g_trace_on = false;
  HIPCHK(ctx, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
  int st = enqueue_upload(ctx, items, gs);
  if (!st) st = enqueue_compress(ctx, P, w, tu, gs, nullptr);
  hipError_t e = hipStreamEndCapture(gs, &graph);
  g_trace_on = trace_was_on;
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(ctx, PCBZ_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  GraphEntry g;
  g.key = key;
  g.items = tu.radix_items;
  g.rounds = tu.rounds;
  g.seg_mask = tu.seg_mask;
  g.gen = ctx->gen;
  HIPCHK(ctx, hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  (void)hipGraphDestroy(graph);
  ctx->graphs.push_back(g);
  *out = &ctx->graphs.back();
  return PCBZ_OK;
}

// Runs a captured graph ordered after the caller's stream and before its
// later work.
int launch_graph(pcbz_ctx *ctx, GraphEntry *g, hipStream_t s, float *ms) {
  HIPCHK(ctx, hipEventRecord(ctx->ev[0], s));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->gstream, ctx->ev[0], 0));
  HIPCHK(ctx, hipEventRecord(ctx->ev[1], ctx->gstream));
  HIPCHK(ctx, hipGraphLaunch(g->exec, ctx->gstream));
  HIPCHK(ctx, hipEventRecord(ctx->ev[2], ctx->gstream));
  HIPCHK(ctx, hipStreamWaitEvent(s, ctx->ev[2], 0));
  if (ms) {
    HIPCHK(ctx, hipEventSynchronize(ctx->ev[2]));
    HIPCHK(ctx, hipEventElapsedTime(ms, ctx->ev[1], ctx->ev[2]));
  }
  return PCBZ_OK;
}

// Batched compression through a captured graph per batch shape.  The first
// call of a shape runs eagerly (to learn the round count and the reference
// lengths), then the autotuner times a second eager call and one replay of a
// captured graph per candidate schedule (host clock, read-backs included)
// and keeps the fastest: later calls replay that graph, or run eagerly when
// the eager call won (unless graphs are forced).  If a replay ends with
// unresolved rotations (data needing more rounds than the tuned budget), the
// call is redone eagerly and the budget raised.
int run_compress_graph(pcbz_ctx *ctx, const std::vector<FrameIn> &fin, hipStream_t s, std::vector<size_t> &lens) {
  const std::string key = shape_key(ctx, fin);
  TuneRec *rec = nullptr;
  for (TuneRec &r : ctx->tune)
    if (r.key == key) rec = &r;
  if (!rec) {
    // learn: eager run gives the correct output and the rounds needed
    int st = run_compress(ctx, fin, s, lens, {});
    if (st) return st;
    TuneRec r;
    r.key = key;
    r.rounds = (int)ctx->last_rounds + 1;
    r.seg_mask = seg_schedule(ctx);
    const auto ms_since = [](std::chrono::steady_clock::time_point t) {
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
    };
    // the eager call is a candidate too (items 0)
    std::vector<size_t> le;
    auto t0 = std::chrono::steady_clock::now();
    if ((st = run_compress(ctx, fin, s, le, {}))) return st;
    r.items = 0;
    r.ms = ms_since(t0);
    double best = ctx->use_graphs == 2 ? 1e30 : r.ms;
    Plan P;
    Work w{};
    if ((st = prepare(ctx, fin, P, w))) return st;
    std::vector<UploadItem> items;
    const int choices[2] = {8, 16};
    // the replays write into the caller's output buffers: after one that did
    // not reproduce the eager result those bytes are rewritten before returning
    bool outs_stale = false;
    for (int c : choices) {
      Tuning tu;
      tu.radix_items = c;
      tu.rounds = ctx->tune_rounds > 0 ? ctx->tune_rounds : r.rounds;
      tu.seg_mask = r.seg_mask;
      if ((st = stage_plan(ctx, P, w, s, items))) return st;
      GraphEntry *g = nullptr;
      if ((st = capture(ctx, P, w, items, key, tu, &g))) return st;
      std::vector<size_t> l2;
      uint32_t ctr[16];
      if ((st = launch_graph(ctx, g, s, nullptr))) return st;  // warm
      if ((st = read_results(ctx, P, w, s, l2, ctr))) return st;
      t0 = std::chrono::steady_clock::now();
      if ((st = stage_plan(ctx, P, w, s, items))) return st;
      if ((st = launch_graph(ctx, g, s, nullptr))) return st;
      if ((st = read_results(ctx, P, w, s, l2, ctr))) return st;
      const double ms = ms_since(t0);
      if (ctr[9] != 0 || l2 != lens) {  // schedule did not reproduce the eager result
        outs_stale = true;
        continue;
      }
      outs_stale = false;  // this replay rewrote every output with the eager bytes
      if (ms < best) {
        best = ms;
        r.items = c;
        r.ms = ms;
        r.rounds = tu.rounds;
      }
    }
    if (r.items == 0) r.rounds = (int)ctx->last_rounds + 1;
    ctx->tune_failed_replays = 0;
    if (outs_stale) {
      ctx->tune_failed_replays = 1;
      if ((st = run_compress(ctx, fin, s, le, {}))) return st;
    }
    ctx->tune.push_back(r);
    save_tuning(ctx);
    return PCBZ_OK;  // lens from the eager run
  }
  if (rec->items == 0) return run_compress(ctx, fin, s, lens, {});  // the eager call was faster
  Plan P;
  Work w{};
  int st = prepare(ctx, fin, P, w);
  if (st) return st;
  Tuning tu;
  tu.radix_items = rec->items;
  tu.rounds = rec->rounds;
  tu.seg_mask = rec->seg_mask;
  std::vector<UploadItem> items;
  if ((st = stage_plan(ctx, P, w, s, items))) return st;
  GraphEntry *g = find_graph(ctx, key, tu);
  if (!g && (st = capture(ctx, P, w, items, key, tu, &g))) return st;
  if ((st = launch_graph(ctx, g, s, nullptr))) return st;
  uint32_t ctr[16];
  if ((st = read_results(ctx, P, w, s, lens, ctr))) return st;
  ctx->last_raw = P.ntot;
  ctx->last_rle = ctr[3];
  ctx->last_blocks = ctr[1];
  ctx->last_rounds = (uint32_t)tu.rounds;
  ctx->last_graph = 1;
  ctx->last_sel_bands = P.selector ? (uint32_t)P.bands.size() : 0;
  ctx->last_sel_fallback = P.selector ? ctr[14] : 0;
  if (ctr[9] != 0) {
    // more rounds needed than the budget, or a group too large for the
    // in-group sort: redo eagerly and remember
    st = run_compress(ctx, fin, s, lens, {});
    if (st) return st;
    rec->rounds = std::max(rec->rounds, (int)ctx->last_rounds + 1);
    rec->seg_mask &= seg_schedule(ctx);
    save_tuning(ctx);
    return PCBZ_OK;
  }
  return check_results(ctx, fin, lens, ctr);
}

}  // namespace

int pcbz::context_device(const pcbz_ctx *ctx) { return ctx->device; }

// ---------------------------------------------------------------- fixed workspace
// pcbz_judge_noalloc takes its workspace (plan tables, candidate bytes, pair
// histograms, segment tables, scores) from `scratch` and its Tq table from
// `tq_fixed` instead of the context's arena.  Each device holds one copy of
// both for as long as the process runs; in host code their names are only
// stand-ins, so the device addresses come from hipGetSymbolAddress, once per
// device, while pcbz_create sets that device up.
namespace {
constexpr size_t kScratchBytes = 48ull << 20;  // the judge of one 2040 x 2040 frame, 4 candidates: ~44 MB
constexpr size_t kTqFixed = 900002;            // pair counts of any band up to the level-9 block limit
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];
static __device__ __align__(256) int64_t tq_fixed[kTqFixed];

namespace {
std::mutex g_fixed_mu;
uint8_t *g_scratch_ptr[kMaxDevices];
int64_t *g_tq_fixed_ptr[kMaxDevices];

// Device addresses of the fixed workspace and Tq table of the current device
// (which is `dev`), filling the table on the device's first use.
int setup_fixed(pcbz_ctx *ctx, int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ctx, PCBZ_EDEVICE, "device %d has no fixed workspace", dev);
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (g_scratch_ptr[dev] && g_tq_fixed_ptr[dev]) return PCBZ_OK;
  void *ps = nullptr, *pt = nullptr;
  HIPCHK(ctx, hipGetSymbolAddress(&ps, HIP_SYMBOL(scratch)));
  HIPCHK(ctx, hipGetSymbolAddress(&pt, HIP_SYMBOL(tq_fixed)));
  if (!ps || !pt) return fail(ctx, PCBZ_EDEVICE, "no device address for the fixed workspace");
  std::vector<int64_t> t(kTqFixed);
  fill_tq(t.data(), kTqFixed);
  HIPCHK(ctx, hipMemcpy(pt, t.data(), kTqFixed * sizeof(int64_t), hipMemcpyHostToDevice));
  g_tq_fixed_ptr[dev] = (int64_t *)pt;
  g_scratch_ptr[dev] = (uint8_t *)ps;
  return PCBZ_OK;
}
}  // namespace

// ---------------------------------------------------------------- decompression host side
namespace pcbz {

uint32_t rd_le(const uint8_t *p, int k) {
  uint32_t v = 0;
  for (int i = 0; i < k; i++) v |= (uint32_t)p[i] << (8 * i);
  return v;
}

// Container header (Sec. 2.1.4: the 8-bit arrangement id of each band is
// stored in the header): geometry, level, band ids and stream lengths; the
// lengths must add up to the container.  Host only.
int peek_container(const uint8_t *in, size_t in_len, pcbz_params *out, uint32_t *n_bands, std::vector<uint8_t> *ids,
                   std::vector<uint32_t> *lens) {
  if (in_len < 20 || memcmp(in, "PCBZ", 4) != 0 || in[4] != 1) return PCBZ_EDATA;
  pcbz_params p;
  p.level = in[5];
  p.pitch = rd_le(in + 6, 2);
  p.h = rd_le(in + 8, 4);
  p.w = rd_le(in + 12, 4);
  const uint32_t nb = rd_le(in + 16, 2);
  p.cand_mask = 0;
  if (p.level < 1 || p.level > 9 || p.pitch == 0 || p.h == 0 || p.w == 0 || p.h % p.pitch || p.w % p.pitch)
    return PCBZ_EDATA;
  if (in_len < 20 + 5ull * nb) return PCBZ_EDATA;
  uint64_t total = 20 + 5ull * nb;
  for (uint32_t b = 0; b < nb; b++) {
    const uint8_t id = in[20 + 5 * b];
    const uint32_t l = rd_le(in + 20 + 5 * b + 1, 4);
    if (id >= kNumCand) return PCBZ_EDATA;
    p.cand_mask |= 1u << id;
    if (ids) ids->push_back(id);
    if (lens) lens->push_back(l);
    total += l;
  }
  if (total != in_len) return PCBZ_EDATA;
  // the band count must match the plan for this geometry
  uint64_t r = (100000ull * p.level - 19) / (2ull * p.pitch * p.w);
  if (r < 1) r = 1;
  const uint64_t ns = p.h / p.pitch;
  if ((ns + r - 1) / r != nb) return PCBZ_EDATA;
  *out = p;
  if (n_bands) *n_bands = nb;
  return PCBZ_OK;
}

}  // namespace pcbz

namespace {

struct DecIn {
  const uint8_t *in;
  size_t len;
  const uint16_t *prev;
  uint16_t *out;
  size_t out_elems;
};

struct DecPlan {
  std::vector<DecBand> bands;
  std::vector<RowItem> rows;
  uint32_t slots = 0, max_nslots = 0, band_n_max = 0;
  uint64_t sym_total = 0, n_max = 0, raw_total = 0, col0_total = 0;
  uint32_t pred_pixel = 0, pred_lines = 0, pred_sets = 0, nt_max = 0;
};

size_t dec_layout(Arena &A, const DecPlan &P, DecWork &w) {
  w.n_bands = (uint32_t)P.bands.size();
  w.n_slots = P.slots;
  w.max_nslots = P.max_nslots;
  w.sym_total = (uint32_t)P.sym_total;
  w.n_max = (uint32_t)P.n_max;
  w.raw_total = (uint32_t)P.raw_total;
  w.n_rows = (uint32_t)P.rows.size();
  w.pred_pixel = P.pred_pixel;
  w.pred_lines = P.pred_lines;
  w.pred_sets = P.pred_sets;
  w.nt_max = P.nt_max;
  w.max_chunks = (uint32_t)(P.sym_total / kDecChunk + P.slots + 1);
  w.max_segs = w.max_chunks / kDecSeg + P.slots + 1;
  w.max_spl = (uint32_t)(P.n_max / kDecSplit + 2ull * P.slots + 1);
  w.max_tiles = (uint32_t)(P.n_max / kDecTile + P.slots + 1);
  const size_t S = P.slots, N = P.n_max;
  w.bands = A.get<DecBand>(w.n_bands);
  w.rows = A.get<RowItem>(w.n_rows);
  w.slots = A.get<DecSlot>(S);
  w.ctr = A.get<uint32_t>(kDcWords);
  w.seq = A.get<uint8_t>(S * 256);
  w.sym = A.get<uint16_t>(P.sym_total + 64);
  w.tok = A.get<uint8_t>(P.sym_total + 64);
  w.chunk_slot = A.get<uint32_t>(w.max_chunks);
  w.chunk_tot = A.get<uint32_t>(w.max_chunks);
  w.chunk_off = A.get<uint32_t>(w.max_chunks);
  w.chunk_fin = A.get<uint8_t>((size_t)w.max_chunks * 256);
  w.chunk_in = A.get<uint8_t>((size_t)w.max_chunks * 256);
  w.seg_slot = A.get<uint32_t>(w.max_segs);
  w.seg_perm = A.get<uint8_t>((size_t)w.max_segs * 256);
  w.seg_in = A.get<uint8_t>((size_t)w.max_segs * 256);
  w.seg_tot = A.get<uint32_t>(w.max_segs);
  w.seg_off = A.get<uint32_t>(w.max_segs);
  w.L = A.get<uint8_t>(N + 16);
  w.T = A.get<uint8_t>(N + 16);
  w.key[0] = A.get<uint64_t>(N + 1);
  w.key[1] = A.get<uint64_t>(N + 1);
  w.val[0] = A.get<uint32_t>(N + 1);
  w.val[1] = A.get<uint32_t>(N + 1);
  w.E = A.get<uint32_t>(N + 1);
  w.counts = A.get<uint32_t>(radix_counts_words((uint32_t)N, (uint32_t)S));
  w.blk_start = A.get<uint32_t>(S + 1);
  w.blk_slot = A.get<uint32_t>(S + 1);
  w.blk_spl0 = A.get<uint32_t>(S + 1);
  w.blk_tile0 = A.get<uint32_t>(S + 1);
  w.spl_nxt = A.get<uint32_t>(w.max_spl);
  w.spl_len = A.get<uint32_t>(w.max_spl);
  w.spl_pos = A.get<uint32_t>(w.max_spl);
  w.tile_agg = A.get<uint32_t>((size_t)w.max_tiles * 6);
  w.tile_in = A.get<uint32_t>((size_t)w.max_tiles * 2);
  w.raw = A.get<uint8_t>(P.raw_total + 16);
  w.col0_total = (uint32_t)P.col0_total;
  w.col0 = A.get<uint16_t>(P.col0_total + 8);
  w.blocks = A.get<BlockDesc>(S + 1);
  w.blk_raw_start = A.get<uint32_t>(S + 1);
  w.crc_acc = A.get<uint32_t>(S + 1);
  return A.off;
}

const char *dec_err_text(uint32_t bits) {
  if (bits & kDecErrStream) return "malformed bzip2 stream";
  if (bits & kDecErrSlots) return "band streams do not end where the band does";
  if (bits & kDecErrMtf) return "bad move-to-front index, zero run or block length";
  if (bits & kDecErrBwt) return "inverse BWT does not form one cycle";
  if (bits & kDecErrLen) return "band decodes to the wrong number of bytes";
  if (bits & kDecErrCrc) return "block CRC mismatch";
  return "corrupt data";
}

// The decompression path (Fig. 1c, Fig. 2b) for containers in device memory:
// the headers come back to the host (one copy each), every band of every
// container is decoded on the device at once, and the counters come back
// twice (after the move-to-front stage, to size the later launches, and at
// the end for the status).
int run_decompress(pcbz_ctx *ctx, const std::vector<DecIn> &in, hipStream_t s) {
  constexpr size_t kHead = 4096;
  const size_t n = in.size();
  if (n * kHead > ctx->h_dec_size) {
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (ctx->h_dec) HIPCHK(ctx, hipHostFree(ctx->h_dec));
    ctx->h_dec = nullptr;
    ctx->h_dec_size = 0;
    HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_dec, n * kHead, hipHostMallocDefault));
    ctx->h_dec_size = n * kHead;
  }
  for (size_t i = 0; i < n; i++)
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_dec + i * kHead, in[i].in, std::min(in[i].len, kHead), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  DecPlan P;
  std::vector<uint8_t> big;
  for (size_t i = 0; i < n; i++) {
    const uint8_t *h = ctx->h_dec + i * kHead;
    const size_t avail = std::min(in[i].len, kHead);
    if (avail < 20) return fail(ctx, PCBZ_EDATA, "container %zu: too short", i);
    const uint32_t nb_hdr = rd_le(h + 16, 2);
    const size_t hdr = 20 + 5ull * nb_hdr;
    if (hdr > avail) {  // a long band table: read the whole table
      if (hdr > in[i].len) return fail(ctx, PCBZ_EDATA, "container %zu: truncated band table", i);
      big.resize(hdr);
      HIPCHK(ctx, hipMemcpy(big.data(), in[i].in, hdr, hipMemcpyDeviceToHost));
      h = big.data();
    }
    pcbz_params p;
    uint32_t nb = 0;
    std::vector<uint8_t> ids;
    std::vector<uint32_t> lens;
    if (peek_container(h, in[i].len, &p, &nb, &ids, &lens))
      return fail(ctx, PCBZ_EDATA, "container %zu: bad header", i);
    pcbz_params q = p;
    q.cand_mask = 1;
    if (check_params(&q)) return fail(ctx, PCBZ_EDATA, "container %zu: geometry outside the library's limits", i);
    const size_t npix = (size_t)p.h * p.w;
    if (in[i].out_elems < npix)
      return fail(ctx, PCBZ_ENOSPC, "container %zu: output holds %zu pixels, frame has %zu", i, in[i].out_elems, npix);
    uint32_t R, nbp;
    plan_rows(&p, &R, &nbp);
    const uint32_t P0 = p.pitch, W = p.w, ns = p.h / P0;
    const uint32_t lim = 100000u * p.level - 19u;
    size_t pos = hdr;
    for (uint32_t k = 0; k < nb; k++) {
      if (lens[k] > (64u << 20)) return fail(ctx, PCBZ_EDATA, "container %zu: band %u longer than 64 MiB", i, k);
      if (ids[k] == PCBZ_VIEW_DT && !in[i].prev)
        return fail(ctx, PCBZ_ENEEDPREV, "container %zu: band %u uses the temporal arrangement", i, k);
      DecBand B{};
      B.src = in[i].in + pos;
      B.src_len = lens[k];
      B.out = in[i].out;
      B.prev = in[i].prev;
      B.id = ids[k];
      B.W = W;
      B.pitch = P0;
      B.Nt = W / P0;
      B.Rb = std::min(R, ns - k * R);
      B.y0 = k * R * P0;
      B.n = 2u * B.Rb * P0 * W;
      B.level = p.level;
      B.raw_off = (uint32_t)P.raw_total;
      B.col0_off = (uint32_t)P.col0_total;
      if (B.id >= 4) {
        const uint32_t domain = (B.id - 4) / 4;
        if (domain == 0) {
          P.pred_pixel = 1;
        } else {
          if (B.Nt > 32768)
            return fail(ctx, PCBZ_EINVAL, "container %zu: predictor bands wider than 32768 lenses are not decoded", i);
          P.pred_lines = 1;
          P.pred_sets = std::max<uint32_t>(P.pred_sets, domain == 1 ? P0 * P0 : B.Rb * P0);
          P.nt_max = std::max<uint32_t>(P.nt_max, B.Nt);
        }
      }
      if (B.id == PCBZ_VIEW_DX) P.col0_total += (uint64_t)P0 * P0 * B.Rb;
      const uint64_t cap = (uint64_t)B.n + B.n / 4 + 8;
      B.blk_cap = (uint32_t)cap;
      B.nslots = (uint32_t)((cap + (lim - 4) - 1) / (lim - 4) + 1);
      B.slot0 = P.slots;
      B.sym_base = (uint32_t)P.sym_total;
      B.sym_end = (uint32_t)(P.sym_total + cap + B.nslots + 1);
      P.slots += B.nslots;
      P.max_nslots = std::max(P.max_nslots, B.nslots);
      P.sym_total = B.sym_end;
      P.n_max += cap;
      P.raw_total += B.n;
      P.band_n_max = std::max(P.band_n_max, B.n);
      const uint32_t bi = (uint32_t)P.bands.size();
      for (uint32_t r = 0; r < B.Rb; r++) P.rows.push_back(RowItem{bi, r});
      P.bands.push_back(B);
      pos += lens[k];
    }
    if (P.raw_total >= (1ull << 31) || P.n_max >= (1ull << 31) || P.sym_total >= (1ull << 31))
      return fail(ctx, PCBZ_EINVAL, "batch too large to decode in one call");
  }
  if (P.bands.empty()) return PCBZ_OK;
  DecWork w{};
  Arena meas{nullptr};
  const size_t need = dec_layout(meas, P, w);
  int st;
  if ((st = ensure_arena(ctx, need))) return st;
  if ((st = ensure_tables(ctx, P.band_n_max))) return st;
  Arena A{ctx->arena};
  dec_layout(A, P, w);
  ctx->last_dec = w;
  ctx->last_dec_valid = true;
  // plan tables through the pinned staging area (one copy)
  {
    std::vector<uint8_t> buf;
    std::vector<UploadItem> items;
    auto add = [&](const void *src, size_t bytes, void *dst) {
      size_t off = align_up(buf.size(), 256);
      buf.resize(off + bytes + 16);
      if (!bytes || !dst) return;
      memcpy(buf.data() + off, src, bytes);
      items.push_back({off, bytes, dst});
    };
    add(P.bands.data(), P.bands.size() * sizeof(DecBand), w.bands);
    add(P.rows.data(), P.rows.size() * sizeof(RowItem), w.rows);
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (buf.size() > ctx->h_stage_size) {
      if (ctx->h_stage) HIPCHK(ctx, hipHostFree(ctx->h_stage));
      ctx->h_stage = nullptr;
      size_t sz = align_up(buf.size() * 2, 1 << 16);
      HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_stage, sz, hipHostMallocDefault));
      ctx->h_stage_size = sz;
      ctx->gen++;
    }
    memcpy(ctx->h_stage, buf.data(), buf.size());
    if ((st = enqueue_upload(ctx, items, s))) return st;
  }
  trace_stage("decode");
  ZeroSpans z;
  z.add(w.ctr, kDcWords);
  z.add(w.slots, (size_t)P.slots * sizeof(DecSlot) / 4);
  z.add(w.crc_acc, (size_t)P.slots + 1);
  zero_spans(z, s);
  fill_u32(w.ctr + kDcBand, 0xFFFFFFFFu, 1, s);
  launch_dec_front(w, s);
  if ((st = ensure_small(ctx))) return st;
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_small, w.ctr, kDcWords * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  uint32_t hc[kDcWords];
  memcpy(hc, ctx->h_small, sizeof hc);
  if (hc[kDcErr]) {
    trace_stage(nullptr);
    return fail(ctx, PCBZ_EDATA, "%s (band %u of the call)", dec_err_text(hc[kDcErr]), hc[kDcBand]);
  }
  launch_dec_back(w, hc, ctx->eager_items, ctx->d_xchunk, ctx->d_xbyte, ctx->d_xpow2, s);
  trace_stage(nullptr);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_small, w.ctr, 2 * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  trace_settle(s);
  const uint32_t err = ctx->h_small[kDcErr], band = ctx->h_small[kDcBand];
  if (err) return fail(ctx, PCBZ_EDATA, "%s (band %u of the call)", dec_err_text(err), band);
  return PCBZ_OK;
}

}  // namespace

extern "C" {

int pcbz_create(pcbz_ctx **out, int hip_device, size_t hbm_budget_bytes) {
  if (!out) return PCBZ_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
    (void)hipGetLastError();
    return PCBZ_EDEVICE;
  }
  if (hipSetDevice(hip_device) != hipSuccess) return PCBZ_EDEVICE;
  pcbz_ctx *c = new pcbz_ctx();
  c->device = hip_device;
  c->budget = hbm_budget_bytes;
  if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    *out = nullptr;
    return PCBZ_EDEVICE;
  }
  for (hipEvent_t &e : c->ev) (void)hipEventCreate(&e);
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) c->side = nullptr;
  for (hipEvent_t &e : c->fev)
    if (c->side && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
  for (hipEvent_t e : c->fev)
    if (!e && c->side) {  // without its events the side stream is not used
      (void)hipStreamDestroy(c->side);
      c->side = nullptr;
    }
  // the fixed workspace of pcbz_judge_noalloc; a failure here only disables
  // that entry point (it then reports the error)
  if (setup_fixed(c, hip_device) != PCBZ_OK) c->fixed_err = c->err;
  const char *tp = getenv("PCBZ_TUNE_CACHE");
  if (tp) c->tune_path = tp;
  const char *ri = getenv("PCBZ_RADIX_ITEMS");  // radix tile of eager calls: 8 or 16
  if (ri && (atoi(ri) == 8 || atoi(ri) == 16)) c->eager_items = atoi(ri);
  const char *tr = getenv("PCBZ_TUNE_ROUNDS");  // fixed round budget for tuned graphs (1..40)
  if (tr && atoi(tr) >= 1 && atoi(tr) <= 40) c->tune_rounds = atoi(tr);
  load_tuning(c);
  *out = c;
  return PCBZ_OK;
}

void pcbz_destroy(pcbz_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->arena) (void)hipFree(c->arena);
  if (c->d_tq) (void)hipFree(c->d_tq);
  if (c->d_xpow2) (void)hipFree(c->d_xpow2);
  if (c->d_xbyte) (void)hipFree(c->d_xbyte);
  if (c->d_xchunk) (void)hipFree(c->d_xchunk);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->h_small) (void)hipHostFree(c->h_small);
  if (c->h_dec) (void)hipHostFree(c->h_dec);
  for (pcbz::GraphEntry &g : c->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->fev)
    if (e) (void)hipEventDestroy(e);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
}

const char *pcbz_last_error(const pcbz_ctx *c) { return c ? c->err.c_str() : "null context"; }

int pcbz_plan(const pcbz_params *prm, uint32_t *n_bands, size_t *compress_bound) {
  int st = check_params(prm);
  if (st) return st;
  uint32_t R, nb;
  plan_rows(prm, &R, &nb);
  if (n_bands) *n_bands = nb;
  if (compress_bound) {
    const uint32_t lim = 100000u * prm->level - 19u;
    const uint64_t raw = 2ull * prm->h * prm->w;
    const uint64_t band_max = 2ull * R * prm->pitch * prm->w;
    const uint64_t slots_per_band = (band_max + band_max / 4 + 8 + (lim - 4) - 1) / (lim - 4) + 1;
    const uint64_t rle = raw + raw / 4 + 8ull * nb;
    *compress_bound = (size_t)(20 + 5ull * nb + rle * 9 / 8 + 64 + nb * slots_per_band * 20600ull);
  }
  return PCBZ_OK;
}

int pcbz_judge(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
               uint8_t *d_choice, double *d_entropy, int64_t *d_score, void *stream) {
  if (!ctx || !prm || !d_frame || !d_choice) return fail(ctx, PCBZ_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<FrameIn> fin(1);
  fin[0] = FrameIn{*prm, d_frame, d_prev, nullptr, nullptr, 0};
  Plan P;
  int st = build_plan(ctx, fin, true, P);
  if (st) return st;
  Work w{};
  Arena meas{nullptr};
  size_t need = layout(meas, P, false, w);
  if ((st = ensure_arena(ctx, need))) return st;
  if ((st = ensure_tables(ctx, P.band_n_max))) return st;
  Arena A{ctx->arena};
  layout(A, P, false, w);
  std::vector<UploadItem> items;
  if ((st = stage_plan(ctx, P, w, s, items))) return st;
  if ((st = enqueue_upload(ctx, items, s))) return st;
  ZeroSpans z;
  z.add(w.hist, P.tasks.size() * 65536);
  z.add(w.score, P.tasks.size() * 2);
  zero_spans(z, s);
  enqueue_judge(ctx->d_tq, P, w, s);
  launch_choose2(w.bands, (uint32_t)P.bands.size(), w.task_of, w.score, w.tasks, nullptr, d_choice, d_entropy,
                 d_score, s);
  trace_stage(nullptr);
  HIPCHK(ctx, hipGetLastError());
  return PCBZ_OK;
}

int pcbz_judge_noalloc(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
                       uint8_t *d_choice, double *d_entropy, int64_t *d_score, void *stream) {
  if (!ctx || !prm || !d_frame || !d_choice) return fail(ctx, PCBZ_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int dev = ctx->device;
  if (!ctx->fixed_err.empty()) return fail(ctx, PCBZ_EDEVICE, "fixed workspace unavailable: %s", ctx->fixed_err.c_str());
  uint8_t *const base = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
  const int64_t *const tq = (dev >= 0 && dev < kMaxDevices) ? g_tq_fixed_ptr[dev] : nullptr;
  if (!base || !tq) return fail(ctx, PCBZ_EDEVICE, "fixed workspace of device %d not set up", dev);
  std::vector<FrameIn> fin(1);
  fin[0] = FrameIn{*prm, d_frame, d_prev, nullptr, nullptr, 0};
  Plan P;
  int st = build_plan(ctx, fin, true, P);
  if (st) return st;
  if ((size_t)P.band_n_max + 2 > kTqFixed)
    return fail(ctx, PCBZ_EINVAL, "band of %u bytes exceeds the fixed Tq table (%zu entries)", P.band_n_max, kTqFixed);
  Work w{};
  Arena meas{nullptr};
  const size_t need = layout(meas, P, false, w);
  if (need > kScratchBytes)
    return fail(ctx, PCBZ_ENOMEM, "pcbz_judge_noalloc needs %zu bytes of workspace; its fixed workspace holds %zu",
                need, kScratchBytes);
  Arena A{base};
  layout(A, P, false, w);
  // plan tables from pageable host memory, in stream order after earlier work
  // on `stream` (which may still read the workspace); the stream is
  // synchronised before the host buffer goes away
  auto put = [&](const void *src, size_t bytes, void *dst) -> int {
    if (!bytes || !dst) return PCBZ_OK;
    HIPCHK(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return PCBZ_OK;
  };
  if ((st = put(P.bands.data(), P.bands.size() * sizeof(BandDesc), w.bands)) ||
      (st = put(P.rows.data(), P.rows.size() * sizeof(RowItem), w.rows)) ||
      (st = put(P.tasks.data(), P.tasks.size() * sizeof(JudgeTask), w.tasks)) ||
      (st = put(P.tile_task.data(), P.tile_task.size() * sizeof(uint32_t), w.tile_task)) ||
      (st = put(P.tile_local.data(), P.tile_local.size() * sizeof(uint32_t), w.tile_local)) ||
      (st = put(P.task_of.data(), P.task_of.size() * sizeof(int32_t), w.task_of)) ||
      (st = put(P.band_start.data(), P.band_start.size() * sizeof(uint32_t), w.band_start)) ||
      (st = put(P.frames.data(), P.frames.size() * sizeof(FrameOut), w.frames)))
    return st;
  HIPCHK(ctx, hipStreamSynchronize(s));
  ZeroSpans z;  // the workspace keeps the previous call's contents
  z.add(w.hist, P.tasks.size() * 65536);
  z.add(w.score, P.tasks.size() * 2);
  zero_spans(z, s);
  enqueue_judge(tq, P, w, s);
  launch_choose2(w.bands, (uint32_t)P.bands.size(), w.task_of, w.score, w.tasks, nullptr, d_choice, d_entropy,
                 d_score, s);
  trace_stage(nullptr);
  HIPCHK(ctx, hipGetLastError());
  return PCBZ_OK;
}

int pcbz_compress(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
                  const uint8_t *d_forced_choice, uint8_t *d_out, size_t out_cap, size_t *out_len,
                  uint8_t *d_choice_out, void *stream) {
  if (!ctx || !prm || !d_frame || !d_out || !out_len) return fail(ctx, PCBZ_EINVAL, "null argument");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<FrameIn> fin(1);
  fin[0] = FrameIn{*prm, d_frame, d_prev, d_forced_choice, d_out, out_cap};
  const hipStream_t s = (hipStream_t)stream;
  std::vector<size_t> lens;
  // a shape seen before runs the schedule its last read-back call needed
  // (one round spare) and syncs once, for the results
  const bool sched = ctx->use_fixed && !getenv("PCBZ_NO_FIXED");
  const std::string key = sched ? shape_key(ctx, fin) : std::string();
  TuneRec *rec = nullptr;
  for (TuneRec &r : ctx->fixed)
    if (sched && r.key == key) rec = &r;
  int st;
  if (rec) {
    Tuning tu;
    tu.radix_items = ctx->eager_items;
    tu.rounds = rec->rounds;
    tu.seg_mask = rec->seg_mask;
    st = run_compress(ctx, fin, s, lens, {d_choice_out}, &tu);
    if (st != kRedo) {
      if (!lens.empty()) *out_len = lens[0];
      return st;
    }
  }
  st = run_compress(ctx, fin, s, lens, {d_choice_out});
  if (!lens.empty()) *out_len = lens[0];
  if (st || !sched) return st;
  if (rec) {  // the data needed more: widen the shape's schedule
    rec->rounds = std::max(rec->rounds, (int)ctx->last_rounds + 1);
    rec->seg_mask &= seg_schedule(ctx);
  } else {
    if (ctx->fixed.size() >= 64) ctx->fixed.erase(ctx->fixed.begin());
    TuneRec r;
    r.key = key;
    r.items = ctx->eager_items;
    r.rounds = (int)ctx->last_rounds + 1;
    r.seg_mask = seg_schedule(ctx);
    ctx->fixed.push_back(r);
  }
  return st;
}

int pcbz_compress_batch(pcbz_ctx *ctx, uint32_t n, const pcbz_params *prm, const uint16_t *const *d_frames,
                        const uint16_t *const *d_prevs, const uint8_t *const *d_forced, const pcbz_selector *sel,
                        float min_conf, uint8_t *const *d_outs, const size_t *caps, size_t *lens, void *stream) {
  if (!ctx || !prm || !d_frames || !d_outs || !caps || !lens) return fail(ctx, PCBZ_EINVAL, "null argument");
  if (sel && !(min_conf >= 0.f)) return fail(ctx, PCBZ_EINVAL, "min_conf must be >= 0");
  if (n == 0) return PCBZ_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<FrameIn> fin(n);
  for (uint32_t i = 0; i < n; i++)
    fin[i] = FrameIn{prm[i], d_frames[i], d_prevs ? d_prevs[i] : nullptr, d_forced ? d_forced[i] : nullptr, d_outs[i],
                     caps[i]};
  // the call's selector replaces the context's (pcbz_set_selector) for its duration
  pcbz_selector *const ctx_sel = ctx->sel;
  const float ctx_conf = ctx->min_conf;
  ctx->sel = const_cast<pcbz_selector *>(sel);
  ctx->min_conf = sel ? min_conf : 1.f;
  std::vector<size_t> out;
  int st = (!ctx->use_graphs || getenv("PCBZ_NO_GRAPH")) ? run_compress(ctx, fin, (hipStream_t)stream, out, {})
                                                       : run_compress_graph(ctx, fin, (hipStream_t)stream, out);
  ctx->sel = ctx_sel;
  ctx->min_conf = ctx_conf;
  for (uint32_t i = 0; i < n && i < out.size(); i++) lens[i] = out[i];
  return st;
}

int pcbz_peek(const uint8_t *in, size_t in_len, pcbz_params *out, uint32_t *n_bands) {
  if (!in || !out) return PCBZ_EINVAL;
  return peek_container(in, in_len, out, n_bands, nullptr, nullptr);
}

int pcbz_decompress(pcbz_ctx *ctx, const uint8_t *d_in, size_t in_len, const uint16_t *d_prev, uint16_t *d_out,
                    size_t out_elems, void *stream) {
  return pcbz_decompress_batch(ctx, 1, &d_in, &in_len, &d_prev, &d_out, &out_elems, stream);
}

int pcbz_decompress_batch(pcbz_ctx *ctx, uint32_t n, const uint8_t *const *d_ins, const size_t *in_lens,
                          const uint16_t *const *d_prevs, uint16_t *const *d_outs, const size_t *out_elems,
                          void *stream) {
  if (!ctx || !d_ins || !in_lens || !d_outs || !out_elems) return fail(ctx, PCBZ_EINVAL, "null argument");
  if (n == 0) return PCBZ_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  std::vector<DecIn> in(n);
  for (uint32_t i = 0; i < n; i++) {
    if (!d_ins[i] || !d_outs[i]) return fail(ctx, PCBZ_EINVAL, "container %u: null pointer", i);
    in[i] = DecIn{d_ins[i], in_lens[i], d_prevs ? d_prevs[i] : nullptr, d_outs[i], out_elems[i]};
  }
  return run_decompress(ctx, in, (hipStream_t)stream);
}

int pcbz_decompress_inspect(const pcbz_ctx *ctx, int which, void *host, size_t bytes) {
  if (!ctx || !host) return PCBZ_EINVAL;
  if (!ctx->last_dec_valid) return PCBZ_EINVAL;
  const DecWork &w = ctx->last_dec;
  const void *src = nullptr;
  size_t size = 0;
  switch (which) {
    case 0: src = w.slots; size = (size_t)w.n_slots * sizeof(DecSlot); break;
    case 1: src = w.sym; size = (size_t)w.sym_total * 2; break;
    case 2: src = w.L; size = w.n_max; break;
    case 3: src = w.T; size = w.n_max; break;
    case 4: src = w.raw; size = w.raw_total; break;
    case 5: src = w.ctr; size = kDcWords * 4; break;
    default: return PCBZ_EINVAL;
  }
  if (bytes > size) return PCBZ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return PCBZ_EDEVICE;
  if (hipMemcpy(host, src, bytes, hipMemcpyDeviceToHost) != hipSuccess) return PCBZ_EDEVICE;
  return PCBZ_OK;
}

int pcbz_trace_enable(pcbz_ctx *c, int on, const char *filter) {
  if (!c) return PCBZ_EINVAL;
  pcbz::g_tracer.collect();
  pcbz::g_tracer.filter = filter ? filter : "";
  pcbz::g_trace_on = on != 0;
  return PCBZ_OK;
}

int pcbz_trace_read(pcbz_ctx *c, char *names, size_t name_stride, double *ms, uint64_t *calls, uint64_t *bytes,
                    uint32_t max, uint32_t *n, int reset) {
  if (!c || !n) return PCBZ_EINVAL;
  HIPCHK(c, hipSetDevice(c->device));
  pcbz::g_tracer.collect();
  const uint32_t k = (uint32_t)std::min<size_t>(max, pcbz::g_tracer.names.size());
  for (uint32_t i = 0; i < k; i++) {
    if (names && name_stride) {
      strncpy(names + i * name_stride, pcbz::g_tracer.names[i].c_str(), name_stride - 1);
      names[i * name_stride + name_stride - 1] = 0;
    }
    if (ms) ms[i] = pcbz::g_tracer.ms[i];
    if (calls) calls[i] = pcbz::g_tracer.calls[i];
    if (bytes) bytes[i] = pcbz::g_tracer.bytes[i];
  }
  *n = (uint32_t)pcbz::g_tracer.names.size();
  if (reset) {
    pcbz::g_tracer.names.clear();
    pcbz::g_tracer.ms.clear();
    pcbz::g_tracer.calls.clear();
    pcbz::g_tracer.bytes.clear();
  }
  return PCBZ_OK;
}

int pcbz_set_selector(pcbz_ctx *ctx, pcbz_selector *sel, float min_conf) {
  if (!ctx) return PCBZ_EINVAL;
  if (!(min_conf >= 0.f)) return fail(ctx, PCBZ_EINVAL, "min_conf must be >= 0");
  ctx->sel = sel;
  ctx->min_conf = min_conf;
  return PCBZ_OK;
}

int pcbz_set_graphs(pcbz_ctx *ctx, int on) {
  if (!ctx) return PCBZ_EINVAL;
  if (on < 0 || on > 2) return fail(ctx, PCBZ_EINVAL, "graph mode must be 0, 1 or 2");
  ctx->use_graphs = on;
  return PCBZ_OK;
}

int pcbz_selector_stats(const pcbz_ctx *ctx, uint32_t *n_bands, uint32_t *n_judged) {
  if (!ctx) return PCBZ_EINVAL;
  if (n_bands) *n_bands = ctx->last_sel_bands;
  if (n_judged) *n_judged = ctx->last_sel_fallback;
  return PCBZ_OK;
}

int pcbz_features(pcbz_ctx *ctx, const pcbz_params *prm, const uint16_t *d_frame, const uint16_t *d_prev,
                  float *d_feat, void *stream) {
  if (!ctx || !prm || !d_frame || !d_feat) return fail(ctx, PCBZ_EINVAL, "null argument");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  int st = check_params(prm);
  if (st) return fail(ctx, st, "invalid parameters");
  uint32_t R, nb;
  plan_rows(prm, &R, &nb);
  std::vector<BandDesc> bands(nb);
  const uint32_t ns = prm->h / prm->pitch;
  for (uint32_t k = 0; k < nb; k++) {
    BandDesc B{};
    B.frame = d_frame;
    B.prev = d_prev;
    B.W = prm->w;
    B.pitch = prm->pitch;
    B.Nt = prm->w / prm->pitch;
    B.Rb = std::min(R, ns - k * R);
    B.y0 = k * R * prm->pitch;
    B.band_in_frame = k;
    B.cand_mask = prm->cand_mask;
    B.level = prm->level;
    B.n = 2u * B.Rb * prm->pitch * prm->w;
    bands[k] = B;
  }
  if ((st = ensure_arena(ctx, nb * sizeof(BandDesc) + 256))) return st;
  HIPCHK(ctx, hipStreamSynchronize(s));
  HIPCHK(ctx, hipMemcpy(ctx->arena, bands.data(), nb * sizeof(BandDesc), hipMemcpyHostToDevice));
  launch_features((const BandDesc *)ctx->arena, nb, d_feat, s);
  HIPCHK(ctx, hipStreamSynchronize(s));
  HIPCHK(ctx, hipGetLastError());
  return PCBZ_OK;
}

int pcbz_last_stats(const pcbz_ctx *c, uint64_t *raw_bytes, uint64_t *rle_bytes, uint32_t *n_blocks,
                    uint32_t *bwt_rounds) {
  if (!c) return PCBZ_EINVAL;
  if (raw_bytes) *raw_bytes = c->last_raw;
  if (rle_bytes) *rle_bytes = c->last_rle;
  if (n_blocks) *n_blocks = c->last_blocks;
  if (bwt_rounds) *bwt_rounds = c->last_rounds;
  return PCBZ_OK;
}

}  // extern "C"
