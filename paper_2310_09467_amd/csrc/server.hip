// server.hip -- serving loop: frames from many cameras arrive over time, are
// admitted under an HBM budget, batched continuously and compressed by
// several worker contexts whose batches overlap on the device.
//
// Life of a frame: pcbz_server_submit queues it (host memory owned by the
// caller) -> admission allocates its device frame and output blocks from the
// server's pool when the pool has room (first in, first out) and starts the
// upload on the upload stream -> a free worker takes every admitted frame up
// to its batch limit and compresses them with one pcbz_compress_batch call
// on its own stream and context (while other workers run theirs) -> the
// containers are copied back to host memory, the device blocks return to the
// pool and the result waits for pcbz_server_poll.
//
// Temporal candidate: the device copy of each camera's last frame of a given
// shape stays resident (it is camera state, counted in the pool) and is the
// previous frame of that camera's next frame of the same shape.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "pcbz.h"
#include "pcbz_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device region (256-byte granules); adjacent
// free ranges merge on release.
class DevicePool {
 public:
  ~DevicePool() {
    if (base_) (void)hipFree(base_);
  }
  int init(size_t bytes) {
    bytes = bytes / 256 * 256;
    if (hipMalloc((void **)&base_, bytes) != hipSuccess) {
      (void)hipGetLastError();
      base_ = nullptr;
      return PCBZ_ENOMEM;
    }
    size_ = bytes;
    free_[0] = bytes;
    return PCBZ_OK;
  }
  uint8_t *alloc(size_t n) {
    n = (n + 255) / 256 * 256;
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used_ += n;
      peak_ = std::max(peak_, used_);
      return base_ + off;
    }
    return nullptr;
  }
  void release(uint8_t *p, size_t n) {
    if (!p) return;
    n = (n + 255) / 256 * 256;
    std::lock_guard<std::mutex> lk(mu_);
    size_t off = (size_t)(p - base_);
    used_ -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  uint8_t *base_ = nullptr;
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
  std::mutex mu_;
};

// A device block that returns to the pool when the last reference goes.
struct DevBlock {
  DevicePool *pool;
  uint8_t *p;
  size_t n;
  DevBlock(DevicePool *pl, uint8_t *q, size_t m) : pool(pl), p(q), n(m) {}
  ~DevBlock() { pool->release(p, n); }
};

struct Job {
  uint64_t tag = 0;
  uint32_t camera = 0;
  pcbz_params prm{};
  const uint16_t *host = nullptr;
  double t_submit = 0.0, t_done = 0.0;
  size_t raw = 0, cap = 0;
  std::shared_ptr<DevBlock> frame, out;
  std::shared_ptr<Job> prev_job;        // the camera's previous frame of this shape (until admission)
  std::shared_ptr<DevBlock> prev;       // its device copy (from admission until completion)
  uint64_t prev_tag = UINT64_MAX;
  hipEvent_t uploaded = nullptr;
  int status = PCBZ_OK;
  bool finished = false;
  uint32_t prev_refs = 0;  // later jobs naming this one as their previous frame, not yet admitted
  std::vector<uint8_t> bytes;
};

struct BatchLog {
  double t0, t1;
  uint32_t frames;
  uint64_t raw;
  int worker;
};

}  // namespace

struct pcbz_server {
  int device = 0;
  DevicePool pool;
  hipStream_t upload = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Job>> pending, admitted;
  std::vector<std::shared_ptr<Job>> done, returned;
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::shared_ptr<Job>> last;  // (camera, h, w)
  std::vector<std::thread> workers;
  std::vector<pcbz_ctx *> ctxs;
  std::vector<pcbz_selector *> sels;
  size_t max_batch_bytes = 0;
  uint32_t max_batch_frames = 64;
  float min_conf = 1.f;
  bool stop = false;
  uint32_t in_flight = 0;  // frames inside worker calls
  uint64_t submitted = 0, completed = 0, batches = 0, batched_frames = 0;
  std::vector<BatchLog> log;
  std::string err;
};

namespace {

bool is_state(pcbz_server *s, const Job &j) {
  auto it = s->last.find(std::make_tuple(j.camera, j.prm.h, j.prm.w));
  return it != s->last.end() && it->second.get() == &j;
}

// A finished job's device frame goes back to the pool once it is neither its
// camera's state nor awaited as a previous frame.  Caller holds s->mu.
void maybe_drop_frame(pcbz_server *s, Job &j) {
  if (j.finished && j.prev_refs == 0 && !is_state(s, j)) j.frame.reset();
}

// Moves pending jobs to the admitted queue while the pool has room (FIFO;
// the head blocks the queue).  Caller holds s->mu.
void admit(pcbz_server *s) {
  bool any = false;
  while (!s->pending.empty()) {
    std::shared_ptr<Job> &j = s->pending.front();
    const size_t fb = j->raw;
    uint8_t *pf = s->pool.alloc(fb);
    if (!pf) break;
    uint8_t *po = s->pool.alloc(j->cap);
    if (!po) {
      s->pool.release(pf, fb);
      break;
    }
    j->frame = std::make_shared<DevBlock>(&s->pool, pf, fb);
    j->out = std::make_shared<DevBlock>(&s->pool, po, j->cap);
    if (j->prev_job) {
      // admitted earlier (FIFO) and kept since (prev_refs), so its block exists
      Job &pj = *j->prev_job;
      j->prev = pj.frame;
      j->prev_tag = pj.tag;
      pj.prev_refs--;
      maybe_drop_frame(s, pj);
      j->prev_job.reset();
    }
    (void)hipEventCreateWithFlags(&j->uploaded, hipEventDisableTiming);
    if (hipMemcpyAsync(pf, j->host, fb, hipMemcpyHostToDevice, s->upload) != hipSuccess ||
        hipEventRecord(j->uploaded, s->upload) != hipSuccess) {
      j->status = PCBZ_EDEVICE;
    }
    s->admitted.push_back(j);
    s->pending.pop_front();
    any = true;
  }
  if (any) s->cv_work.notify_all();
}

void finish(pcbz_server *s, std::vector<std::shared_ptr<Job>> &jobs) {
  const double t = now_ms();
  std::lock_guard<std::mutex> lk(s->mu);
  for (auto &j : jobs) {
    j->t_done = t;
    if (j->uploaded) (void)hipEventDestroy(j->uploaded);
    j->uploaded = nullptr;
    j->out.reset();
    j->prev.reset();
    j->finished = true;
    maybe_drop_frame(s, *j);
    s->done.push_back(j);
    s->completed++;
  }
  s->in_flight -= (uint32_t)jobs.size();
  admit(s);
  s->cv_done.notify_all();
}

void worker_main(pcbz_server *s, int wi) {
  (void)hipSetDevice(s->device);
  pcbz_ctx *ctx = s->ctxs[wi];
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  uint8_t *h_buf = nullptr;
  size_t h_cap = 0;
  for (;;) {
    std::vector<std::shared_ptr<Job>> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->admitted.empty(); });
      if (s->admitted.empty() && s->stop) break;
      size_t bytes = 0;
      while (!s->admitted.empty() && batch.size() < s->max_batch_frames) {
        const size_t r = s->admitted.front()->raw;
        if (!batch.empty() && bytes + r > s->max_batch_bytes) break;
        bytes += r;
        batch.push_back(s->admitted.front());
        s->admitted.pop_front();
      }
      s->in_flight += (uint32_t)batch.size();
    }
    const double t0 = now_ms();
    // frames whose upload failed keep their status and stay out of the call
    std::vector<std::shared_ptr<Job>> failed;
    {
      std::vector<std::shared_ptr<Job>> ok;
      for (auto &j : batch) (j->status == PCBZ_OK ? ok : failed).push_back(j);
      if (!failed.empty()) {
        finish(s, failed);
        batch.swap(ok);
      }
    }
    // run what is admitted; on a workspace shortfall, split the batch; when a
    // call of several frames fails otherwise, run them one by one so that
    // each frame gets its own status
    size_t k0 = 0;
    bool singly = false;
    while (k0 < batch.size()) {
      size_t k1 = singly ? k0 + 1 : batch.size();
      int rc = PCBZ_OK;
      for (;;) {
        const uint32_t n = (uint32_t)(k1 - k0);
        std::vector<pcbz_params> prm(n);
        std::vector<const uint16_t *> fr(n), pv(n);
        std::vector<uint8_t *> outs(n);
        std::vector<size_t> caps(n), lens(n, 0);
        for (uint32_t i = 0; i < n; i++) {
          Job &j = *batch[k0 + i];
          if (j.uploaded) (void)hipStreamWaitEvent(st, j.uploaded, 0);
          prm[i] = j.prm;
          if (!j.prev) prm[i].cand_mask &= ~0x8u;
          fr[i] = (const uint16_t *)j.frame->p;
          pv[i] = j.prev ? (const uint16_t *)j.prev->p : nullptr;
          outs[i] = j.out->p;
          caps[i] = j.cap;
        }
        rc = pcbz_compress_batch(ctx, n, prm.data(), fr.data(), pv.data(), nullptr,
                                 s->sels.empty() ? nullptr : s->sels[wi], s->min_conf, outs.data(), caps.data(),
                                 lens.data(), st);
        if (rc == PCBZ_ENOMEM && n > 1) {
          k1 = k0 + n / 2;
          continue;
        }
        if (rc != PCBZ_OK && n > 1) {
          singly = true;
          k1 = k0 + 1;
          continue;
        }
        size_t tot = 0;
        for (uint32_t i = 0; i < n; i++) tot += rc == PCBZ_OK ? lens[i] : 0;
        if (rc == PCBZ_OK && tot > h_cap) {
          if (h_buf) (void)hipHostFree(h_buf);
          h_cap = tot * 2;
          if (hipHostMalloc((void **)&h_buf, h_cap, hipHostMallocDefault) != hipSuccess) {
            h_buf = nullptr;
            h_cap = 0;
            rc = PCBZ_ENOMEM;
          }
        }
        size_t off = 0;
        for (uint32_t i = 0; i < n && rc == PCBZ_OK; i++) {
          if (hipMemcpyAsync(h_buf + off, outs[i], lens[i], hipMemcpyDeviceToHost, st) != hipSuccess)
            rc = PCBZ_EDEVICE;
          off += lens[i];
        }
        if (rc == PCBZ_OK && hipStreamSynchronize(st) != hipSuccess) rc = PCBZ_EDEVICE;
        off = 0;
        for (uint32_t i = 0; i < n; i++) {
          Job &j = *batch[k0 + i];
          j.status = rc;
          if (rc == PCBZ_OK) j.bytes.assign(h_buf + off, h_buf + off + lens[i]);
          off += lens[i];
        }
        break;
      }
      std::vector<std::shared_ptr<Job>> part(batch.begin() + k0, batch.begin() + k1);
      finish(s, part);
      k0 = k1;
    }
    const double t1 = now_ms();
    if (batch.empty()) continue;
    std::lock_guard<std::mutex> lk(s->mu);
    uint64_t raw = 0;
    for (auto &j : batch) raw += j->raw;
    s->log.push_back(BatchLog{t0, t1, (uint32_t)batch.size(), raw, wi});
    s->batches++;
    s->batched_frames += batch.size();
  }
  if (h_buf) (void)hipHostFree(h_buf);
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

int pcbz_server_create(int hip_device, size_t hbm_budget, uint32_t n_workers, size_t max_batch_bytes,
                       const pcbz_selector *sel, float min_conf, pcbz_server **out) {
  if (!out || n_workers == 0 || n_workers > 8 || hbm_budget < (64u << 20)) return PCBZ_EINVAL;
  *out = nullptr;
  if (hipSetDevice(hip_device) != hipSuccess) return PCBZ_EDEVICE;
  pcbz_server *s = new pcbz_server();
  s->device = hip_device;
  s->min_conf = min_conf;
  // an eighth of the budget holds frames, outputs and camera state (about
  // 2.3 bytes per input byte); the rest is split between the workers'
  // workspaces (about 100 bytes per input byte of a batch)
  if (sel && !(min_conf >= 0.f)) return PCBZ_EINVAL;
  const size_t pool = hbm_budget / 8;
  const size_t per_ws = (hbm_budget - pool) / n_workers;
  s->max_batch_bytes = max_batch_bytes ? max_batch_bytes : per_ws / 128;
  int rc = s->pool.init(pool);
  if (rc) {
    delete s;
    return rc;
  }
  if (hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return PCBZ_EDEVICE;
  }
  std::vector<float> params;
  float norm[8];
  if (sel) {
    params.resize(pcbz_selector_num_params());
    if ((rc = pcbz_selector_get_params(sel, params.data(), norm))) {
      pcbz_server_destroy(s);
      return rc;
    }
  }
  for (uint32_t w = 0; w < n_workers; w++) {
    pcbz_ctx *c = nullptr;
    if ((rc = pcbz_create(&c, hip_device, per_ws))) {
      pcbz_server_destroy(s);
      return rc;
    }
    pcbz_set_graphs(c, 0);  // batch shapes vary from call to call
    s->ctxs.push_back(c);
    if (sel) {
      // each worker has its own copy: a selector serves one call at a time
      pcbz_selector *ws = nullptr;
      if ((rc = pcbz_selector_create(c, params.data(), norm, &ws))) {
        pcbz_server_destroy(s);
        return rc;
      }
      s->sels.push_back(ws);
    }
  }
  for (uint32_t w = 0; w < n_workers; w++) s->workers.emplace_back(worker_main, s, (int)w);
  *out = s;
  return PCBZ_OK;
}

int pcbz_server_submit(pcbz_server *s, const pcbz_params *prm, const uint16_t *host_frame, uint32_t camera,
                       uint64_t tag) {
  if (!s || !prm || !host_frame) return PCBZ_EINVAL;
  uint32_t nb = 0;
  size_t bound = 0;
  int rc = pcbz_plan(prm, &nb, &bound);
  if (rc) return rc;
  auto j = std::make_shared<Job>();
  j->tag = tag;
  j->camera = camera;
  j->prm = *prm;
  j->host = host_frame;
  j->raw = 2ull * prm->h * prm->w;
  j->cap = bound;
  j->t_submit = now_ms();
  if (j->raw + j->cap > s->pool.size()) return PCBZ_ENOMEM;
  std::lock_guard<std::mutex> lk(s->mu);
  auto key = std::make_tuple(camera, prm->h, prm->w);
  std::shared_ptr<Job> old;
  auto it = s->last.find(key);
  if (it != s->last.end()) old = it->second;
  // the first frame of a camera and shape has no previous frame: it is coded
  // without the temporal candidate, so it needs another one
  if (!old && (prm->cand_mask & ~8u) == 0) return PCBZ_ENEEDPREV;
  if ((prm->cand_mask & 8u) && old) {
    j->prev_job = old;
    old->prev_refs++;
  }
  s->last[key] = j;
  if (old) maybe_drop_frame(s, *old);
  s->pending.push_back(j);
  s->submitted++;
  admit(s);
  return PCBZ_OK;
}

int pcbz_server_poll(pcbz_server *s, pcbz_server_result *res, uint32_t max, uint32_t *n, int timeout_ms) {
  if (!s || !n || (max && !res)) return PCBZ_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->returned.clear();  // the previous poll's byte buffers
  if (s->done.empty() && timeout_ms != 0) {
    auto pred = [&] { return !s->done.empty(); };
    if (timeout_ms < 0)
      s->cv_done.wait(lk, pred);
    else
      s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  }
  const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size());
  for (uint32_t i = 0; i < k; i++) {
    const Job &j = *s->done[i];
    pcbz_server_result &r = res[i];
    r.tag = j.tag;
    r.prev_tag = j.prev_tag;
    r.camera = j.camera;
    r.status = j.status;
    r.data = j.bytes.data();
    r.len = j.bytes.size();
    r.latency_ms = j.t_done - j.t_submit;
    r.submit_ms = j.t_submit;
  }
  s->returned.assign(s->done.begin(), s->done.begin() + k);
  s->done.erase(s->done.begin(), s->done.begin() + k);
  *n = k;
  return PCBZ_OK;
}

int pcbz_server_stats(const pcbz_server *cs, pcbz_server_info *st) {
  if (!cs || !st) return PCBZ_EINVAL;
  pcbz_server *s = const_cast<pcbz_server *>(cs);
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof *st);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->pending = s->pending.size();
  st->admitted = s->admitted.size();
  st->in_flight = s->in_flight;
  st->batches = s->batches;
  st->batched_frames = s->batched_frames;
  st->pool_bytes = s->pool.size();
  st->pool_used = s->pool.used();
  st->pool_peak = s->pool.peak();
  // time with two or more batches on the device at once (from the batch log)
  std::vector<std::pair<double, int>> ev;
  for (const BatchLog &b : s->log) {
    ev.push_back({b.t0, +1});
    ev.push_back({b.t1, -1});
  }
  std::sort(ev.begin(), ev.end());
  int depth = 0;
  double last = 0.0, busy = 0.0, overlap = 0.0;
  for (auto &e : ev) {
    if (depth >= 1) busy += e.first - last;
    if (depth >= 2) overlap += e.first - last;
    depth += e.second;
    last = e.first;
  }
  st->busy_ms = busy;
  st->overlap_ms = overlap;
  return PCBZ_OK;
}

void pcbz_server_destroy(pcbz_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->pending.clear();  // never admitted: nothing on the device
  }
  s->cv_work.notify_all();
  for (std::thread &t : s->workers) t.join();
  (void)hipSetDevice(s->device);
  if (s->upload) {
    (void)hipStreamSynchronize(s->upload);
    (void)hipStreamDestroy(s->upload);
  }
  for (pcbz_selector *w : s->sels) pcbz_selector_free(w);
  for (pcbz_ctx *c : s->ctxs) pcbz_destroy(c);
  s->done.clear();
  s->returned.clear();
  s->last.clear();
  delete s;
}

}  // extern "C"
