// Serving loop: continuous batching of propagator solves on one GPU.
//
// Host-side scheduler.  Gauge fields live permanently in the caller's arena;
// every admitted request borrows a contiguous piece of the arena for its
// workspace and its source/solution staging, runs lqcd_solve on its worker's
// stream, and returns the piece.  Admission is first-fit over the queue in
// arrival order; a head request that does not fit may be passed by later
// ones at most kMaxBypass times in a row.  All bookkeeping is host memory; the
// device memory is the caller's arena.  In simulation mode (no arena) no HIP
// call is made at all.
//
// Gauge fields are imported, and kernels autotuned (lqcd_server_warmup), on a
// private stream while no request is queued or running: the arena space that
// queued requests were admitted against never shrinks, and a tuning is never
// timed on a GPU shared with requests.  A request reads the process-wide
// tuning cache for its lattice, precision and rhs count and never tunes.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "lqcd_internal.h"

using namespace lqcd;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxBypass = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct GaugeEntry {
  lqcd_geom_t* geom = nullptr;
  lqcd_gauge_t* gauge = nullptr;
  size_t off = 0, bytes = 0;
  int pmask = 0;
};

struct Request {
  uint64_t ticket;
  int gauge_id;
  lqcd_solve_params p;
  const void* eta;
  void* psi;
  size_t bytes;
  size_t off = 0;
  int status = LQCD_PENDING;
  std::vector<lqcd_solve_info> info;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int bypassed = 0;
  bool finished = false;  // set under the server lock once status/info are final
};

int request_pmask(const lqcd_solve_params* p) {
  return LQCD_PM_F64 | (p->inner_prec == LQCD_F32 ? LQCD_PM_F32 : 0) |
         (p->inner_prec == LQCD_BF16 ? LQCD_PM_BF16 : 0);
}

}  // namespace

struct lqcd_server {
  char* arena = nullptr;
  bool sim = false;
  double sim_seconds = 0.0;
  int max_streams = 1, queue_cap = 1;
  std::mutex mu;
  std::condition_variable cv;
  Arena alloc;
  size_t gauge_bytes_total = 0;
  std::vector<GaugeEntry> gauges;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> tickets;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  hipStream_t import_stream = nullptr;  // gauge import and warm-up tuning
  int running = 0;                      // requests admitted and not finished
  bool exclusive = false;               // gauge import or warm-up in progress: admit nothing
  bool stopping = false;
  bool stopped = false;
  uint64_t next_ticket = 1;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker(int idx);
  Request* pick_locked();
  void run(Request* r, const GaugeEntry& g, int idx);
};

static size_t footprint(const lqcd_server* s, const GaugeEntry& g, const lqcd_solve_params* p) {
  const size_t canon = (size_t)p->nrhs * (size_t)lqcd_geom_volume(g.geom) * 12 * 16;
  return align_up(lqcd_ws_bytes(g.geom, request_pmask(p), p->nrhs)) + 2 * align_up(canon);
}

Request* lqcd_server::pick_locked() {
  if (exclusive) return nullptr;
  for (size_t i = 0; i < queue.size(); ++i) {
    Request* q = queue[i];
    size_t off;
    if (alloc.alloc(q->bytes, &off)) {
      q->off = off;
      if (i > 0) queue.front()->bypassed++;
      queue.erase(queue.begin() + i);
      return q;
    }
    if (i == 0 && q->bypassed >= kMaxBypass) break;  // keep the space for the head
  }
  return nullptr;
}

void lqcd_server::run(Request* r, const GaugeEntry& g, int idx) {
  r->info.assign(r->p.nrhs, lqcd_solve_info{});
  if (sim) {
    std::this_thread::sleep_for(std::chrono::duration<double>(sim_seconds));
    for (auto& i : r->info) i.status = LQCD_OK;
    r->status = LQCD_OK;
    return;
  }
  hipStream_t st = streams[idx];
  (void)hipSetDevice(0);
  const int pm = request_pmask(&r->p);
  const size_t ws_bytes = lqcd_ws_bytes(g.geom, pm, r->p.nrhs);
  const size_t canon = (size_t)r->p.nrhs * (size_t)lqcd_geom_volume(g.geom) * 12 * 16;
  char* base = arena + r->off;
  char* eta_dev = base + align_up(ws_bytes);
  char* psi_dev = eta_dev + align_up(canon);
  lqcd_ws_t* ws = nullptr;
  lqcd_solve_params p = r->p;
  int rc = lqcd_ws_create(g.geom, pm, p.nrhs, base, ws_bytes, &ws);
  if (rc == LQCD_OK) {
    // the cached tuning of this lattice, inner precision and rhs count, if
    // lqcd_server_warmup (or an earlier lqcd_autotune) filled one; otherwise
    // the default.  Never tuned here, and no tuning changes a result.
    lqcd_tuning t;
    if (lqcd_tune_cache_find(g.gauge, p.inner_prec, p.nrhs, p.d.mu != 0.0, 0, &t) == LQCD_OK)
      lqcd_ws_set_tuning(ws, p.inner_prec, &t);
    // the FP64 tuning of the reliable updates of a mixed solve
    if (p.inner_prec != LQCD_F64 && lqcd_tune_cache_find(g.gauge, LQCD_F64, p.nrhs, p.d.mu != 0.0, 0, &t) == LQCD_OK)
      lqcd_ws_set_tuning(ws, LQCD_F64, &t);
    hipError_t e = hipMemcpyAsync(eta_dev, r->eta, canon, hipMemcpyHostToDevice, st);
    // an initial guess travels in the solution buffer (lqcd_solve reads x0
    // before it writes psi)
    if (e == hipSuccess && p.x0) {
      e = hipMemcpyAsync(psi_dev, p.x0, canon, hipMemcpyHostToDevice, st);
      p.x0 = psi_dev;
    }
    if (e != hipSuccess) rc = hip_status(e, "request source upload");
  }
  if (rc == LQCD_OK) {
    rc = lqcd_solve(g.gauge, &p, eta_dev, psi_dev, ws, st, r->info.data());
    if (rc == LQCD_OK || rc == LQCD_ENOCONV) {
      hipError_t e = hipMemcpyAsync(r->psi, psi_dev, canon, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) rc = hip_status(e, "request solution download");
    }
  }
  if (ws) lqcd_ws_free(ws);
  if (rc != LQCD_OK)
    for (auto& i : r->info)
      if (i.status == LQCD_OK) i.status = rc;
  r->status = rc;
}

void lqcd_server::worker(int idx) {
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    Request* r = pick_locked();
    if (!r) {
      if (stopping && queue.empty()) return;
      cv.wait(lk);
      continue;
    }
    r->t_admit = now();
    ++running;
    const GaugeEntry g = gauges[r->gauge_id];  // copied under the lock
    lk.unlock();
    run(r, g, idx);
    lk.lock();
    alloc.release(r->off, r->bytes);
    r->t_done = now();
    r->finished = true;
    --running;
    cv.notify_all();
  }
}

extern "C" int lqcd_server_create(void* arena, size_t arena_bytes, int max_streams, int queue_cap,
                                  double sim_seconds, lqcd_server_t** out) {
  if (!out) return fail(LQCD_EINVAL, "lqcd_server_create: null pointer");
  *out = nullptr;
  if (max_streams < 1 || max_streams > 16) return fail(LQCD_EINVAL, "lqcd_server_create: max_streams in [1,16]");
  if (queue_cap < 1) return fail(LQCD_EINVAL, "lqcd_server_create: queue_cap >= 1");
  if (arena && ((uintptr_t)arena % kAlign)) return fail(LQCD_EINVAL, "lqcd_server_create: arena not 256-byte aligned");
  if (arena_bytes < kAlign) return fail(LQCD_ENOMEM, "lqcd_server_create: arena too small");
  lqcd_server* s = new (std::nothrow) lqcd_server;
  if (!s) return fail(LQCD_ENOMEM, "lqcd_server_create: host allocation failed");
  s->arena = (char*)arena;
  s->sim = (arena == nullptr);
  s->sim_seconds = sim_seconds > 0 ? sim_seconds : 0.0;
  s->max_streams = max_streams;
  s->queue_cap = queue_cap;
  s->alloc.init(arena_bytes & ~(kAlign - 1));
  if (!s->sim) {
    for (int i = 0; i <= max_streams; ++i) {  // one per worker, then the import stream
      hipStream_t st;
      hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e != hipSuccess) {
        for (auto x : s->streams) (void)hipStreamDestroy(x);
        if (s->import_stream) (void)hipStreamDestroy(s->import_stream);
        delete s;
        return hip_status(e, "lqcd_server_create: stream");
      }
      if (i < max_streams)
        s->streams.push_back(st);
      else
        s->import_stream = st;
    }
  }
  for (int i = 0; i < max_streams; ++i) s->workers.emplace_back(&lqcd_server::worker, s, i);
  *out = s;
  return LQCD_OK;
}

extern "C" int lqcd_server_add_gauge(lqcd_server_t* s, const lqcd_geom_desc* desc, const void* U_host,
                                     int pmask, int* gauge_id) {
  if (!s || !desc || !gauge_id || (!U_host && !s->sim))
    return fail(LQCD_EINVAL, "lqcd_server_add_gauge: null pointer");
  if (pmask & ~15) return fail(LQCD_EINVAL, "lqcd_server_add_gauge: bad precision mask");
  lqcd_geom_t* geom = nullptr;
  int rc = lqcd_geom(desc, &geom);
  if (rc) return rc;
  GaugeEntry g;
  g.geom = geom;
  g.pmask = pmask | LQCD_PM_F64;
  g.bytes = lqcd_gauge_bytes(geom, g.pmask);
  const size_t canon = (size_t)lqcd_geom_volume(geom) * 4 * 9 * 16;
  size_t tmp_off = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping || s->exclusive || s->running > 0 || !s->queue.empty()) {
      lqcd_geom_free(geom);
      return fail(LQCD_EBUSY, "lqcd_server_add_gauge: requests are queued or running");
    }
    if (!s->alloc.alloc(g.bytes, &g.off)) {
      lqcd_geom_free(geom);
      return fail(LQCD_ENOMEM, "lqcd_server_add_gauge: arena full (%zu bytes needed)", g.bytes);
    }
    if (!s->sim && !s->alloc.alloc(canon, &tmp_off)) {
      s->alloc.release(g.off, g.bytes);
      lqcd_geom_free(geom);
      return fail(LQCD_ENOMEM, "lqcd_server_add_gauge: no room to stage the field");
    }
    s->exclusive = true;  // nothing is admitted until the field is in place
    // counted at once, so that a request submitted meanwhile is checked
    // against the arena that will remain for requests
    s->gauge_bytes_total += align_up(g.bytes);
  }
  if (!s->sim) {
    hipStream_t st = s->import_stream;
    char* dev = s->arena + tmp_off;
    hipError_t e = hipMemcpyAsync(dev, U_host, canon, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      rc = lqcd_gauge_create(geom, dev, g.pmask, s->arena + g.off, g.bytes, st, &g.gauge);
      e = hipStreamSynchronize(st);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->alloc.release(tmp_off, canon);
    if (e != hipSuccess || rc != LQCD_OK) {
      s->alloc.release(g.off, g.bytes);
      s->gauge_bytes_total -= align_up(g.bytes);
      lqcd_geom_free(geom);
      s->exclusive = false;
      s->cv.notify_all();
      return rc != LQCD_OK ? rc : hip_status(e, "lqcd_server_add_gauge");
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->gauges.push_back(g);
  *gauge_id = (int)s->gauges.size() - 1;
  s->exclusive = false;
  s->cv.notify_all();
  return LQCD_OK;
}

extern "C" int lqcd_server_warmup(lqcd_server_t* s, int gauge_id, int inner_prec, int nrhs) {
  if (!s) return fail(LQCD_EINVAL, "lqcd_server_warmup: null server");
  if (inner_prec < LQCD_F64 || inner_prec > LQCD_BF16 || nrhs < 1 || nrhs > 64)
    return fail(LQCD_EINVAL, "lqcd_server_warmup: bad precision or nrhs");
  GaugeEntry g;
  size_t off = 0, bytes = 0;
  bool need_inner = false, need64 = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (gauge_id < 0 || gauge_id >= (int)s->gauges.size())
      return fail(LQCD_ENOTFOUND, "lqcd_server_warmup: unknown gauge id %d", gauge_id);
    g = s->gauges[gauge_id];
    if (!(g.pmask & (1 << inner_prec)))
      return fail(LQCD_EINVAL, "lqcd_server_warmup: gauge field %d not stored in precision %d", gauge_id,
                  inner_prec);
    if (s->stopping || s->exclusive || s->running > 0 || !s->queue.empty())
      return fail(LQCD_EBUSY, "lqcd_server_warmup: requests are queued or running");
    if (s->sim) return LQCD_OK;
    lqcd_tuning t;
    need_inner = lqcd_tune_cache_find(g.gauge, inner_prec, nrhs, 0, 0, &t) != LQCD_OK;
    // the FP64 hops of the reliable updates of a multi-rhs mixed solve run in
    // the FP64 tuning of the same rhs count
    need64 = inner_prec != LQCD_F64 && nrhs > 1 && lqcd_tune_cache_find(g.gauge, LQCD_F64, nrhs, 0, 0, &t) != LQCD_OK;
    if (!need_inner && !need64) return LQCD_OK;
    const int pm = LQCD_PM_F64 | (inner_prec == LQCD_F32 ? LQCD_PM_F32 : 0) |
                   (inner_prec == LQCD_BF16 ? LQCD_PM_BF16 : 0);
    bytes = lqcd_ws_bytes(g.geom, pm, nrhs);
    if (!s->alloc.alloc(bytes, &off))
      return fail(LQCD_ENOMEM, "lqcd_server_warmup: no room for a %zu-byte workspace", bytes);
    s->exclusive = true;  // the GPU stays idle apart from the tuning runs
  }
  const int pm = LQCD_PM_F64 | (inner_prec == LQCD_F32 ? LQCD_PM_F32 : 0) |
                 (inner_prec == LQCD_BF16 ? LQCD_PM_BF16 : 0);
  lqcd_ws_t* ws = nullptr;
  int rc = lqcd_ws_create(g.geom, pm, nrhs, s->arena + off, bytes, &ws);
  if (rc == LQCD_OK) {
    // any Dirac parameters: the clover values do not change kernel timings
    const lqcd_dirac d{0.13, 1.9, 1.0, 0.0};
    if (need_inner) rc = lqcd_autotune(g.gauge, &d, inner_prec, nrhs, ws, s->import_stream, nullptr, nullptr);
    if (rc == LQCD_OK && need64)
      rc = lqcd_autotune(g.gauge, &d, LQCD_F64, nrhs, ws, s->import_stream, nullptr, nullptr);
    const hipError_t e = hipStreamSynchronize(s->import_stream);
    if (rc == LQCD_OK && e != hipSuccess) rc = hip_status(e, "lqcd_server_warmup");
    lqcd_ws_free(ws);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->alloc.release(off, bytes);
  s->exclusive = false;
  s->cv.notify_all();
  return rc;
}

extern "C" size_t lqcd_request_bytes(lqcd_server_t* s, int gauge_id, const lqcd_solve_params* p) {
  if (!s || !p || p->nrhs < 1) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  if (gauge_id < 0 || gauge_id >= (int)s->gauges.size()) return 0;
  return footprint(s, s->gauges[gauge_id], p);
}

extern "C" int lqcd_submit(lqcd_server_t* s, int gauge_id, const lqcd_solve_params* p, const void* eta,
                           void* psi, uint64_t* ticket) {
  if (!s || !p || !ticket || ((!eta || !psi) && !s->sim)) return fail(LQCD_EINVAL, "lqcd_submit: null pointer");
  if (p->nrhs < 1 || p->nrhs > 64) return fail(LQCD_EINVAL, "lqcd_submit: nrhs=%d out of range", p->nrhs);
  if (p->inner_prec < LQCD_F64 || p->inner_prec > LQCD_BF16)
    return fail(LQCD_EINVAL, "lqcd_submit: bad inner precision");
  int rc = check_dirac(&p->d);
  if (rc) return rc;
  if (!(p->tol > 0.0 && p->tol < 1.0) || p->maxiter < 1) return fail(LQCD_EINVAL, "lqcd_submit: bad tol/maxiter");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail(LQCD_EINVAL, "lqcd_submit: server is stopping");
  if (gauge_id < 0 || gauge_id >= (int)s->gauges.size())
    return fail(LQCD_ENOTFOUND, "lqcd_submit: unknown gauge id %d", gauge_id);
  const GaugeEntry& g = s->gauges[gauge_id];
  if (!(g.pmask & (1 << p->inner_prec)))
    return fail(LQCD_EINVAL, "lqcd_submit: gauge field %d not stored in precision %d", gauge_id, p->inner_prec);
  const size_t bytes = footprint(s, g, p);
  if (bytes > s->alloc.size() - s->gauge_bytes_total)
    return fail(LQCD_ENOMEM, "lqcd_submit: request needs %zu bytes, arena can never hold it", bytes);
  if ((int)s->queue.size() >= s->queue_cap) return fail(LQCD_EBUSY, "lqcd_submit: queue full");
  Request* r = new (std::nothrow) Request;
  if (!r) return fail(LQCD_ENOMEM, "lqcd_submit: host allocation failed");
  r->ticket = s->next_ticket++;
  r->gauge_id = gauge_id;
  r->p = *p;
  r->eta = eta;
  r->psi = psi;
  r->bytes = bytes;
  r->t_submit = s->now();
  s->queue.push_back(r);
  s->tickets[r->ticket] = r;
  *ticket = r->ticket;
  s->cv.notify_all();
  return LQCD_OK;
}

extern "C" int lqcd_poll(lqcd_server_t* s, uint64_t ticket, lqcd_solve_info* info, double* times) {
  if (!s) return fail(LQCD_EINVAL, "lqcd_poll: null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(LQCD_ENOTFOUND, "lqcd_poll: unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  if (!r->finished) return LQCD_PENDING;
  if (info)
    for (size_t i = 0; i < r->info.size(); ++i) info[i] = r->info[i];
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_admit;
    times[2] = r->t_done;
  }
  const int st = r->status;
  s->tickets.erase(it);
  delete r;
  return st;
}

extern "C" size_t lqcd_server_peak_bytes(lqcd_server_t* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->alloc.peak();
}

extern "C" int lqcd_server_stop(lqcd_server_t* s, int cancel_pending) {
  if (!s) return fail(LQCD_EINVAL, "lqcd_server_stop: null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopped) return LQCD_OK;
    s->stopping = true;
    if (cancel_pending) {
      for (Request* r : s->queue) {
        r->status = LQCD_ECANCELED;
        r->info.assign(r->p.nrhs, lqcd_solve_info{});
        for (auto& i : r->info) i.status = LQCD_ECANCELED;
        r->t_done = s->now();
        r->finished = true;
      }
      s->queue.clear();
    }
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  s->workers.clear();
  std::lock_guard<std::mutex> lk(s->mu);
  s->stopped = true;
  return LQCD_OK;
}

extern "C" int lqcd_server_destroy(lqcd_server_t* s, int cancel_pending) {
  if (!s) return fail(LQCD_EINVAL, "lqcd_server_destroy: null server");
  lqcd_server_stop(s, cancel_pending);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  if (s->import_stream) (void)hipStreamDestroy(s->import_stream);
  for (auto& g : s->gauges) {
    if (g.gauge) lqcd_gauge_free(g.gauge);
    lqcd_geom_free(g.geom);
  }
  for (auto& kv : s->tickets) delete kv.second;
  delete s;
  return LQCD_OK;
}
