// server.cpp -- continuous-batching request server for dd Rgemm / Rsyrk.
//
// Requests (an SDP interior-point iteration issues many Rgemm / Rsyrk updates
// of uneven sizes; the manual motivates MPBLAS by SDPA, section
// "Introduction") are submitted from any host thread and complete
// asynchronously.  One scheduler thread:
//   1. polls the in-flight groups (one per slot stream) and completes them:
//      stamps the end time, releases their memory budget, wakes waiters;
//   2. admits queued requests in FIFO order while the HBM budget (bytes of
//      the operands they keep resident: 16 bytes per dd entry of A, B, C) and
//      the in-flight request limit allow -- a request larger than the whole
//      budget fails with MPDD_ERR_BUDGET, others wait;
//   3. whenever a slot is free and requests are admitted, launches them all
//      as one group: their C tiles become a work list (longest k first), the
//      list is copied to the slot's device buffer and a captured hipGraph of
//      persistent grouped kernels (one per tile shape) walks it; a group of
//      one request launches its tile kernel directly.  Groups on different
//      slots overlap on the device, so requests that arrive while others run
//      start as soon as a slot and budget free up.
// When the server is idle, a submitted request is launched by the submitting
// thread itself, as a group of one (no hand-off to the scheduler).
// The thread polls without sleeping while groups are in flight and for
// kIdleSpin seconds after its last activity (so steady traffic never waits
// for a thread wake-up); after that it sleeps until the next submission.
// The tile shape of each request is the handle's tuned choice (restricted to
// the shapes the grouped graph holds), so a request's result is bit-identical
// to a standalone call with that tile.
//
// A fake-device mode (no HIP calls; groups "complete" after a simulated time)
// exercises admission, FIFO order, grouping, failure isolation and the timing
// records on machines without a GPU.  Failures can be injected per request
// from the host (mpdd_request.inject) in both modes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/mpdd.h"
#include "../../include/mpdd_testing.h"
#include "kernels.hpp"
#include "tuner.hpp"

using namespace mpdd;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

bool lsame(char c, char ref) {
  if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
  return c == ref;
}

// Tile shapes the grouped graph runs: a small one for small requests and the
// large one that the dense products use (tile-table entries).
constexpr int kServeTiles[] = {2, 4};
constexpr int kNumServeTiles = 2;
constexpr int kSlots = 4;
constexpr int kMaxGroupReqs = 1024;
constexpr int kMaxGroupItems = 1 << 18;
// the scheduler polls (yielding) for this long after its last activity before
// it sleeps on the condition variable: under steady traffic a request never
// waits for a thread wake-up
constexpr double kIdleSpin = 0.05;

struct Req {
  mpdd_request r;
  uint64_t ticket = 0;
  size_t bytes = 0;
  int info = 0;
  bool done = false;
  mpdd_timing t{};
  int tile = 0;        // index into kServeTiles
  int64_t items = 0;   // C tiles
  double flops = 0.0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  void* host_buf = nullptr;   // pinned: header | reqs | items
  void* dev_buf = nullptr;
  size_t buf_bytes = 0;
  hipGraphExec_t exec = nullptr;
  bool busy = false;
  bool failed = false;
  double fake_done = 0.0;
  int group_id = 0;
  std::vector<Req*> reqs;
};

// Device buffer layout of a group: header | request descriptors | work items,
// packed so that one copy of exactly the used bytes moves a group.
struct GroupHeader {
  int count[kNumServeTiles];   // items per tile shape
  int items_offset;            // byte offset of the work items from the buffer start
  int pad[64 - kNumServeTiles - 1];
};

}  // namespace

struct mpdd_server_s {
  mpdd_handle h = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_inflight = 0;
  bool fake = false;
  double fake_rate = 1e12;       // simulated dd-flop/s
  double fake_latency = 20e-6;   // simulated per-group latency

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Req*> pending;
  std::vector<Req*> admitted;
  std::map<uint64_t, Req*> table;
  size_t inflight_bytes = 0;
  int inflight_count = 0;
  uint64_t next_ticket = 1;
  int next_group = 1;
  bool stop = false;
  bool shutdown = false;
  Slot slots[kSlots];
  std::thread thr;
  int fatal = 0;
  mpdd_server_stats stats{};
};

namespace {

int check_request(const mpdd_request& r) {
  if (r.op == MPDD_OP_GEMM) {
    const char ta = r.flag1, tb = r.flag2;
    const bool nota = lsame(ta, 'N'), notb = lsame(tb, 'N');
    const mpdd_int nrowa = nota ? r.m : r.k, nrowb = notb ? r.k : r.n;
    if (!nota && !lsame(ta, 'T') && !lsame(ta, 'C')) return 1;
    if (!notb && !lsame(tb, 'T') && !lsame(tb, 'C')) return 2;
    if (r.m < 0) return 3;
    if (r.n < 0) return 4;
    if (r.k < 0) return 5;
    if (r.lda < std::max<mpdd_int>(1, nrowa)) return 8;
    if (r.ldb < std::max<mpdd_int>(1, nrowb)) return 10;
    if (r.ldc < std::max<mpdd_int>(1, r.m)) return 13;
    return 0;
  }
  if (r.op == MPDD_OP_SYRK) {
    const bool upper = lsame(r.flag1, 'U');
    const mpdd_int nrowa = lsame(r.flag2, 'N') ? r.n : r.k;
    if (!upper && !lsame(r.flag1, 'L')) return 1;
    if (!lsame(r.flag2, 'N') && !lsame(r.flag2, 'T') && !lsame(r.flag2, 'C')) return 2;
    if (r.n < 0) return 3;
    if (r.k < 0) return 4;
    if (r.lda < std::max<mpdd_int>(1, nrowa)) return 7;
    if (r.ldc < std::max<mpdd_int>(1, r.n)) return 10;
    return 0;
  }
  return MPDD_ERR_ARG;
}

bool dd_zero(mpdd_dd x) { return x.hi == 0.0 && x.lo == 0.0; }
bool dd_one(mpdd_dd x) { return x.hi == 1.0 && x.lo == 0.0; }

// Rows x columns of C that a request updates, and whether it is a no-op.
void shape_of(const mpdd_request& r, int64_t& m, int64_t& n, int64_t& k) {
  if (r.op == MPDD_OP_GEMM) { m = r.m; n = r.n; k = r.k; }
  else { m = r.n; n = r.n; k = r.k; }
}

bool quick_return(const mpdd_request& r) {
  int64_t m, n, k;
  shape_of(r, m, n, k);
  return m == 0 || n == 0 || ((dd_zero(r.alpha) || k == 0) && dd_one(r.beta));
}

size_t footprint(const mpdd_request& r) {
  int64_t m, n, k;
  shape_of(r, m, n, k);
  size_t a, b = 0;
  if (r.op == MPDD_OP_GEMM) {
    a = (size_t)r.lda * (size_t)(lsame(r.flag1, 'N') ? k : m);
    b = (size_t)r.ldb * (size_t)(lsame(r.flag2, 'N') ? n : k);
  } else {
    a = (size_t)r.lda * (size_t)(lsame(r.flag2, 'N') ? k : n);
  }
  const size_t c = (size_t)r.ldc * (size_t)n;
  return 16 * (a + b + c);
}

int serve_tile_index(mpdd_server_s* s, const mpdd_request& r) {
  int64_t m, n, k;
  shape_of(r, m, n, k);
  int tile = -1;
  if (s->h) {
    TuneEntry e;
    const bool syrk = r.op == MPDD_OP_SYRK;
    const bool ta = syrk ? !lsame(r.flag2, 'N') : !lsame(r.flag1, 'N');
    const bool tb = syrk ? !ta : !lsame(r.flag2, 'N');
    if (handle_tune_lookup(s->h, syrk ? 1 : 0, ta, tb, m, n, k, e))
      tile = e.serve_tile >= 0 ? e.serve_tile : e.tile;
  }
  if (tile < 0) tile = default_tile(m, n, k, r.op == MPDD_OP_SYRK);
  for (int i = 0; i < kNumServeTiles; ++i)
    if (kServeTiles[i] == tile) return i;
  // not a grouped shape: small tiles for small C, else the large ones
  return (m * n <= 512 * 512) ? 0 : 1;
}

void finish(mpdd_server_s* s, Req* q, int info, double t_end) {
  q->info = info;
  q->t.end = t_end;
  q->t.info = info;
  q->done = true;
  s->stats.completed += 1;
  if (info != 0) s->stats.failed += 1;
}

// Build the request descriptors and work list of a group into the slot's
// pinned buffer.  Returns false if it does not fit.
// The update of one request as the tile kernels take it (k = 0 and alpha = 0
// when it is C <- beta C only), with its op flags and output shape.
void make_params(const mpdd_request& r, GemmParams& p, bool& ta, bool& tb, int64_t& m,
                 int64_t& n) {
  const bool syrk = r.op == MPDD_OP_SYRK;
  int64_t k;
  shape_of(r, m, n, k);
  const bool scale_only = dd_zero(r.alpha) || k == 0;
  p.m = m; p.n = n; p.k = scale_only ? 0 : k;
  p.kchunk = p.k;
  p.alpha_hi = scale_only ? 0.0 : r.alpha.hi;
  p.alpha_lo = scale_only ? 0.0 : r.alpha.lo;
  p.beta_hi = r.beta.hi; p.beta_lo = r.beta.lo;
  p.beta_zero = dd_zero(r.beta) ? 1 : 0;
  p.c_hi = r.C_hi; p.c_lo = r.C_lo; p.ldc = r.ldc;
  if (syrk) {
    ta = !lsame(r.flag2, 'N');
    tb = !ta;
    p.a_hi = r.A_hi; p.a_lo = r.A_lo; p.lda = r.lda;
    p.b_hi = r.A_hi; p.b_lo = r.A_lo; p.ldb = r.lda;
    p.tri = lsame(r.flag1, 'U') ? 1 : 2;
  } else {
    ta = !lsame(r.flag1, 'N');
    tb = !lsame(r.flag2, 'N');
    p.a_hi = r.A_hi; p.a_lo = r.A_lo; p.lda = r.lda;
    p.b_hi = r.B_hi; p.b_lo = r.B_lo; p.ldb = r.ldb;
    p.tri = 0;
  }
}

bool build_group(Slot& sl, const std::vector<Req*>& g, size_t& used, int counts[kNumServeTiles]) {
  char* base = (char*)sl.host_buf;
  GroupHeader* hdr = (GroupHeader*)base;
  ServeReq* reqs = (ServeReq*)(base + sizeof(GroupHeader));
  ServeItem* items0 = (ServeItem*)(reqs + g.size());
  std::vector<std::vector<std::pair<int64_t, ServeItem>>> lists(kNumServeTiles);
  for (size_t qi = 0; qi < g.size(); ++qi) {
    const mpdd_request& r = g[qi]->r;
    ServeReq d{};
    GemmParams& p = d.p;
    int64_t m, n;
    bool ta, tb;
    make_params(r, p, ta, tb, m, n);
    d.flags = (ta ? 1 : 0) | (tb ? 2 : 0);
    reqs[qi] = d;
    const TileInfo* t = tile_info(kServeTiles[g[qi]->tile]);
    const int tm = (int)((m + t->bm - 1) / t->bm), tn = (int)((n + t->bn - 1) / t->bn);
    auto& L = lists[g[qi]->tile];
    for (int bj = 0; bj < tn; ++bj)
      for (int bi = 0; bi < tm; ++bi) {
        if (p.tri == 1 && bi > bj) continue;
        if (p.tri == 2 && bi < bj) continue;
        L.push_back({p.k, ServeItem{(int)qi, bi, bj}});
      }
  }
  size_t total = 0;
  for (auto& L : lists) total += L.size();
  if (total > (size_t)kMaxGroupItems) return false;
  std::memset(hdr, 0, sizeof(GroupHeader));
  hdr->items_offset = (int)((char*)items0 - base);
  ServeItem* out = items0;
  for (int c = 0; c < kNumServeTiles; ++c) {
    auto& L = lists[c];
    std::stable_sort(L.begin(), L.end(),
                     [](const std::pair<int64_t, ServeItem>& a,
                        const std::pair<int64_t, ServeItem>& b) { return a.first > b.first; });
    for (auto& e : L) *out++ = e.second;
    hdr->count[c] = (int)L.size();
    counts[c] = (int)L.size();
  }
  used = (size_t)((char*)out - base);
  return true;
}

// Capture the grouped schedule of a slot once: one persistent kernel per tile
// shape, reading its work list and item count from the slot's device buffer.
int capture_graph(Slot& sl) {
  const char* dbase = (const char*)sl.dev_buf;
  const GroupHeader* hdr = (const GroupHeader*)dbase;
  const ServeReq* reqs = (const ServeReq*)(dbase + sizeof(GroupHeader));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPDD_ERR_HIP;
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return MPDD_ERR_HIP;
  hipError_t e = hipSuccess;
  for (int c = 0; c < kNumServeTiles && e == hipSuccess; ++c)
    e = launch_grouped_list(kServeTiles[c], dbase, reqs, hdr->count, &hdr->items_offset, c,
                            2 * cus, sl.stream);
  hipError_t e2 = hipStreamEndCapture(sl.stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return MPDD_ERR_HIP;
  }
  e = hipGraphInstantiate(&sl.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e == hipSuccess ? 0 : MPDD_ERR_HIP;
}

size_t slot_bytes() {
  return sizeof(GroupHeader) + sizeof(ServeReq) * kMaxGroupReqs +
         sizeof(ServeItem) * (size_t)kMaxGroupItems;
}

int init_slot(Slot& sl) {
  sl.buf_bytes = slot_bytes();
  if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) return MPDD_ERR_HIP;
  if (hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess) return MPDD_ERR_HIP;
  if (hipHostMalloc(&sl.host_buf, sl.buf_bytes, hipHostMallocDefault) != hipSuccess)
    return MPDD_ERR_ALLOC;
  if (hipMalloc(&sl.dev_buf, sl.buf_bytes) != hipSuccess) return MPDD_ERR_ALLOC;
  std::memset(sl.host_buf, 0, sizeof(GroupHeader));
  if (hipMemcpy(sl.dev_buf, sl.host_buf, sizeof(GroupHeader), hipMemcpyHostToDevice) != hipSuccess)
    return MPDD_ERR_HIP;
  return capture_graph(sl);
}

void free_slot(Slot& sl) {
  if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
  if (sl.dev_buf) (void)hipFree(sl.dev_buf);
  if (sl.host_buf) (void)hipHostFree(sl.host_buf);
  if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  sl = Slot();
}

// Launch a group on a slot (called with the lock held).  Returns 0 or an error.
int launch_group(mpdd_server_s* s, Slot& sl, std::vector<Req*>& g) {
  const double t0 = now_s();
  for (Req* q : g) {
    q->t.start = t0;
    q->t.group = s->next_group;
  }
  sl.group_id = s->next_group++;
  s->stats.groups += 1;
  for (Req* q : g)
    if (q->r.inject == MPDD_INJECT_DEVICE_ERROR) return MPDD_ERR_HIP;
  if (s->fake) {
    double flops = 0.0;
    for (Req* q : g) flops += q->flops;
    sl.fake_done = t0 + s->fake_latency + flops / s->fake_rate;
    return 0;
  }
  if (g.size() == 1) {
    // a group of one: launch its tile kernel directly with the update passed
    // by value (no descriptor copy); the same tile code as the grouped
    // kernel, so the result is the same
    GemmParams p{};
    bool ta, tb;
    int64_t m, n;
    make_params(g[0]->r, p, ta, tb, m, n);
    const int tile = kServeTiles[g[0]->tile];
    const TileInfo* ti = tile_info(tile);
    p.tiles_m = (int)((m + ti->bm - 1) / ti->bm);
    p.tiles_n = (int)((n + ti->bn - 1) / ti->bn);
    if (launch_gemm(tile, p, ta, tb, false, 1, sl.stream) != hipSuccess) return MPDD_ERR_HIP;
    if (hipEventRecord(sl.done_ev, sl.stream) != hipSuccess) return MPDD_ERR_HIP;
    return 0;
  }
  size_t used = 0;
  int counts[kNumServeTiles];
  if (!build_group(sl, g, used, counts)) return MPDD_ERR_UNSUPPORTED;
  if (hipMemcpyAsync(sl.dev_buf, sl.host_buf, used, hipMemcpyHostToDevice, sl.stream) !=
      hipSuccess)
    return MPDD_ERR_HIP;
  if (hipGraphLaunch(sl.exec, sl.stream) != hipSuccess) return MPDD_ERR_HIP;
  if (hipEventRecord(sl.done_ev, sl.stream) != hipSuccess) return MPDD_ERR_HIP;
  return 0;
}

void release(mpdd_server_s* s, Req* q) {
  s->inflight_bytes -= q->bytes;
  s->inflight_count -= 1;
}

void scheduler(mpdd_server_s* s) {
  if (!s->fake) (void)hipSetDevice(s->device);   // HIP's current device is per thread
  std::unique_lock<std::mutex> lk(s->mu);
  double last_active = now_s();
  for (;;) {
    bool progressed = false;
    // 1. completions
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      bool done;
      if (s->fake) done = now_s() >= sl.fake_done;
      else {
        hipError_t q = hipEventQuery(sl.done_ev);
        done = (q != hipErrorNotReady);
        if (done && q != hipSuccess) sl.failed = true;
      }
      if (!done) continue;
      const double t_end = now_s();
      for (Req* q : sl.reqs) {
        finish(s, q, sl.failed ? MPDD_ERR_HIP : 0, t_end);
        release(s, q);
      }
      sl.reqs.clear();
      sl.busy = false;
      sl.failed = false;
      progressed = true;
      s->cv_done.notify_all();
    }
    // 2. admission, FIFO
    while (!s->pending.empty()) {
      Req* q = s->pending.front();
      if (s->inflight_count >= s->max_inflight) break;
      if (s->inflight_bytes + q->bytes > s->budget) break;
      s->pending.pop_front();
      q->t.admit = now_s();
      if (q->r.inject == MPDD_INJECT_ALLOC_FAILURE) {
        finish(s, q, MPDD_ERR_ALLOC, q->t.admit);
        s->cv_done.notify_all();
        continue;
      }
      s->inflight_bytes += q->bytes;
      s->inflight_count += 1;
      s->admitted.push_back(q);
      progressed = true;
    }
    // 3. launch admitted requests as a group on a free slot
    while (!s->admitted.empty()) {
      Slot* free_sl = nullptr;
      for (Slot& sl : s->slots)
        if (!sl.busy) { free_sl = &sl; break; }
      if (!free_sl) break;
      std::vector<Req*> g;
      int64_t items = 0;
      size_t take = 0;
      while (take < s->admitted.size() && (int)g.size() < kMaxGroupReqs &&
             items + s->admitted[take]->items <= kMaxGroupItems) {
        items += s->admitted[take]->items;
        g.push_back(s->admitted[take++]);
      }
      if (g.empty()) {       // a single request with too many tiles
        Req* q = s->admitted.front();
        s->admitted.erase(s->admitted.begin());
        finish(s, q, MPDD_ERR_UNSUPPORTED, now_s());
        release(s, q);
        s->cv_done.notify_all();
        continue;
      }
      s->admitted.erase(s->admitted.begin(), s->admitted.begin() + take);
      int rc = launch_group(s, *free_sl, g);
      if (rc != 0 && g.size() > 1) {
        // isolate the failure: run the requests one by one.  The slot stays
        // marked busy meanwhile (holding no requests), so the submit path,
        // which may run while the fake device's wait below drops the lock,
        // cannot launch on it.
        free_sl->busy = true;
        for (Req* q : g) {
          std::vector<Req*> one{q};
          int r1 = launch_group(s, *free_sl, one);
          if (r1 == 0 && !s->fake) {
            hipError_t w = hipEventSynchronize(free_sl->done_ev);
            if (w != hipSuccess) r1 = MPDD_ERR_HIP;
          }
          if (r1 == 0 && s->fake) {
            const double until = free_sl->fake_done;
            lk.unlock();
            while (now_s() < until) std::this_thread::yield();
            lk.lock();
          }
          finish(s, q, r1, now_s());
          release(s, q);
        }
        free_sl->busy = false;
        s->cv_done.notify_all();
      } else if (rc != 0) {
        finish(s, g[0], rc, now_s());
        release(s, g[0]);
        s->cv_done.notify_all();
      } else {
        free_sl->reqs = g;
        free_sl->busy = true;
      }
      progressed = true;
    }
    bool busy = false;
    for (Slot& sl : s->slots) busy = busy || sl.busy;
    if (s->stop && !busy && s->pending.empty() && s->admitted.empty()) break;
    if (progressed) {
      last_active = now_s();
      continue;
    }
    if (busy) last_active = now_s();
    if (busy || now_s() - last_active < kIdleSpin) {
      // groups in flight, or recent traffic: poll without sleeping (a timed
      // wait, or a wake-up from the condition variable, would add tens of
      // microseconds to every request)
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      s->cv_sched.wait(lk);
      last_active = now_s();
    }
  }
}

// An idle server (nothing queued or admitted) with a free slot and room in
// the budget launches a request from the submitting thread itself: the
// request skips the hand-off to the scheduler, which then only has to see it
// complete.  FIFO order holds because nothing waits ahead of it.  Requests
// with an injected failure take the scheduler's path.  Called with the lock
// held; true when the request was launched (or failed at launch).
bool launch_from_submit(mpdd_server_s* s, Req* q) {
  if (!s->pending.empty() || !s->admitted.empty() || q->r.inject != MPDD_INJECT_NONE) return false;
  if (s->inflight_count >= s->max_inflight || s->inflight_bytes + q->bytes > s->budget ||
      q->items > kMaxGroupItems)
    return false;
  if (!s->fake) {
    // the slot streams belong to the server's device; a caller thread with
    // another device current goes through the scheduler (which set it)
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != s->device) return false;
  }
  Slot* free_sl = nullptr;
  for (Slot& sl : s->slots)
    if (!sl.busy) { free_sl = &sl; break; }
  if (!free_sl) return false;
  q->t.admit = now_s();
  s->inflight_bytes += q->bytes;
  s->inflight_count += 1;
  std::vector<Req*> g{q};
  const int rc = launch_group(s, *free_sl, g);
  if (rc != 0) {
    finish(s, q, rc, now_s());
    release(s, q);
    s->cv_done.notify_all();
  } else {
    free_sl->reqs = g;
    free_sl->busy = true;
  }
  s->cv_sched.notify_one();   // the scheduler watches for its completion
  return true;
}

}  // namespace

extern "C" {

double mpdd_clock(void) { return now_s(); }

int mpdd_server_create(mpdd_server* out, mpdd_handle h, size_t hbm_budget_bytes,
                       int max_inflight, int flags) {
  if (!out) return MPDD_ERR_ARG;
  *out = nullptr;
  const bool fake = (flags & MPDD_SERVER_FAKE_DEVICE) != 0;
  if (!fake && !handle_valid(h)) return MPDD_ERR_HANDLE;
  if (hbm_budget_bytes == 0 || max_inflight < 1) return MPDD_ERR_ARG;
  auto* s = new (std::nothrow) mpdd_server_s();
  if (!s) return MPDD_ERR_ALLOC;
  s->h = fake ? nullptr : h;
  s->device = fake ? 0 : handle_device(h);
  if (!fake && hipSetDevice(s->device) != hipSuccess) {
    delete s;
    return MPDD_ERR_HIP;
  }
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  s->fake = fake;
  if (!fake) {
    for (Slot& sl : s->slots) {
      int rc = init_slot(sl);
      if (rc != 0) {
        for (Slot& x : s->slots) free_slot(x);
        delete s;
        return rc;
      }
    }
  }
  s->thr = std::thread(scheduler, s);
  *out = s;
  return 0;
}

int mpdd_server_set_fake_rate(mpdd_server s, double dd_flops_per_s, double group_latency_s) {
  if (!s || !s->fake || dd_flops_per_s <= 0 || group_latency_s < 0) return MPDD_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->fake_rate = dd_flops_per_s;
  s->fake_latency = group_latency_s;
  return 0;
}

int mpdd_server_submit(mpdd_server s, const mpdd_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return MPDD_ERR_ARG;
  auto* q = new (std::nothrow) Req();
  if (!q) return MPDD_ERR_ALLOC;
  q->r = *r;
  const double t = now_s();
  q->t.arrival = r->arrival >= 0.0 ? r->arrival : t;
  q->t.submit = t;
  q->t.tile = -1;
  int64_t m, n, k;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->shutdown) {
    delete q;
    return MPDD_ERR_SHUTDOWN;
  }
  q->ticket = s->next_ticket++;
  *ticket = q->ticket;
  s->table[q->ticket] = q;
  s->stats.submitted += 1;
  const int info = check_request(*r);
  if (info != 0) {
    q->t.admit = q->t.start = t;
    finish(s, q, info, t);
    s->cv_done.notify_all();
    return 0;
  }
  shape_of(*r, m, n, k);
  if (quick_return(*r)) {
    q->t.admit = q->t.start = t;
    finish(s, q, 0, t);
    s->cv_done.notify_all();
    return 0;
  }
  const bool scale_only = dd_zero(r->alpha) || k == 0;
  if (!r->C_hi || !r->C_lo ||
      (!scale_only && (!r->A_hi || !r->A_lo ||
                       (r->op == MPDD_OP_GEMM && (!r->B_hi || !r->B_lo))))) {
    finish(s, q, MPDD_ERR_ARG, t);
    s->cv_done.notify_all();
    return 0;
  }
  q->bytes = footprint(*r);
  if (q->bytes > s->budget) {
    q->t.admit = q->t.start = t;
    finish(s, q, MPDD_ERR_BUDGET, t);
    s->cv_done.notify_all();
    return 0;
  }
  q->tile = serve_tile_index(s, *r);
  q->t.tile = kServeTiles[q->tile];
  const TileInfo* ti = tile_info(kServeTiles[q->tile]);
  const int64_t tm = (m + ti->bm - 1) / ti->bm, tn = (n + ti->bn - 1) / ti->bn;
  q->items = (r->op == MPDD_OP_SYRK) ? tm * (tm + 1) / 2 : tm * tn;
  q->flops = (r->op == MPDD_OP_SYRK) ? (double)n * (n + 1) * k : 2.0 * m * n * k;
  if (launch_from_submit(s, q)) return 0;
  s->pending.push_back(q);
  s->cv_sched.notify_one();
  return 0;
}

int mpdd_server_wait(mpdd_server s, uint64_t ticket, int* info, mpdd_timing* t) {
  if (!s) return MPDD_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->table.find(ticket);
  if (it == s->table.end()) return MPDD_ERR_ARG;
  Req* q = it->second;
  s->cv_done.wait(lk, [&] { return q->done; });
  if (info) *info = q->info;
  if (t) *t = q->t;
  s->table.erase(it);
  delete q;
  return 0;
}

int mpdd_server_poll(mpdd_server s, uint64_t ticket, int* done) {
  if (!s || !done) return MPDD_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->table.find(ticket);
  if (it == s->table.end()) return MPDD_ERR_ARG;
  *done = it->second->done ? 1 : 0;
  return 0;
}

int mpdd_server_get_stats(mpdd_server s, mpdd_server_stats* st) {
  if (!s || !st) return MPDD_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  st->inflight_bytes = s->inflight_bytes;
  st->inflight_requests = s->inflight_count;
  st->queued_requests = (int64_t)s->pending.size();
  return 0;
}

int mpdd_server_destroy(mpdd_server s) {
  if (!s) return MPDD_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->shutdown = true;
    s->cv_sched.notify_all();
  }
  s->thr.join();
  for (auto& kv : s->table) delete kv.second;
  s->table.clear();
  if (!s->fake)
    for (Slot& sl : s->slots) free_slot(sl);
  delete s;
  return 0;
}

}  // extern "C"
