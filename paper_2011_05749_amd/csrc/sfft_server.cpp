// sfft_server.cpp -- serving loop: continuous batching of independent solves
// (each the problem of Sect. 2.1) on one device.
//
// Requests carry a plan (kept by the caller and reused: plans stay resident),
// device pointers to a signal and its outputs, and a release time.  A
// scheduler thread forms a batch whenever a lane is free and released
// requests wait: it takes them in release order while their workspaces --
// computed on the host from the plans (make_layout) -- fit the lane's slab of
// device memory (admission by HBM footprint), lays the batch out in that slab
// and launches the same kernels as sfft_exec_batch eagerly on the lane's
// stream.  Lanes run concurrently, so requests that arrive while batches are
// on the device are admitted into the next free lane and their work overlaps
// with the batches in flight.  A waiter thread per lane blocks on the lane's
// completion event and time-stamps the batch's requests.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "sfft_host.h"

using namespace sfft;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  const sfft_plan_s *plan;
  SigIO io;
  int64_t bytes;        // workspace of the request alone
  int64_t release_ns, launch_ns, done_ns;
  int32_t batch, lane, status;
};

struct Lane {
  int id = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void *slab = nullptr;
  size_t cap = 0;
  char *staging = nullptr;   // pinned: descriptors, lists and per-signal pointers
  size_t staging_cap = 0;
  Layout lay;
  std::vector<int64_t> tickets;
  bool busy = false;         // a batch is on the device (or being launched)
  bool go = false;           // the waiter has a batch to wait for
  int32_t err = 0;
  std::thread waiter;
};

}  // namespace

struct sfft_server_s {
  sfft_server_params_t prm{};
  int device = 0;
  int ncu = 256;
  const float2 *tw = nullptr;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_lane;
  std::deque<Req> reqs;                       // index = ticket
  std::multimap<int64_t, int64_t> pending;   // release time -> ticket
  std::map<const sfft_plan_s *, int64_t> footprint;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::thread sched;
  bool stop = false;
  int64_t outstanding = 0;

  ~sfft_server_s() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_sched.notify_all();
    cv_lane.notify_all();
    if (sched.joinable()) sched.join();
    for (auto &l : lanes)
      if (l->waiter.joinable()) l->waiter.join();
    (void)hipSetDevice(device);
    for (auto &l : lanes) {
      if (l->stream) (void)hipStreamSynchronize(l->stream);
      if (l->ev) (void)hipEventDestroy(l->ev);
      if (l->stream) (void)hipStreamDestroy(l->stream);
      if (l->slab) (void)hipFree(l->slab);
      if (l->staging) (void)hipHostFree(l->staging);
    }
  }

  // Lay out and launch the batch `tk` on lane L (called without the lock).
  // Tickets that do not fit the slab once the batch's layout is known (the
  // class-vector stride is the batch's widest) are handed back in `back`.
  int32_t launch(Lane &L, std::vector<int64_t> &tk, std::vector<int64_t> &back) {
    std::vector<const sfft_plan_s *> ps;
    std::vector<SigIO> io;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int64_t t : tk) {
        ps.push_back(reqs[(size_t)t].plan);
        io.push_back(reqs[(size_t)t].io);
      }
    }
    for (;;) {
      const int32_t rc = make_layout(ps, false, ncu, L.lay);
      if (rc != SFFT_OK) return rc;
      if (L.lay.bytes <= L.cap || ps.size() == 1) break;
      back.push_back(tk.back());
      tk.pop_back();
      ps.pop_back();
      io.pop_back();
    }
    if (L.lay.bytes > L.cap) return SFFT_ETOOBIG;
    const Layout &Y = L.lay;
    const size_t nd = sizeof(SigDesc) * Y.desc.size(), nl = sizeof(int32_t) * Y.lists.size(),
                 ni = sizeof(SigIO) * io.size();
    if (nd + nl + ni > L.staging_cap) return SFFT_EINVAL;
    memcpy(L.staging, Y.desc.data(), nd);
    memcpy(L.staging + nd, Y.lists.data(), nl);
    memcpy(L.staging + nd + nl, io.data(), ni);
    char *base = (char *)L.slab;
    LaunchCtx c;
    bind_layout(Y, base, tw, c);
    c.io = (const SigIO *)(base + Y.o_io);
    if (hipMemcpyAsync(base + Y.o_desc, L.staging, nd, hipMemcpyHostToDevice, L.stream) != hipSuccess ||
        hipMemcpyAsync(base + Y.o_lists, L.staging + nd, nl, hipMemcpyHostToDevice, L.stream) != hipSuccess ||
        hipMemcpyAsync(base + Y.o_io, L.staging + nd + nl, ni, hipMemcpyHostToDevice, L.stream) != hipSuccess ||
        launch_pipeline(Y, c, L.stream, nullptr) != hipSuccess ||
        hipEventRecord(L.ev, L.stream) != hipSuccess)
      return SFFT_EDEVICE;
    return SFFT_OK;
  }

  void sched_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      if (stop) return;
      Lane *L = nullptr;
      for (auto &l : lanes)
        if (!l->busy) {
          L = l.get();
          break;
        }
      const int64_t now = now_ns();
      if (!L || pending.empty() || pending.begin()->first > now) {
        if (L && !pending.empty()) {
          const auto at = std::chrono::steady_clock::time_point(
              std::chrono::nanoseconds(pending.begin()->first));
          cv_sched.wait_until(lk, at);
        } else {
          cv_sched.wait(lk);
        }
        continue;
      }
      // released requests in release order, while their workspaces fit
      std::vector<int64_t> tk;
      int64_t est = 0;
      for (auto it = pending.begin(); it != pending.end() && it->first <= now &&
                                      (int)tk.size() < prm.max_batch;) {
        const int64_t b = reqs[(size_t)it->second].bytes;
        if (!tk.empty() && est + b > (int64_t)L->cap) break;
        est += b;
        tk.push_back(it->second);
        it = pending.erase(it);
      }
      L->busy = true;
      lk.unlock();
      std::vector<int64_t> back;
      const int64_t t_launch = now_ns();
      const int32_t rc = launch(*L, tk, back);
      lk.lock();
      for (int64_t t : back) pending.insert({reqs[(size_t)t].release_ns, t});
      for (int64_t t : tk) {
        Req &r = reqs[(size_t)t];
        r.launch_ns = t_launch;
        r.batch = (int32_t)tk.size();
        r.lane = L->id;
      }
      L->tickets = tk;
      L->err = rc;
      L->go = true;
      cv_lane.notify_all();
    }
  }

  void wait_loop(Lane *L) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_lane.wait(lk, [&] { return stop || L->go; });
      if (!L->go) return;
      int32_t rc = L->err;
      lk.unlock();
      if (rc == SFFT_OK && hipEventSynchronize(L->ev) != hipSuccess) rc = SFFT_EDEVICE;
      const int64_t t = now_ns();
      lk.lock();
      for (int64_t k : L->tickets) {
        Req &r = reqs[(size_t)k];
        r.done_ns = t;
        r.status = rc == SFFT_OK ? 1 : rc;
      }
      outstanding -= (int64_t)L->tickets.size();
      L->tickets.clear();
      L->go = false;
      L->busy = false;
      cv_sched.notify_all();
      cv_done.notify_all();
    }
  }

  int64_t plan_bytes(const sfft_plan_s *p) {
    auto it = footprint.find(p);
    if (it != footprint.end()) return it->second;
    Layout Y;
    if (make_layout({p}, false, ncu, Y) != SFFT_OK) return -1;
    footprint[p] = (int64_t)Y.bytes;
    return (int64_t)Y.bytes;
  }
};

extern "C" {

void sfft_server_params_init(sfft_server_params_t *p) {
  memset(p, 0, sizeof(*p));
  p->hbm_bytes = int64_t(8) << 30;
  p->lanes = 2;
  p->max_batch = 256;
}

int64_t sfft_server_clock_ns(void) { return now_ns(); }

sfft_server_t sfft_server_create(const sfft_server_params_t *p) {
  if (!p || p->lanes < 1 || p->lanes > 8 || p->max_batch < 1 || p->max_batch > 65536 ||
      p->hbm_bytes < p->lanes * (int64_t(1) << 20)) {
    set_last_error(SFFT_EINVAL);
    return nullptr;
  }
  std::unique_ptr<sfft_server_s> s(new sfft_server_s());
  s->prm = *p;
  if (hipGetDevice(&s->device) != hipSuccess || device_twiddles(s->device, &s->tw) != hipSuccess) {
    set_last_error(SFFT_EDEVICE);
    return nullptr;
  }
  s->ncu = device_cus(s->device);
  const size_t cap = (size_t)(p->hbm_bytes / p->lanes) & ~size_t(255);
  // staging: descriptors, lists (at most 3 n + 3 entries) and pointers of a full batch
  const size_t stage = (sizeof(SigDesc) + sizeof(SigIO) + 4 * sizeof(int32_t)) * (size_t)p->max_batch + 64;
  for (int i = 0; i < p->lanes; i++) {
    std::unique_ptr<Lane> L(new Lane());
    L->id = i;
    L->cap = cap;
    L->staging_cap = stage;
    if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L->ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&L->staging, stage, 0) != hipSuccess) {
      s->lanes.push_back(std::move(L));
      set_last_error(SFFT_EDEVICE);
      return nullptr;
    }
    if (hipMalloc(&L->slab, cap) != hipSuccess) {
      (void)hipGetLastError();
      s->lanes.push_back(std::move(L));
      set_last_error(SFFT_ENOMEM);
      return nullptr;
    }
    s->lanes.push_back(std::move(L));
  }
  sfft_server_s *sp = s.get();
  for (auto &l : s->lanes) {
    Lane *lp = l.get();
    l->waiter = std::thread([sp, lp] { sp->wait_loop(lp); });
  }
  s->sched = std::thread([sp] { sp->sched_loop(); });
  return s.release();
}

int32_t sfft_server_submit_many(sfft_server_t s, int32_t n, const sfft_plan_t *plans,
                                const void *const *xs, int64_t *const *idx, void *const *vals,
                                int64_t *d_counts, int32_t *d_status, const int64_t *release_ns,
                                int64_t *tickets) {
  if (!s || n < 1 || !plans || !xs || !idx || !vals || !d_counts || !d_status)
    return set_last_error(SFFT_EINVAL);
  if (!is_device_ptr(d_counts) || !is_device_ptr(d_status)) return set_last_error(SFFT_EINVAL);
  std::vector<int64_t> bytes((size_t)n);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i = 0; i < n; i++) {
      if (!plans[i]) return set_last_error(SFFT_EINVAL);
      bytes[(size_t)i] = s->plan_bytes(plans[i]);
      if (bytes[(size_t)i] < 0) return set_last_error(SFFT_EINVAL);
      if ((size_t)bytes[(size_t)i] > s->lanes[0]->cap) return set_last_error(SFFT_ETOOBIG);
    }
  }
  for (int i = 0; i < n; i++)
    if (!is_device_ptr(xs[i]) || !is_device_ptr(idx[i]) || !is_device_ptr(vals[i]))
      return set_last_error(SFFT_EINVAL);
  const int64_t now = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_last_error(SFFT_EINVAL);
    for (int i = 0; i < n; i++) {
      Req r{};
      r.plan = plans[i];
      r.io.x = (const float2 *)xs[i];
      r.io.idx = idx[i];
      r.io.val = (float2 *)vals[i];
      r.io.count = d_counts + i;
      r.io.status = d_status + i;
      r.bytes = bytes[(size_t)i];
      r.release_ns = (release_ns && release_ns[i] > 0) ? release_ns[i] : now;
      const int64_t t = (int64_t)s->reqs.size();
      s->reqs.push_back(r);
      s->pending.insert({r.release_ns, t});
      s->outstanding++;
      if (tickets) tickets[i] = t;
    }
  }
  s->cv_sched.notify_all();
  return SFFT_OK;
}

int64_t sfft_server_submit(sfft_server_t s, sfft_plan_t plan, const void *x, int64_t *out_idx,
                           void *out_val, int64_t *d_count, int32_t *d_status, int64_t release_ns) {
  int64_t t = -1;
  const void *xs[1] = {x};
  int64_t *ix[1] = {out_idx};
  void *vs[1] = {out_val};
  const int32_t rc = sfft_server_submit_many(s, 1, &plan, xs, ix, vs, d_count, d_status, &release_ns, &t);
  return rc == SFFT_OK ? t : rc;
}

int32_t sfft_server_requests(sfft_server_t s, int64_t first, int32_t n, sfft_request_t *out) {
  if (!s || !out || first < 0 || n < 0) return set_last_error(SFFT_EINVAL);
  std::lock_guard<std::mutex> lk(s->mu);
  if (first + n > (int64_t)s->reqs.size()) return set_last_error(SFFT_EINVAL);
  for (int32_t i = 0; i < n; i++) {
    const Req &r = s->reqs[(size_t)(first + i)];
    sfft_request_t &o = out[i];
    memset(&o, 0, sizeof(o));
    o.release_ns = r.release_ns;
    o.launch_ns = r.launch_ns;
    o.done_ns = r.done_ns;
    o.batch = r.batch;
    o.lane = r.lane;
    o.status = r.status;
  }
  return SFFT_OK;
}

int32_t sfft_server_wait(sfft_server_t s, int64_t ticket) {
  if (!s || ticket < 0) return set_last_error(SFFT_EINVAL);
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket >= (int64_t)s->reqs.size()) return set_last_error(SFFT_EINVAL);
  s->cv_done.wait(lk, [&] { return s->reqs[(size_t)ticket].status != 0; });
  const int32_t st = s->reqs[(size_t)ticket].status;
  return st == 1 ? SFFT_OK : set_last_error(st);
}

int32_t sfft_server_drain(sfft_server_t s) {
  if (!s) return set_last_error(SFFT_EINVAL);
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  for (const Req &r : s->reqs)
    if (r.status < 0) return set_last_error(r.status);
  return SFFT_OK;
}

void sfft_server_destroy(sfft_server_t s) {
  if (!s) return;
  (void)sfft_server_drain(s);
  delete s;
}

}  // extern "C"
