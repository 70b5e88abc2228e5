// Serving runtime: continuous batching of single QPs of uneven sizes.
//
// A scheduler thread owns a device arena and kLanes streams ("lanes").
// Resident QPs are grouped into size-class buckets (threads per QP,
// rows-per-lane variant, factor placement).  Whenever a lane is idle, the
// scheduler
//  1. admits queued requests while a slot is free and the arena has room for
//     the request's footprint (inputs + iterate + factor storage if the
//     factor does not fit LDS);
//  2. launches the serving kernel on the lane for one bucket of resident QPs
//     that are not in flight (the bucket holding the longest-waiting QP):
//     the new requests' data are uploaded first on the same stream, every QP
//     resumes its Newton loop from the iterate kept in the arena for a
//     bounded number of iterations (a fresh QP first runs the
//     initialisation), and the kernel also writes each QP's iterate to the
//     lane's staging buffer, which comes back to the host with the status
//     words in the same stream;
//  3. when a lane's launch has completed (polled with an event), retires
//     the QPs of that launch that finished (converged, failed, or out of
//     iterations), copying their solution from the staging buffer, and
//     frees their arena space and slot.
// Lanes complete independently: a bucket of small QPs is retired, refilled
// and launched again while a bucket of large ones is still running, and
// one lane serves only the small size classes, so a small request's latency
// does not wait for the largest size class.
// Requests that arrive while others are on the device join at the next
// launch of their bucket.  Each QP's arithmetic is independent of the others
// in its launch, its per-launch iteration budget depends only on its own
// size and progress, and resuming from the stored iterate and arithmetic
// state repeats exactly what an uninterrupted solve computes, so a request
// gives the same result alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/qpx.h"
#include "qp_internal.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

struct Request {
  uint64_t ticket = 0;
  int n = 0, m = 0, p = 0;
  qpk::Plan plan;
  std::vector<float> data;  // Q q A b G h, packed
  std::vector<float> sol;   // x y z s
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = 0, iters = 0;
  bool done = false;
  bool fresh = false;      // not yet launched: the kernel runs the initialisation
  bool in_flight = false;  // part of a launch that has not completed
  uint64_t order = 0;      // admission order (oldest bucket first)
  // arena placement (byte offsets relative to the request's block)
  size_t off = 0, bytes = 0;
  size_t o_Q, o_q, o_A, o_b, o_G, o_h, o_state, o_ws;
};

// First-fit allocator over [0, size) with coalescing of free blocks.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
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

 private:
  std::map<size_t, size_t> free_;
};

void layout_request(Request *r) {
  const size_t n = r->n, m = r->m, p = r->p;
  size_t o = 0;
  auto take = [&](size_t floats) { size_t b = o; o += al256(floats * 4); return b; };
  r->o_Q = take(n * n); r->o_q = take(n); r->o_A = take(p * n); r->o_b = take(p);
  r->o_G = take(m * n); r->o_h = take(m); r->o_state = take(n + p + 2 * m + 1);
  r->o_ws = r->plan.m_in_lds ? 0 : take((size_t)r->plan.ws_stride);
  r->bytes = o;
}

struct Bucket {
  int threads;
  int rpl;
  bool mlds;
};

// Floats of a request's iterate (x, y, z, s), and of its place in a lane's
// staging buffer (64-float aligned).
size_t state_floats(int n, int m, int p) { return (size_t)n + p + 2 * (size_t)m; }
size_t staged_floats(const Request *r) { return (state_floats(r->n, r->m, r->p) + 63) & ~size_t(63); }

// One stream with the buffers of the launch in flight on it.
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  qpk::SlotDesc *d_desc = nullptr, *h_desc = nullptr;
  int32_t *d_status = nullptr, *d_iters = nullptr, *h_status = nullptr, *h_iters = nullptr;
  float *d_res = nullptr;
  float *d_out = nullptr, *h_out = nullptr;  // staging of the iterates
  std::vector<Request *> batch;              // the launch in flight (launch order)
  std::vector<size_t> out_off;               // each QP's place in the staging buffer
  bool busy = false;
};

}  // namespace

struct qpx_server {
  qpx_ctx *ctx = nullptr;
  qp_server_opts o{};
  qp_opts so{};
  // lanes run at the default stream priority
  static constexpr int kLanes = 4;
  Lane lane[kLanes];
  size_t staging = 0;  // staging buffer floats per lane
  char *arena_dev = nullptr;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> by_ticket;
  std::vector<Request *> active;  // resident (admitted, not retired)
  std::thread th;
  std::atomic<bool> stop{false};
  std::atomic<int> error{0};
  uint64_t next_ticket = 1, admitted = 0, completed = 0, admit_order = 0;
  int peak = 0;
};

namespace {

Bucket bucket_of(const Request *r) {
  const int N = r->n + r->plan.kb + r->p;
  return Bucket{r->plan.threads, (N + 63) / 64, r->plan.m_in_lds};
}

// Launch one bucket of idle resident QPs on lane L.  Called with S->mu held
// (reads the active list).  With small_only, only buckets of systems of at
// most 128 rows qualify.  Returns false if nothing was launched.
bool launch_bucket(qpx_server *S, Lane &L, bool small_only) {
  // the bucket of the longest-waiting idle QP
  const Request *oldest = nullptr;
  for (const Request *r : S->active)
    if (!r->in_flight && (!small_only || bucket_of(r).rpl <= 2) &&
        (!oldest || r->order < oldest->order))
      oldest = r;
  if (!oldest) return false;
  const Bucket bk = bucket_of(oldest);
  std::vector<Request *> cand;
  for (Request *r : S->active) {
    if (r->in_flight) continue;
    const Bucket b = bucket_of(r);
    if (b.threads == bk.threads && b.rpl == bk.rpl && b.mlds == bk.mlds) cand.push_back(r);
  }
  std::sort(cand.begin(), cand.end(),
            [](const Request *a, const Request *b) { return a->order < b->order; });
  // oldest first, as many as the staging buffer holds (at least one)
  L.batch.clear();
  L.out_off.clear();
  size_t lds = 0, used = 0;
  for (Request *r : cand) {
    const size_t f = staged_floats(r);
    if (!L.batch.empty() && used + f > S->staging) break;
    L.batch.push_back(r);
    L.out_off.push_back(used);
    used += f;
    lds = std::max(lds, r->plan.lds);
  }
  // data of QPs launched for the first time, then the descriptors
  for (Request *r : L.batch) {
    r->in_flight = true;
    if (!r->fresh) continue;
    char *base = S->arena_dev + r->off;
    const size_t n = r->n, m = r->m, p = r->p;
    const float *src = r->data.data();
    auto put = [&](size_t o, size_t floats) {
      if (floats) (void)hipMemcpyAsync(base + o, src, floats * 4, hipMemcpyHostToDevice, L.stream);
      src += floats;
    };
    put(r->o_Q, n * n); put(r->o_q, n); put(r->o_A, p * n); put(r->o_b, p);
    put(r->o_G, m * n); put(r->o_h, m);
  }
  for (int k = 0; k < (int)L.batch.size(); ++k) {
    const Request *r = L.batch[k];
    char *base = S->arena_dev + r->off;
    qpk::SlotDesc &d = L.h_desc[k];
    std::memset(&d, 0, sizeof(d));
    d.n = r->n; d.m = r->m; d.p = r->p; d.kb = r->plan.kb;
    d.flags = (r->fresh ? 1 : 0) | (r->plan.amode << 1);
    // small size classes run more iterations per launch (their launches end
    // well before the largest class's); the iterate persists between
    // launches, so how iterations are split over them does not change them.
    // No QP runs past max_iter in total.
    const int mult = bk.rpl <= 1 ? 4 : (bk.rpl <= 2 ? 2 : 1);
    d.budget = std::min(S->o.iters_per_step * mult, S->so.max_iter - r->iters);
    d.Q = (const float *)(base + r->o_Q); d.q = (const float *)(base + r->o_q);
    d.A = r->p ? (const float *)(base + r->o_A) : nullptr;
    d.b = r->p ? (const float *)(base + r->o_b) : nullptr;
    d.G = r->m ? (const float *)(base + r->o_G) : nullptr;
    d.h = r->m ? (const float *)(base + r->o_h) : nullptr;
    d.state = (float *)(base + r->o_state);
    d.ws = r->plan.m_in_lds ? nullptr : (float *)(base + r->o_ws);
    d.out = L.d_out + L.out_off[k];
    d.status = L.d_status + k; d.iters = L.d_iters + k; d.res = L.d_res + k;
  }
  const int cnt = (int)L.batch.size();
  (void)hipMemcpyAsync(L.d_desc, L.h_desc, cnt * sizeof(qpk::SlotDesc), hipMemcpyHostToDevice,
                       L.stream);
  qpk::Params P;
  std::memset(&P, 0, sizeof(P));
  P.n = 64 * bk.rpl;  // dispatch only: rows-per-lane variant
  P.form = S->so.form; P.max_iter = S->so.max_iter; P.pc = S->so.pc;
  P.tol = S->so.tol; P.sigma = S->so.sigma; P.delta_reg = S->so.delta_reg;
  P.refine = S->so.refine_steps;
  P.rmode = S->so.fp64_residual;
  P.backoff = S->so.backoff > 0.f ? S->so.backoff : (S->so.form == QPX_STANDARD ? 0.99f : 1.f);
  P.desc = L.d_desc;
  P.mode = qpk::kServe;
  if (qpk::launch(P, bk.threads, bk.mlds, lds, cnt, L.stream) != hipSuccess) S->error = QPX_ERR_HIP;
  (void)hipMemcpyAsync(L.h_status, L.d_status, cnt * 4, hipMemcpyDeviceToHost, L.stream);
  (void)hipMemcpyAsync(L.h_iters, L.d_iters, cnt * 4, hipMemcpyDeviceToHost, L.stream);
  (void)hipMemcpyAsync(L.h_out, L.d_out, used * 4, hipMemcpyDeviceToHost, L.stream);
  (void)hipEventRecord(L.done, L.stream);
  L.busy = true;
  return true;
}

// Retire the finished QPs of lane L's completed launch.  Called with S->mu.
void complete_lane(qpx_server *S, Lane &L) {
  const double t = now_s();
  std::vector<Request *> keep;
  keep.reserve(S->active.size());
  for (int k = 0; k < (int)L.batch.size(); ++k) {
    Request *r = L.batch[k];
    r->in_flight = false;
    r->fresh = false;
    r->iters += L.h_iters[k];
    const int st = L.h_status[k] & 0xff;
    if (st == 1 && r->iters < S->so.max_iter) continue;  // still running
    r->status = L.h_status[k];
    const float *src = L.h_out + L.out_off[k];
    r->sol.assign(src, src + state_floats(r->n, r->m, r->p));
    S->arena.release(r->off, r->bytes);
    r->t_done = t;
    r->done = true;
    std::vector<float>().swap(r->data);
    ++S->completed;
  }
  for (Request *r : S->active)
    if (!r->done) keep.push_back(r);
  S->active.swap(keep);
  L.batch.clear();
  L.busy = false;
}

void scheduler(qpx_server *S) {
  if (hipSetDevice(S->ctx->device) != hipSuccess) {
    S->error = QPX_ERR_HIP;
    return;
  }
  for (;;) {
    bool progress = false;
    std::unique_lock<std::mutex> lk(S->mu);
    // retire completed launches
    for (Lane &L : S->lane) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) S->error = QPX_ERR_HIP;
      complete_lane(S, L);
      progress = true;
    }
    // admit while slots and arena space last
    while ((int)S->active.size() < S->o.max_slots && !S->pending.empty()) {
      Request *r = S->pending.front();
      size_t off;
      if (!S->arena.alloc(r->bytes, &off)) break;  // wait for memory to free up
      S->pending.pop_front();
      r->off = off;
      r->t_admit = now_s();
      r->fresh = true;
      r->order = S->admit_order++;
      S->active.push_back(r);
      ++S->admitted;
      progress = true;
    }
    S->peak = std::max(S->peak, (int)S->active.size());
    // launch on idle lanes; lane 0 serves only the small size classes, so
    // their launches (a few milliseconds) never wait behind the large ones
    for (int li = 0; li < qpx_server::kLanes; ++li) {
      Lane &L = S->lane[li];
      if (!L.busy && launch_bucket(S, L, li == 0)) progress = true;
    }
    bool any_busy = false;
    for (Lane &L : S->lane) any_busy |= L.busy;
    if (!any_busy && S->active.empty() && S->pending.empty() && S->stop) return;
    if (!progress) {
      if (!any_busy) S->cv.wait_for(lk, std::chrono::milliseconds(1));
      else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  }
}

}  // namespace

extern "C" {

int qp_server_create(qpx_ctx *ctx, const qp_server_opts *opts, const qp_opts *solver,
                     qpx_server **srv) {
  if (!srv) return QPX_ERR_ARG;
  *srv = nullptr;
  if (!ctx) return QPX_ERR_ARG;
  qpx_server *S = new (std::nothrow) qpx_server();
  if (!S) return QPX_ERR_OOM;
  S->ctx = ctx;
  S->o.max_slots = 256;
  S->o.iters_per_step = 4;
  S->o.n_max = 256;
  S->o.arena_bytes = 0;
  if (opts) S->o = *opts;
  if (S->o.arena_bytes == 0) S->o.arena_bytes = (size_t)256 << 20;
  if (solver) S->so = *solver; else qp_default_opts(&S->so);
  if (S->o.max_slots < 1 || S->o.max_slots > 65536 || S->o.iters_per_step < 1 ||
      S->o.n_max < 1 || S->o.n_max > qpk::kMaxN || !(S->so.tol > 0.f) || S->so.max_iter < 1) {
    delete S;
    return QPX_ERR_ARG;
  }
  // staging per lane: max_slots iterates of n_max variables with m = 2 n_max,
  // and at least one of the largest a request may have (m <= 4096); a launch
  // takes as many QPs as fit
  S->staging = std::max((size_t)S->o.max_slots * (state_floats(S->o.n_max, 2 * S->o.n_max,
                                                               S->o.n_max) + 64),
                        state_floats(S->o.n_max, 4096, S->o.n_max) + 64);
  if (hipSetDevice(ctx->device) != hipSuccess) { delete S; return QPX_ERR_HIP; }
  const size_t ns = S->o.max_slots;
  bool ok = hipMalloc(&S->arena_dev, S->o.arena_bytes) == hipSuccess;
  for (Lane &L : S->lane) {
    ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L.done, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(&L.d_desc, ns * sizeof(qpk::SlotDesc)) == hipSuccess;
    ok = ok && hipMalloc(&L.d_status, ns * 4) == hipSuccess;
    ok = ok && hipMalloc(&L.d_iters, ns * 4) == hipSuccess;
    ok = ok && hipMalloc(&L.d_res, ns * 4) == hipSuccess;
    ok = ok && hipMalloc(&L.d_out, S->staging * 4) == hipSuccess;
    ok = ok && hipHostMalloc(&L.h_desc, ns * sizeof(qpk::SlotDesc), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(&L.h_status, ns * 4, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(&L.h_iters, ns * 4, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(&L.h_out, S->staging * 4, hipHostMallocDefault) == hipSuccess;
  }
  if (!ok) {
    qp_server_destroy(S);
    return QPX_ERR_OOM;
  }
  S->arena.reset(S->o.arena_bytes);
  S->th = std::thread(scheduler, S);
  *srv = S;
  return QPX_OK;
}

int qp_serve_submit(qpx_server *S, int32_t n, int32_t m, int32_t p, const float *Q,
                    const float *q, const float *A, const float *b, const float *G,
                    const float *h, uint64_t *ticket) {
  if (!S || !ticket) return QPX_ERR_ARG;
  if (S->stop) return QPX_ERR_STATE;
  if (const int e = S->error.load()) return e;
  if (n < 1 || m < 0 || p < 0 || p >= n || n > S->o.n_max) return QPX_ERR_ARG;
  if (!Q || !q || (p && (!A || !b)) || (m && (!G || !h))) return QPX_ERR_ARG;
  Request *r = new (std::nothrow) Request();
  if (!r) return QPX_ERR_OOM;
  r->n = n; r->m = m; r->p = p;
  int rc = qpk::make_plan(n, m, p, S->so, &r->plan);
  if (rc) { delete r; return rc; }
  layout_request(r);
  if (r->bytes > S->o.arena_bytes) { delete r; return QPX_ERR_ARG; }
  const size_t nn = n, mm = m, pp = p;
  try {
    r->data.resize(nn * nn + nn + pp * nn + pp + mm * nn + mm);
  } catch (...) {
    delete r;
    return QPX_ERR_OOM;
  }
  float *d = r->data.data();
  std::memcpy(d, Q, nn * nn * 4); d += nn * nn;
  std::memcpy(d, q, nn * 4); d += nn;
  if (pp) { std::memcpy(d, A, pp * nn * 4); d += pp * nn; std::memcpy(d, b, pp * 4); d += pp; }
  if (mm) { std::memcpy(d, G, mm * nn * 4); d += mm * nn; std::memcpy(d, h, mm * 4); }
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    S->by_ticket[r->ticket] = r;
    S->pending.push_back(r);
  }
  S->cv.notify_one();
  *ticket = r->ticket;
  return QPX_OK;
}

int qp_serve_poll(qpx_server *S, uint64_t ticket, float *x, float *y, float *z, float *s,
                  qp_timing *timing) {
  if (!S) return QPX_ERR_ARG;
  Request *r;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->by_ticket.find(ticket);
    if (it == S->by_ticket.end()) return QPX_ERR_ARG;
    r = it->second;
    if (!r->done) {
      const int e = S->error.load();
      return e ? e : QPX_PENDING;
    }
    S->by_ticket.erase(it);
  }
  const size_t n = r->n, m = r->m, p = r->p;
  const float *st = r->sol.data();
  if (x) std::memcpy(x, st, n * 4);
  if (y && p) std::memcpy(y, st + n, p * 4);
  if (z && m) std::memcpy(z, st + n + p, m * 4);
  if (s && m) std::memcpy(s, st + n + p + m, m * 4);
  if (timing) {
    timing->t_submit = r->t_submit;
    timing->t_admit = r->t_admit;
    timing->t_done = r->t_done;
    timing->status = r->status;
    timing->iters = r->iters;
  }
  delete r;
  return QPX_OK;
}

int qp_serve_stats(qpx_server *S, uint64_t *admitted, uint64_t *completed, int32_t *peak) {
  if (!S) return QPX_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (admitted) *admitted = S->admitted;
  if (completed) *completed = S->completed;
  if (peak) *peak = S->peak;
  return QPX_OK;
}

int qp_server_destroy(qpx_server *S) {
  if (!S) return QPX_OK;
  S->stop = true;
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  for (Lane &L : S->lane)
    if (L.stream) (void)hipStreamSynchronize(L.stream);
  for (auto &kv : S->by_ticket) delete kv.second;
  if (S->arena_dev) (void)hipFree(S->arena_dev);
  for (Lane &L : S->lane) {
    if (L.d_desc) (void)hipFree(L.d_desc);
    if (L.d_status) (void)hipFree(L.d_status);
    if (L.d_iters) (void)hipFree(L.d_iters);
    if (L.d_res) (void)hipFree(L.d_res);
    if (L.d_out) (void)hipFree(L.d_out);
    if (L.h_desc) (void)hipHostFree(L.h_desc);
    if (L.h_status) (void)hipHostFree(L.h_status);
    if (L.h_iters) (void)hipHostFree(L.h_iters);
    if (L.h_out) (void)hipHostFree(L.h_out);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  delete S;
  return QPX_OK;
}

}  // extern "C"
