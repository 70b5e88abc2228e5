// Serving runtime: continuous batching of single QPs of uneven sizes.
//
// A scheduler thread owns one HIP stream and a device arena.  Each step it
//  1. admits queued requests while a slot is free and the arena has room for
//     the request's footprint (inputs + iterate + factor storage if the
//     factor does not fit LDS), copying the request's data into the arena;
//  2. launches the serving kernel once per size bucket (threads per QP,
//     rows-per-lane variant, factor placement); every resident QP resumes
//     its Newton loop from the iterate kept in the arena for at most
//     `iters_per_step` iterations (a fresh QP first runs the initialisation);
//  3. reads back the per-slot status and retires finished QPs (converged,
//     failed, or out of iterations), copying their solution to the host and
//     freeing their arena space and slot for the next admissions.
// Requests that arrive while others are on the device join at the next step,
// so work of different requests overlaps on the GPU.  Each QP's arithmetic
// is independent of the others in its launch, and resuming from a stored
// iterate repeats exactly what an uninterrupted solve computes, so a request
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
  bool fresh = false;  // admitted this step: the kernel runs the initialisation
  // arena placement (floats offsets relative to the request's block)
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
  r->o_G = take(m * n); r->o_h = take(m); r->o_state = take(n + p + 2 * m);
  r->o_ws = r->plan.m_in_lds ? 0 : take((size_t)r->plan.ws_stride);
  r->bytes = o;
}

struct Bucket {
  int threads;
  int rpl;
  bool mlds;
};
bool operator<(const Bucket &a, const Bucket &b) {
  if (a.threads != b.threads) return a.threads < b.threads;
  if (a.rpl != b.rpl) return a.rpl < b.rpl;
  return a.mlds < b.mlds;
}

}  // namespace

struct qpx_server {
  qpx_ctx *ctx = nullptr;
  qp_server_opts o{};
  qp_opts so{};
  hipStream_t stream = nullptr;
  // size-class buckets of one device step run concurrently on the main
  // stream and these (all at the default priority); events order them after
  // the descriptor upload and before the status download
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t ev_ready = nullptr, ev_done[kSide] = {};
  char *arena_dev = nullptr;
  Arena arena;
  qpk::SlotDesc *d_desc = nullptr, *h_desc = nullptr;
  int32_t *d_status = nullptr, *d_iters = nullptr, *h_status = nullptr, *h_iters = nullptr;
  float *d_res = nullptr, *h_res = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> by_ticket;
  std::vector<Request *> active;
  std::thread th;
  std::atomic<bool> stop{false};
  std::atomic<int> error{0};
  uint64_t next_ticket = 1, admitted = 0, completed = 0;
  int peak = 0;
};

namespace {

void scheduler(qpx_server *S) {
  if (hipSetDevice(S->ctx->device) != hipSuccess) {
    S->error = QPX_ERR_HIP;
    return;
  }
  std::vector<Request *> fresh;
  for (;;) {
    fresh.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while ((int)S->active.size() < S->o.max_slots && !S->pending.empty()) {
        Request *r = S->pending.front();
        size_t off;
        if (!S->arena.alloc(r->bytes, &off)) break;  // wait for memory to free up
        S->pending.pop_front();
        r->off = off;
        r->t_admit = now_s();
        r->fresh = true;
        S->active.push_back(r);
        fresh.push_back(r);
        ++S->admitted;
      }
      S->peak = std::max(S->peak, (int)S->active.size());
      if (S->active.empty()) {
        if (S->stop) return;
        S->cv.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
    }
    // copy the admitted requests' data into the arena
    for (Request *r : fresh) {
      char *base = S->arena_dev + r->off;
      const size_t n = r->n, m = r->m, p = r->p;
      const float *src = r->data.data();
      auto put = [&](size_t o, size_t floats) {
        if (floats) (void)hipMemcpyAsync(base + o, src, floats * 4, hipMemcpyHostToDevice, S->stream);
        src += floats;
      };
      put(r->o_Q, n * n); put(r->o_q, n); put(r->o_A, p * n); put(r->o_b, p);
      put(r->o_G, m * n); put(r->o_h, m);
    }
    // descriptors grouped by bucket
    std::map<Bucket, std::vector<int>> groups;
    for (int i = 0; i < (int)S->active.size(); ++i) {
      const Request *r = S->active[i];
      const int N = r->n + r->plan.kb + r->p;
      groups[Bucket{r->plan.threads, (N + 63) / 64, r->plan.m_in_lds}].push_back(i);
    }
    std::vector<int> order;
    order.reserve(S->active.size());
    for (auto &g : groups) order.insert(order.end(), g.second.begin(), g.second.end());
    for (int k = 0; k < (int)order.size(); ++k) {
      const Request *r = S->active[order[k]];
      char *base = S->arena_dev + r->off;
      qpk::SlotDesc &d = S->h_desc[k];
      d.n = r->n; d.m = r->m; d.p = r->p; d.kb = r->plan.kb;
      d.flags = (r->fresh ? 1 : 0) | (r->plan.amode << 1);
      d.Q = (const float *)(base + r->o_Q); d.q = (const float *)(base + r->o_q);
      d.A = r->p ? (const float *)(base + r->o_A) : nullptr;
      d.b = r->p ? (const float *)(base + r->o_b) : nullptr;
      d.G = r->m ? (const float *)(base + r->o_G) : nullptr;
      d.h = r->m ? (const float *)(base + r->o_h) : nullptr;
      d.state = (float *)(base + r->o_state);
      d.ws = r->plan.m_in_lds ? nullptr : (float *)(base + r->o_ws);
      d.status = S->d_status + k; d.iters = S->d_iters + k; d.res = S->d_res + k;
    }
    (void)hipMemcpyAsync(S->d_desc, S->h_desc, order.size() * sizeof(qpk::SlotDesc),
                         hipMemcpyHostToDevice, S->stream);
    // one launch per bucket; the buckets, largest estimated cost first, are
    // dealt to the main and side streams so a step lasts about as long as
    // its most expensive bucket rather than the sum of all of them
    struct Launch { Bucket b; int k0, cnt; size_t lds; double cost; };
    std::vector<Launch> launches;
    int k0 = 0;
    for (auto &g : groups) {
      const int cnt = (int)g.second.size();
      size_t lds = 0;
      double cost = 0.0;
      for (int idx : g.second) {
        const Request *r = S->active[idx];
        lds = std::max(lds, r->plan.lds);
        const double N = r->n + r->plan.kb + r->p;
        cost += N * N * N;
      }
      launches.push_back(Launch{g.first, k0, cnt, lds, cost});
      k0 += cnt;
    }
    std::sort(launches.begin(), launches.end(),
              [](const Launch &a, const Launch &b) { return a.cost > b.cost; });
    const int nstreams = 1 + S->kSide;
    bool used[1 + qpx_server::kSide] = {};
    (void)hipEventRecord(S->ev_ready, S->stream);
    for (size_t j = 0; j < launches.size(); ++j) {
      const Launch &L = launches[j];
      const int si = (int)(j % nstreams);
      hipStream_t st = si == 0 ? S->stream : S->side[si - 1];
      if (si > 0 && !used[si]) (void)hipStreamWaitEvent(st, S->ev_ready, 0);
      used[si] = true;
      qpk::Params P;
      std::memset(&P, 0, sizeof(P));
      P.n = 64 * L.b.rpl;  // dispatch only: rows-per-lane variant
      // small size classes run more iterations per step (their launches end
      // well before the largest class's); the iterate persists between
      // steps, so how iterations are split over steps does not change them
      const int mult = L.b.rpl <= 1 ? 4 : (L.b.rpl <= 2 ? 2 : 1);
      P.form = S->so.form; P.max_iter = S->o.iters_per_step * mult; P.pc = S->so.pc;
      P.tol = S->so.tol; P.sigma = S->so.sigma; P.delta_reg = S->so.delta_reg;
      P.refine = S->so.refine_steps;
      P.desc = S->d_desc + L.k0;
      P.mode = qpk::kServe;
      if (qpk::launch(P, L.b.threads, L.b.mlds, L.lds, L.cnt, st) != hipSuccess) S->error = QPX_ERR_HIP;
    }
    for (int si = 1; si < nstreams; ++si) {
      if (!used[si]) continue;
      (void)hipEventRecord(S->ev_done[si - 1], S->side[si - 1]);
      (void)hipStreamWaitEvent(S->stream, S->ev_done[si - 1], 0);
    }
    const size_t na = order.size();
    (void)hipMemcpyAsync(S->h_status, S->d_status, na * 4, hipMemcpyDeviceToHost, S->stream);
    (void)hipMemcpyAsync(S->h_iters, S->d_iters, na * 4, hipMemcpyDeviceToHost, S->stream);
    if (hipStreamSynchronize(S->stream) != hipSuccess) S->error = QPX_ERR_HIP;
    // retire finished QPs
    std::vector<Request *> keep, done;
    for (int k = 0; k < (int)na; ++k) {
      Request *r = S->active[order[k]];
      r->iters += S->h_iters[k];
      const int st = S->h_status[k] & 0xff;
      const bool running = st == 1 && r->iters < S->so.max_iter;
      r->fresh = false;
      if (running) {
        keep.push_back(r);
      } else {
        r->status = S->h_status[k];
        done.push_back(r);
      }
    }
    for (Request *r : done) {
      r->sol.resize((size_t)r->n + r->p + 2 * r->m);
      (void)hipMemcpyAsync(r->sol.data(), S->arena_dev + r->off + r->o_state, r->sol.size() * 4,
                           hipMemcpyDeviceToHost, S->stream);
    }
    if (!done.empty() && hipStreamSynchronize(S->stream) != hipSuccess) S->error = QPX_ERR_HIP;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t = now_s();
      for (Request *r : done) {
        S->arena.release(r->off, r->bytes);
        r->t_done = t;
        r->done = true;
        std::vector<float>().swap(r->data);
        ++S->completed;
      }
      S->active.swap(keep);
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
  if (hipSetDevice(ctx->device) != hipSuccess) { delete S; return QPX_ERR_HIP; }
  bool ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i < qpx_server::kSide; ++i) {
    ok = ok && hipStreamCreateWithFlags(&S->side[i], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&S->ev_done[i], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreateWithFlags(&S->ev_ready, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipMalloc(&S->arena_dev, S->o.arena_bytes) == hipSuccess;
  const size_t ns = S->o.max_slots;
  ok = ok && hipMalloc(&S->d_desc, ns * sizeof(qpk::SlotDesc)) == hipSuccess;
  ok = ok && hipMalloc(&S->d_status, ns * 4) == hipSuccess;
  ok = ok && hipMalloc(&S->d_iters, ns * 4) == hipSuccess;
  ok = ok && hipMalloc(&S->d_res, ns * 4) == hipSuccess;
  ok = ok && hipHostMalloc(&S->h_desc, ns * sizeof(qpk::SlotDesc), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(&S->h_status, ns * 4, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(&S->h_iters, ns * 4, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc(&S->h_res, ns * 4, hipHostMallocDefault) == hipSuccess;
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
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (int i = 0; i < qpx_server::kSide; ++i)
    if (S->side[i]) (void)hipStreamSynchronize(S->side[i]);
  for (auto &kv : S->by_ticket) delete kv.second;
  if (S->arena_dev) (void)hipFree(S->arena_dev);
  if (S->d_desc) (void)hipFree(S->d_desc);
  if (S->d_status) (void)hipFree(S->d_status);
  if (S->d_iters) (void)hipFree(S->d_iters);
  if (S->d_res) (void)hipFree(S->d_res);
  if (S->h_desc) (void)hipHostFree(S->h_desc);
  if (S->h_status) (void)hipHostFree(S->h_status);
  if (S->h_iters) (void)hipHostFree(S->h_iters);
  if (S->h_res) (void)hipHostFree(S->h_res);
  for (int i = 0; i < qpx_server::kSide; ++i) {
    if (S->ev_done[i]) (void)hipEventDestroy(S->ev_done[i]);
    if (S->side[i]) (void)hipStreamDestroy(S->side[i]);
  }
  if (S->ev_ready) (void)hipEventDestroy(S->ev_ready);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
  return QPX_OK;
}

}  // extern "C"
