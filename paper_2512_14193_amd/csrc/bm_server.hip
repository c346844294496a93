// Request server for contour solves (declared in include/bm.h).
//
// A worker thread owns `lanes` HIP streams and a cache of problem handles keyed
// by (lane, N, reuse_key).  It admits queued requests in submission order,
// enqueues each one's work on a lane (assembly, factorisation, solve, error-flag
// readback, two timing events) and polls the completion events of the requests
// in flight.  Requests with N <= concurrent_max_n run side by side on different
// lanes; a larger request is fenced on the device against every other lane
// after its assembly (it then waits for the work already enqueued there), so that
// it forms its Schur complement alone; later requests wait for that, not for its
// LU, which runs beside them.  The host enqueues up to max_inflight requests per lane
// ahead, so the device never waits for the host.  (The lanes' streams only run
// side by side if the process has enough hardware queues: GPU_MAX_HW_QUEUES.)
//
// Why concurrency is limited to small problems: the panel factorisation needs
// its P workgroups resident at once (P = ceil(rows / 64) <= 16 for N <= 1024).
// With lanes * P <= CUs / 2 every panel of every lane fits beside the others,
// and each kernel of a small request is short (well under a millisecond at
// N <= 1024), so a panel workgroup waits at most that long for a free CU.  A
// large request's Schur complement GEMM occupies every CU for tens of
// milliseconds, which could hold off another lane's panel for as long.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bm_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct srv_handle {
  bm_problem *p = nullptr;
  int lane = 0;
  int n = 0;
  uint64_t key = 0;
  int bslot = 0;           // position in a batched factorisation (one handle each)
  int64_t bytes = 0;
  bool factored = false;   // factors for `prm` are (or will be, in stream order) held
  bm_params prm{};
  int pending = 0;         // requests using it that have not completed
  uint64_t last_use = 0;
  // graph of bm_block_lu + bm_solve on the staging buffers
  hipGraphExec_t gexec = nullptr;
  bool graph_failed = false;
  int graph_nrhs = 0;
  cplx *stage_b = nullptr, *stage_x = nullptr;
};

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct srv_request {
  uint64_t ticket = 0;
  bm_request req{};
  int state = RQ_QUEUED;
  bm_request_result res{};
  srv_handle *h = nullptr;
  int lane = 0;
  int slot = -1;           // event pair and pinned error words
};

struct srv_lane {
  hipStream_t stream = nullptr;
  hipEvent_t fence = nullptr;  // recorded when a large request must wait for this lane
  int inflight = 0;
  bool used = false;           // work was enqueued since the last large request
};

bool same_params(const bm_params &a, const bm_params &b) { return memcmp(&a, &b, sizeof(bm_params)) == 0; }

}  // namespace

struct bm_server {
  int device = 0;
  int64_t budget = 0;
  int max_inflight = 4;        // per lane
  int graph_max_n = 0;
  int concurrent_max_n = 0;
  int batch_max = 1;       // requests of one N factored together (FP64)
  int ncu = 0;
  int quad = BM_QUAD_KRESS;    // quadrature of every handle
  int prec = BM_PREC_FP64;     // precision of every handle (FP64 or mixed, refined on the device)
  int refine_steps = 2;
  double refine_tol = 1e-12;

  std::mutex mu;
  std::condition_variable cv_work;   // worker: new request or stop
  std::condition_variable cv_done;   // waiters: a request finished
  std::deque<srv_request *> queue;   // submitted, not started
  std::unordered_map<uint64_t, srv_request *> by_ticket;
  uint64_t next_ticket = 1;
  bool stop = false;
  bm_server_counters st{};

  // worker-only state
  std::thread worker;
  std::vector<srv_lane> lanes;
  hipEvent_t big_fence = nullptr;    // recorded after each large request
  bool big_recorded = false;
  std::vector<srv_handle *> handles;
  std::vector<srv_request *> inflight;
  std::vector<hipEvent_t> ev_start, ev_done;
  std::vector<int> free_slots;
  int32_t *pinned = nullptr;         // 4 words per slot: error flag, info, domain flag, 0
  uint64_t use_clock = 0;
};

namespace {

int64_t live_bytes(const bm_server *s) {
  int64_t live = 0;
  for (const srv_handle *h : s->handles) live += h->bytes;
  return live;
}

void update_live(bm_server *s) {  // with s->mu held
  const int64_t live = live_bytes(s);
  s->st.bytes_live = live;
  s->st.handles_live = (int64_t)s->handles.size();
  if (live > s->st.bytes_peak) s->st.bytes_peak = live;
}

void release_handle(srv_handle *h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  (void)hipFree(h->stage_b);
  (void)hipFree(h->stage_x);
  if (h->p) bm_destroy(h->p);
  delete h;
}

bool is_small(const bm_server *s, int n) { return s->lanes.size() > 1 && n <= s->concurrent_max_n; }
// workgroups of the widest panel of an N-node factorisation (64 rows each up to
// 32 workgroups, then 128)
int panel_p(int n) { return (n <= 64 * 32) ? (n + 63) / 64 : (n + 127) / 128; }
// requests of N nodes that may be factored together: their panels within one
// lane's share of the panel workgroups all lanes may hold, half the CUs
int batch_limit(const bm_server *s, int n) {
  if (s->batch_max < 2 || !is_small(s, n)) return 1;
  const int fit = (s->ncu / 2 / (int)s->lanes.size()) / panel_p(n);
  const int b = (s->batch_max < fit) ? s->batch_max : fit;
  return (b < BM_LU_BATCH_MAX) ? (b > 1 ? b : 1) : BM_LU_BATCH_MAX;
}

// Lane for a request: the lane that holds its keyed factors, else the least
// loaded lane for a small request, else lane 0.
int choose_lane(const bm_server *s, const bm_request &r) {
  if (r.reuse_key != 0)
    for (const srv_handle *h : s->handles)
      if (h->n == r.n && h->key == r.reuse_key) return h->lane;
  if (!is_small(s, r.n)) return 0;
  int best = 0;
  for (int l = 1; l < (int)s->lanes.size(); ++l)
    if (s->lanes[l].inflight < s->lanes[best].inflight) best = l;
  return best;
}

// Find the handle for request r on `lane` or make room for it and create it.
// Returns BM_OK with *out set, BM_OK with *out == nullptr (wait for
// completions) or an error for the request.
int acquire(bm_server *s, const bm_request &r, int lane, int bslot, srv_handle **out) {
  *out = nullptr;
  for (srv_handle *h : s->handles)
    if (h->lane == lane && h->n == r.n && h->key == r.reuse_key && h->bslot == bslot) {
      *out = h;
      return BM_OK;
    }
  int64_t need = 0;
  if (int rc = bm_problem_bytes(r.n, BM_MIXED, &need)) return rc;
  int64_t live = live_bytes(s);
  while (live + need > s->budget) {  // evict the least recently used idle handle
    srv_handle *victim = nullptr;
    for (srv_handle *h : s->handles)
      if (h->pending == 0 && (!victim || h->last_use < victim->last_use)) victim = h;
    if (!victim) return BM_OK;  // everything busy: wait
    live -= victim->bytes;
    for (size_t i = 0; i < s->handles.size(); ++i)
      if (s->handles[i] == victim) {
        s->handles.erase(s->handles.begin() + (long)i);
        break;
      }
    release_handle(victim);
    std::lock_guard<std::mutex> g(s->mu);
    ++s->st.evictions;
    update_live(s);
  }
  srv_handle *h = new (std::nothrow) srv_handle();
  if (!h) return BM_E_NOMEM;
  int rc = bm_create(r.n, BM_MIXED, (void *)s->lanes[lane].stream, &h->p);
  if (!rc && s->quad != BM_QUAD_KRESS) {
    rc = bm_set_quadrature(h->p, s->quad);
    if (rc) bm_destroy(h->p);
  }
  // served factorisations form U33 first: the segmented product holds most CUs
  // for its whole length, which requests overlapping on other lanes would share
  if (!rc) (void)bm_set_lu_overlap(h->p, 0);
  if (!rc && s->prec != BM_PREC_FP64) {
    rc = bm_set_precision(h->p, s->prec, s->refine_tol, s->refine_steps);
    if (rc) bm_destroy(h->p);
  }
  if (rc) {
    delete h;
    return rc;
  }
  h->lane = lane;
  h->n = r.n;
  h->key = r.reuse_key;
  h->bslot = bslot;
  h->bytes = need;
  s->handles.push_back(h);
  std::lock_guard<std::mutex> g(s->mu);
  ++s->st.handles_created;
  update_live(s);
  *out = h;
  return BM_OK;
}

// Capture bm_block_lu + bm_solve on the staging buffers of h into a graph.
// The handle must be assembled (state) when this is called.
int capture(bm_server *s, srv_handle *h, int nrhs) {
  const size_t rows = 3 * (size_t)h->n;
  const hipStream_t st = s->lanes[h->lane].stream;
  if (!h->stage_b) {
    const int64_t extra = (int64_t)(2 * sizeof(cplx) * rows * nrhs);
    if (live_bytes(s) + extra > s->budget) return BM_E_BUDGET;
    if (hipMalloc(&h->stage_b, sizeof(cplx) * rows * nrhs) != hipSuccess) return BM_E_NOMEM;
    if (hipMalloc(&h->stage_x, sizeof(cplx) * rows * nrhs) != hipSuccess) return BM_E_NOMEM;
    h->bytes += extra;
  }
  BM_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  int rc = bm_block_lu(h->p, nullptr);
  if (!rc) rc = bm_solve(h->p, nrhs, h->stage_b, (int64_t)rows, h->stage_x, (int64_t)rows);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : BM_E_HIP;
  }
  const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    h->gexec = nullptr;
    return BM_E_HIP;
  }
  h->graph_nrhs = nrhs;
  return BM_OK;
}

// Device-side ordering of a request on its lane against the other lanes: a large
// request waits for everything enqueued on the other lanes; a small one waits
// for the latest large request.
int fence(bm_server *s, const srv_request *rq) {
  srv_lane &L = s->lanes[rq->lane];
  if (is_small(s, rq->req.n)) {
    if (s->big_recorded && rq->lane != 0) BM_HIP_TRY(hipStreamWaitEvent(L.stream, s->big_fence, 0));
    return BM_OK;
  }
  for (int l = 0; l < (int)s->lanes.size(); ++l) {
    if (l == rq->lane || !s->lanes[l].used) continue;
    BM_HIP_TRY(hipEventRecord(s->lanes[l].fence, s->lanes[l].stream));
    BM_HIP_TRY(hipStreamWaitEvent(L.stream, s->lanes[l].fence, 0));
    s->lanes[l].used = false;
  }
  return BM_OK;
}

// Enqueue the work of r on its lane.
int enqueue(bm_server *s, srv_request *rq) {
  const bm_request &r = rq->req;
  srv_handle *h = rq->h;
  const hipStream_t st = s->lanes[rq->lane].stream;
  const int64_t rows = 3 * (int64_t)r.n;
  const bool reuse = r.reuse_key != 0 && h->factored && same_params(h->prm, r.params);
  // a large request's assembly (vector work on its own buffers) runs beside the
  // other lanes' work; its product, LU and solve wait for them
  const bool late_fence = !reuse && !is_small(s, r.n);
  if (!late_fence)
    if (int rc = fence(s, rq)) return rc;
  BM_HIP_TRY(hipEventRecord(s->ev_start[rq->slot], st));
  int rc = BM_OK;
  if (reuse) {
    rc = bm_solve(h->p, r.nrhs, r.B, r.ldb, r.X, r.ldx);
    rq->res.reused_factors = 1;
  } else {
    h->factored = false;
    rc = bm_assemble(h->p, &r.geometry, &r.params);
    if (rc) return rc;
    if (late_fence)
      if (int rc2 = fence(s, rq)) return rc2;
    const bool want_graph = r.n <= s->graph_max_n && !h->graph_failed;
    if (want_graph && h->gexec && h->graph_nrhs != r.nrhs) {
      (void)hipGraphExecDestroy(h->gexec);  // captured for another block width
      h->gexec = nullptr;
      (void)hipFree(h->stage_b);
      (void)hipFree(h->stage_x);
      h->bytes -= (int64_t)(2 * sizeof(cplx) * rows * h->graph_nrhs);
      h->stage_b = h->stage_x = nullptr;
    }
    if (want_graph && !h->gexec && capture(s, h, r.nrhs) != BM_OK) h->graph_failed = true;
    if (want_graph && h->gexec) {
      BM_HIP_TRY(hipMemcpy2DAsync(h->stage_b, sizeof(cplx) * rows, r.B, sizeof(cplx) * r.ldb, sizeof(cplx) * rows,
                                  r.nrhs, hipMemcpyDeviceToDevice, st));
      BM_HIP_TRY(hipGraphLaunch(h->gexec, st));
      BM_HIP_TRY(hipMemcpy2DAsync(r.X, sizeof(cplx) * r.ldx, h->stage_x, sizeof(cplx) * rows, sizeof(cplx) * rows,
                                  r.nrhs, hipMemcpyDeviceToDevice, st));
      rq->res.graph = 1;
    } else {
      // a large request holds the device alone only while it forms U33; the small
      // requests after it start beside its LU (the panels of the lanes together
      // stay within half the CUs, see bm_server_create)
      const bool big = !is_small(s, r.n) && s->lanes.size() > 1;
      if (big) h->p->after_schur = s->big_fence;
      rc = bm_block_lu(h->p, nullptr);
      h->p->after_schur = nullptr;
      if (big && !rc) s->big_recorded = true;
      if (!rc) rc = bm_solve(h->p, r.nrhs, r.B, r.ldb, r.X, r.ldx);
    }
    if (!rc) {
      h->factored = true;
      h->prm = r.params;
    }
  }
  if (rc) return rc;
  BM_HIP_TRY(hipMemcpyAsync(s->pinned + 4 * rq->slot, h->p->dev_err, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  BM_HIP_TRY(hipEventRecord(s->ev_done[rq->slot], st));
  s->lanes[rq->lane].used = true;
  if (!is_small(s, r.n) && (rq->res.graph || rq->res.reused_factors)) {
    BM_HIP_TRY(hipEventRecord(s->big_fence, st));
    s->big_recorded = true;
  }
  return BM_OK;
}

// Enqueue requests of one N (no reuse key, FP64) on one lane with their
// factorisations in shared launches: each is assembled on its own handle, the
// handles are factored together, then each is solved.
int enqueue_batch(bm_server *s, const std::vector<srv_request *> &rqs) {
  const hipStream_t st = s->lanes[rqs[0]->lane].stream;
  bm_problem *ps[BM_LU_BATCH_MAX];
  const int count = (int)rqs.size();
  for (int k = 0; k < count; ++k) {
    srv_request *rq = rqs[k];
    if (int rc = fence(s, rq)) return rc;
    BM_HIP_TRY(hipEventRecord(s->ev_start[rq->slot], st));
    rq->h->factored = false;
    if (int rc = bm_assemble(rq->h->p, &rq->req.geometry, &rq->req.params)) return rc;
    ps[k] = rq->h->p;
  }
  if (int rc = bm_block_lu_batch(ps, count, nullptr)) return rc;
  for (int k = 0; k < count; ++k) {
    srv_request *rq = rqs[k];
    const bm_request &r = rq->req;
    if (int rc = bm_solve(rq->h->p, r.nrhs, r.B, r.ldb, r.X, r.ldx)) return rc;
    rq->h->factored = true;
    rq->h->prm = r.params;
    rq->res.batched = count;
    BM_HIP_TRY(hipMemcpyAsync(s->pinned + 4 * rq->slot, rq->h->p->dev_err, 4 * sizeof(int32_t),
                              hipMemcpyDeviceToHost, st));
    BM_HIP_TRY(hipEventRecord(s->ev_done[rq->slot], st));
  }
  s->lanes[rqs[0]->lane].used = true;
  return BM_OK;
}

void finish(bm_server *s, srv_request *rq, int status) {
  if (rq->h) --rq->h->pending;
  if (rq->slot >= 0) {
    s->free_slots.push_back(rq->slot);
    --s->lanes[rq->lane].inflight;
  }
  rq->slot = -1;
  std::lock_guard<std::mutex> g(s->mu);
  rq->res.status = status;
  rq->res.t_done = now_s();
  rq->state = RQ_DONE;
  if (status == BM_OK) {
    ++s->st.completed;
    if (rq->res.batched > 1) ++s->st.batched;
    if (rq->res.reused_factors) ++s->st.factor_reuses;
    if (rq->res.graph) ++s->st.graph_launches;
  } else if (status == BM_E_CANCELED) {
    ++s->st.canceled;
  } else {
    ++s->st.failed;
  }
  update_live(s);
  s->cv_done.notify_all();
}

// Completions of the requests in flight (in any order across lanes).
bool poll(bm_server *s) {
  bool any = false;
  for (size_t i = 0; i < s->inflight.size();) {
    srv_request *rq = s->inflight[i];
    const hipError_t e = hipEventQuery(s->ev_done[rq->slot]);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    s->inflight.erase(s->inflight.begin() + (long)i);
    int status = BM_OK;
    if (e != hipSuccess) {
      status = BM_E_HIP;
    } else {
      const int32_t *w = s->pinned + 4 * rq->slot;
      if (w[2]) status = BM_E_DOMAIN;
      else if (w[0]) status = BM_E_DEVICE;
      else if (w[1] > 0) status = w[1];
      else if (w[3]) status = BM_E_NOCONV;  // the device refinement missed its target
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, s->ev_start[rq->slot], s->ev_done[rq->slot]) == hipSuccess)
        rq->res.device_ms = ms;
    }
    if (status != BM_OK && rq->h) rq->h->factored = false;
    finish(s, rq, status);
    any = true;
  }
  return any;
}

void worker_main(bm_server *s) {
  (void)hipSetDevice(s->device);
  // a batch takes same-N requests from this many queue positions after the front
  constexpr size_t kBatchWindow = 8;
  for (;;) {
    const bool progress = poll(s);
    srv_request *next = nullptr;
    bm_request req{};
    int lane = 0;
    std::vector<srv_request *> extra;  // requests factored together with `next`
    std::vector<bm_request> extra_req;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop && s->queue.empty() && s->inflight.empty()) break;
      if (!s->queue.empty()) {
        req = s->queue.front()->req;  // a copy: the request may be canceled once the lock is released
        lane = choose_lane(s, req);
        if (s->lanes[lane].inflight < s->max_inflight) {
          next = s->queue.front();
          // (a batch may take the lane up to batch_max - 1 requests beyond max_inflight)
          int lim = batch_limit(s, req.n);
          if (req.reuse_key == 0)
            for (size_t qi = 1; qi < s->queue.size() && qi <= kBatchWindow && (int)extra.size() + 1 < lim; ++qi) {
              srv_request *c = s->queue[qi];
              if (c->req.n == req.n && c->req.reuse_key == 0) {
                extra.push_back(c);
                extra_req.push_back(c->req);
              }
            }
        }
      }
      if (!next && !progress) {
        if (s->inflight.empty())
          s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
        else
          s->cv_work.wait_for(lk, std::chrono::microseconds(50));
        continue;
      }
    }
    if (!next) continue;
    srv_handle *h = nullptr;
    int rc = acquire(s, req, lane, 0, &h);
    if (rc == BM_OK && !h) {
      if (!s->inflight.empty()) {  // no room until a request completes
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        continue;
      }
      rc = BM_E_BUDGET;  // not reached: the submission check guarantees that one handle fits
    }
    // the other members' handles (slots 1, 2, ...): the batch ends at the first
    // that cannot be had now; each handle is held (pending) once acquired, so that
    // a later acquisition does not evict it
    std::vector<srv_handle *> extra_h;
    if (!rc) {
      ++h->pending;
      for (size_t k = 0; k < extra.size(); ++k) {
        srv_handle *hk = nullptr;
        if (acquire(s, extra_req[k], lane, (int)k + 1, &hk) != BM_OK || !hk) break;
        ++hk->pending;
        extra_h.push_back(hk);
      }
      for (size_t k = extra_h.size(); k < extra.size(); ++k) extra[k] = nullptr;
    }
    {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->queue.empty() || s->queue.front() != next) {  // canceled meanwhile
        if (!rc) --h->pending;
        for (srv_handle *hk : extra_h) --hk->pending;
        continue;
      }
      s->queue.pop_front();
      next->state = RQ_RUNNING;  // from here on only the worker touches it until it is done
      for (size_t k = 0; k < extra_h.size(); ++k) {
        auto it = std::find(s->queue.begin(), s->queue.end(), extra[k]);
        if (it == s->queue.end()) {  // canceled meanwhile: its handle stays idle
          --extra_h[k]->pending;
          extra[k] = nullptr;
          continue;
        }
        s->queue.erase(it);
        extra[k]->state = RQ_RUNNING;
      }
    }
    next->res.t_start = now_s();
    next->lane = lane;
    if (rc) {
      finish(s, next, rc);
      continue;
    }
    std::vector<srv_request *> group{next};
    next->h = h;
    for (size_t k = 0; k < extra_h.size(); ++k)
      if (extra[k]) {
        extra[k]->h = extra_h[k];
        extra[k]->res.t_start = next->res.t_start;
        extra[k]->lane = lane;
        group.push_back(extra[k]);
      }
    for (srv_request *rq : group) {
      rq->h->last_use = ++s->use_clock;
      rq->slot = s->free_slots.back();
      s->free_slots.pop_back();
      ++s->lanes[lane].inflight;
    }
    rc = (group.size() == 1) ? enqueue(s, next) : enqueue_batch(s, group);
    if (rc) {
      for (srv_request *rq : group) rq->h->factored = false;
      // the lane may hold part of the requests' work: let everything drain
      (void)hipDeviceSynchronize();
      (void)poll(s);
      for (srv_request *rq : group) finish(s, rq, rc);
      continue;
    }
    for (srv_request *rq : group) s->inflight.push_back(rq);
  }
}

void free_server(bm_server *s) {
  for (auto e : s->ev_start)
    if (e) (void)hipEventDestroy(e);
  for (auto e : s->ev_done)
    if (e) (void)hipEventDestroy(e);
  for (auto &L : s->lanes) {
    if (L.fence) (void)hipEventDestroy(L.fence);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  if (s->big_fence) (void)hipEventDestroy(s->big_fence);
  if (s->pinned) (void)hipHostFree(s->pinned);
  delete s;
}

}  // namespace

extern "C" {

int bm_server_create(const bm_server_config *cfg, bm_server **out) {
  if (!out) return BM_E_ARG;
  *out = nullptr;
  bm_server_config c{};
  if (cfg) c = *cfg;
  if (c.graph_max_n < 0 || c.lanes < 0 || c.lanes > 16 || c.concurrent_max_n < 0) return BM_E_ARG;
  if (c.quadrature != BM_QUAD_KRESS && c.quadrature != BM_QUAD_ZETA1 && c.quadrature != BM_QUAD_ZETA31) return BM_E_ARG;
  if (c.precision != BM_PREC_FP64 && c.precision != BM_PREC_MIXED_DEVICE) return BM_E_ARG;
  const int lanes = c.lanes > 0 ? c.lanes : 4;
  const int cmax = c.concurrent_max_n > 0 ? c.concurrent_max_n : 1024;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BM_E_HIP;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return BM_E_HIP;
  // the panels of all lanes together may take at most half of the CUs
  if (lanes > 1 && (cmax > 2048 || lanes * ((cmax + 63) / 64) > ncu / 2)) return BM_E_ARG;
  bm_server *s = new (std::nothrow) bm_server();
  if (!s) return BM_E_NOMEM;
  s->device = dev;
  s->max_inflight = c.max_inflight > 0 ? c.max_inflight : 4;
  s->graph_max_n = c.graph_max_n;
  s->concurrent_max_n = cmax;
  s->ncu = ncu;
  s->batch_max = (c.batch_max < 1) ? 1 : ((c.batch_max > BM_LU_BATCH_MAX) ? BM_LU_BATCH_MAX : c.batch_max);
  s->quad = c.quadrature;
  s->prec = c.precision;
  s->refine_steps = c.refine_steps > 0 ? c.refine_steps : 2;
  s->refine_tol = c.refine_tol > 0.0 ? c.refine_tol : 1e-12;
  size_t free_b = 0, total_b = 0;
  bool ok = hipMemGetInfo(&free_b, &total_b) == hipSuccess;
  s->budget = c.hbm_budget_bytes > 0 ? c.hbm_budget_bytes : (int64_t)(0.9 * (double)free_b);
  ok = ok && bm_getrf_prepare() == BM_OK;
  s->lanes.resize(lanes);
  for (auto &L : s->lanes) {
    ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&L.fence, hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreateWithFlags(&s->big_fence, hipEventDisableTiming) == hipSuccess;
  const int nslot = (s->max_inflight + s->batch_max - 1) * lanes;  // (a batch may go past max_inflight)
  s->ev_start.assign(nslot, nullptr);
  s->ev_done.assign(nslot, nullptr);
  for (int i = 0; ok && i < nslot; ++i) {
    ok = hipEventCreate(&s->ev_start[i]) == hipSuccess && hipEventCreate(&s->ev_done[i]) == hipSuccess;
    s->free_slots.push_back(nslot - 1 - i);
  }
  ok = ok && hipHostMalloc((void **)&s->pinned, sizeof(int32_t) * 4 * nslot, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_server(s);
    return BM_E_HIP;
  }
  s->st.budget = s->budget;
  s->worker = std::thread(worker_main, s);
  *out = s;
  return BM_OK;
}

int bm_server_submit(bm_server *s, const bm_request *r, uint64_t *ticket) {
  if (!s || !r || !ticket) return BM_E_ARG;
  const int64_t rows = 3 * (int64_t)r->n;
  int64_t need = 0;
  int rc = bm_problem_bytes(r->n, BM_MIXED, &need);
  if (!rc) rc = bm_check_params(&r->params);
  if (!rc && (r->nrhs < 1 || !r->B || !r->X || r->B == r->X || r->ldb < rows || r->ldx < rows)) rc = BM_E_ARG;
  if (!rc && (!r->geometry.x || !r->geometry.dx || !r->geometry.ddx || !r->geometry.d3x)) rc = BM_E_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  if (!rc && need > s->budget) rc = BM_E_BUDGET;
  if (rc) {
    ++s->st.rejected;
    return rc;
  }
  srv_request *rq = new (std::nothrow) srv_request();
  if (!rq) return BM_E_NOMEM;
  rq->ticket = s->next_ticket++;
  rq->req = *r;
  rq->res.n = r->n;
  rq->res.batched = 1;
  rq->res.t_submit = now_s();
  s->queue.push_back(rq);
  s->by_ticket[rq->ticket] = rq;
  ++s->st.submitted;
  *ticket = rq->ticket;
  s->cv_work.notify_one();
  return BM_OK;
}

int bm_server_wait(bm_server *s, uint64_t ticket, double timeout_s, bm_request_result *res) {
  if (!s || !res) return BM_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return BM_E_ARG;
  srv_request *rq = it->second;
  auto done = [rq] { return rq->state == RQ_DONE; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return BM_E_TIMEOUT;
  }
  *res = rq->res;
  s->by_ticket.erase(ticket);
  delete rq;
  return BM_OK;
}

int bm_server_cancel(bm_server *s, uint64_t ticket) {
  if (!s) return BM_E_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return BM_E_ARG;
  srv_request *rq = it->second;
  if (rq->state != RQ_QUEUED) return BM_E_STATE;
  for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
    if (*q == rq) {
      s->queue.erase(q);
      break;
    }
  rq->state = RQ_DONE;
  rq->res.status = BM_E_CANCELED;
  rq->res.t_start = rq->res.t_done = now_s();
  ++s->st.canceled;
  s->cv_done.notify_all();
  return BM_OK;
}

int bm_server_stats(bm_server *s, bm_server_counters *st) {
  if (!s || !st) return BM_E_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  *st = s->st;
  return BM_OK;
}

void bm_server_destroy(bm_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (srv_request *rq : s->queue) {
      rq->state = RQ_DONE;
      rq->res.status = BM_E_CANCELED;
      ++s->st.canceled;
    }
    s->queue.clear();
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (auto &L : s->lanes) (void)hipStreamSynchronize(L.stream);
  for (srv_handle *h : s->handles) release_handle(h);
  s->handles.clear();
  for (auto &kv : s->by_ticket) delete kv.second;
  free_server(s);
}

}  // extern "C"
