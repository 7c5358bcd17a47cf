// Continuous-batching server (the eik_serve_* entry points of include/eik.h).
//
// The server owns one device arena of hbm_budget_bytes.  Every request is
// charged its device bytes (speed, solution and h/F arrays, mask, exit
// nodes, and for FP32 with the residual check the FP64 re-solve buffers)
// and admitted only when the arena can place it.  Lanes, each a host thread
// with its own HIP stream and solver workspace, take every pending request
// that fits when they fall idle and solve them together in one persistent
// launch; launches of different lanes overlap on the device, so requests
// arriving while others run start as soon as a lane, a slot and memory are
// free.  A request's result does not depend on what it was batched with:
// instances in a launch share the workers but no data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/eik.h"
#include "internal.h"

namespace eik {
namespace {

constexpr size_t kAlign = 256;
// Each lane drives two streams (its launches, and the residual checks and
// copies of requests that finish early); with the process's default of four
// hardware queues two lanes keep every stream on a queue of its own.  Maze
// serving measured with 2 / 4 / 8 lanes: 947 / 1008-1074 / 807 requests/s
// saturated, p99 64-81 / 104-226 / 405-1037 ms.
constexpr int kDefaultLanes = 2;
constexpr int kMaxBatch = 256;          // requests per launch
constexpr uint64_t kDefaultBudget = 64ull << 30;
constexpr size_t kPinnedBytes = 1ull << 30;  // pinned staging of submitted inputs
// EIK_SERVE_LOG=1: one line per launched batch on stderr (lane, requests,
// nodes, upload / solve / download milliseconds), a diagnostic
const bool g_serve_log = [] {
  const char* v = std::getenv("EIK_SERVE_LOG");
  return v && v[0] == '1';
}();

size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
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
  std::map<size_t, size_t> free_;  // offset -> length
};

enum ReqState { kReqQueued, kReqRunning, kReqDone };

struct Req {
  uint64_t ticket = 0;
  eik_problem p{};          // the caller's problem (pointers valid until admission)
  // host copies (device_ptrs = 0): in the server's pinned arena when it has
  // room (hoff, hbytes), else in these vectors
  std::vector<char> F;
  std::vector<uint8_t> mask;
  std::vector<int64_t> src;
  std::vector<double> q;
  const void* hF = nullptr;
  const void* hmask = nullptr;
  const void* hsrc = nullptr;
  const void* hq = nullptr;
  size_t hoff = 0, hbytes = 0;  // pinned block (hbytes = 0: none)
  size_t bytes = 0, off = 0;
  ReqState state = kReqQueued;
  int rc = EIK_OK;
  std::string err;
  eik_stats st{};
  double t_submit = 0.0;
  double density = 0.0;     // wall density (host masks; cell-side tuning)
};

// Byte offsets of a request's arrays inside its arena block.
struct Layout {
  size_t F, u, delta, mask, src, q, f64, total;
};

Layout layout(const eik_problem& p, const eik_opts& o) {
  const size_t nn = (size_t)p.nx * p.ny, es = dsize(o.dtype);
  Layout L;
  size_t at = 0;
  L.F = at; at += up(nn * es);
  L.u = at; at += up(nn * es);
  L.delta = at; at += up(nn * es);
  L.mask = at; at += p.mask ? up(nn) : 0;
  L.src = at; at += up(p.nsrc * sizeof(int64_t));
  L.q = at; at += p.q ? up(p.nsrc * sizeof(double)) : 0;
  L.f64 = at; at += (o.dtype == EIK_F32 && o.residual_check) ? up(3 * nn * sizeof(double)) : 0;
  L.total = at;
  return L;
}

}  // namespace
}  // namespace eik

using namespace eik;

struct eik_server {
  eik_serve_cfg cfg{};
  int dev = 0;
  char* base = nullptr;  // device arena
  Arena arena;
  char* pinned = nullptr;  // host staging arena (page-locked)
  Arena host_arena;
  int lanes = kDefaultLanes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  int in_flight = 0;
  bool stop = false;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;
  std::vector<std::unique_ptr<Workspace>> ws;
  // early completion, per lane: a side stream for the finished problems'
  // residual checks and downloads, and pinned host memory the solver writes
  // each problem's completion flag into (kMaxBatch flags) plus a read-back
  // area for the problems' counters (4 x kMaxBatch)
  std::vector<hipStream_t> side;
  std::vector<unsigned int*> flags;
  std::vector<unsigned long long*> counters;

  void lane(int id);
  void solve(int id, std::vector<Req*>& batch);
  void finish(Req* r);
  // frees the lanes' streams, workspaces and pinned memory and the arenas
  void free_lanes() {
    for (auto& w : ws) workspace_free(w.get());
    for (hipStream_t x : streams) (void)hipStreamDestroy(x);
    for (hipStream_t x : side) (void)hipStreamDestroy(x);
    for (unsigned int* f : flags) (void)hipHostFree(f);
    for (unsigned long long* c : counters) (void)hipHostFree(c);
    ws.clear();
    streams.clear();
    side.clear();
    flags.clear();
    counters.clear();
    if (base) (void)hipFree(base);
    base = nullptr;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
  }
};

// Hands a solved request back (result in place, stats set): frees its
// arena block and wakes waiters and idle lanes.
void eik_server::finish(Req* r) {
  {
    std::lock_guard<std::mutex> lk(mu);
    arena.release(r->off, r->bytes);
    if (r->hbytes) host_arena.release(r->hoff, r->hbytes);
    r->hbytes = 0;
    r->state = kReqDone;
    in_flight--;
  }
  cv_work.notify_all();
  cv_done.notify_all();
}

// Takes the requests at the head of the queue while a slot and arena space
// are free (first come, first served: a request that does not fit holds back
// those behind it).
static void take_batch(eik_server* s, std::vector<Req*>& batch) {
  const int max_slots = s->cfg.max_slots ? s->cfg.max_slots : 1024;
  while (!s->pending.empty() && (int)batch.size() < kMaxBatch && s->in_flight < max_slots) {
    Req* r = s->pending.front();
    size_t off = 0;
    if (!s->arena.alloc(r->bytes, &off)) break;
    r->off = off;
    r->state = kReqRunning;
    s->pending.pop_front();
    s->in_flight++;
    batch.push_back(r);
  }
}

void eik_server::lane(int id) {
  (void)hipSetDevice(dev);
  for (;;) {
    std::vector<Req*> batch;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        take_batch(this, batch);
        if (!batch.empty() || (stop && pending.empty())) break;
        cv_work.wait(lk);
      }
      if (batch.empty()) return;
    }
    solve(id, batch);  // finishes every request of the batch
  }
}

// Uploads, solves and downloads one batch on lane `id`.  A batch that fails
// as a whole is retried request by request, so one bad request (speeds or
// sources checked on the device) fails alone.
void eik_server::solve(int id, std::vector<Req*>& batch) {
  const double t_up = now_s();
  hipStream_t st = streams[id];
  eik_opts o = cfg.opts;
  o.device_ptrs = 1;
  o.stream = st;
  const size_t es = dsize(o.dtype);
  const int n = (int)batch.size();
  std::vector<eik_problem> probs(n);
  std::vector<void*> delta(n), f64(n);
  std::vector<double> density(n);
  int rc = EIK_OK;
  for (int k = 0; k < n && !rc; ++k) {
    Req* r = batch[k];
    const eik_problem& p = r->p;
    const Layout L = layout(p, o);
    char* b = base + r->off;
    const size_t nn = (size_t)p.nx * p.ny;
    const hipMemcpyKind kind = cfg.opts.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const void* F = cfg.opts.device_ptrs ? p.F : r->hF;
    const void* M = cfg.opts.device_ptrs ? (const void*)p.mask : r->hmask;
    const void* S = cfg.opts.device_ptrs ? (const void*)p.src : r->hsrc;
    const void* Q = cfg.opts.device_ptrs ? (const void*)p.q : r->hq;
    hipError_t e = hipMemcpyAsync(b + L.F, F, nn * es, kind, st);
    if (e == hipSuccess && p.mask) e = hipMemcpyAsync(b + L.mask, M, nn, kind, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b + L.src, S, p.nsrc * sizeof(int64_t), kind, st);
    if (e == hipSuccess && p.q) e = hipMemcpyAsync(b + L.q, Q, p.nsrc * sizeof(double), kind, st);
    if (e != hipSuccess) rc = fail(EIK_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    eik_problem d = p;
    d.F = b + L.F;
    d.u_out = b + L.u;
    d.mask = p.mask ? (const uint8_t*)(b + L.mask) : nullptr;
    d.src = (const int64_t*)(b + L.src);
    d.q = p.q ? (const double*)(b + L.q) : nullptr;
    probs[k] = d;
    delta[k] = b + L.delta;
    f64[k] = b + L.f64;
    density[k] = r->density;
  }
  if (g_serve_log) (void)hipStreamSynchronize(st);
  const double t_up1 = now_s();
  std::vector<eik_stats> stats(n);
  RunCtx ctx;
  ctx.ws = ws[id].get();
  ctx.delta = delta.data();
  ctx.f64 = f64.data();
  ctx.share = lanes;
  if (!cfg.opts.device_ptrs) ctx.density = density.data();
  // Early completion: while the launch runs, a problem whose cells are all
  // done is checked (FP32: its FP64 residual), downloaded and handed back at
  // once, so a small request does not wait for the largest one of its
  // launch.  A problem that fails its residual check stays for the FP64
  // re-solve at the end of the launch.
  std::vector<char> detached(n, 0), seen(n, 0);
  std::vector<double> t_early(n, 0.0);
  unsigned int* fl = flags[id];
  unsigned long long* cnt = counters[id];
  const bool early = n > 1;
  const bool check32 = o.dtype == EIK_F32 && o.residual_check;
  const double tol = o.residual_tol > 0.0 ? o.residual_tol : 4.0 * std::ldexp(1.0, -24);
  if (early) {
    std::memset(fl, 0, n * sizeof(unsigned int));
    ctx.idone = fl;
    ctx.detached = detached.data();
    ctx.poll = [&](const Engine& e, const std::vector<Inst>& inst) {
      for (int k = 0; k < n; ++k) {
        if (seen[k] || !__atomic_load_n(&fl[k], __ATOMIC_ACQUIRE)) continue;
        seen[k] = 1;
        Req* r = batch[k];
        hipStream_t ss = side[id];
        const size_t nn = (size_t)r->p.nx * r->p.ny;
        hipError_t e1 = check32 ? launch_residual(e, (int64_t)nn, ss, k, 1) : hipSuccess;
        if (e1 == hipSuccess)
          e1 = hipMemcpyAsync(cnt + 4 * k, e.istat + 4 * k, 4 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, ss);
        if (e1 == hipSuccess)
          e1 = hipMemcpyAsync(r->p.u_out, probs[k].u_out, nn * es, hipMemcpyDeviceToHost, ss);
        if (e1 == hipSuccess) e1 = hipStreamSynchronize(ss);
        if (e1 != hipSuccess) continue;  // left to the end of the launch
        double resid = -1.0;
        if (check32) std::memcpy(&resid, &cnt[4 * k + 3], sizeof resid);
        if (check32 && !(resid <= tol)) continue;  // FP64 re-solve at the end
        eik_stats& S = r->st;
        std::memset(&S, 0, sizeof S);
        const double t = now_s();
        S.seconds = t - r->t_submit;
        S.kernel_seconds = t - t_up1;  // launch start to completion (host clock)
        S.cells = (uint64_t)inst[k].kx * inst[k].ky;
        S.cells_total = (uint64_t)e.ncells;
        S.cell_used = inst[k].s;
        S.cell_visits = cnt[4 * k];
        S.sweeps = cnt[4 * k + 1];
        S.checks = cnt[4 * k + 2];
        S.max_residual = check32 ? resid : -1.0;
        S.residual_f32 = check32 ? resid : -1.0;
        S.band_used = -1.0;
        r->rc = EIK_OK;
        detached[k] = 1;
        t_early[k] = t;
        std::vector<char>().swap(r->F);
        std::vector<uint8_t>().swap(r->mask);
        std::vector<int64_t>().swap(r->src);
        std::vector<double>().swap(r->q);
        finish(r);
      }
    };
  }
  if (!rc) rc = run(n, probs.data(), o, stats.data(), nullptr, &ctx);
  if (rc && n > 1) {
    // isolate the failing request(s) (none finished early: a failed launch
    // reports no completed problem before its device-side error)
    for (int k = 0; k < n; ++k) {
      if (detached[k]) continue;
      RunCtx one;  // the request's own arena buffers
      one.ws = ctx.ws;
      one.share = ctx.share;
      one.delta = &delta[k];
      one.f64 = &f64[k];
      one.density = ctx.density ? &density[k] : nullptr;
      batch[k]->rc = run(1, &probs[k], o, &stats[k], nullptr, &one);
      if (batch[k]->rc) batch[k]->err = g_err;
    }
  } else {
    for (int k = 0; k < n; ++k) {
      if (detached[k]) continue;
      batch[k]->rc = rc;
      if (rc) batch[k]->err = g_err;
    }
  }
  const double t_solved = now_s();
  for (int k = 0; k < n; ++k) {
    Req* r = batch[k];
    if (r->rc || detached[k]) continue;
    const size_t nn = (size_t)r->p.nx * r->p.ny;
    hipError_t e = hipMemcpyAsync(r->p.u_out, probs[k].u_out, nn * es, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) {
      r->rc = EIK_EDEVICE;
      r->err = std::string("download failed: ") + hipGetErrorString(e);
    }
  }
  (void)hipStreamSynchronize(st);
  const double t = now_s();
  if (g_serve_log) {
    double nodes = 0;
    int ne = 0;
    for (int k = 0; k < n; ++k) {
      nodes += (double)batch[k]->p.nx * batch[k]->p.ny;
      ne += detached[k];
    }
    std::fprintf(stderr, "[eik serve] lane %d: %d requests (%d finished early), %.2f Mnodes; upload "
                 "%.2f ms, solve %.2f ms (kernel %.2f ms), download %.2f ms\n", id, n, ne,
                 nodes * 1e-6, (t_up1 - t_up) * 1e3, (t_solved - t_up1) * 1e3,
                 stats[0].kernel_seconds * 1e3, (t - t_solved) * 1e3);
  }
  for (int k = 0; k < n; ++k) {
    Req* r = batch[k];
    if (detached[k]) continue;
    r->st = stats[k];
    r->st.seconds = t - r->t_submit;
    std::vector<char>().swap(r->F);
    std::vector<uint8_t>().swap(r->mask);
    std::vector<int64_t>().swap(r->src);
    std::vector<double>().swap(r->q);
    finish(r);
  }
}

extern "C" {

int eik_serve_create(const eik_serve_cfg* cfg, eik_server** out) {
  g_err.clear();
  if (!cfg || !out) return fail(EIK_EINVAL, "cfg and out are required");
  *out = nullptr;
  int rc = check_opts(cfg->opts);
  if (rc) return rc;
  if (cfg->max_slots < 0) return fail(EIK_EINVAL, "max_slots must be >= 0");
  if (cfg->lanes < 0 || cfg->lanes > 16) return fail(EIK_EINVAL, "lanes outside [0, 16]");
  std::unique_ptr<eik_server> s(new eik_server());
  s->cfg = *cfg;
  if (!s->cfg.hbm_budget_bytes) s->cfg.hbm_budget_bytes = kDefaultBudget;
  s->lanes = cfg->lanes ? cfg->lanes : kDefaultLanes;
  HIP_TRY(hipGetDevice(&s->dev));
  void* base = nullptr;
  if (hipMalloc(&base, s->cfg.hbm_budget_bytes) != hipSuccess)
    return fail(EIK_ENOMEM, "cannot allocate a %llu-byte arena",
                (unsigned long long)s->cfg.hbm_budget_bytes);
  s->base = static_cast<char*>(base);
  s->arena.reset(s->cfg.hbm_budget_bytes / kAlign * kAlign);
  if (!s->cfg.opts.device_ptrs) {
    // page-locked staging for submitted inputs; without it, pageable copies
    const size_t pb = std::min<size_t>(kPinnedBytes, s->cfg.hbm_budget_bytes) / kAlign * kAlign;
    void* h = nullptr;
    if (pb && hipHostMalloc(&h, pb, hipHostMallocDefault) == hipSuccess) {
      s->pinned = static_cast<char*>(h);
      s->host_arena.reset(pb);
    }
  }
  for (int i = 0; i < s->lanes; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      s->free_lanes();
      return fail(EIK_EDEVICE, "cannot create a stream");
    }
    s->streams.push_back(st);
    hipStream_t ss = nullptr;
    void* f = nullptr;
    void* c = nullptr;
    if (hipStreamCreateWithFlags(&ss, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(&f, kMaxBatch * sizeof(unsigned int),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostMalloc(&c, 4 * kMaxBatch * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
      if (ss) (void)hipStreamDestroy(ss);
      if (f) (void)hipHostFree(f);
      s->free_lanes();
      return fail(EIK_EDEVICE, "cannot create a lane's side stream or completion flags");
    }
    s->side.push_back(ss);
    s->flags.push_back(static_cast<unsigned int*>(f));
    s->counters.push_back(static_cast<unsigned long long*>(c));
    s->ws.emplace_back(new Workspace());
    workspace_defer_frees(s->ws.back().get());
    if ((rc = workspace_init(s->ws.back().get()))) {
      s->free_lanes();
      return rc;
    }
  }
  eik_server* raw = s.get();
  for (int i = 0; i < s->lanes; ++i) s->threads.emplace_back([raw, i] { raw->lane(i); });
  *out = s.release();
  return EIK_OK;
}

int eik_serve_submit(eik_server* s, const eik_problem* p, uint64_t* ticket) {
  g_err.clear();
  if (!s || !p || !ticket) return fail(EIK_EINVAL, "server, problem and ticket are required");
  int rc = validate_shape(*p);
  if (rc) return rc;
  const eik_opts& o = s->cfg.opts;
  if (!o.device_ptrs && (rc = validate_host(*p, o.dtype))) return rc;
  Tiling t;
  const int cell = o.cell ? o.cell : default_cell(p->nx, p->ny, o.method);
  if ((rc = make_tiling(p->nx, p->ny, cell, o.method, &t))) return rc;
  std::unique_ptr<Req> r(new Req());
  r->p = *p;
  r->bytes = layout(*p, o).total;
  if (r->bytes > s->cfg.hbm_budget_bytes / kAlign * kAlign)
    return fail(EIK_EBUDGET, "request needs %zu device bytes, budget is %llu", r->bytes,
                (unsigned long long)s->cfg.hbm_budget_bytes);
  if (!o.device_ptrs) {
    const size_t nn = (size_t)p->nx * p->ny;
    const size_t bF = up(nn * dsize(o.dtype)), bM = p->mask ? up(nn) : 0;
    const size_t bS = up(p->nsrc * sizeof(int64_t)), bQ = p->q ? up(p->nsrc * sizeof(double)) : 0;
    size_t hoff = 0;
    bool pin = false;
    if (s->pinned) {
      std::lock_guard<std::mutex> lk(s->mu);
      pin = s->host_arena.alloc(bF + bM + bS + bQ, &hoff);
    }
    if (pin) {
      char* h = s->pinned + hoff;
      r->hoff = hoff;
      r->hbytes = bF + bM + bS + bQ;
      std::memcpy(h, p->F, nn * dsize(o.dtype));
      r->hF = h;
      if (p->mask) {
        std::memcpy(h + bF, p->mask, nn);
        r->hmask = h + bF;
      }
      std::memcpy(h + bF + bM, p->src, p->nsrc * sizeof(int64_t));
      r->hsrc = h + bF + bM;
      if (p->q) {
        std::memcpy(h + bF + bM + bS, p->q, p->nsrc * sizeof(double));
        r->hq = h + bF + bM + bS;
      }
    } else {
      r->F.assign((const char*)p->F, (const char*)p->F + nn * dsize(o.dtype));
      if (p->mask) r->mask.assign(p->mask, p->mask + nn);
      r->src.assign(p->src, p->src + p->nsrc);
      if (p->q) r->q.assign(p->q, p->q + p->nsrc);
      r->hF = r->F.data();
      r->hmask = p->mask ? r->mask.data() : nullptr;
      r->hsrc = r->src.data();
      r->hq = p->q ? r->q.data() : nullptr;
    }
    r->density = wall_density_host(*p);
  }
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(EIK_EINVAL, "server is shutting down");
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
  }
  s->cv_work.notify_one();
  return EIK_OK;
}

// Hands out a finished request's result once and forgets the ticket.
static int collect(eik_server* s, std::unique_lock<std::mutex>& lk, uint64_t ticket, eik_stats* stats) {
  (void)lk;
  auto it = s->reqs.find(ticket);
  Req* r = it->second.get();
  const int rc = r->rc;
  if (rc) g_err = r->err;
  else if (stats) *stats = r->st;
  s->reqs.erase(it);
  return rc;
}

int eik_serve_poll(eik_server* s, uint64_t ticket, eik_stats* stats) {
  g_err.clear();
  if (!s) return fail(EIK_EINVAL, "server is required");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(EIK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second->state != kReqDone) return EIK_EBUSY;
  return collect(s, lk, ticket, stats);
}

int eik_serve_wait(eik_server* s, uint64_t ticket, eik_stats* stats) {
  g_err.clear();
  if (!s) return fail(EIK_EINVAL, "server is required");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(EIK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second.get();
  s->cv_done.wait(lk, [r] { return r->state == kReqDone; });
  return collect(s, lk, ticket, stats);
}

int eik_serve_cancel(eik_server* s, uint64_t ticket) {
  g_err.clear();
  if (!s) return fail(EIK_EINVAL, "server is required");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(EIK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second->state != kReqQueued) return fail(EIK_EBUSY, "request already admitted");
  if (it->second->hbytes) s->host_arena.release(it->second->hoff, it->second->hbytes);
  s->pending.erase(std::find(s->pending.begin(), s->pending.end(), it->second.get()));
  s->reqs.erase(it);
  return EIK_OK;
}

int eik_serve_destroy(eik_server* s) {
  g_err.clear();
  if (!s) return fail(EIK_EINVAL, "server is required");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->threads) t.join();
  s->free_lanes();
  delete s;
  return EIK_OK;
}

}  // extern "C"
