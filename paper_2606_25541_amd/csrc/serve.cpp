// Batched solves of same-shape instances in lock-step launches, and the
// continuous-batching solve server.
#include "serve.hpp"

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace psfd {

static bool same_shape(const psfd_problem& a, const psfd_problem& b) {
  return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lx_nm == b.lx_nm && a.ly_nm == b.ly_nm &&
         a.t_nm == b.t_nm;
}

// Workspaces of finished batched solves, kept for the next call with the same
// device, shape, batch size, restart length and precision: fresh device memory
// costs about as much to map and clear as a solve of the same size, so a batch
// that allocated its own workspace on every call would spend most of its time
// there. At most BATCH_CACHE_GROUPS groups are kept (least recently used are
// freed first); psfd_release_cached_workspaces frees them all.
static const size_t BATCH_CACHE_GROUPS = 4;
struct CachedGroup {
  int device;
  std::unique_ptr<Group> g;
};
static std::mutex g_cache_mu;
// never destroyed: at process exit the runtime may be gone before static destructors run
static std::deque<CachedGroup>& g_cache = *new std::deque<CachedGroup>();

static std::unique_ptr<Group> take_group(int device, const Shape& sh, int B, int m, int prec) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
    const Group& g = *it->g;
    if (it->device == device && g.sh.nx == sh.nx && g.sh.ny == sh.ny && g.sh.nz == sh.nz && g.B == B &&
        g.m == m && g.prec == prec) {
      std::unique_ptr<Group> out = std::move(it->g);
      g_cache.erase(it);
      return out;
    }
  }
  return nullptr;
}

static void return_group(int device, std::unique_ptr<Group> g) {
  std::unique_ptr<Group> drop;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.push_front(CachedGroup{device, std::move(g)});
  if (g_cache.size() > BATCH_CACHE_GROUPS) {
    drop = std::move(g_cache.back().g);
    g_cache.pop_back();
  }
}

void release_cached_groups() {
  std::deque<CachedGroup> drop;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  drop.swap(g_cache);
}

Status solve_batch(int n, const psfd_problem* probs, const psfd_opts* opts, const void* const* d_deps,
                   void* const* d_emask, void* const* d_orders, psfd_info* info, hipStream_t s) {
  Status st;
  Opts o;
  st = make_opts(opts, o);
  if (!st.ok()) return st;
  std::vector<Problem> pr(n);
  for (int i = 0; i < n; ++i) {
    st = validate_problem(&probs[i], pr[i]);
    if (!st.ok()) return st;
    if (!same_shape(probs[0], probs[i])) {
      st.code = PSFD_ERR_INVALID_ARG;
      st.msg = "batched instances must share nx, ny, nz, lx, ly and t";
      return st;
    }
  }
  const Shape sh = shape_of(pr[0].p);
  int device = 0;
  hipError_t de = hipGetDevice(&device);
  if (de != hipSuccess) return hip_status(de, "batch device");
  std::unique_ptr<Group> gp = take_group(device, sh, n, o.restart, o.precision);
  if (!gp) {
    gp = std::make_unique<Group>();
    st = group_alloc(*gp, sh, n, o.restart, o.precision);
    if (!st.ok()) return st;
  }
  Group& g = *gp;
  std::vector<double> tab;
  for (int i = 0; i < n; ++i) {
    st = build_table(pr[i], tab);
    if (!st.ok()) return st;
    st = group_set_tables(g, i, pr[i], tab, s);
    if (!st.ok()) return st;
    hipError_t e = hipMemcpyAsync(g.deps64 + (size_t)i * sh.N, d_deps[i], sh.N * 16, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_status(e, "copy contrast");
  }
  std::vector<SolveStats> stats;
  st = solve_group(g, o, stats, s);
  if (!st.ok()) return st;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipMemcpyAsync(d_emask[i], g.x + (size_t)i * sh.n3, sh.n3 * 16, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && d_orders && d_orders[i])
      e = hipMemcpyAsync(d_orders[i], g.ord + (size_t)i * sh.nxny * 3, sh.nxny * 3 * 16, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_status(e, "copy results");
    if (info) {
      info[i].iters = stats[i].iters;
      info[i].outer_iters = stats[i].outer;
      info[i].cycles = stats[i].cycles;
      info[i].status = stats[i].status;
      info[i].rel_residual = stats[i].rel_res;
      info[i].outer_change = stats[i].change;
      info[i].mono_residual = stats[i].mono;
    }
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_status(e, "batch");
  return_group(device, std::move(gp));
  return st;
}

// ---------------------------------------------------------------------------
// Continuous-batching solve server.
//
// Requests are grouped by kind: grid shape, restart length, precision and the
// FP32 cycle reduction (what fixes a group's buffers and launches); tolerance
// and iteration limit are per request. Each kind runs in a slot group (a Group
// of `cap` instances) with its own worker thread and HIP stream, so groups of
// different kinds run concurrently on the device and small requests never wait
// behind the launches of large ones. A worker runs ticks; every tick advances
// every occupied slot of its group by one phase of its own coupled solve
// (monolithic coupling, GMRES(m) with FP64 residuals):
//   INIT  tables, contrast, e_bg, x0 = e_bg, ||b||
//   START FP64 residual r = b - A x: done, or start an Arnoldi cycle
//   ARN   Arnoldi steps (all running slots share each launch)
//   END   y = H^-1 g, x += V y
//   FIN   readouts, E_up, E_layer, E_mask = u - e, orders, copy-out
// Requests that arrive while others run are admitted into free slots at the
// next tick and share the launches from then on. Every kernel works per
// instance with a fixed reduction layout, so a result does not depend on which
// other requests share the group.
//
// Admission by device-memory footprint. A request whose kind has a running
// group joins that group's queue. Otherwise it waits in the server's pending
// list (first come, first served) until its kind can get a group: a group of
// min(max_slots, free budget / slot bytes) slots is created as soon as one
// slot fits what is left of the budget. When it does not fit, idle groups are
// released at once and, if that is not enough, the oldest busy groups are
// drained: they take no new requests, finish the ones already queued to them,
// then free their memory. A group idle for IDLE_RELEASE_S also frees its
// memory. Only a request that cannot fit even an empty budget completes with
// PSFD_ERR_OOM.
// ---------------------------------------------------------------------------
using clk = std::chrono::steady_clock;

static const double IDLE_RELEASE_S = 5.0;

enum Phase { P_FREE = 0, P_INIT, P_START, P_ARN, P_END, P_FIN };

// what fixes a slot group's buffers and launches
struct Kind {
  Shape sh;
  int m = 30, prec = PSFD_MIXED;
  double eta = 1e-4;
  bool operator==(const Kind& k) const {
    return sh.nx == k.sh.nx && sh.ny == k.sh.ny && sh.nz == k.sh.nz && m == k.m && prec == k.prec && eta == k.eta;
  }
};

struct Req {
  uint64_t ticket = 0;
  Problem pr;
  Opts o;
  Kind kind;
  size_t slot_bytes = 0;
  std::vector<double> tab;
  const void* d_deps = nullptr;
  void* d_emask = nullptr;
  void* d_orders = nullptr;
  clk::time_point t_submit, t_done;
  bool done = false;
  int status = PSFD_OK;
  psfd_info info{};
};

struct SlotGroup {
  Kind kind;
  size_t bytes = 0;
  std::unique_ptr<Group> g;
  int cap = 0;
  hipStream_t s = nullptr;
  std::thread worker;
  std::condition_variable cv;
  std::deque<Req*> queue;  // waiting for a free slot of this group (guarded by the server mutex)
  bool draining = false;   // takes no new requests; released once its queue and slots are empty
  bool dead = false;       // released (memory freed, worker exiting)
  std::vector<Req*> req;
  std::vector<int> phase;
  std::vector<int> cycles;
  // residual of the slot's next restart (the policy of the device-driven solve):
  // b - A x (tres) or the last cycle's GMRES residual from its basis (rres);
  // since: restarts since the last b - A x
  std::vector<int> tres, rres, since;
  std::vector<double> bn, tgt, res;
  int occupied() const {
    int n = 0;
    for (auto* r : req) n += r != nullptr;
    return n;
  }
};

}  // namespace psfd

struct psfd_server {
  size_t budget = 0;
  int max_slots = 1;
  psfd::Opts o;
  int device = 0;
  std::mutex mu;  // guards everything below and every group's queue, req slots' ownership, flags
  std::unordered_map<uint64_t, std::unique_ptr<psfd::Req>> reqs;
  std::deque<psfd::Req*> pending;  // waiting for a group of their kind, in ticket order
  uint64_t next = 1;
  bool stop = false;
  size_t allocated = 0;
  std::vector<std::unique_ptr<psfd::SlotGroup>> groups;  // live and released (joined at destroy)
  psfd::Status err;
};

namespace psfd {

static void finish_req(psfd_server* S, Req* r, int status) {
  std::lock_guard<std::mutex> lk(S->mu);
  r->status = status;
  r->info.status = status;
  r->t_done = clk::now();
  r->done = true;
}

template <class T>
static Status tick_group(psfd_server* S, SlotGroup& G) {
  Group& g = *G.g;
  hipStream_t s = G.s;
  const int B = G.cap;
  const Shape& sh = G.kind.sh;
  const long long n3 = sh.n3, nq = sh.nxny * 3, N = sh.N, bsv = (long long)(g.m + 1) * n3;
  auto mask_of = [&](int ph) {
    std::vector<int> m(B, 0);
    bool any = false;
    for (int b = 0; b < B; ++b) if (G.phase[b] == ph) { m[b] = 1; any = true; }
    return std::make_pair(m, any);
  };
  Status st;
  // INIT
  {
    auto mk = mask_of(P_INIT);
    if (mk.second) {
      for (int b = 0; b < B; ++b) {
        if (!mk.first[b]) continue;
        Req* r = G.req[b];
        st = group_set_tables(g, b, r->pr, r->tab, s);
        if (!st.ok()) return st;
        hipError_t e = hipMemcpyAsync(g.deps64 + (size_t)b * N, r->d_deps, N * 16, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(g.adn + (size_t)b * nq, 0, nq * 16, s);
        if (e == hipSuccess) e = hipMemsetAsync(g.st + b, 0, sizeof(GState), s);
        if (e != hipSuccess) return hip_status(e, "server init");
        G.cycles[b] = 0;
        G.tres[b] = 1;
        G.rres[b] = 0;
        G.since[b] = 0;
      }
      st = set_mask(g, g.mask2, mk.first, s);
      if (!st.ok()) return st;
      if (g.prec == PSFD_MIXED)
        vec_axpby<float2, double2, double2>(g.deps32, g.deps64, nullptr, 1.0, 0.0, N, N, g.mask2, B, s);
      st = reflect(g, g.eup, g.mask2, nullptr, s);
      if (!st.ok()) return st;
      inject(g, g.eup, g.b, g.mask2, s);
      vec_axpby<double2, double2, double2>(g.x, g.b, (const double2*)nullptr, 1.0, 0.0, n3, n3, g.mask2, B, s);
      vec_norm2<double2>(g.b, n3, n3, g.dpart, g.n2b, g.mask2, B, s);
      std::vector<double> bn2;
      st = read_norms(g, g.n2b, bn2, s);
      if (!st.ok()) return st;
      for (int b = 0; b < B; ++b)
        if (mk.first[b]) {
          G.bn[b] = std::sqrt(bn2[b]);
          G.tgt[b] = G.req[b]->o.rtol * G.bn[b];
          G.phase[b] = P_START;
        }
      std::memcpy(g.h_dbl, G.tgt.data(), sizeof(double) * B);
      hipError_t e = hipMemcpyAsync(g.abs_target, g.h_dbl, sizeof(double) * B, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_status(e, "server targets");
    }
  }
  // START: the restart's residual (b - A x, or the last cycle's basis residual),
  // convergence test, cycle start; the same decisions as the device-driven
  // solve, so a served request computes exactly what a lone solve does
  {
    auto mk = mask_of(P_START);
    if (mk.second) {
      std::vector<int> mt(B, 0), mr(B, 0);
      for (int b = 0; b < B; ++b)
        if (mk.first[b]) (G.tres[b] ? mt : mr)[b] = 1;
      st = set_mask(g, g.mask, mt, s);
      if (!st.ok()) return st;
      apply_op<double2>(g, g.deps64, vr(g.x, n3), vr(g.r, n3), g.ws64, 0, 0, 1, g.mask, s);  // A x
      // r = b - A x to the first basis vector (unnormalised) and ||r||^2
      krylov_residual<T>(g.b, g.r, (T*)g.basis, n3, n3, bsv, g.dpart, g.n2, g.mask, B, s);
      st = set_mask(g, g.rres, mr, s);
      if (!st.ok()) return st;
      krylov_sum_norm(g.lpart, g.n2, g.rres, B, s);
      std::vector<double> rn2;
      st = read_norms(g, g.n2, rn2, s);
      if (!st.ok()) return st;
      std::vector<GState> hs(B);
      hipError_t e = hipMemcpyAsync(hs.data(), g.st, sizeof(GState) * B, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_status(e, "server state");
      std::vector<int> go(B, 0);
      bool any = false;
      const int every = true_residual_every();
      for (int b = 0; b < B; ++b) {
        if (!mk.first[b]) continue;
        const double rn = std::sqrt(rn2[b]);
        const bool was_true = G.tres[b] != 0;
        Req* r = G.req[b];
        r->info.iters = hs[b].iters;
        r->info.cycles = G.cycles[b];
        if (!std::isfinite(rn)) { r->status = PSFD_ERR_NONFINITE; G.phase[b] = P_FIN; continue; }
        const bool met = rn <= G.tgt[b] || G.bn[b] == 0.0;
        const bool limit = hs[b].iters >= r->o.max_iters;
        if (was_true) {
          r->info.rel_residual = G.bn[b] > 0 ? rn / G.bn[b] : 0.0;
          if (met) { G.phase[b] = P_FIN; continue; }
          if (limit) { r->status = PSFD_NOT_CONVERGED; G.phase[b] = P_FIN; continue; }
        } else if (met || limit) {
          G.tres[b] = 1;  // decide on b - A x at the next tick, without a cycle now
          G.rres[b] = 0;
          continue;
        }
        G.since[b] = was_true ? 0 : G.since[b] + 1;
        const bool next_true = G.since[b] + 1 >= every || rn <= 2.0 * G.tgt[b];
        G.tres[b] = next_true ? 1 : 0;
        G.rres[b] = next_true ? 0 : 1;
        go[b] = 1;
        any = true;
        G.phase[b] = P_ARN;
        G.cycles[b] += 1;
      }
      if (any) {
        st = set_mask(g, g.mask, go, s);
        if (!st.ok()) return st;
        krylov_start(g.st, g.n2, g.abs_target, g.prec == PSFD_MIXED ? G.kind.eta : 0.0, g.m, cancel_threshold(),
                     g.mask, g.run, B, s);
      }
    }
  }
  // FIN: fields and orders, copy-out
  {
    auto mk = mask_of(P_FIN);
    if (mk.second) {
      st = set_mask(g, g.mask2, mk.first, s);
      if (!st.ok()) return st;
      apply_stage<double2>(g, 0, g.deps64, vr(g.x, n3), vr(g.x, n3), g.ws64, 0, 0, 0, g.mask2, s);
      launch_readout(sh.nx, sh.ny, sh.nz, vr(g.ws64, n3), g.tab, g.tab_stride, g.adn, g.aup, nq, g.mask2, B, s);
      st = reflect(g, g.eup, g.mask2, nullptr, s);
      if (!st.ok()) return st;
      inject(g, g.eup, g.e, g.mask2, s);
      launch_orders(sh.nx, sh.ny, g.tab, g.tab_stride, g.eup, g.aup, g.ord, nq, B, s);
      vec_axpby<double2, double2, double2>(g.x, g.x, g.e, 1.0, -1.0, n3, n3, g.mask2, B, s);
      for (int b = 0; b < B; ++b) {
        if (!mk.first[b]) continue;
        Req* r = G.req[b];
        hipError_t e = hipMemcpyAsync(r->d_emask, g.x + (size_t)b * n3, n3 * 16, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && r->d_orders)
          e = hipMemcpyAsync(r->d_orders, g.ord + (size_t)b * nq, nq * 16, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_status(e, "server copy-out");
      }
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_status(e, "server finish");
      for (int b = 0; b < B; ++b) {
        if (!mk.first[b]) continue;
        Req* r = G.req[b];
        r->info.outer_iters = 1;
        r->info.mono_residual = r->info.rel_residual;
        finish_req(S, r, r->status);
        G.req[b] = nullptr;
        G.phase[b] = P_FREE;
      }
    }
  }
  // ARN: Arnoldi steps of every running slot
  {
    bool any = false;
    for (int b = 0; b < B; ++b) any |= G.phase[b] == P_ARN;
    if (any) {
      // issued eagerly: the groups' worker threads, the submitting thread and
      // the caller's own threads all issue work while a group runs, and HIP
      // has failed such work in another thread during a stream capture
      for (int k = 0; k < STEPS_PER_SYNC; ++k) arnoldi_step<T>(g, 0, 1, s);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(g.h_run, g.run, sizeof(int) * B, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_status(e, "server arnoldi");
      std::vector<int> end(B, 0);
      bool anyend = false;
      for (int b = 0; b < B; ++b)
        if (G.phase[b] == P_ARN && g.h_run[b] == 0) { end[b] = 1; anyend = true; G.phase[b] = P_END; }
      // END: solution update of the finished cycles
      if (anyend) {
        st = set_mask(g, g.mask, end, s);
        if (!st.ok()) return st;
        std::vector<int> rec(B, 0);
        for (int b = 0; b < B; ++b) rec[b] = end[b] && G.rres[b];
        st = set_mask(g, g.rres, rec, s);
        if (!st.ok()) return st;
        krylov_solve_small(g.st, g.mask, B, s);
        krylov_lincomb_res<T, double2>((T*)g.basis, n3, bsv, g.x, n3, n3, g.st, g.mask, g.rres, g.lpart, B, s);
        for (int b = 0; b < B; ++b) if (end[b]) G.phase[b] = P_START;
      }
    }
  }
  return Status();
}

static void group_worker(psfd_server* S, SlotGroup* G);

// Merge requests (in ticket order) into the pending list, keeping it in ticket order.
static void to_pending(psfd_server* S, std::deque<Req*>& q) {
  for (Req* r : q) {
    auto it = S->pending.begin();
    while (it != S->pending.end() && (*it)->ticket < r->ticket) ++it;
    S->pending.insert(it, r);
  }
  q.clear();
}

static SlotGroup* live_group(psfd_server* S, const Kind& k) {
  for (auto& gp : S->groups)
    if (!gp->dead && !gp->draining && gp->kind == k) return gp.get();
  return nullptr;
}

// A new slot group of kind k with cap slots: workspace, stream and worker.
static Status make_group(psfd_server* S, const Kind& k, size_t per, int cap, SlotGroup*& out) {
  auto ng = std::make_unique<SlotGroup>();
  ng->kind = k;
  ng->g = std::make_unique<Group>();
  Status st = group_alloc(*ng->g, k.sh, cap, k.m, k.prec);
  if (!st.ok()) return st;
  hipError_t e = hipStreamCreateWithFlags(&ng->s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_status(e, "server stream");
  ng->cap = cap;
  ng->bytes = per * (size_t)cap;
  ng->req.assign(cap, nullptr);
  ng->phase.assign(cap, P_FREE);
  ng->cycles.assign(cap, 0);
  ng->tres.assign(cap, 1);
  ng->rres.assign(cap, 0);
  ng->since.assign(cap, 0);
  ng->bn.assign(cap, 0.0);
  ng->tgt.assign(cap, 0.0);
  ng->res.assign(cap, 0.0);
  S->allocated += ng->bytes;
  out = ng.get();
  S->groups.push_back(std::move(ng));
  out->worker = std::thread(group_worker, S, out);
  return Status();
}

// Admission of the pending list, first come, first served (server mutex held).
static void admit_pending(psfd_server* S) {
  while (!S->pending.empty()) {
    Req* r = S->pending.front();
    if (SlotGroup* G = live_group(S, r->kind)) {
      S->pending.pop_front();
      G->queue.push_back(r);
      G->cv.notify_one();
      continue;
    }
    const size_t per = r->slot_bytes;
    const size_t avail = S->budget > S->allocated ? S->budget - S->allocated : 0;
    if (avail >= per) {
      const int cap = (int)std::min<size_t>((size_t)S->max_slots, avail / per);
      SlotGroup* G = nullptr;
      Status st = make_group(S, r->kind, per, cap, G);
      if (!st.ok()) {
        // the device refused the memory: the request ends with that status
        S->pending.pop_front();
        S->err = st;
        r->status = st.code;
        r->info.status = st.code;
        r->t_done = clk::now();
        r->done = true;
        continue;
      }
      S->pending.pop_front();
      G->queue.push_back(r);
      G->cv.notify_one();
      continue;
    }
    // not enough memory left: release idle groups, then drain the oldest busy ones
    size_t freeing = 0;
    for (auto& gp : S->groups)
      if (!gp->dead && gp->draining) freeing += gp->bytes;
    for (int pass = 0; pass < 2 && avail + freeing < per; ++pass)
      for (auto& gp : S->groups) {
        if (gp->dead || gp->draining || avail + freeing >= per) continue;
        const bool idle = gp->occupied() == 0 && gp->queue.empty();
        if (pass == 0 && !idle) continue;
        gp->draining = true;
        freeing += gp->bytes;
        gp->cv.notify_one();
      }
    break;  // the head waits for the memory; later requests keep their place behind it
  }
}

// Release of a group by its own worker (server mutex held, queue empty): memory
// freed, then admission of the pending list.
static void release_group(psfd_server* S, SlotGroup* G) {
  G->dead = true;
  to_pending(S, G->queue);
  if (G->s) {
    (void)hipStreamSynchronize(G->s);
    (void)hipStreamDestroy(G->s);
    G->s = nullptr;
  }
  G->g.reset();
  S->allocated -= G->bytes;
  G->bytes = 0;
  admit_pending(S);
}

// Worker of one slot group: admits its queued requests into free slots and
// ticks while any slot is occupied. With no slot occupied it waits for work;
// it releases the group when asked to drain, after IDLE_RELEASE_S without work,
// or at shutdown once nothing is left for it.
static void group_worker(psfd_server* S, SlotGroup* G) {
  (void)hipSetDevice(S->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (G->occupied() == 0) {
        const bool work = G->cv.wait_for(lk, std::chrono::duration<double>(IDLE_RELEASE_S), [&] {
          return S->stop || G->draining || !G->queue.empty();
        });
        if (G->queue.empty() && (G->draining || S->stop || !work)) {
          release_group(S, G);
          return;
        }
      }
      // requests already in the queue were admitted to this group: a draining
      // group still runs them, it only takes no new ones
      for (int b = 0; b < G->cap && !G->queue.empty(); ++b) {
        if (G->req[b]) continue;
        G->req[b] = G->queue.front();
        G->phase[b] = P_INIT;
        G->queue.pop_front();
      }
    }
    Status st = G->kind.prec == PSFD_MIXED ? tick_group<float2>(S, *G) : tick_group<double2>(S, *G);
    if (!st.ok()) {
      // a runtime failure ends every request of the group
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->err = st;
      }
      for (int b = 0; b < G->cap; ++b)
        if (G->req[b]) { finish_req(S, G->req[b], st.code); G->req[b] = nullptr; G->phase[b] = P_FREE; }
    }
  }
}

Status server_create(size_t hbm_budget, int max_slots, const psfd_opts* opts, psfd_server** out) {
  Status st;
  auto S = std::make_unique<psfd_server>();
  st = make_opts(opts, S->o);
  if (!st.ok()) return st;
  S->o.coupling = PSFD_COUPLING_MONO;
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  hipError_t e = hipGetDevice(&S->device);
  if (e != hipSuccess) return hip_status(e, "server device");
  *out = S.release();
  return st;
}

Status server_submit(psfd_server* S, const psfd_problem* prob, const psfd_opts* opts, const void* d_deps,
                     void* d_emask, void* d_orders, uint64_t* ticket) {
  auto r = std::make_unique<Req>();
  Status st = validate_problem(prob, r->pr);
  if (!st.ok()) return st;
  if (opts) {
    st = make_opts(opts, r->o);
    if (!st.ok()) return st;
  } else {
    r->o = S->o;
  }
  r->o.coupling = PSFD_COUPLING_MONO;
  st = build_table(r->pr, r->tab);
  if (!st.ok()) return st;
  r->kind.sh = shape_of(r->pr.p);
  r->kind.m = r->o.restart;
  r->kind.prec = r->o.precision;
  r->kind.eta = r->o.precision == PSFD_MIXED ? r->o.inner_eta : 0.0;
  r->slot_bytes = group_bytes(r->kind.sh, 1, r->kind.m, r->kind.prec);
  r->d_deps = d_deps;
  r->d_emask = d_emask;
  r->d_orders = d_orders;
  r->t_submit = clk::now();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) { st.code = PSFD_ERR_INVALID_ARG; st.msg = "server is shutting down"; return st; }
  r->ticket = S->next++;
  *ticket = r->ticket;
  Req* raw = r.get();
  S->reqs.emplace(r->ticket, std::move(r));
  if (raw->slot_bytes > S->budget) {
    // cannot fit even an empty budget: the ticket completes at once
    raw->status = PSFD_ERR_OOM;
    raw->info.status = PSFD_ERR_OOM;
    raw->t_done = clk::now();
    raw->done = true;
    return Status();
  }
  if (SlotGroup* G = S->pending.empty() ? live_group(S, raw->kind) : nullptr) {
    G->queue.push_back(raw);
    G->cv.notify_one();
    return Status();
  }
  S->pending.push_back(raw);
  admit_pending(S);
  return Status();
}

Status server_poll(psfd_server* S, uint64_t ticket, int* done, psfd_info* info, double* latency_s) {
  Status st;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) { st.code = PSFD_ERR_INVALID_ARG; st.msg = "unknown ticket"; return st; }
  Req* r = it->second.get();
  *done = r->done ? 1 : 0;
  if (!r->done) return st;
  if (info) *info = r->info;
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  S->reqs.erase(it);
  return st;
}

Status server_destroy(psfd_server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (auto& G : S->groups) G->cv.notify_all();
  }
  // Workers finish every submitted request; a group released at shutdown may
  // admit pending requests into new groups, so join until no worker is left.
  for (;;) {
    std::vector<std::thread*> th;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto& G : S->groups)
        if (G->worker.joinable()) th.push_back(&G->worker);
    }
    if (th.empty()) break;
    for (auto* t : th) t->join();
  }
  Status st = S->err;
  delete S;
  return st;
}

}  // namespace psfd
