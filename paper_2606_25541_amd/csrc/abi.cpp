// extern "C" entry points declared in include/psfd.h.
#include <cstring>
#include <memory>
#include <string>

#include "engine.hpp"
#include "diff.hpp"
#include "iso.hpp"
#include "noalloc.hpp"
#include "serve.hpp"

using namespace psfd;

static thread_local std::string g_last_error;

static int fail(const Status& st) {
  g_last_error = st.msg;
  return st.code;
}
static int fail(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

struct psfd_plan {
  Problem pr;
  Opts o;
  Shape sh;
  std::vector<double> tab;
  int device = 0;
  std::unique_ptr<Group> solve;   // full solve workspace (lazily)
  std::unique_ptr<Group> lite;    // tables + apply scratch for psfd_apply
  void* scratch32 = nullptr;
  void* scratch64 = nullptr;
  ~psfd_plan() {
    if (scratch32) (void)hipFree(scratch32);
    if (scratch64) (void)hipFree(scratch64);
  }
};

static Status ensure_lite(psfd_plan* p, hipStream_t s);

extern "C" {

const char* psfd_version(void) { return "psfd-mi355x 0.1"; }

const char* psfd_last_error(void) { return g_last_error.c_str(); }

const char* psfd_status_string(int s) {
  switch (s) {
    case PSFD_OK: return "ok";
    case PSFD_NOT_CONVERGED: return "not converged";
    case PSFD_ERR_INVALID_ARG: return "invalid argument";
    case PSFD_ERR_UNSUPPORTED_SIZE: return "unsupported size";
    case PSFD_ERR_OOM: return "out of device memory";
    case PSFD_ERR_SINGULAR: return "singular (grazing order)";
    case PSFD_ERR_NONFINITE: return "non-finite value";
    case PSFD_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int psfd_plan_create(const psfd_problem* prob, const psfd_opts* opts, psfd_plan** out) {
  if (!out) return fail(PSFD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  auto plan = std::make_unique<psfd_plan>();
  Status st = validate_problem(prob, plan->pr);
  if (!st.ok()) return fail(st);
  st = make_opts(opts, plan->o);
  if (!st.ok()) return fail(st);
  plan->sh = shape_of(plan->pr.p);
  st = build_table(plan->pr, plan->tab);
  if (!st.ok()) return fail(st);
  if (hipGetDevice(&plan->device) != hipSuccess) return fail(PSFD_ERR_HIP, "hipGetDevice failed");
  // device tables now, so that the applies allocate no table memory later; the
  // device's scratch array of the allocation-free apply is looked up here too
  st = ensure_lite(plan.get(), nullptr);
  if (st.ok()) {
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) st = hip_status(e, "plan tables");
  }
  if (!st.ok()) return fail(st);
  void* sp = nullptr;
  st = noalloc_scratch(plan->device, &sp);
  if (!st.ok()) return fail(st);
  *out = plan.release();
  return PSFD_OK;
}

void psfd_plan_destroy(psfd_plan* plan) { delete plan; }

int psfd_plan_footprint(const psfd_plan* plan, size_t* device_bytes) {
  if (!plan || !device_bytes) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  *device_bytes = group_bytes(plan->sh, 1, plan->o.restart, plan->o.precision);
  return PSFD_OK;
}

static Status ensure_lite(psfd_plan* p, hipStream_t s) {
  if (p->lite) return Status();
  auto g = std::make_unique<Group>();
  Status st = device_consts(g->dc);
  if (!st.ok()) return st;
  g->sh = p->sh;
  g->B = 1;
  g->tab_stride = (long long)p->tab.size();
  void* t = nullptr;
  hipError_t e = hipMalloc(&t, p->tab.size() * 8);
  if (e != hipSuccess) return hip_status(e, "hipMalloc");
  g->owned.push_back(t);
  g->tab = (double*)t;
  e = hipMalloc(&t, (LAYER_CAP + 2) * sizeof(double4));
  if (e != hipSuccess) return hip_status(e, "hipMalloc");
  g->owned.push_back(t);
  g->lay = (double4*)t;
  st = group_set_tables(*g, 0, p->pr, p->tab, s);
  if (!st.ok()) return st;
  p->lite = std::move(g);
  return Status();
}

int psfd_apply(psfd_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, int flags, void* stream) {
  if (!plan || !d_deps || !d_x || !d_y) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  if (d_x == d_y) return fail(PSFD_ERR_INVALID_ARG, "d_y must not alias d_x");
  if (dtype != PSFD_C64 && dtype != PSFD_C128) return fail(PSFD_ERR_INVALID_ARG, "dtype must be PSFD_C64 or PSFD_C128");
  hipStream_t s = (hipStream_t)stream;
  Status st = ensure_lite(plan, s);
  if (!st.ok()) return fail(st);
  const size_t esz = dtype == PSFD_C64 ? 8 : 16;
  void*& scratch = dtype == PSFD_C64 ? plan->scratch32 : plan->scratch64;
  if (!scratch) {
    hipError_t e = hipMalloc(&scratch, (size_t)plan->sh.n3 * esz);
    if (e != hipSuccess) return fail(hip_status(e, "hipMalloc"));
  }
  const int kmode = (flags & PSFD_APPLY_K_ONLY) ? 1 : 0;
  const int tr = (flags & PSFD_APPLY_TRANSPOSE) ? 1 : 0;
  const int rf = (flags & PSFD_APPLY_REFLECT) ? 1 : 0;
  Group& g = *plan->lite;
  if (dtype == PSFD_C64)
    apply_op<float2>(g, (const float2*)d_deps, vr(d_x), vr(d_y), (float2*)scratch, kmode, tr, rf, nullptr, s);
  else
    apply_op<double2>(g, (const double2*)d_deps, vr(d_x), vr(d_y), (double2*)scratch, kmode, tr, rf, nullptr, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(hip_status(e, "apply launch"));
  return PSFD_OK;
}

int psfd_apply_noalloc(psfd_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, int flags,
                       void* stream) {
  if (!plan || !d_deps || !d_x || !d_y) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  if (d_x == d_y) return fail(PSFD_ERR_INVALID_ARG, "d_y must not alias d_x");
  if (dtype != PSFD_C64 && dtype != PSFD_C128) return fail(PSFD_ERR_INVALID_ARG, "dtype must be PSFD_C64 or PSFD_C128");
  if (!plan->lite) return fail(PSFD_ERR_INVALID_ARG, "the plan has no device tables");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(PSFD_ERR_HIP, "hipGetDevice failed");
  if (cur != plan->device) return fail(PSFD_ERR_INVALID_ARG, "the plan's device is not the current device");
  Status st = apply_noalloc(*plan->lite, cur, d_deps, d_x, d_y, dtype, flags, (hipStream_t)stream);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_bench_stage(psfd_plan* plan, int stage, const void* d_deps, const void* d_x, void* d_y, int dtype,
                     int reps, float* ms, void* stream) {
  if (!plan || !d_deps || !d_x || !d_y || !ms || reps < 1 || stage < 0 || stage > 2)
    return fail(PSFD_ERR_INVALID_ARG, "bad arguments");
  if (dtype != PSFD_C64 && dtype != PSFD_C128) return fail(PSFD_ERR_INVALID_ARG, "bad dtype");
  hipStream_t s = (hipStream_t)stream;
  Status st = ensure_lite(plan, s);
  if (!st.ok()) return fail(st);
  const size_t esz = dtype == PSFD_C64 ? 8 : 16;
  void*& scratch = dtype == PSFD_C64 ? plan->scratch32 : plan->scratch64;
  if (!scratch) {
    hipError_t e = hipMalloc(&scratch, (size_t)plan->sh.n3 * esz);
    if (e != hipSuccess) return fail(hip_status(e, "hipMalloc"));
    (void)hipMemsetAsync(scratch, 0, (size_t)plan->sh.n3 * esz, s);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(PSFD_ERR_HIP, "hipEventCreate");
  Group& g = *plan->lite;
  const bool qp = quarter_planes(g, esz);  // the stage as psfd_apply runs it
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) {
    if (dtype == PSFD_C64)
      apply_stage<float2>(g, stage, (const float2*)d_deps, vr(d_x), vr(d_y), (float2*)scratch, 0, 0, 1, nullptr, s,
                          nullptr, 0, nullptr, qp);
    else
      apply_stage<double2>(g, stage, (const double2*)d_deps, vr(d_x), vr(d_y), (double2*)scratch, 0, 0, 1,
                           nullptr, s, nullptr, 0, nullptr, qp);
  }
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(hip_status(e, "stage timing"));
  *ms = t / reps;
  return PSFD_OK;
}

int psfd_bench_gram_schmidt(psfd_plan* plan, int pass, int j, const void* d_x, int dtype, int reps, float* ms,
                            void* stream) {
  if (!plan || !d_x || !ms || reps < 1 || pass < 0 || pass > 3 || j < 0 || j >= MAXM)
    return fail(PSFD_ERR_INVALID_ARG, "bad arguments");
  if (dtype != PSFD_C64 && dtype != PSFD_C128) return fail(PSFD_ERR_INVALID_ARG, "bad dtype");
  hipStream_t s = (hipStream_t)stream;
  const int prec = dtype == PSFD_C64 ? PSFD_MIXED : PSFD_FP64;
  Group g;
  Status st = group_alloc(g, plan->sh, 1, j + 1, prec);
  if (st.ok()) st = bench_gram_schmidt(g, pass, j, d_x, reps, ms, s);
  if (st.ok()) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_status(e, "Gram-Schmidt timing");
  }
  if (!st.ok()) return fail(st);
  return PSFD_OK;
}

static void fill_info(psfd_info* info, const SolveStats& s) {
  if (!info) return;
  info->iters = s.iters;
  info->outer_iters = s.outer;
  info->cycles = s.cycles;
  info->status = s.status;
  info->rel_residual = s.rel_res;
  info->outer_change = s.change;
  info->mono_residual = s.mono;
}

static Status ensure_solve(psfd_plan* p, hipStream_t s) {
  if (p->solve) return Status();
  auto g = std::make_unique<Group>();
  Status st = group_alloc(*g, p->sh, 1, p->o.restart, p->o.precision);
  if (!st.ok()) return st;
  st = group_set_tables(*g, 0, p->pr, p->tab, s);
  if (!st.ok()) return st;
  p->solve = std::move(g);
  return Status();
}

int psfd_solve(psfd_plan* plan, const void* d_deps, void* d_emask, void* d_orders, void* d_u, psfd_info* info,
               void* stream) {
  if (!plan || !d_deps || !d_emask) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  Status st = ensure_solve(plan, s);
  if (!st.ok()) return fail(st);
  Group& g = *plan->solve;
  const Shape& sh = plan->sh;
  hipError_t e = hipMemcpyAsync(g.deps64, d_deps, sh.N * 16, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(hip_status(e, "copy contrast"));
  std::vector<SolveStats> stats;
  st = solve_group(g, plan->o, stats, s);
  if (!st.ok()) return fail(st);
  e = hipMemcpyAsync(d_emask, g.x, sh.n3 * 16, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && d_orders) e = hipMemcpyAsync(d_orders, g.ord, sh.nxny * 3 * 16, hipMemcpyDeviceToDevice, s);
  // total field u = E_mask + E_inc + E_layer (g.x + g.e after either coupling)
  if (e == hipSuccess && d_u) {
    vec_axpby<double2, double2, double2>((double2*)d_u, g.x, g.e, 1.0, 1.0, sh.n3, sh.n3, nullptr, 1, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(hip_status(e, "copy results"));
  fill_info(info, stats[0]);
  if (stats[0].status < 0) return fail(stats[0].status, "non-finite residual");
  if (stats[0].status == PSFD_NOT_CONVERGED) {
    g_last_error = "iteration limit reached";
    return PSFD_NOT_CONVERGED;
  }
  return PSFD_OK;
}

int psfd_solve_adjoint(psfd_plan* plan, const void* d_deps, const void* d_u, const void* d_grad_orders, void* d_grad,
                       psfd_info* info, void* stream) {
  if (!plan || !d_deps || !d_u || !d_grad_orders || !d_grad) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  if (d_grad == d_u || d_grad == d_grad_orders || d_grad == d_deps)
    return fail(PSFD_ERR_INVALID_ARG, "d_grad must not alias an input");
  hipStream_t s = (hipStream_t)stream;
  Status st = ensure_solve(plan, s);
  if (!st.ok()) return fail(st);
  Group& g = *plan->solve;
  const Shape& sh = plan->sh;
  hipError_t e = hipMemcpyAsync(g.deps64, d_deps, sh.N * 16, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(hip_status(e, "copy contrast"));
  std::vector<SolveStats> ast;
  st = adjoint_group(g, plan->o, (const double2*)d_u, (const double2*)d_grad_orders, (double2*)d_grad, ast, s);
  if (!st.ok()) return fail(st);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(hip_status(e, "adjoint"));
  fill_info(info, ast[0]);
  if (ast[0].status < 0) return fail(ast[0].status, "non-finite residual");
  if (ast[0].status == PSFD_NOT_CONVERGED) {
    g_last_error = "iteration limit reached";
    return PSFD_NOT_CONVERGED;
  }
  return PSFD_OK;
}

int psfd_solve_batch(int32_t n, const psfd_problem* probs, const psfd_opts* opts, const void* const* d_deps,
                     void* const* d_emask, void* const* d_orders, psfd_info* info, void* stream) {
  if (n <= 0 || !probs || !d_deps || !d_emask) return fail(PSFD_ERR_INVALID_ARG, "bad batch arguments");
  Status st = solve_batch(n, probs, opts, d_deps, d_emask, d_orders, info, (hipStream_t)stream);
  if (!st.ok()) return fail(st);
  bool nc = false;
  for (int i = 0; info && i < n; ++i) nc |= info[i].status == PSFD_NOT_CONVERGED;
  return nc ? PSFD_NOT_CONVERGED : PSFD_OK;
}

int psfd_release_cached_workspaces(void) {
  release_cached_groups();
  return PSFD_OK;
}

int psfd_server_create(size_t hbm_budget, int32_t max_slots, const psfd_opts* opts, psfd_server** out) {
  if (!out || max_slots < 1 || hbm_budget == 0) return fail(PSFD_ERR_INVALID_ARG, "bad server arguments");
  Status st = server_create(hbm_budget, max_slots, opts, out);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_server_submit(psfd_server* srv, const psfd_problem* prob, const psfd_opts* opts, const void* d_deps,
                       void* d_emask, void* d_orders, uint64_t* ticket) {
  if (!srv || !prob || !d_deps || !d_emask || !ticket) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  Status st = server_submit(srv, prob, opts, d_deps, d_emask, d_orders, ticket);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_server_poll(psfd_server* srv, uint64_t ticket, int32_t* done, psfd_info* info, double* latency_s) {
  if (!srv || !done) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  Status st = server_poll(srv, ticket, done, info, latency_s);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_server_destroy(psfd_server* srv) {
  if (!srv) return fail(PSFD_ERR_INVALID_ARG, "NULL server");
  Status st = server_destroy(srv);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_diff_plan_create(const psfd_diff_problem* prob, psfd_diff_plan** out) {
  if (!prob || !out) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  Status st = diff_create(*prob, *out);
  return st.ok() ? PSFD_OK : fail(st);
}

void psfd_diff_plan_destroy(psfd_diff_plan* plan) { diff_destroy(plan); }

int psfd_diff_apply(psfd_diff_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, int precond,
                    void* stream) {
  if (!plan || !d_deps || !d_x || !d_y) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  if (d_x == d_y) return fail(PSFD_ERR_INVALID_ARG, "d_y must not alias d_x");
  if (dtype != PSFD_C64 && dtype != PSFD_C128) return fail(PSFD_ERR_INVALID_ARG, "dtype must be PSFD_C64 or PSFD_C128");
  Status st = diff_apply(plan, d_deps, d_x, d_y, dtype, precond, (hipStream_t)stream);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_diff_solve(psfd_diff_plan* plan, const void* d_deps, void* d_e, void* d_orders, const psfd_opts* opts,
                    int precond, psfd_info* info, void* stream) {
  if (!plan || !d_deps || !d_e) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  psfd_info inf{};
  Status st = diff_solve(plan, d_deps, d_e, d_orders, opts, precond, &inf, (hipStream_t)stream);
  if (info) *info = inf;
  if (!st.ok()) return fail(st);
  if (inf.status == PSFD_NOT_CONVERGED) {
    g_last_error = "iteration limit reached";
    return PSFD_NOT_CONVERGED;
  }
  return PSFD_OK;
}

int psfd_iso_plan_create(const psfd_iso_problem* prob, psfd_iso_plan** out) {
  if (!prob || !out) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  Status st = iso_create(*prob, *out);
  return st.ok() ? PSFD_OK : fail(st);
}

void psfd_iso_plan_destroy(psfd_iso_plan* plan) { iso_destroy(plan); }

int psfd_iso_apply(psfd_iso_plan* plan, const void* d_deps, const void* d_x, void* d_y, int dtype, void* stream) {
  if (!plan || !d_deps || !d_x || !d_y) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  if (d_x == d_y) return fail(PSFD_ERR_INVALID_ARG, "d_y must not alias d_x");
  Status st = iso_apply(plan, d_deps, d_x, d_y, dtype, -1, (hipStream_t)stream);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_iso_solve(psfd_iso_plan* plan, const void* d_deps, const void* d_b, void* d_u, double rtol, int32_t restart,
                   int32_t max_iters, int32_t precision, psfd_info* info, void* stream) {
  if (!plan || !d_deps || !d_b || !d_u) return fail(PSFD_ERR_INVALID_ARG, "NULL argument");
  if (d_b == d_u) return fail(PSFD_ERR_INVALID_ARG, "d_u must not alias d_b");
  psfd_info inf{};
  Status st = iso_solve(plan, d_deps, d_b, d_u, rtol, restart, max_iters, precision, &inf, (hipStream_t)stream);
  if (info) *info = inf;
  if (!st.ok()) return fail(st);
  if (inf.status == PSFD_NOT_CONVERGED) {
    g_last_error = "iteration limit reached";
    return PSFD_NOT_CONVERGED;
  }
  return PSFD_OK;
}

int psfd_iso_table(psfd_iso_plan* plan, void* d_table, int32_t* over, double* radius_nm, void* stream) {
  if (!plan) return fail(PSFD_ERR_INVALID_ARG, "NULL plan");
  Status st = iso_table(plan, d_table, over, radius_nm, (hipStream_t)stream);
  return st.ok() ? PSFD_OK : fail(st);
}

int psfd_iso_bench_stage(psfd_iso_plan* plan, int stage, const void* d_deps, const void* d_x, void* d_y, int dtype,
                         int reps, float* ms, void* stream) {
  if (!plan || !d_deps || !d_x || !d_y || !ms || reps < 1) return fail(PSFD_ERR_INVALID_ARG, "bad arguments");
  if (d_x == d_y) return fail(PSFD_ERR_INVALID_ARG, "d_y must not alias d_x");
  hipStream_t s = (hipStream_t)stream;
  Status st = iso_apply(plan, d_deps, d_x, d_y, dtype, stage, s);  // untimed first launch
  if (!st.ok()) return fail(st);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(PSFD_ERR_HIP, "hipEventCreate");
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps && st.ok(); ++r) st = iso_apply(plan, d_deps, d_x, d_y, dtype, stage, s);
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!st.ok()) return fail(st);
  if (e != hipSuccess) return fail(PSFD_ERR_HIP, hipGetErrorString(e));
  *ms = t / reps;
  return PSFD_OK;
}

}  // extern "C"
