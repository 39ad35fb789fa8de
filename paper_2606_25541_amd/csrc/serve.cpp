// Batched solves of same-shape instances in lock-step launches, and the
// continuous-batching solve server.
#include "serve.hpp"

#include <cmath>
#include <cstring>

namespace psfd {

static bool same_shape(const psfd_problem& a, const psfd_problem& b) {
  return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lx_nm == b.lx_nm && a.ly_nm == b.ly_nm &&
         a.t_nm == b.t_nm;
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
  Group g;
  st = group_alloc(g, sh, n, o.restart, o.precision);
  if (!st.ok()) return st;
  std::vector<double> tab;
  for (int i = 0; i < n; ++i) {
    st = build_table(pr[i], tab);
    if (!st.ok()) return st;
    st = group_set_tables(g, i, tab, s);
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
  return st;
}

Status server_create(size_t, int, const psfd_opts*, psfd_server**) {
  Status st; st.code = PSFD_ERR_INVALID_ARG; st.msg = "server not available"; return st;
}
Status server_submit(psfd_server*, const psfd_problem*, const void*, void*, void*, uint64_t*) {
  Status st; st.code = PSFD_ERR_INVALID_ARG; st.msg = "server not available"; return st;
}
Status server_poll(psfd_server*, uint64_t, int*, psfd_info*, double*) {
  Status st; st.code = PSFD_ERR_INVALID_ARG; st.msg = "server not available"; return st;
}
Status server_destroy(psfd_server*) {
  Status st; st.code = PSFD_ERR_INVALID_ARG; st.msg = "server not available"; return st;
}

}  // namespace psfd
