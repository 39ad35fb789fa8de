// The Givens step of restarted GMRES as a block-level device task, shared by
// the update-final kernel and by the first operator-apply kernel of the next
// Arnoldi step, which runs it in one extra block on a CU its planes leave free.
// Both callers get bitwise the same ||w||^2 (and so the same scale of the new
// vector) from the same fixed-order sum of the norm partials.
#pragma once
#include "krylov.hpp"

namespace psfd {


PSFD_D double gv_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ||w||^2 from the nblk (<= RED_BLOCKS) norm partials of one instance, in two
// halves for callers with barriers of their own between them. norm_wave_sums:
// the first GIVENS_THREADS threads take partials tid, tid + 256, ... in order
// and leave their four wavefront sums in gs (LDS; the other threads do
// nothing). norm_total, after a barrier: the four sums in order.
PSFD_D void norm_wave_sums(const double2* pb, int nblk, double2* gs) {
  constexpr int PK = RED_BLOCKS / GIVENS_THREADS;
  const int tid = threadIdx.x;
  if (tid < GIVENS_THREADS) {
    double2 pv[PK];
    double2 acc = make_double2(0, 0);
#pragma unroll
    for (int k = 0; k < PK; ++k) pv[k] = pb[min(tid + k * GIVENS_THREADS, nblk - 1)];
#pragma unroll
    for (int k = 0; k < PK; ++k)
      if (tid + k * GIVENS_THREADS < nblk) acc = cadd(acc, pv[k]);
    const double re = gv_wave_sum(acc.x), im = gv_wave_sum(acc.y);
    if ((tid & 63) == 0) gs[tid >> 6] = make_double2(re, im);
  }
}
PSFD_D double norm_total(const double2* gs) {
  double2 t = gs[0];
  for (int wv = 1; wv < GIVENS_THREADS / 64; ++wv) t = cadd(t, gs[wv]);
  return t.x;
}

// Both halves with their barriers: every thread of the block must call it, and
// the block must have at least GIVENS_THREADS threads; all of them get the total.
PSFD_D double norm_from_partials(const double2* pb, int nblk) {
  __shared__ double2 gsm[GIVENS_THREADS / 64];
  __shared__ double gtot;
  norm_wave_sums(pb, nblk, gsm);
  __syncthreads();
  if (threadIdx.x == 0) gtot = norm_total(gsm);
  __syncthreads();
  return gtot;
}

// scale of the new vector from ||w||^2: v_{j+1} = -w / ||w||
PSFD_D double inv_norm_of(double wn2) {
  const double hn = sqrt(wn2);
  return hn > 0.0 ? -1.0 / hn : 0.0;
}

// ||w||^2 over the norm partials, then the Givens step of column j of A's
// Hessenberg for instance b. Arnoldi runs on B with A = I - B: column j of A's
// Hessenberg is e_j - h, and v_{j+1} = -(B v_j - V h) / ||.|| keeps the
// subdiagonal positive. Severe cancellation (||w||^2 after the update below
// cancel_thr times its value before) ends the cycle at this column instead of
// a second Gram-Schmidt pass: the columns so far are kept, and the restart's
// residual, computed afresh, carries the solve on with a new orthonormal basis.
// Every global read is issued at the start, before the first wait (flag,
// partials, this column's Givens inputs, the scalars), so the task pays one
// memory latency; the rotations of the earlier columns are staged in LDS, so
// the single-thread recurrence reads no global memory. Every thread of the
// block must call it (blockDim >= GIVENS_THREADS).
// PROJ: the caller passes this thread's projection hp (h_t of the column), ||w||^2
// before the update (wn2in_p) and after it (wn2_p) instead of the state and the
// norm partials, and the column's slot j + 1 keeps w (raw_last = j + 1).
template <bool PROJ>
PSFD_D void givens_impl(GState* st, int* run, const double2* part, int nblk, int b, double2 hp, double wn2in_p,
                        double wn2_p) {
  static_assert(GIVENS_THREADS > MAXM, "one thread per Hessenberg row");
  __shared__ double2 col[MAXM + 1], snl[MAXM], gj_s;
  __shared__ double csl[MAXM];
  const int tid = threadIdx.x;
  GState& S = st[b];
  const int runb = run[b], j = S.j;
  const double2 hv = PROJ ? hp : S.h[min(tid, MAXM)], gv = S.g[min(tid, MAXM)], snv = S.sn[min(tid, MAXM - 1)];
  const double csv = S.cs[min(tid, MAXM - 1)];
  const double thr = S.cancel_thr, wn2in = PROJ ? wn2in_p : S.wn2_in, beta = S.beta, target = S.target;
  const int m = S.m, iters = S.iters, ncancel = S.ncancel;
  // values used only under a branch below: tie them here, or the compiler sinks
  // their loads into the branch, each then costing a full memory latency
  asm volatile("" ::"v"(hv.x), "v"(hv.y), "v"(gv.x), "v"(gv.y), "v"(snv.x), "v"(snv.y), "v"(csv));
  asm volatile("" ::"s"(thr), "s"(wn2in), "s"(beta), "s"(target), "s"(m), "s"(iters), "s"(ncancel));
  if (!runb) return;
  const double wn2 = PROJ ? wn2_p : norm_from_partials(part + (long long)b * nblk, nblk);
  const bool cancel = wn2 < thr * wn2in;
  if (tid <= j) col[tid] = make_double2((tid == j ? 1.0 : 0.0) - hv.x, -hv.y);
  if (tid < j) { csl[tid] = csv; snl[tid] = snv; }
  if (tid == j) gj_s = gv;
  __syncthreads();
  if (tid == 0) {
    const double hn = sqrt(wn2);
    for (int i = 0; i < j; ++i) {
      const double2 a = col[i], c = col[i + 1];
      const double2 sn = snl[i];
      const double cs = csl[i];
      col[i] = cadd(cscale(a, cs), cmul(sn, c));
      col[i + 1] = csub(cscale(c, cs), cmulc(a, sn) /* a * conj(sn) */);
    }
    const double2 a = col[j];
    const double aa = sqrt(cabs2(a));
    const double den = hypot(aa, hn);
    double cs;
    double2 sn;
    if (aa == 0.0) { cs = 0.0; sn = make_double2(1.0, 0.0); }
    else { cs = aa / den; sn = make_double2(a.x / aa * hn / den, a.y / aa * hn / den); }
    col[j] = cadd(cscale(a, cs), cscale(sn, hn));
    S.cs[j] = cs;
    S.sn[j] = sn;
    const double2 gj = gj_s;
    // g_{j+1} = -conj(sn) g_j ; g_j = cs g_j
    const double2 gn = cmul(make_double2(sn.x, -sn.y), gj);
    S.g[j + 1] = make_double2(-gn.x, -gn.y);
    S.g[j] = cscale(gj, cs);
    const double res = sqrt(cabs2(gn));
    S.res = res;
    S.iters = iters + 1;
    S.ncols = j + 1;
    S.inv_norm = inv_norm_of(wn2);
    S.sc[j + 1] = S.inv_norm;
    const bool conv = res <= target;
    S.conv = conv;
    S.jcur = j;
    S.j = j + 1;  // slot j + 1 holds the unnormalised new vector; the next apply scales it
    const bool breakdown = !(hn > 1e-300 * (beta > 0 ? beta : 1.0));
    const bool stop = conv || (j + 1 >= m) || breakdown || cancel || !(res == res);
    S.wn2 = wn2;
    S.raw_last = PROJ ? j + 1 : 0;
    if (cancel) S.ncancel = ncancel + 1;
    S.stop = stop;
    run[b] = stop ? 0 : 1;
  }
  __syncthreads();
  if (tid <= j) S.H[tid][j] = col[tid];
}

PSFD_D void givens_task(GState* st, int* run, const double2* part, int nblk, int b) {
  givens_impl<false>(st, run, part, nblk, b, make_double2(0, 0), 0.0, 0.0);
}

}  // namespace psfd
