// Restarted GMRES state and Krylov kernel launchers (device-side Arnoldi/Givens).
//
// Every launcher works on a batch of independent instances: instance b finds
// its vectors at b * bstride and its state at st[b]; run[b] == 0 makes every
// kernel skip that instance (converged, finished cycle or empty slot).
// Reductions are two-stage with a fixed block count and a fixed summation
// order, so results are bitwise reproducible and independent of the batch.
#pragma once
#include "layout.hpp"

namespace psfd {

constexpr int MAXM = 32;          // largest supported restart length
constexpr int RED_BLOCKS = 1024;  // blocks per instance of the first reduction stage
constexpr int LIN_BLOCKS = 2048;  // blocks per instance of the solution update (its norm partials)
// blocks per instance of the projection pass: 256 of 1024 threads (FP32 vectors)
// or 512 of 512 threads (FP64)
template <class T> struct DotBlocks { static constexpr int value = sizeof(T) == 8 ? 256 : 512; };
constexpr int DOT_BLOCKS_MAX = 512;
constexpr int PSTR = MAXM + 2;    // partial stride: up to MAXM + 1 dots and ||w||^2
// threads of a block that take part in the Givens task and its norm sum; a
// kernel that runs them needs at least this many threads per block
constexpr int GIVENS_THREADS = 256;

// What a solve's cycle start reports to the host per instance, in host memory
// mapped for the device: still active, b - A x wanted at the next restart,
// ||r|| / target at the last restart that formed a residual, and the cycles
// started by then.
struct HostFlags {
  int act;
  int want;
  double ratio;
  int cycles;
  int pad;
};

// Device-resident state of one GMRES(m) instance. All scalars are FP64.
struct GState {
  int j;            // index of the newest basis vector v_j (the column being built)
  int m;            // restart length
  int stop;         // cycle finished (converged, full or breakdown)
  int conv;         // residual estimate at or below target
  int iters;        // Arnoldi steps taken (all cycles)
  int ncols;        // Hessenberg columns completed in the current cycle
  int ncancel;      // cycles ended early by severe cancellation (all cycles)
  int since_true;   // restarts since the last one with b - A x evaluated (basis residuals in between)
  int raw_last;     // k > 0: slot k holds w before its Gram-Schmidt update (last column of the
                    // cycle, Givens step from the projections); 0: every slot is updated
  int pend;         // 1: slot j + 1 holds B v_j with its projections stored, and the update of
                    // column j is left to the next forward plane kernel (set by the inverse
                    // kernel that forms the projections, cleared at a cycle start)
  double target;    // stopping threshold of the residual estimate
  double res;       // |g_{j+1}|: current residual estimate
  double beta;      // ||r0|| of the current cycle
  double inv_norm;  // scale of the newest slot, sc[j] (-1 / ||w||; 1 / ||r|| for v_0)
  double wn2;       // ||w||^2 after the last orthogonalisation pass
  double wn2_in;    // ||w||^2 before the pass
  double cancel_thr;  // the cycle ends when ||w||^2 after the update < cancel_thr * ||w||^2 before
  int jcur;         // column index of the last step
  int cycles;       // restart cycles of the current linear solve
  int status;       // PSFD_OK, PSFD_NOT_CONVERGED or PSFD_ERR_NONFINITE (linear solve)
  int iter_limit;   // the linear solve stops once iters reaches it
  double bnorm;     // ||b|| of the current linear solve
  double rel_res;   // ||b - A x|| / ||b|| at the last FP64 residual
  double2 H[MAXM + 1][MAXM];  // rotated Hessenberg matrix (upper triangle used)
  double cs[MAXM];
  double2 sn[MAXM];
  double2 g[MAXM + 1];
  double2 y[MAXM];
  double2 h[MAXM + 1];        // Gram-Schmidt coefficients of the current column
  double2 cres[MAXM + 1];     // GMRES residual of the cycle in the basis: r = sum_i cres_i slot_i
  double sc[MAXM + 1];        // slot scales: v_i = sc[i] slot_i (slots keep the unnormalised vectors)
};

// The Arnoldi process runs on B for systems A = I - B (B = K V or M V): the apply
// writes B v_j into slot j+1, Gram-Schmidt orthogonalises it, and the Givens step
// forms column j of A's Hessenberg as e_j - h (same Krylov space, no cancellation
// against the identity part).
// Classical Gram-Schmidt on w = v_{j+1} (the new apply output), one pass:
// h[i] = <v_i, w> for i = 0..j and wn2_in = ||w||^2. The projection kernel
// leaves per-block partials in dpart (PSTR * DotBlocks<T> complex values per
// instance); the update kernel sums them.
// jh >= 0: every running instance stands at step j = jh (lock-step callers),
// which spares the kernels the read of j; jh < 0: j from the state.
template <class T>
void krylov_dots(const T* V, long long ldv, long long bsv, long long n, GState* st, const int* run,
                 double2* dpart, int nbatch, hipStream_t s, int jh = -1);
// w = v_{j+1}: h from the projection partials, w -= sum_{i<=j} h_i v_i,
// wn2 = ||w||^2 afterwards (partials in part, RED_BLOCKS per instance), then the
// Givens step (rotated Hessenberg column, residual estimate, inv_norm,
// stop/run). Severe cancellation (wn2 < cancel_thr * wn2_in) ends the cycle at
// this column: the restart's fresh residual replaces a second pass.
// givens == false leaves the Givens step to a later launch (krylov_givens, or
// the first apply kernel of the next step, which reads the same norm partials).
template <class T>
void krylov_update(T* V, long long ldv, long long bsv, long long n, GState* st, int* run,
                   const double2* dpart, double2* part, int nbatch, hipStream_t s, int jh = -1,
                   bool givens = true);
// the Givens step of the newest column from the norm partials of krylov_update
// (RED_BLOCKS per instance in part): one block per instance
void krylov_givens(GState* st, int* run, const double2* part, int nbatch, hipStream_t s);
// The last column of a cycle without its update pass: h and ||w||^2 from the
// projection partials (DotBlocks<float2> per value in dpart, as the update pass
// sums them), ||w - V h||^2 = ||w||^2 - sum |h_i|^2 (orthonormal basis), then the
// Givens step. Slot j + 1 keeps w; the residual coefficients of the restart fold
// the update in (krylov_solve_small). One block per instance; FP32 bases.
void krylov_givens_proj(GState* st, int* run, const double2* dpart, int nbatch, hipStream_t s, int jh);
// y = H^{-1} g over the k = j + 1 completed columns, and the coefficients of the
// cycle's GMRES residual in the basis, cres = Q^H (g_k e_k) (Q: the Givens
// rotations); both are stored times the slot scales sc[i], as coefficients of
// the slots themselves. When slot k holds w before its update (raw_last == k),
// cres_i -= cres_k h_i sc_i for i < k, so that cres applies to the slots as they are
void krylov_solve_small(GState* st, const int* mask, int nbatch, hipStream_t s);
// krylov_givens_proj (column jh) followed by krylov_solve_small (mask) in one launch
void krylov_givens_proj_solve(GState* st, int* run, const double2* dpart, const int* mask, int nbatch, hipStream_t s,
                              int jh);
// x += sum_{i<k} y_i v_i for the instances with mask[b]; for those with rec[b]
// also the restart residual from the basis, r = sum_{i<=k} cres_i slot_i, into
// slot 0 (unnormalised) with ||r||^2 partials in part (LIN_BLOCKS per instance),
// read by krylov_sum_norm. Slot 0 is read before it is overwritten, element by
// element, in the same thread.
template <class T, class TX>
void krylov_lincomb_res(T* V, long long ldv, long long bsv, TX* x, long long bsx, long long n, GState* st,
                        const int* mask, const int* rec, double* part, int nbatch, hipStream_t s);
// n2[b] = sum of the LIN_BLOCKS partials of krylov_lincomb_res in part, for the instances with mask[b]
void krylov_sum_norm(const double* part, double* n2, const int* mask, int nbatch, hipStream_t s);
// Device-driven restarted solve of the instances with act[b] set.
// krylov_solve_init: bnorm = sqrt(bnorm2[b]), abs_target[b] = rtol[b] bnorm,
// iter_limit = iters + max_iters, cycles = 0, status = PSFD_OK.
void krylov_solve_init(GState* st, const double* bnorm2, const double* rtol, double* abs_target, int max_iters,
                       const int* act, int nbatch, hipStream_t s);
// r = b - ax (FP64) for the instances with mask[b]: ||r||^2 to n2[b] (partials
// in part, RED_BLOCKS per instance) and r, unnormalised, to the first basis
// vector v0 (instance stride bsv) in the working precision
template <class T>
void krylov_residual(const double2* b, const double2* ax, T* v0, long long n, long long bs, long long bsv,
                     double* part, double* n2, const int* mask, int nbatch, hipStream_t s);
// the same without the sum of the partials (krylov_cycle_start_sum sums them)
template <class T>
void krylov_residual_parts(const double2* b, const double2* ax, T* v0, long long n, long long bs, long long bsv,
                           double* part, const int* mask, int nbatch, hipStream_t s);
// krylov_cycle_start, at a restart of an active instance with ||r||^2 in
// rnorm2[b]. The restart's residual is b - A x (FP64; tres[b] set) or the
// previous cycle's GMRES residual in its basis (rres[b] set).
// - A non-finite residual ends the solve with status NONFINITE.
// - After b - A x: records rel_res, and ends the solve (act[b] = 0) when the
//   residual meets abs_target[b] (or b = 0), or with status NOT_CONVERGED when
//   the iteration limit is reached.
// - After a basis residual that meets the target, or at the iteration limit:
//   runs no cycle; the next restart evaluates b - A x to decide.
// - Otherwise starts a cycle like krylov_start, with inv_norm = 1 / ||r|| for
//   the unnormalised v0, and chooses the next restart's residual: b - A x when
//   `every` restarts have passed since the last one, or when ||r|| is within
//   twice the target; the basis residual otherwise.
// cyc[b] and run[b] are set for the instances whose cycle starts and cleared
// for all others; tres and rres are rewritten for the next restart.
void krylov_cycle_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                        double cancel_thr, int every, int* act, int* tres, int* rres, int* run, int* cyc,
                        int nbatch, hipStream_t s);
// krylov_cycle_start with ||r||^2 summed in the same launch, in the order of
// krylov_residual / krylov_sum_norm: from the b - A x partials in tpart
// (RED_BLOCKS per instance) where tres is set, from the basis-residual partials
// in lpart (LIN_BLOCKS) where rres is; the sum is also stored to rnorm2. With
// host (host memory the device can write) each instance's HostFlags are
// written there. fp64 = false: no b - A x was formed for this restart; an
// instance that asked for one keeps its request and starts no cycle (it waits
// for a restart with b - A x).
void krylov_cycle_start_sum(GState* st, double* rnorm2, const double* tpart, const double* lpart,
                            const double* abs_target, double eta, int m, double cancel_thr, int every, int* act,
                            int* tres, int* rres, int* run, int* cyc, int nbatch, hipStream_t s,
                            HostFlags* host = nullptr, bool fp64 = true);
// start a cycle from rnorm2[b] = ||r_b||^2 (v0 = r unnormalised, as left by
// krylov_residual; inv_norm = 1 / ||r||): g = (||r||, 0, ...), j = 0,
// target = max(abs_target[b], eta ||r||); run[b] = mask[b] && ||r|| > abs_target[b]
void krylov_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                  double cancel_thr, const int* mask, int* run, int nbatch, hipStream_t s);

// ---- batched vector kernels (instance b at offset b * bstride) ---------------
// out = a x + c y (any mix of precisions; y may be null)
template <class TO, class TX, class TY>
void vec_axpby(TO* out, const TX* x, const TY* y, double a, double c, long long n, long long bstride,
               const int* mask, int nbatch, hipStream_t s);
// out[b] = ||x_b||^2
template <class T>
void vec_norm2(const T* x, long long n, long long bstride, double* part, double* out, const int* mask,
               int nbatch, hipStream_t s);
// out[b] = ||x_b - y_b||^2 and ||x_b||^2 (for relative changes); out has 2 doubles per instance
template <class T>
void vec_diff2(const T* x, const T* y, long long n, long long bstride, double* part, double* out,
               int nbatch, hipStream_t s);

}  // namespace psfd
