// Host engine: problem tables, device workspaces of a group of same-shape
// instances, operator apply orchestration and the solve drivers.
#pragma once
#include <functional>
#include <string>
#include <vector>

#include "../../include/psfd.h"
#include "kernels.hpp"
#include "krylov.hpp"

namespace psfd {

struct Status {
  int code = PSFD_OK;
  std::string msg;
  bool ok() const { return code == PSFD_OK; }
};

struct Shape {
  int nx = 0, ny = 0, nz = 0, pz = 0;
  long long nxny = 0, N = 0, n3 = 0;
};

// validated copy of a problem statement
struct Problem {
  psfd_problem p{};
  std::vector<psfd_layer> layers;
};

struct Opts {
  double rtol = 1e-6, outer_rtol = 1e-6, inner_eta = 1e-4;
  int restart = 30, max_iters = 5000, max_outer = 100, precision = PSFD_MIXED;
  int coupling = PSFD_COUPLING_MONO;
};

Status validate_problem(const psfd_problem* p, Problem& out);
// restart limited to max_restart (the device-driven solves: MAXM)
Status make_opts(const psfd_opts* o, Opts& out, int max_restart = MAXM);
Shape shape_of(const psfd_problem& p);
// per-instance FP64 tables (TabLayout) of a problem; SINGULAR on a grazing order
// Host part of an instance table (scalars, kx, ky, incident order); fails with
// SINGULAR at a Wood anomaly.
Status build_table(const Problem& pr, std::vector<double>& tab);
// Copies the host part to d_tab and computes the per-order part on the device
// (d_lay: scratch for LAYER_CAP + 2 layers).
Status upload_table(double* d_tab, double4* d_lay, const Problem& pr, const std::vector<double>& tab,
                    hipStream_t s);
// largest layer count of a stack
const int LAYER_CAP = 2048;
// twiddle tables of all power-of-two lengths up to TW_MAX_N (tw[n + i] = exp(-2 pi i i / n))
constexpr int TW_MAX_N = 1024;
void build_twiddles(std::vector<double>& tw64);

// Launch configurations of the transverse FFT and z-pencil kernels.
struct XYCfg {
  bool fused;
  TileShape full, rows, cols;
};
XYCfg xy_config(const Shape& sh, size_t esz);
struct ZCfg { int bx, nthr; size_t lds; };
ZCfg z_config(const Shape& sh, size_t esz);

// Device tables shared by every group on a device (twiddles).
struct DeviceConsts {
  int device = -1;
  float2* tw32 = nullptr;
  double2* tw64 = nullptr;
};
Status device_consts(DeviceConsts*& out);

// Snapshots of the solve flags in flight: ring slots, and how many may be
// outstanding before the host waits for the oldest. Kernels launched for
// finished instances are no-ops (every kernel tests its flags).
constexpr int FLAG_SLOTS = 4;
constexpr int FLAG_EVERY = 2;  // a solve records an event after every FLAG_EVERY-th cycle
constexpr int FLAG_LAG = 1;    // and runs at most FLAG_LAG such events ahead of the GPU

// B instances of one grid shape with every device buffer a solve needs.
struct Group {
  Shape sh;
  int B = 0;
  int m = 30;
  int prec = PSFD_MIXED;
  bool alloc_solve = false;
  DeviceConsts* dc = nullptr;
  // per instance tables
  double* tab = nullptr;
  long long tab_stride = 0;
  double4* lay = nullptr;  // layer stack per instance (LAYER_CAP + 2 entries), table input
  // contrast (FP64 copy of the user data, FP32 copy for mixed precision)
  double2* deps64 = nullptr;
  float2* deps32 = nullptr;
  // FP64 fields [B][n3]
  double2 *x = nullptr, *b = nullptr, *r = nullptr, *e = nullptr, *u = nullptr, *ws64 = nullptr;
  // Krylov basis [B][m+1][n3] of the working precision and its apply scratch [B][n3]
  void* basis = nullptr;
  void* wsP = nullptr;
  GState* st = nullptr;
  int* run = nullptr;
  int* mask = nullptr;
  int* mask2 = nullptr;
  int* cyc = nullptr;        // a restart cycle started for the instance (device-driven solve)
  int* tres = nullptr;       // the next restart evaluates b - A x (device-driven solve)
  int* rres = nullptr;       // the next restart takes the GMRES residual from the basis
  double* rtol = nullptr;    // relative tolerance per instance of the current linear solve
  double2* part = nullptr;
  double2* dpart2 = nullptr;  // projection partials of the Gram-Schmidt passes (value-major)
  double* n2 = nullptr;
  double* n2b = nullptr;
  double* abs_target = nullptr;
  double* dpart = nullptr;
  double* lpart = nullptr;   // norm partials of the basis residual (LIN_BLOCKS per instance)
  double2 *adn = nullptr, *aup = nullptr, *eup = nullptr, *ord = nullptr, *eup2 = nullptr;
  double* rpart = nullptr;
  int rblk = 1;
  HostFlags* h_flags = nullptr;  // the solve flags in mapped, coherent host memory (B), and
  HostFlags* d_flags = nullptr;  // the device's address of it, written by each cycle start
  hipEvent_t flag_ev[FLAG_SLOTS] = {};
  int* h_run = nullptr;      // pinned host mirrors
  double* h_dbl = nullptr;
  // Captured launch sequences (HIP graphs), replayed on the caller's stream:
  // one restart cycle of the device-driven solve. A graph is re-captured when
  // its key (the launch choices baked into it) changes; a capture that HIP
  // refuses leaves `failed` set for that key, and the cycles run eagerly.
  struct Captured {
    hipGraphExec_t exec = nullptr;
    std::string key;
    bool failed = false;
  };
  Captured cycle_graph[2][2][2];   // [transpose][refl][restart with b - A x]
  hipStream_t cap_stream = nullptr;  // capture only (launches are not executed there)
  std::vector<void*> owned;
  ~Group();
};

// Whether restart cycles and the server's Arnoldi blocks run as captured HIP
// graphs (PSFD_GRAPH=0 issues the same launches one by one; read per call).
bool use_graphs();
// Whether a solve may leave b - A x out of the restarts that do not use it
// (PSFD_LITE_RESTARTS=0: every restart launches it; read per call).
bool lite_restarts();
// Replays the captured sequence `c` on stream s, capturing `issue(cs)` first when
// the key differs (cs is the group's capture stream).
Status replay(Group& g, Group::Captured& c, const std::string& key, hipStream_t s,
              const std::function<void(hipStream_t)>& issue);
// The launch choices read from the environment that a captured sequence bakes in.
std::string launch_key(double eta, int every);

size_t group_bytes(const Shape& sh, int B, int m, int prec);
Status group_alloc(Group& g, const Shape& sh, int B, int m, int prec);
Status group_set_tables(Group& g, int b, const Problem& pr, const std::vector<double>& tab, hipStream_t s);

// y = x - K(V x) (kmode 0) or y = K(V x) (kmode 1); transpose uses the kernel at -k.
// refl adds the layered-stack response R_vol T_R K_top to K (monolithic operator M).
// in_scale (optional): per-instance factor at in_scale[b * scale_stride] applied to
// x on load, and the scaled x written back to in (normalisation of the newest
// Arnoldi vector inside the apply).
// gt (optional): a pending Givens step to take along with the first kernel.
template <class T>
void apply_op(Group& g, const T* deps, VecRef in, VecRef out, T* ws, int kmode, int transpose, int refl,
              const int* active, hipStream_t s, const double* in_scale = nullptr, long long scale_stride = 0,
              const GivensTask* gt = nullptr);
// one of the three launches of apply_op: 0 transverse forward, 1 z-pencil, 2 transverse inverse.
// qp: the quarter-plane kernels and layout (all three stages of one apply alike;
// only where quarter_planes holds and with no gt)
template <class T>
void apply_stage(Group& g, int stage, const T* deps, VecRef in, VecRef out, T* ws, int kmode, int transpose,
                 int refl, const int* active, hipStream_t s, const double* in_scale = nullptr,
                 long long scale_stride = 0, const GivensTask* gt = nullptr, bool qp = false);
// whether the operator apply of this group's shape takes the quarter-plane
// kernels (FP32 128 x 128 planes with the compile-time pencil; PSFD_QUARTER_PLANES=0
// turns them off)
bool quarter_planes(const Group& g, size_t esz);

struct SolveStats {
  int iters = 0, outer = 0, cycles = 0, status = PSFD_OK;
  double rel_res = 0, change = 0, mono = 0;
};

// Forward solve of every instance (deps64 filled). Results stay in g.x / g.ord.
Status solve_group(Group& g, const Opts& o, std::vector<SolveStats>& stats, hipStream_t s);
// Vector-Jacobian product of the reflected orders (adjoint solve, transposed
// coupled system): u [B][n3] the forward total field, grad_orders [B][nx ny 3]
// the cotangent dL/dRe a + i dL/dIm a; grad [B][N] receives dL/dRe + i dL/dIm of
// delta_eps. The contrast must be in g.deps64 and the tables set.
Status adjoint_group(Group& g, const Opts& o, const double2* u, const double2* grad_orders, double2* grad,
                     std::vector<SolveStats>& stats, hipStream_t s);

Status hip_status(hipError_t e, const char* what);

// Times one Gram-Schmidt pass of the Arnoldi step at column j on a group of one
// instance (pass 0: projections, pass 1: update; reps launches between two
// events on s): slots 0..j+1 of the basis are copied from x (n3 values of the
// group's working precision), every slot scale is 1, the instance runs.
Status bench_gram_schmidt(Group& g, int pass, int j, const void* x, int reps, float* ms, hipStream_t s);

// ---- building blocks shared with the serving runtime (all masked per instance) ----
// e = E_inc + IFFT_xy(E_up exp(i beta z)) on every plane (FP64)
void inject(Group& g, const double2* eup, double2* out, const int* active, hipStream_t s);
// per-order plane-wave readouts adn / aup of V (x + e) (e may be null only through apply_stage)
void readout(Group& g, const double2* x, const double2* e, const int* active, hipStream_t s);
// eup <- T_R (adn + e_inc); relative change per instance when change != null
Status reflect(Group& g, double2* eup, const int* active, std::vector<double>* change, hipStream_t s);
Status set_mask(Group& g, int* dmask, const std::vector<int>& h, hipStream_t s);
Status read_norms(Group& g, const double* d, std::vector<double>& out, hipStream_t s);
double cancel_threshold();
int true_residual_every();
extern const int STEPS_PER_SYNC;
// one Arnoldi step (apply of B, Gram-Schmidt, Givens, scale) for every instance with run[b];
// jh >= 0 when every running instance stands at step jh (the Krylov slots are
// then fixed at launch), jh < 0 to take each instance's step from its state.
// solve_mask: at the last step of a lock-step cycle with the fused update, the
// back substitution (krylov_solve_small over solve_mask) runs in the launch of
// the last column's Givens step, and the call returns true; false otherwise.
template <class T>
bool arnoldi_step(Group& g, int transpose, int refl, hipStream_t s, int jh = -1, const int* solve_mask = nullptr);

}  // namespace psfd
