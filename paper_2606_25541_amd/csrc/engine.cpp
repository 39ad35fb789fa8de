// Host engine of the solver: FP64 problem tables, grouped device workspaces,
// operator apply orchestration and the GMRES / outer-loop drivers.
#include "engine.hpp"

#include <deque>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>

namespace psfd {

using cd = std::complex<double>;
static const double PI = 3.14159265358979323846;
static const size_t LDS_MAX = 163840;
// inner (eq. (18)) tolerance policy of the outer loop
static const double INNER_FACTOR = 0.1;     // final inner rtol = INNER_FACTOR * rtol
static const double FIRST_INNER_TOL = 1e-3; // first outer step
static const double OUTER_TO_INNER = 0.1;   // inner rtol <= OUTER_TO_INNER * last outer change

Status hip_status(hipError_t e, const char* what) {
  Status st;
  if (e != hipSuccess) {
    st.code = (e == hipErrorOutOfMemory) ? PSFD_ERR_OOM : PSFD_ERR_HIP;
    st.msg = std::string(what) + ": " + hipGetErrorString(e);
  }
  return st;
}

#define HIPCHK(call)                                     \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_status(e_, #call);  \
  } while (0)

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

Status validate_problem(const psfd_problem* p, Problem& out) {
  Status st;
  auto bad = [&](int code, const std::string& m) { st.code = code; st.msg = m; return st; };
  if (!p) return bad(PSFD_ERR_INVALID_ARG, "problem is NULL");
  if (!pow2_in(p->nx, 4, 256) || !pow2_in(p->ny, 4, 256) || !pow2_in(p->nz, 2, 128))
    return bad(PSFD_ERR_UNSUPPORTED_SIZE, "nx, ny must be powers of two in [4, 256] and nz in [2, 128]");
  if (!(p->lx_nm > 0) || !(p->ly_nm > 0) || !(p->t_nm > 0) || !(p->wavelength_nm > 0) || !(p->eps_bg > 0))
    return bad(PSFD_ERR_INVALID_ARG, "lengths, wavelength and eps_bg must be positive");
  if (!(std::fabs(p->theta_deg) < 90.0) || !std::isfinite(p->phi_deg))
    return bad(PSFD_ERR_INVALID_ARG, "theta must lie in (-90, 90) degrees");
  if (p->pol != PSFD_TE && p->pol != PSFD_TM) return bad(PSFD_ERR_INVALID_ARG, "pol must be PSFD_TE or PSFD_TM");
  if (p->n_layers < 0 || (p->n_layers > 0 && !p->layers)) return bad(PSFD_ERR_INVALID_ARG, "bad layer list");
  if (p->n_layers > LAYER_CAP) return bad(PSFD_ERR_UNSUPPORTED_SIZE, "at most 2048 layers");
  out.p = *p;
  out.layers.assign(p->layers, p->layers + p->n_layers);
  for (auto& l : out.layers)
    if (!(l.thickness_nm >= 0) || !std::isfinite(l.eps_re) || !std::isfinite(l.eps_im))
      return bad(PSFD_ERR_INVALID_ARG, "bad layer parameters");
  out.p.layers = out.layers.empty() ? nullptr : out.layers.data();
  return st;
}

Status make_opts(const psfd_opts* o, Opts& out, int max_restart) {
  Status st;
  out = Opts();
  if (!o) return st;
  if (!(o->rtol > 0) || o->restart < 1 || o->restart > max_restart || o->max_iters < 1 || o->max_outer < 1 ||
      (o->precision != PSFD_FP64 && o->precision != PSFD_MIXED)) {
    st.code = PSFD_ERR_INVALID_ARG;
    st.msg = "bad options (rtol > 0, 1 <= restart <= " + std::to_string(max_restart) +
             ", max_iters, max_outer >= 1, precision)";
    return st;
  }
  out.rtol = o->rtol;
  out.outer_rtol = o->outer_rtol > 0 ? o->outer_rtol : o->rtol;
  out.restart = o->restart;
  out.max_iters = o->max_iters;
  out.max_outer = o->max_outer;
  out.precision = o->precision;
  out.inner_eta = o->inner_eta > 0 ? o->inner_eta : 1e-4;
  if (o->coupling != PSFD_COUPLING_OUTER && o->coupling != PSFD_COUPLING_MONO) {
    st.code = PSFD_ERR_INVALID_ARG;
    st.msg = "coupling must be PSFD_COUPLING_OUTER or PSFD_COUPLING_MONO";
    return st;
  }
  out.coupling = o->coupling;
  return st;
}

Shape shape_of(const psfd_problem& p) {
  Shape s;
  s.nx = p.nx; s.ny = p.ny; s.nz = p.nz; s.pz = 2 * p.nz;
  s.nxny = (long long)p.nx * p.ny;
  s.N = s.nxny * p.nz;
  s.n3 = 3 * s.N;
  return s;
}

// ---------------------------------------------------------------------------
// z-wavenumber branch with Im >= 0 (outgoing or decaying for e^{-i omega t})
static inline cd kz_branch(cd k2) {
  cd r = std::sqrt(k2);
  if (r.imag() < 0 || (r.imag() == 0 && r.real() < 0)) r = -r;
  return r;
}

static void cross3(const cd* a, const cd* b, cd* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

Status build_table(const Problem& pr, std::vector<double>& tab) {
  Status st;
  const psfd_problem& p = pr.p;
  const int nx = p.nx, ny = p.ny, nz = p.nz, pz = 2 * nz;
  TabLayout L{nx, ny};
  tab.assign((size_t)L.size(), 0.0);
  const double k0 = 2.0 * PI / p.wavelength_nm;
  const double kbg = k0 * std::sqrt(p.eps_bg);
  const double th = p.theta_deg * PI / 180.0, ph = p.phi_deg * PI / 180.0;
  const double kx0 = kbg * std::sin(th) * std::cos(ph), ky0 = kbg * std::sin(th) * std::sin(ph);
  const double dz = p.t_nm / nz;
  tab[TS_KBG] = kbg;
  tab[TS_L] = p.t_nm;
  tab[TS_DZ] = dz;
  tab[TS_KAPPA] = 2.0 * PI / (pz * dz);
  tab[TS_SCALE] = 1.0 / ((double)nx * ny * pz);
  tab[TS_K0SQ] = k0 * k0;
  tab[TS_T] = p.t_nm;
  tab[TS_INVNXNY] = 1.0 / ((double)nx * ny);
  tab[TS_ST] = std::sin(th) * std::cos(ph);
  tab[TS_ST + 1] = std::sin(th) * std::sin(ph);
  double* kx = tab.data() + L.off_kx();
  double* ky = tab.data() + L.off_ky();
  for (int i = 0; i < nx; ++i) { int m = i < nx / 2 ? i : i - nx; kx[i] = kx0 + 2.0 * PI * m / p.lx_nm; }
  for (int j = 0; j < ny; ++j) { int n = j < ny / 2 ? j : j - ny; ky[j] = ky0 + 2.0 * PI * n / p.ly_nm; }
  // Wood anomaly check: every order needs |beta| > 0 (the kernel and the
  // readouts divide by beta). The per-order tables themselves (beta, exp(i beta L),
  // keep mask, T_R) are computed on the device by upload_table.
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double kt = std::hypot(kx[i], ky[j]);
      if (std::abs(kz_branch(cd(kbg * kbg - kt * kt, 0.0))) < 1e-6 * kbg) {
        st.code = PSFD_ERR_SINGULAR;
        st.msg = "a transverse order grazes the surface (beta = 0, Wood anomaly)";
        return st;
      }
    }
  // incident order (0, 0): polarisation vector s (TE) or p- (TM) and its beta
  {
    const double kt = std::hypot(kx[0], ky[0]);
    const cd b = kz_branch(cd(kbg * kbg - kt * kt, 0.0));
    cd sv[3];
    if (kt > 0) { sv[0] = -ky[0] / kt; sv[1] = kx[0] / kt; }
    else { sv[0] = -std::sin(ph); sv[1] = std::cos(ph); }
    sv[2] = 0.0;
    cd km[3] = {kx[0], ky[0], -b}, pm[3];
    cross3(km, sv, pm);
    for (int c = 0; c < 3; ++c) pm[c] /= kbg;
    tab[TS_INCQ] = 0.0;
    const cd* ev = (p.pol == PSFD_TE) ? sv : pm;
    for (int c = 0; c < 3; ++c) { tab[TS_EINC + 2 * c] = ev[c].real(); tab[TS_EINC + 2 * c + 1] = ev[c].imag(); }
    tab[TS_BINC] = b.real();
    tab[TS_BINC + 1] = b.imag();
  }
  return st;
}

Status upload_table(double* d_tab, double4* d_lay, const Problem& pr, const std::vector<double>& tab,
                    hipStream_t s) {
  const psfd_problem& p = pr.p;
  const int nl = (int)pr.layers.size();
  std::vector<double4> lay(nl + 2);
  lay[0] = make_double4(p.eps_bg, 0.0, 0.0, 0.0);
  for (int i = 0; i < nl; ++i)
    lay[i + 1] = make_double4(pr.layers[i].eps_re, pr.layers[i].eps_im, pr.layers[i].thickness_nm, 0.0);
  lay[nl + 1] = make_double4(p.eps_sub_re, p.eps_sub_im, 0.0, 0.0);
  const TabLayout L{p.nx, p.ny};
  HIPCHK(hipMemcpyAsync(d_tab, tab.data(), (size_t)L.off_beta() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_lay, lay.data(), lay.size() * sizeof(double4), hipMemcpyHostToDevice, s));
  const double k0 = 2.0 * PI / p.wavelength_nm;
  launch_stack_table(p.nx, p.ny, d_tab, d_lay, nl, k0 * k0, p.phi_deg * PI / 180.0, s);
  HIPCHK(hipGetLastError());
  return Status();
}

void build_twiddles(std::vector<double>& tw) {
  tw.assign(2 * 2 * TW_MAX_N, 0.0);
  for (int n = 2; n <= TW_MAX_N; n <<= 1)
    for (int i = 0; i < n; ++i) {
      // exp(-2 pi i i / n); the angle is reduced to the first octant by symmetry
      const double a = 2.0 * PI * i / n;
      tw[2 * (n + i)] = std::cos(a);
      tw[2 * (n + i) + 1] = -std::sin(a);
    }
}

// ---------------------------------------------------------------------------
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
// launch-shape overrides for tuning sweeps (read at every call)
static int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}
static double env_double(const char* name, double dflt) {
  const char* e = std::getenv(name);
  return e ? std::atof(e) : dflt;
}
// complex values per thread of an LDS FFT pass (see FftBudget)
static int fft_elems(size_t esz) { return esz == 8 ? 16 : 8; }

// LDS row pitch of a transverse tile. The LDS serves a 64-bit access 16 lanes at a
// time (a 128-bit one 8 lanes at a time). The FFT passes give consecutive lanes
// consecutive sequences at the same butterfly: a column pass then reads
// consecutive words, and with an odd pitch the 16 (8) rows of a row pass fall
// into distinct banks, so neither pass conflicts.
static int tile_pitch(int tx, size_t esz) {
  (void)esz;
  return tx + 1;
}
static int ceil64(int v) { return (v + 63) / 64 * 64; }

XYCfg xy_config(const Shape& sh, size_t esz) {
  XYCfg c{};
  const int nx = sh.nx, ny = sh.ny;
  const size_t full_lds = (size_t)ny * tile_pitch(nx, esz) * esz;
  c.fused = full_lds <= LDS_MAX && (long long)nx * ny <= 16 * 1024;
  c.full = TileShape{nx, ny, 1, 1, clampi(nx * ny / 8, 64, 1024), full_lds, tile_pitch(nx, esz)};
  if (nx * ny > fft_elems(esz) * c.full.nthr) c.fused = false;
  if (env_int("PSFD_XY_SPLIT", 0)) c.fused = false;
  int rb = clampi(4096 / nx, 1, ny);
  int rel = rb * nx;
  c.rows = TileShape{nx, rb, 1, 0, clampi(ceil64(rel / 8), 64, 1024), (size_t)rb * tile_pitch(nx, esz) * esz,
                     tile_pitch(nx, esz)};
  int cb = std::min(nx, 16);
  int cel = cb * ny;
  c.cols = TileShape{cb, ny, 0, 1, clampi(ceil64(cel / 8), 64, 1024), (size_t)ny * tile_pitch(cb, esz) * esz,
                     tile_pitch(cb, esz)};
  return c;
}

// Threads of a pencil block: at most 8 values per thread in its FFT passes.
static int pencil_threads(const Shape& sh, int bx) {
  int nthr = clampi(ceil64(3 * bx * sh.pz / 8), 64, 768);
  if (nthr < 4 * 3 * bx) nthr = ceil64(4 * 3 * bx);  // at least four readout partial sums per sequence
  return nthr;
}

// LDS bytes of a pencil block (the regions of PencilLds)
static size_t pencil_lds(const Shape& sh, int bx, int nthr, size_t esz) {
  return (size_t)PencilLds(sh.pz, bx, nthr, (int)esz).total;
}

ZCfg z_config(const Shape& sh, size_t esz) {
  ZCfg z{};
  int bx = std::min(sh.nx, env_int("PSFD_ZBX", 16));
  // pencil FFT passes take at most 8 values per thread and 768 threads per block
  while (bx > 1 && (pencil_lds(sh, bx, pencil_threads(sh, bx), esz) > 150 * 1024 || 3 * bx * sh.pz > 8 * 768))
    bx >>= 1;
  z.bx = bx;
  z.nthr = pencil_threads(sh, bx);
  z.lds = pencil_lds(sh, bx, z.nthr, esz);
  return z;
}

// ---------------------------------------------------------------------------
static std::mutex g_dc_mu;
static std::vector<DeviceConsts*> g_dc;

Status device_consts(DeviceConsts*& out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dc_mu);
  for (auto* d : g_dc)
    if (d->device == dev) { out = d; return Status(); }
  std::vector<double> tw;
  build_twiddles(tw);
  std::vector<float> tw32(tw.size());
  for (size_t i = 0; i < tw.size(); ++i) tw32[i] = (float)tw[i];
  auto* d = new DeviceConsts();
  d->device = dev;
  HIPCHK(hipMalloc((void**)&d->tw64, tw.size() * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d->tw32, tw32.size() * sizeof(float)));
  HIPCHK(hipMemcpy(d->tw64, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d->tw32, tw32.data(), tw32.size() * sizeof(float), hipMemcpyHostToDevice));
  for (int t : {0}) (void)t;
  g_dc.push_back(d);
  out = d;
  return Status();
}

// ---------------------------------------------------------------------------
Group::~Group() {
  for (auto& a : cycle_graph)
    for (auto& b2 : a)
      for (auto& c : b2)
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (void* p : owned) (void)hipFree(p);
  for (hipEvent_t e : flag_ev)
    if (e) (void)hipEventDestroy(e);
  if (h_flags) (void)hipHostFree(h_flags);
  if (h_run) (void)hipHostFree(h_run);
  if (h_dbl) (void)hipHostFree(h_dbl);
}

size_t group_bytes(const Shape& sh, int B, int m, int prec) {
  const size_t n3 = (size_t)sh.n3, N = (size_t)sh.N;
  const size_t esz = prec == PSFD_FP64 ? 16 : 8;
  size_t per = 0;
  per += (size_t)TabLayout{sh.nx, sh.ny}.size() * 8;
  per += N * 16 + (prec == PSFD_MIXED ? N * 8 : 0);
  per += 6 * n3 * 16;
  per += (size_t)(m + 1) * n3 * esz;
  per += prec == PSFD_MIXED ? n3 * esz : 0;
  per += sizeof(GState) + RED_BLOCKS * PSTR * 16 + DOT_BLOCKS_MAX * PSTR * 16 + RED_BLOCKS * 2 * 8 + LIN_BLOCKS * 8 + 6 * sizeof(int);
  per += 5 * (size_t)sh.nxny * 3 * 16 + (size_t)((sh.nxny + 255) / 256) * 2 * 8 + 64;
  per += (size_t)(LAYER_CAP + 2) * sizeof(double4);
  return per * (size_t)B;
}

template <class P>
static Status galloc(Group& g, P*& p, size_t bytes) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) return hip_status(e, "hipMalloc");
  g.owned.push_back(v);
  p = (P*)v;
  return Status();
}

#define GALLOC(ptr, bytes)                         \
  do {                                             \
    Status s_ = galloc(g, ptr, (bytes));           \
    if (!s_.ok()) return s_;                       \
  } while (0)

Status group_alloc(Group& g, const Shape& sh, int B, int m, int prec) {
  Status st = device_consts(g.dc);
  if (!st.ok()) return st;
  g.sh = sh;
  g.B = B;
  g.m = m;
  g.prec = prec;
  const size_t n3 = (size_t)sh.n3, N = (size_t)sh.N, nq = (size_t)sh.nxny * 3;
  g.tab_stride = TabLayout{sh.nx, sh.ny}.size();
  GALLOC(g.tab, (size_t)g.tab_stride * 8 * B);
  GALLOC(g.lay, (size_t)(LAYER_CAP + 2) * sizeof(double4) * B);
  GALLOC(g.deps64, N * 16 * B);
  if (prec == PSFD_MIXED) GALLOC(g.deps32, N * 8 * B);
  GALLOC(g.x, n3 * 16 * B);
  GALLOC(g.b, n3 * 16 * B);
  GALLOC(g.r, n3 * 16 * B);
  GALLOC(g.e, n3 * 16 * B);
  GALLOC(g.u, n3 * 16 * B);
  GALLOC(g.ws64, n3 * 16 * B);
  const size_t esz = prec == PSFD_FP64 ? 16 : 8;
  GALLOC(g.basis, (size_t)(m + 1) * n3 * esz * B);
  if (prec == PSFD_MIXED) GALLOC(g.wsP, n3 * esz * B);
  else g.wsP = g.ws64;
  GALLOC(g.st, sizeof(GState) * B);
  GALLOC(g.run, sizeof(int) * B);
  GALLOC(g.mask, sizeof(int) * B);
  GALLOC(g.mask2, sizeof(int) * B);
  GALLOC(g.cyc, sizeof(int) * B);
  GALLOC(g.tres, sizeof(int) * B);
  GALLOC(g.rres, sizeof(int) * B);
  GALLOC(g.rtol, sizeof(double) * B);
  GALLOC(g.part, (size_t)RED_BLOCKS * PSTR * 16 * B);
  GALLOC(g.dpart2, (size_t)DOT_BLOCKS_MAX * PSTR * 16 * B);
  GALLOC(g.n2, 8 * B);
  GALLOC(g.n2b, 8 * B);
  GALLOC(g.abs_target, 8 * B);
  GALLOC(g.dpart, (size_t)RED_BLOCKS * 2 * 8 * B);
  GALLOC(g.lpart, (size_t)LIN_BLOCKS * 8 * B);
  GALLOC(g.adn, nq * 16 * B);
  GALLOC(g.aup, nq * 16 * B);
  GALLOC(g.eup, nq * 16 * B);
  GALLOC(g.eup2, nq * 16 * B);
  GALLOC(g.ord, nq * 16 * B);
  g.rblk = (int)((sh.nxny + 255) / 256);
  GALLOC(g.rpart, (size_t)g.rblk * 2 * 8 * B);
  HIPCHK(hipHostMalloc((void**)&g.h_run, sizeof(int) * B * 4, hipHostMallocDefault));
  // the solve flags, written by the cycle-start kernel itself (coherent, mapped)
  HIPCHK(hipHostMalloc((void**)&g.h_flags, sizeof(HostFlags) * B, hipHostMallocCoherent | hipHostMallocMapped));
  HIPCHK(hipHostGetDevicePointer((void**)&g.d_flags, g.h_flags, 0));
  for (int b = 0; b < B; ++b) g.h_flags[b] = HostFlags{0, 0, 0.0, -1, 0};
  for (int i = 0; i < FLAG_SLOTS; ++i) HIPCHK(hipEventCreateWithFlags(&g.flag_ev[i], hipEventDisableTiming));
  HIPCHK(hipHostMalloc((void**)&g.h_dbl, sizeof(double) * (size_t)B * 2 * std::max(8, g.rblk), hipHostMallocDefault));
  HIPCHK(hipMemset(g.st, 0, sizeof(GState) * B));
  HIPCHK(hipMemset(g.run, 0, sizeof(int) * B));
  g.alloc_solve = true;
  return Status();
}

Status group_set_tables(Group& g, int b, const Problem& pr, const std::vector<double>& tab, hipStream_t s) {
  return upload_table(g.tab + (size_t)b * g.tab_stride, g.lay + (size_t)b * (LAYER_CAP + 2), pr, tab, s);
}

// ---------------------------------------------------------------------------
template <class T> static const T* twiddles(const Group& g);
template <> const float2* twiddles<float2>(const Group& g) { return g.dc->tw32; }
template <> const double2* twiddles<double2>(const Group& g) { return g.dc->tw64; }

static TileArgs tile_base(const Group& g, const void* tw, const TileShape& t) {
  TileArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nx = g.sh.nx; a.ny = g.sh.ny; a.nz = g.sh.nz;
  a.log2nx = ilog2i(g.sh.nx); a.log2ny = ilog2i(g.sh.ny);
  a.tx = t.tx; a.ty = t.ty; a.pitch = t.pitch;
  a.tiles_x = g.sh.nx / t.tx; a.tiles_y = g.sh.ny / t.ty;
  a.do_x = t.do_x; a.do_y = t.do_y;
  a.tab = g.tab; a.tab_stride = g.tab_stride;
  a.tw = tw;
  a.alpha = 0; a.gamma = 1;
  return a;
}

bool quarter_planes(const Group& g, size_t esz) {
  const Shape& sh = g.sh;
  if ((esz != 8 && esz != 16) || env_int("PSFD_QUARTER_PLANES", 1) == 0) return false;
  const ZCfg z = z_config(sh, esz);
  return qplane_shape(sh.nx, sh.ny, sh.nz, sh.pz, z.bx, z.nthr, esz);
}

template <class T>
void apply_stage(Group& g, int stage, const T* deps, VecRef in, VecRef out, T* ws, int kmode, int transpose,
                 int refl, const int* active, hipStream_t s, const double* in_scale, long long scale_stride,
                 const GivensTask* gt, bool qp) {
  const Shape& sh = g.sh;
  const XYCfg c = xy_config(sh, sizeof(T));
  const int np = 3 * sh.nz;
  const T* tw = twiddles<T>(g);
  VecRef wsr = vr(ws, sh.n3);
  if (qp && !quarter_planes(g, sizeof(T))) {
    std::fprintf(stderr, "psfd: internal error: quarter-plane apply stage on an unsupported shape\n");
    std::abort();
  }
  if (stage == 0) {
    // forward: w = FFT_xy(k0^2 delta_eps x)
    if (qp) {
      // a pending Givens step takes a launch of its own first
      if (gt) krylov_givens(gt->st, gt->run, gt->part, g.B, s);
      TileArgs a = tile_base(g, tw, c.full);
      a.in = in; a.vol = vr(deps, sh.N); a.out = wsr; a.active = active;
      a.in_scale = in_scale; a.scale_stride = scale_stride;
      launch_qplane<T, false, LD_VX, ST_PLAIN>(a, np, g.B, s);
    } else if (c.fused) {
      TileArgs a = tile_base(g, tw, c.full);
      a.in = in; a.vol = vr(deps, sh.N); a.out = wsr; a.active = active;
      a.in_scale = in_scale; a.scale_stride = scale_stride;
      if (gt) {
        // the pending Givens step rides along with the square-plane kernel;
        // other kernels take it as a launch of its own first
        if (tile_is_plane(a, sizeof(T))) a.gv = *gt;
        else krylov_givens(gt->st, gt->run, gt->part, g.B, s);
      }
      launch_tile<T, false, LD_VX, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
    } else {
      if (gt) krylov_givens(gt->st, gt->run, gt->part, g.B, s);
      TileArgs a = tile_base(g, tw, c.rows);
      a.in = in; a.vol = vr(deps, sh.N); a.out = wsr; a.active = active;
      a.in_scale = in_scale; a.scale_stride = scale_stride;
      launch_tile<T, false, LD_VX, ST_PLAIN>(a, np, g.B, c.rows.nthr, c.rows.lds, s);
      TileArgs b2 = tile_base(g, tw, c.cols);
      b2.in = wsr; b2.out = wsr; b2.active = active;
      launch_tile<T, false, LD_PLAIN, ST_PLAIN>(b2, np, g.B, c.cols.nthr, c.cols.lds, s);
    }
  } else if (stage == 1) {
    // z: pad, FFT, kernel, IFFT, restrict (in place)
    const ZCfg z = z_config(sh, sizeof(T));
    PencilArgs p;
    std::memset(&p, 0, sizeof(p));
    p.nx = sh.nx; p.ny = sh.ny; p.nz = sh.nz; p.pz = sh.pz; p.log2pz = ilog2i(sh.pz);
    p.bx = z.bx; p.pitch = sh.pz + 1; p.nblk_x = qp ? sh.nx / 4 : sh.nx / z.bx; p.yq = qp;
    p.w = wsr; p.tab = g.tab; p.tab_stride = g.tab_stride; p.tw = tw; p.transpose = transpose; p.reflect = refl;
    p.active = active;
    if (gt) p.gv = *gt;  // the pending Givens step, and the scale of the input from its partials
    launch_pencil<T>(p, g.B, z.nthr, z.lds, s);
  } else {
    // inverse: out = in - IFFT_xy(w) (kmode 0) or out = IFFT_xy(w) (kmode 1, no read of in)
    if (qp) {
      TileArgs a = tile_base(g, tw, c.full);
      a.in = wsr; a.aux = in; a.out = out; a.alpha = 1.0; a.gamma = -1.0; a.active = active;
      if (kmode == 0) launch_qplane<T, true, LD_PLAIN, ST_AXPBY>(a, np, g.B, s);
      else launch_qplane<T, true, LD_PLAIN, ST_PLAIN>(a, np, g.B, s);
    } else if (c.fused) {
      TileArgs a = tile_base(g, tw, c.full);
      a.in = wsr; a.aux = in; a.out = out; a.alpha = 1.0; a.gamma = -1.0; a.active = active;
      if (kmode == 0) launch_tile<T, true, LD_PLAIN, ST_AXPBY>(a, np, g.B, c.full.nthr, c.full.lds, s);
      else launch_tile<T, true, LD_PLAIN, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
    } else {
      TileArgs a = tile_base(g, tw, c.cols);
      a.in = wsr; a.out = wsr; a.active = active;
      launch_tile<T, true, LD_PLAIN, ST_PLAIN>(a, np, g.B, c.cols.nthr, c.cols.lds, s);
      TileArgs b2 = tile_base(g, tw, c.rows);
      b2.in = wsr; b2.aux = in; b2.out = out; b2.alpha = 1.0; b2.gamma = -1.0; b2.active = active;
      if (kmode == 0) launch_tile<T, true, LD_PLAIN, ST_AXPBY>(b2, np, g.B, c.rows.nthr, c.rows.lds, s);
      else launch_tile<T, true, LD_PLAIN, ST_PLAIN>(b2, np, g.B, c.rows.nthr, c.rows.lds, s);
    }
  }
}
template void apply_stage<float2>(Group&, int, const float2*, VecRef, VecRef, float2*, int, int, int, const int*,
                                  hipStream_t, const double*, long long, const GivensTask*, bool);
template void apply_stage<double2>(Group&, int, const double2*, VecRef, VecRef, double2*, int, int, int,
                                   const int*, hipStream_t, const double*, long long, const GivensTask*, bool);

template <class T>
void apply_op(Group& g, const T* deps, VecRef in, VecRef out, T* ws, int kmode, int transpose, int refl,
              const int* active, hipStream_t s, const double* in_scale, long long scale_stride,
              const GivensTask* gt) {
  // the quarter-plane kernels where the shape takes them
  const bool qp = quarter_planes(g, sizeof(T));
  for (int stage = 0; stage < 3; ++stage)
    apply_stage<T>(g, stage, deps, in, out, ws, kmode, transpose, refl, active, s, in_scale, scale_stride,
                   stage == 0 ? gt : nullptr, qp);
}
template void apply_op<float2>(Group&, const float2*, VecRef, VecRef, float2*, int, int, int, const int*,
                               hipStream_t, const double*, long long, const GivensTask*);
template void apply_op<double2>(Group&, const double2*, VecRef, VecRef, double2*, int, int, int, const int*,
                                hipStream_t, const double*, long long, const GivensTask*);

// e = E_inc + IFFT_xy(E_up exp(i beta z)) per plane (FP64)
void inject(Group& g, const double2* eup, double2* out, const int* active, hipStream_t s) {
  const Shape& sh = g.sh;
  const XYCfg c = xy_config(sh, 16);
  const int np = 3 * sh.nz;
  VecRef o = vr(out, sh.n3);
  if (c.fused) {
    TileArgs a = tile_base(g, g.dc->tw64, c.full);
    a.in = o; a.out = o; a.eup = eup; a.eup_stride = sh.nxny * 3; a.active = active;
    launch_tile<double2, true, LD_INJECT, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
  } else {
    TileArgs a = tile_base(g, g.dc->tw64, c.cols);
    a.in = o; a.out = o; a.eup = eup; a.eup_stride = sh.nxny * 3; a.active = active;
    launch_tile<double2, true, LD_INJECT, ST_PLAIN>(a, np, g.B, c.cols.nthr, c.cols.lds, s);
    TileArgs b2 = tile_base(g, g.dc->tw64, c.rows);
    b2.in = o; b2.out = o; b2.active = active;
    launch_tile<double2, true, LD_PLAIN, ST_PLAIN>(b2, np, g.B, c.rows.nthr, c.rows.lds, s);
  }
}

// spectra of k0^2 delta_eps (x + e) into ws64, then per-order plane-wave readouts
void readout(Group& g, const double2* x, const double2* e, const int* active, hipStream_t s) {
  const Shape& sh = g.sh;
  const XYCfg c = xy_config(sh, 16);
  const int np = 3 * sh.nz;
  VecRef w = vr(g.ws64, sh.n3);
  if (c.fused) {
    TileArgs a = tile_base(g, g.dc->tw64, c.full);
    a.in = vr(x, sh.n3); a.aux = vr(e, sh.n3); a.vol = vr(g.deps64, sh.N); a.out = w; a.active = active;
    launch_tile<double2, false, LD_VXE, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
  } else {
    TileArgs a = tile_base(g, g.dc->tw64, c.rows);
    a.in = vr(x, sh.n3); a.aux = vr(e, sh.n3); a.vol = vr(g.deps64, sh.N); a.out = w; a.active = active;
    launch_tile<double2, false, LD_VXE, ST_PLAIN>(a, np, g.B, c.rows.nthr, c.rows.lds, s);
    TileArgs b2 = tile_base(g, g.dc->tw64, c.cols);
    b2.in = w; b2.out = w; b2.active = active;
    launch_tile<double2, false, LD_PLAIN, ST_PLAIN>(b2, np, g.B, c.cols.nthr, c.cols.lds, s);
  }
  launch_readout(sh.nx, sh.ny, sh.nz, w, g.tab, g.tab_stride, g.adn, g.aup, sh.nxny * 3, active, g.B, s);
}

// eup <- T_R (adn + e_inc); returns per-instance relative change (host)
Status reflect(Group& g, double2* eup, const int* active, std::vector<double>* change, hipStream_t s) {
  const Shape& sh = g.sh;
  launch_reflect(sh.nx, sh.ny, g.tab, g.tab_stride, g.adn, eup, sh.nxny * 3, g.rpart, g.rblk, active, g.B, s);
  if (!change) return Status();
  HIPCHK(hipMemcpyAsync(g.h_dbl, g.rpart, sizeof(double) * 2 * g.rblk * g.B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  change->assign(g.B, 0.0);
  for (int b = 0; b < g.B; ++b) {
    double d2 = 0, n2 = 0;
    for (int k = 0; k < g.rblk; ++k) { d2 += g.h_dbl[((size_t)b * g.rblk + k) * 2]; n2 += g.h_dbl[((size_t)b * g.rblk + k) * 2 + 1]; }
    (*change)[b] = n2 > 0 ? std::sqrt(d2 / n2) : 0.0;
  }
  return Status();
}

Status set_mask(Group& g, int* dmask, const std::vector<int>& h, hipStream_t s) {
  std::memcpy(g.h_run + g.B, h.data(), sizeof(int) * g.B);
  HIPCHK(hipMemcpyAsync(dmask, g.h_run + g.B, sizeof(int) * g.B, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return Status();
}

Status read_norms(Group& g, const double* d, std::vector<double>& out, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(g.h_dbl, d, sizeof(double) * g.B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out.assign(g.h_dbl, g.h_dbl + g.B);
  return Status();
}

// A Gram-Schmidt update that leaves less than this fraction of ||w||^2
// (||w'|| < 0.32 ||w||, the cancellation at which one classical pass stops
// keeping the basis orthogonal to working accuracy) ends the Arnoldi cycle at
// that column; the restart recomputes the residual and starts a fresh basis.
// On the solver workloads it never triggers: iteration counts are those of a
// basis orthogonalised twice. PSFD_CANCEL overrides it (read at every solve)
// for experiments and for the test that forces the early restarts.
double cancel_threshold() {
  const char* e = std::getenv("PSFD_CANCEL");
  return e ? std::atof(e) : 0.1;
}

// Restarts of the device-driven solve evaluate b - A x (the FP64 residual of
// the refinement) at least every this many restarts; the ones in between take
// the cycle's GMRES residual from its basis, r = V_{k+1} Q^H (g_k e_k), formed
// in the solution-update kernel without an operator apply. The basis residual
// differs from b - A x by the rounding of the working precision, which the
// next evaluation of b - A x removes; convergence is only ever declared on
// b - A x. On the 128x128x64 contact-hole solve, periods 1, 2, 3, 4 and 6 all
// took 328 iterations to the same final residual. PSFD_TRUE_EVERY overrides it
// (1: b - A x at every restart).
int true_residual_every() {
  const char* e = std::getenv("PSFD_TRUE_EVERY");
  const int v = e ? std::atoi(e) : 6;
  return v < 1 ? 1 : v;
}

bool use_graphs() {
  const char* e = std::getenv("PSFD_GRAPH");
  return !(e && std::atoi(e) == 0);
}

bool lite_restarts() {
  const char* e = std::getenv("PSFD_LITE_RESTARTS");
  return !(e && std::atoi(e) == 0);
}

Status replay(Group& g, Group::Captured& c, const std::string& key, hipStream_t s,
              const std::function<void(hipStream_t)>& issue) {
  if (c.key != key) {
    if (c.exec) HIPCHK(hipGraphExecDestroy(c.exec));
    c.exec = nullptr;
    c.failed = false;
    c.key = key;
  }
  if (!c.exec && !c.failed) {
    // relaxed mode: the capture puts no restriction on what other threads of
    // the process do meanwhile. If HIP still refuses it (a capture invalidated
    // by work elsewhere), the error is cleared and this key runs eagerly.
    if (!g.cap_stream) HIPCHK(hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      issue(g.cap_stream);
      e = hipStreamEndCapture(g.cap_stream, &graph);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      c.exec = nullptr;
      c.failed = true;
      (void)hipGetLastError();
    }
  }
  if (c.exec) {
    HIPCHK(hipGraphLaunch(c.exec, s));
  } else {
    issue(s);
  }
  return Status();
}

std::string launch_key(double eta, int every) {
  char buf[192];
  const char* d = std::getenv("PSFD_FUSE_DOTS");
  const char* u = std::getenv("PSFD_FUSE_UPDATE");
  const char* q = std::getenv("PSFD_QUARTER_PLANES");
  std::snprintf(buf, sizeof(buf), "%.17g|%.17g|%d|%s|%s|%s", cancel_threshold(), eta, every, d ? d : "-",
                u ? u : "-", q ? q : "-");
  return buf;
}

template <class T> static T* deps_of_mut(Group& g);
template <> float2* deps_of_mut<float2>(Group& g) { return g.deps32; }
template <> double2* deps_of_mut<double2>(Group& g) { return g.deps64; }

// Whether the inverse transverse kernel of an Arnoldi step also forms the
// Gram-Schmidt projections of the vector it writes (FP32 64 x 64 and 128 x 128 square planes;
// PSFD_FUSE_DOTS=0 keeps the separate projection pass, read per call).
static bool fuse_dots(const Group& g, size_t esz) {
  const char* e = std::getenv("PSFD_FUSE_DOTS");
  if (e && std::atoi(e) == 0) return false;
  const XYCfg c = xy_config(g.sh, esz);
  return c.fused && tile_takes_dots(tile_base(g, nullptr, c.full), esz);
}

// Whether the forward transverse kernel of an Arnoldi step also does the
// Gram-Schmidt update of the previous column (FP32 64 x 64 and 128 x 128 square planes, and
// pencil blocks large enough to run the Givens task: at least GIVENS_THREADS
// threads, i.e. padded z lengths of 64 and more; with the projections in the
// inverse kernel, which also marks the update pending; PSFD_FUSE_UPDATE=0 keeps
// the separate update pass, read per call).
static bool fuse_update(const Group& g, size_t esz) {
  const char* e = std::getenv("PSFD_FUSE_UPDATE");
  if (e && std::atoi(e) == 0) return false;
  const XYCfg c = xy_config(g.sh, esz);
  return c.fused && tile_takes_update(tile_base(g, nullptr, c.full), esz) &&
         z_config(g.sh, esz).nthr >= GIVENS_THREADS && fuse_dots(g, esz);
}

// The inverse transverse stage of an Arnoldi step: the slot vout (j + 1) =
// IFFT_xy of the workspace. Returns true when the kernel also stored the
// projection partials of the new vector (fuse_dots), false when the separate
// projection pass must follow.
template <class T>
static bool arnoldi_inverse(Group& g, VecRef vout, int jh, hipStream_t s, bool qp = false) {
  T* ws = (T*)g.wsP;
  if constexpr (std::is_same<T, float2>::value) {
    if (fuse_dots(g, sizeof(T))) {
      const long long n3 = g.sh.n3, bsv = (long long)(g.m + 1) * n3;
      const XYCfg c = xy_config(g.sh, sizeof(T));
      TileArgs a = tile_base(g, twiddles<T>(g), c.full);
      a.in = vr(ws, n3); a.out = vout; a.active = g.run;
      a.dt = DotTask{g.basis, n3, bsv, g.st, g.dpart2, jh};
      launch_tile<T, true, LD_PLAIN, ST_DOTS>(a, 3 * g.sh.nz, g.B, c.full.nthr, c.full.lds, s);
      return true;
    }
  }
  apply_stage<T>(g, 2, (const T*)nullptr, vout, vout, ws, 1, 0, 0, g.run, s, nullptr, 0, nullptr, qp);
  return false;
}

template <class T>
static Status bench_gs_t(Group& g, int pass, int j, const T* x, int reps, float* ms, hipStream_t s) {
  T* V = (T*)g.basis;
  const long long n3 = g.sh.n3, bsv = (long long)(g.m + 1) * n3;
  for (int i = 0; i <= j + 1; ++i)
    HIPCHK(hipMemcpyAsync(V + (size_t)i * n3, x, sizeof(T) * n3, hipMemcpyDeviceToDevice, s));
  GState hs;
  std::memset(&hs, 0, sizeof(hs));
  hs.j = j;
  hs.m = g.m;
  for (int i = 0; i <= MAXM; ++i) hs.sc[i] = 1.0;
  const int one = 1;
  HIPCHK(hipMemcpyAsync(g.st, &hs, sizeof(GState), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(g.run, &one, sizeof(int), hipMemcpyHostToDevice, s));
  // the projections the update pass consumes
  krylov_dots<T>(V, n3, bsv, n3, g.st, g.run, g.dpart2, 1, s, j);
  // pass 2: the inverse transverse stage of the step, from a workspace holding x
  VecRef vout;
  std::memset(&vout, 0, sizeof(vout));
  vout.base = V; vout.bstride = bsv; vout.jstride = n3; vout.joff = j + 1;
  if (pass == 2) HIPCHK(hipMemcpyAsync(g.wsP, x, sizeof(T) * n3, hipMemcpyDeviceToDevice, s));
  // pass 3: the forward transverse stage of step j + 1 carrying the update of
  // column j where the shape allows it (else the plain forward stage); the
  // contrast is the first N values of x
  bool fwd_upd = false;
  TileArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  if (pass == 3) {
    HIPCHK(hipMemcpyAsync(deps_of_mut<T>(g), x, sizeof(T) * g.sh.N, hipMemcpyDeviceToDevice, s));
    if constexpr (std::is_same<T, float2>::value) fwd_upd = fuse_update(g, sizeof(T));
    if (fwd_upd) {
      const XYCfg c = xy_config(g.sh, sizeof(T));
      fa = tile_base(g, twiddles<T>(g), c.full);
      fa.in = vout; fa.vol = vr(deps_of_mut<T>(g), g.sh.N); fa.out = vr(g.wsP, n3); fa.active = g.run;
      fa.up = UpdateTask{V, n3, bsv, g.st, g.dpart2, g.part, j + 1};
    }
  }
  auto run_pass = [&]() {
    if (pass == 0) krylov_dots<T>(V, n3, bsv, n3, g.st, g.run, g.dpart2, 1, s, j);
    else if (pass == 1) krylov_update<T>(V, n3, bsv, n3, g.st, g.run, g.dpart2, g.part, 1, s, j, false);
    else if (pass == 2) arnoldi_inverse<T>(g, vout, j, s);
    else if (fwd_upd) {
      if constexpr (std::is_same<T, float2>::value) {
        const XYCfg c = xy_config(g.sh, sizeof(T));
        launch_tile<T, false, LD_UPD_VX, ST_PLAIN>(fa, 3 * g.sh.nz, 1, c.full.nthr, c.full.lds, s);
      }
    } else {
      apply_stage<T>(g, 0, deps_of_mut<T>(g), vout, vout, (T*)g.wsP, 1, 0, 0, g.run, s);
    }
  };
  run_pass();  // untimed: a kernel's first launch in the process carries set-up costs
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) run_pass();
  HIPCHK(hipEventRecord(e1, s));
  hipError_t e = hipEventSynchronize(e1);
  float t = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_status(e, "Gram-Schmidt timing");
  *ms = t / reps;
  return Status();
}

Status bench_gram_schmidt(Group& g, int pass, int j, const void* x, int reps, float* ms, hipStream_t s) {
  if (g.prec == PSFD_MIXED) return bench_gs_t<float2>(g, pass, j, (const float2*)x, reps, ms, s);
  return bench_gs_t<double2>(g, pass, j, (const double2*)x, reps, ms, s);
}

// Arnoldi steps the server issues per host check of the run flags.
const int STEPS_PER_SYNC = 4;

template <class T> static const T* deps_of(const Group& g);
template <> const float2* deps_of<float2>(const Group& g) { return g.deps32; }
template <> const double2* deps_of<double2>(const Group& g) { return g.deps64; }

template <class T>
bool arnoldi_step(Group& g, int transpose, int refl, hipStream_t s, int jh, const int* solve_mask) {
  T* V = (T*)g.basis;
  const long long n3 = g.sh.n3, bsv = (long long)(g.m + 1) * n3;
  VecRef vin;
  vin.base = V; vin.bstride = bsv; vin.jstride = n3;
  if (jh >= 0) {  // every running instance stands at step jh: fixed slots
    vin.idx = nullptr; vin.idx_stride = 0; vin.joff = jh;
  } else {
    vin.idx = &g.st[0].j; vin.idx_stride = (int)(sizeof(GState) / sizeof(int)); vin.joff = 0;
  }
  VecRef vout = vin;
  vout.joff = vin.joff + 1;
  // B v_j; slots keep the unnormalised vectors (v_i = sc[i] slot_i): the first
  // apply kernel scales slot j by inv_norm = sc[j] on load. In lock-step solves
  // the Givens step of step j - 1 rides along with this apply (gt), and the
  // last step of the cycle takes it at once. The last apply kernel also forms
  // the projections of the new vector where the shape allows (arnoldi_inverse);
  // elsewhere the projection pass follows it.
  const bool lock = jh >= 0;
  const GivensTask gt{g.st, g.run, g.part, RED_BLOCKS, 0};
  const double* isc = &g.st[0].inv_norm;
  const long long iss = (long long)(sizeof(GState) / sizeof(double));
  bool upd = false, upd_slots = false;
  if constexpr (std::is_same<T, float2>::value) {
    upd = lock && fuse_update(g, sizeof(T));
    upd_slots = !lock && fuse_update(g, sizeof(T));
  }
  if (upd_slots) {
    // instances at different steps (server slots): the same fused kernels, each
    // instance taking the update, the scale and the Givens step only while an
    // update is pending (GState::pend), and the last column's Givens step from
    // the projections, so that a slot computes exactly what a lone solve does
    const int np = 3 * g.sh.nz;
    const XYCfg c = xy_config(g.sh, sizeof(T));
    TileArgs a = tile_base(g, twiddles<T>(g), c.full);
    a.in = vin; a.vol = vr(deps_of<T>(g), g.sh.N); a.out = vr((T*)g.wsP, n3); a.active = g.run;
    a.up = UpdateTask{V, n3, bsv, g.st, g.dpart2, g.part, -1};
    if constexpr (std::is_same<T, float2>::value)
      launch_tile<T, false, LD_UPD_SLOT, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
    const GivensTask gp{g.st, g.run, g.part, np, 1};
    apply_stage<T>(g, 1, deps_of<T>(g), vin, vout, (T*)g.wsP, 1, transpose, refl, g.run, s, nullptr, 0, &gp);
    if (!arnoldi_inverse<T>(g, vout, jh, s)) krylov_dots<T>(V, n3, bsv, n3, g.st, g.run, g.dpart2, g.B, s, jh);
    krylov_givens_proj(g.st, g.run, g.dpart2, g.B, s, -1);
    return false;
  }
  if (upd) {
    // the update of column jh - 1 in the forward plane kernel, which transforms
    // slot jh unscaled; the pencil kernel scales it from the plane norm
    // partials and runs the Givens step of column jh - 1 in one extra block
    const int np = 3 * g.sh.nz;
    const XYCfg c = xy_config(g.sh, sizeof(T));
    TileArgs a = tile_base(g, twiddles<T>(g), c.full);
    a.in = vin; a.vol = vr(deps_of<T>(g), g.sh.N); a.out = vr((T*)g.wsP, n3); a.active = g.run;
    a.up = UpdateTask{V, n3, bsv, g.st, g.dpart2, g.part, jh};
    // at step 0 the per-slot kernel loads slot 0 scaled (no update, as the
    // server's first step does), and no Givens step is pending
    if constexpr (std::is_same<T, float2>::value) {
      if (jh > 0) launch_tile<T, false, LD_UPD_VX, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
      else launch_tile<T, false, LD_UPD_SLOT, ST_PLAIN>(a, np, g.B, c.full.nthr, c.full.lds, s);
    }
    const GivensTask gp{g.st, g.run, g.part, np, 0};
    apply_stage<T>(g, 1, deps_of<T>(g), vin, vout, (T*)g.wsP, 1, transpose, refl, g.run, s, nullptr, 0,
                   jh > 0 ? &gp : nullptr);
  }
  // steps on planes the quarter split takes run the quarter-plane kernels,
  // except where the one-block-per-plane kernels carry the Gram-Schmidt work
  // (FP32 128 x 128: the update in the forward kernel, the projections in the
  // inverse one)
  const bool qp = !upd && quarter_planes(g, sizeof(T)) &&
                  (std::is_same<T, double2>::value || !fuse_dots(g, sizeof(T)));
  if (!upd) {
    apply_stage<T>(g, 0, deps_of<T>(g), vin, vout, (T*)g.wsP, 1, transpose, refl, g.run, s, isc, iss,
                   lock && jh > 0 ? &gt : nullptr, qp);
    apply_stage<T>(g, 1, deps_of<T>(g), vin, vout, (T*)g.wsP, 1, transpose, refl, g.run, s, nullptr, 0, nullptr, qp);
  }
  if (!arnoldi_inverse<T>(g, vout, jh, s, qp)) krylov_dots<T>(V, n3, bsv, n3, g.st, g.run, g.dpart2, g.B, s, jh);
  // with the fused update, the last column of a cycle takes no update pass: its
  // Givens step uses the projections alone, and slot m keeps w (the restart's
  // residual coefficients fold the update in)
  // (with solve_mask the back substitution of the cycle follows in the same launch)
  if (upd && jh == g.m - 1) {
    if (solve_mask) {
      krylov_givens_proj_solve(g.st, g.run, g.dpart2, solve_mask, g.B, s, jh);
      return true;
    }
    krylov_givens_proj(g.st, g.run, g.dpart2, g.B, s, jh);
  } else if (!upd) {
    krylov_update<T>(V, n3, bsv, n3, g.st, g.run, g.dpart2, g.part, g.B, s, jh, !lock || jh == g.m - 1);
  }
  return false;
}

template bool arnoldi_step<float2>(Group&, int, int, hipStream_t, int, const int*);
template bool arnoldi_step<double2>(Group&, int, int, hipStream_t, int, const int*);

// Restarted GMRES on (I - K V) x = b for the instances with act[b] set, driven
// from the device. Each restart takes the residual of the active instances,
// either the FP64 r = b - A x or the last cycle's GMRES residual from its basis
// (see true_residual_every); krylov_cycle_start ends the solve of the converged
// (on b - A x) or failed ones and starts a cycle of the others (the Arnoldi
// cycle runs in the working precision T, x accumulates in FP64). The host only
// launches cycles and reads the active flags every few cycles; launches for
// finished instances, and for the residual path an instance does not take, are
// no-ops.
template <class T>
static Status linear_solve(Group& g, const Opts& o, const std::vector<int>& act, const std::vector<double>& rtol,
                           std::vector<SolveStats>& stats, int transpose, int refl, hipStream_t s) {
  const int B = g.B;
  const long long n3 = g.sh.n3, bsv = (long long)(g.m + 1) * n3;
  Status st = set_mask(g, g.mask, act, s);
  if (!st.ok()) return st;
  // the first restart evaluates b - A x for every active instance
  HIPCHK(hipMemcpyAsync(g.tres, g.mask, sizeof(int) * B, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(g.rres, 0, sizeof(int) * B, s));
  const int every = true_residual_every();
  std::memcpy(g.h_dbl, rtol.data(), sizeof(double) * B);
  HIPCHK(hipMemcpyAsync(g.rtol, g.h_dbl, sizeof(double) * B, hipMemcpyHostToDevice, s));
  vec_norm2<double2>(g.b, n3, n3, g.dpart, g.n2b, g.mask, B, s);
  krylov_solve_init(g.st, g.n2b, g.rtol, g.abs_target, o.max_iters, g.mask, B, s);
  const double eta = g.prec == PSFD_MIXED ? o.inner_eta : 0.0;
  // Each cycle start writes the active flags to mapped host memory. The host
  // reads them before every launch and stops launching once no instance is
  // active; an instance's flag only ever goes from 1 to 0, so any read is a
  // valid snapshot. An event after every FLAG_EVERY-th cycle paces the host:
  // it blocks only when more than FLAG_LAG events are outstanding, so the GPU
  // queue stays full while few cycles are queued past convergence.
  std::deque<int> pending;  // event slots in flight, oldest first
  bool done = false;
  volatile HostFlags* hf = g.h_flags;
  auto snapshot_live = [&]() {
    for (int b = 0; b < B; ++b)
      if (hf[b].act) return true;
    return false;
  };
  // Restarts with and without b - A x. Most restarts take the basis residual,
  // and the launches of an unused b - A x (the FP64 apply and the residual
  // kernel, launches that return at once) are left out of them. A restart
  // includes b - A x at every `every`-th cycle (the device's cadence from the
  // first restart), whenever the flags show a pending request, and once any
  // instance may be near its target: the host runs a few cycles ahead of the
  // flags, so it extrapolates each instance's ||r|| / target from its last two
  // readings (per cycle started) to the restart it is about to launch; while an
  // instance has fewer than two readings, every restart includes b - A x. Near
  // stays on for the rest of the solve (the device asks for b - A x near
  // convergence and before it declares convergence). An instance whose request
  // meets a restart without b - A x keeps it and waits (cycle_start), so the
  // choice affects speed, never results. PSFD_LITE_RESTARTS=0 includes b - A x
  // in every restart; PSFD_NEAR_RATIO overrides NEAR_RATIO (0: requests are
  // only seen in the flags and every instance counts as far, so that a test
  // can make instances wait).
  const double NEAR_RATIO = env_double("PSFD_NEAR_RATIO", 64.0);
  // an event every FLAG_EVERY cycles, at most FLAG_LAG of them outstanding
  // (PSFD_EV_EVERY, PSFD_EV_LAG override them for tuning)
  const int EV_EVERY = std::max(1, env_int("PSFD_EV_EVERY", FLAG_EVERY)), EV_LAG = env_int("PSFD_EV_LAG", FLAG_LAG);
  // every cycle that starts takes at least one step; restarts without b - A x
  // can make an instance wait (below) for as many cycles as the host runs
  // ahead, near convergence and at the iteration limit
  const int max_cycles = o.max_iters + 2 + 2 * (EV_EVERY * (EV_LAG + 1) + 2);
  const bool lite_ok = lite_restarts();
  bool near = false;
  struct Reading { int c = -1; double r = 0.0; };
  std::vector<Reading> last(B), prev(B);
  auto want_full = [&](int cyc) {
    if (!lite_ok || near) return true;
    bool full = cyc % every == 0;
    for (int b = 0; b < B; ++b) {
      if (!hf[b].act) continue;
      if (hf[b].want) full = true;
      const int c = hf[b].cycles;
      const double r = hf[b].ratio;
      if (r > 0.0 && c != last[b].c) {
        prev[b] = last[b];
        last[b] = Reading{c, r};
      }
      if (NEAR_RATIO <= 0.0) continue;
      if (prev[b].c < 0 || last[b].c <= prev[b].c) {
        full = true;  // fewer than two readings: this restart includes b - A x
        continue;
      }
      const double rate = std::pow(last[b].r / prev[b].r, 1.0 / (last[b].c - prev[b].c));
      if (last[b].r * std::pow(std::min(rate, 1.0), std::max(0, cyc - last[b].c)) <= NEAR_RATIO) near = true;
    }
    return full || near;
  };
  const double cancel = cancel_threshold();
  // the restart's residual: b - A x (FP64) where tres is set, the previous
  // cycle's basis residual (left in v0 and its norm partials) where rres is;
  // ||r||^2 from the partials of b - A x or of the basis residual, summed in the
  // cycle start
  auto cycle_start = [&](hipStream_t q, bool full) {
    if (full) {
      apply_op<double2>(g, g.deps64, vr(g.x, n3), vr(g.r, n3), g.ws64, 0, transpose, refl, g.tres, q);  // A x
      krylov_residual_parts<T>(g.b, g.r, (T*)g.basis, n3, n3, bsv, g.dpart, g.tres, B, q);
    }
    krylov_cycle_start_sum(g.st, g.n2, g.dpart, g.lpart, g.abs_target, eta, g.m, cancel, every, g.mask, g.tres,
                           g.rres, g.run, g.cyc, B, q, g.d_flags, full);
  };
  // every instance that runs a cycle starts it at j = 0 and stops for good
  // when it ends, so the running ones all stand at step `step`; the cycle's
  // solution update and the next restart's residual follow
  auto cycle_body = [&](hipStream_t q, bool full) {
    bool solved = false;
    for (int step = 0; step < g.m; ++step)
      solved = arnoldi_step<T>(g, transpose, refl, q, step, step == g.m - 1 ? g.cyc : nullptr);
    if (!solved) krylov_solve_small(g.st, g.cyc, B, q);
    krylov_lincomb_res<T, double2>((T*)g.basis, n3, bsv, g.x, n3, n3, g.st, g.cyc, g.rres, g.lpart, B, q);
    cycle_start(q, full);
  };
  const bool graphs = use_graphs();
  const std::string key = launch_key(eta, every);
  for (int b = 0; b < B; ++b) {
    hf[b].act = act[b] ? 1 : 0;  // until the first cycle start writes it
    hf[b].want = 0;
    hf[b].ratio = 0.0;
    hf[b].cycles = -1;
  }
  cycle_start(s, true);  // the first restart evaluates b - A x
  for (int cyc = 0; cyc < max_cycles && !done; ++cyc) {
    if (cyc > 0) {
      const bool full = want_full(cyc);
      if (graphs) {
        Status gs = replay(g, g.cycle_graph[transpose ? 1 : 0][refl ? 1 : 0][full ? 1 : 0], key, s,
                           [&](hipStream_t q) { cycle_body(q, full); });
        if (!gs.ok()) return gs;
      } else {
        cycle_body(s, full);
      }
      HIPCHK(hipGetLastError());
    }
    // the flags are valid at any time (an instance's act only goes to 0, and
    // only once its solve has ended); events every EV_EVERY cycles keep the
    // host at most FLAG_LAG events ahead
    if (!snapshot_live()) break;
    if (cyc % EV_EVERY == 0) {
      const int slot = (cyc / EV_EVERY) % FLAG_SLOTS;
      HIPCHK(hipEventRecord(g.flag_ev[slot], s));
      pending.push_back(slot);
    }
    while (!pending.empty()) {
      const int old = pending.front();
      hipError_t q = (int)pending.size() > EV_LAG ? hipEventSynchronize(g.flag_ev[old]) : hipEventQuery(g.flag_ev[old]);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return hip_status(q, "solve flags");
      pending.pop_front();
      if (!snapshot_live()) { done = true; break; }
    }
    if (done) break;
  }
  std::vector<GState> hs(B);
  HIPCHK(hipMemcpyAsync(hs.data(), g.st, sizeof(GState) * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b) {
    if (!act[b]) continue;
    stats[b].iters = hs[b].iters;
    stats[b].cycles += hs[b].cycles;
    stats[b].rel_res = hs[b].rel_res;
    if (hs[b].status != PSFD_OK) stats[b].status = hs[b].status;
  }
  return Status();
}


// Forward solve: outer fixed point over the multilayer reflection (eqs. (8)-(9))
// around the Lippmann-Schwinger solve of eq. (18). Step i: E_up = T_R(E_inc +
// E_mask,down(z_top)); e = E_inc + E_layer; b = K V e; solve (I - K V) x = b
// (warm start); read the downgoing mask field at z_top off V (x + e); stop when
// the reflected spectrum changes by at most outer_rtol.
template <class T>
static Status solve_group_t(Group& g, const Opts& o, std::vector<SolveStats>& stats, hipStream_t s) {
  const int B = g.B;
  const Shape& sh = g.sh;
  const long long n3 = sh.n3, nq = sh.nxny * 3;
  stats.assign(B, SolveStats());
  if (g.prec == PSFD_MIXED)
    vec_axpby<float2, double2, double2>(g.deps32, g.deps64, nullptr, 1.0, 0.0, sh.N, sh.N, nullptr, B, s);
  HIPCHK(hipMemsetAsync(g.x, 0, sizeof(double2) * n3 * B, s));
  HIPCHK(hipMemsetAsync(g.adn, 0, sizeof(double2) * nq * B, s));
  HIPCHK(hipMemsetAsync(g.eup, 0, sizeof(double2) * nq * B, s));
  HIPCHK(hipMemsetAsync(g.st, 0, sizeof(GState) * B, s));
  std::vector<int> act(B, 1);
  Status st = set_mask(g, g.mask2, act, s);
  if (!st.ok()) return st;
  st = reflect(g, g.eup, g.mask2, nullptr, s);
  if (!st.ok()) return st;
  std::vector<double> ebg2, change;
  // Inexact outer iteration: the first solves only need to resolve the current
  // change of the reflected spectrum; the last ones run at INNER_FACTOR * rtol so
  // that solver noise stays below the outer tolerance.
  const double final_tol = INNER_FACTOR * o.rtol;
  std::vector<double> tol(B, std::max(final_tol, FIRST_INNER_TOL));
  for (int outer = 1; outer <= o.max_outer; ++outer) {
    st = set_mask(g, g.mask2, act, s);
    if (!st.ok()) return st;
    inject(g, g.eup, g.e, g.mask2, s);
    if (outer == 1) {
      vec_norm2<double2>(g.e, n3, n3, g.dpart, g.n2, g.mask2, B, s);
      st = read_norms(g, g.n2, ebg2, s);
      if (!st.ok()) return st;
    }
    apply_op<double2>(g, g.deps64, vr(g.e, n3), vr(g.b, n3), g.ws64, 1, 0, 0, g.mask2, s);
    st = linear_solve<T>(g, o, act, tol, stats, 0, 0, s);
    if (!st.ok()) return st;
    st = set_mask(g, g.mask2, act, s);
    if (!st.ok()) return st;
    readout(g, g.x, g.e, g.mask2, s);
    st = reflect(g, g.eup, g.mask2, &change, s);
    if (!st.ok()) return st;
    bool any = false;
    for (int b = 0; b < B; ++b) {
      if (!act[b]) continue;
      stats[b].outer = outer;
      stats[b].change = change[b];
      if (stats[b].status < 0 || (change[b] <= o.outer_rtol && tol[b] <= final_tol)) { act[b] = 0; continue; }
      tol[b] = std::max(final_tol, std::min(tol[b], OUTER_TO_INNER * change[b]));
      any = true;
    }
    if (!any) break;
  }
  for (int b = 0; b < B; ++b)
    if (act[b] && stats[b].status == PSFD_OK) stats[b].status = PSFD_NOT_CONVERGED;
  // final fields with the converged reflection: e, readouts, orders
  std::vector<int> all(B, 1);
  st = set_mask(g, g.mask2, all, s);
  if (!st.ok()) return st;
  inject(g, g.eup, g.e, g.mask2, s);
  readout(g, g.x, g.e, g.mask2, s);
  launch_orders(sh.nx, sh.ny, g.tab, g.tab_stride, g.eup, g.aup, g.ord, nq, B, s);
  // monolithic residual: u - K V u - (E_inc + R_vol T_R (E_inc + K_top V u)) with u = x + e
  vec_axpby<double2, double2, double2>(g.u, g.x, g.e, 1.0, 1.0, n3, n3, nullptr, B, s);
  st = reflect(g, g.eup2, g.mask2, nullptr, s);
  if (!st.ok()) return st;
  inject(g, g.eup2, g.r, g.mask2, s);
  apply_op<double2>(g, g.deps64, vr(g.u, n3), vr(g.b, n3), g.ws64, 0, 0, 0, g.mask2, s);  // b = u - K V u
  vec_axpby<double2, double2, double2>(g.b, g.b, g.r, 1.0, -1.0, n3, n3, nullptr, B, s);
  vec_norm2<double2>(g.b, n3, n3, g.dpart, g.n2, nullptr, B, s);
  std::vector<double> m2;
  st = read_norms(g, g.n2, m2, s);
  if (!st.ok()) return st;
  for (int b = 0; b < B; ++b) {
    stats[b].mono = ebg2[b] > 0 ? std::sqrt(m2[b] / ebg2[b]) : 0.0;
    if (!std::isfinite(stats[b].mono) && stats[b].status >= 0) stats[b].status = PSFD_ERR_NONFINITE;
  }
  return Status();
}

// Monolithic coupling: GMRES directly on (I - (K + R_vol T_R K_top) V) u = e_bg for
// the total field u in the slab, e_bg = E_inc + R_vol T_R E_inc. Its solution is
// the fixed point of the outer loop above; E_mask = u - E_inc - E_layer(u).
template <class T>
static Status solve_group_mono_t(Group& g, const Opts& o, std::vector<SolveStats>& stats, hipStream_t s) {
  const int B = g.B;
  const Shape& sh = g.sh;
  const long long n3 = sh.n3, nq = sh.nxny * 3;
  stats.assign(B, SolveStats());
  if (g.prec == PSFD_MIXED)
    vec_axpby<float2, double2, double2>(g.deps32, g.deps64, nullptr, 1.0, 0.0, sh.N, sh.N, nullptr, B, s);
  HIPCHK(hipMemsetAsync(g.adn, 0, sizeof(double2) * nq * B, s));
  HIPCHK(hipMemsetAsync(g.eup, 0, sizeof(double2) * nq * B, s));
  HIPCHK(hipMemsetAsync(g.st, 0, sizeof(GState) * B, s));
  std::vector<int> all(B, 1);
  Status st = set_mask(g, g.mask2, all, s);
  if (!st.ok()) return st;
  st = reflect(g, g.eup, g.mask2, nullptr, s);  // E_up of the incident wave alone
  if (!st.ok()) return st;
  inject(g, g.eup, g.b, g.mask2, s);             // b = e_bg
  HIPCHK(hipMemcpyAsync(g.x, g.b, sizeof(double2) * n3 * B, hipMemcpyDeviceToDevice, s));  // u0 = e_bg
  std::vector<double> tol(B, o.rtol);
  st = linear_solve<T>(g, o, all, tol, stats, 0, 1, s);
  if (!st.ok()) return st;
  // E_up = T_R (E_inc + K_top V u), E_layer, E_mask = u - e, orders
  apply_stage<double2>(g, 0, g.deps64, vr(g.x, n3), vr(g.x, n3), g.ws64, 0, 0, 0, g.mask2, s);
  launch_readout(sh.nx, sh.ny, sh.nz, vr(g.ws64, n3), g.tab, g.tab_stride, g.adn, g.aup, nq, g.mask2, B, s);
  st = reflect(g, g.eup, g.mask2, nullptr, s);
  if (!st.ok()) return st;
  inject(g, g.eup, g.e, g.mask2, s);
  launch_orders(sh.nx, sh.ny, g.tab, g.tab_stride, g.eup, g.aup, g.ord, nq, B, s);
  vec_axpby<double2, double2, double2>(g.x, g.x, g.e, 1.0, -1.0, n3, n3, nullptr, B, s);
  for (int b = 0; b < B; ++b) {
    stats[b].outer = 1;
    stats[b].mono = stats[b].rel_res;
  }
  HIPCHK(hipGetLastError());
  return Status();
}

Status solve_group(Group& g, const Opts& o, std::vector<SolveStats>& stats, hipStream_t s) {
  if (o.coupling == PSFD_COUPLING_MONO) {
    if (g.prec == PSFD_MIXED) return solve_group_mono_t<float2>(g, o, stats, s);
    return solve_group_mono_t<double2>(g, o, stats, s);
  }
  if (g.prec == PSFD_MIXED) return solve_group_t<float2>(g, o, stats, s);
  return solve_group_t<double2>(g, o, stats, s);
}

// Vector-Jacobian product of the reflected orders a = c0 + W V u, with u the total
// field of (I - M V) u = e_bg, for a cotangent G = dL/dRe a + i dL/dIm a of a real
// loss L: dL = Re sum_r k0^2 d(delta_eps) sum_c lam_c u_c with
// (I - M^T V) lam = W^T conj(G),  W = diag(e^{i beta T}) T_R K_top + K_up,
// so dL/dRe + i dL/dIm of delta_eps is conj(k0^2 sum_c lam_c u_c).
// u and G are device arrays [B][n3] and [B][nx ny 3]; the contrast is in g.deps64.
template <class T>
static Status adjoint_group_t(Group& g, const Opts& o, const double2* u, const double2* gord, double2* grad,
                              long long gstride, std::vector<SolveStats>& stats, hipStream_t s) {
  const int B = g.B;
  const Shape& sh = g.sh;
  const long long n3 = sh.n3, nq = sh.nxny * 3;
  stats.assign(B, SolveStats());
  if (g.prec == PSFD_MIXED)
    vec_axpby<float2, double2, double2>(g.deps32, g.deps64, nullptr, 1.0, 0.0, sh.N, sh.N, nullptr, B, s);
  launch_adjoint_source(sh.nx, sh.ny, g.tab, g.tab_stride, gord, g.adn, g.aup, nq, B, s);
  // s = W^T c: transposed plane-wave injection into b
  std::vector<int> all(B, 1);
  Status st = set_mask(g, g.mask2, all, s);
  if (!st.ok()) return st;
  {
    const XYCfg cfg = xy_config(sh, 16);
    const int np = 3 * sh.nz;
    VecRef ob = vr(g.b, n3);
    if (cfg.fused) {
      TileArgs ta = tile_base(g, g.dc->tw64, cfg.full);
      ta.in = ob; ta.out = ob; ta.eup = g.adn; ta.eup2 = g.aup; ta.eup_stride = nq; ta.active = g.mask2;
      launch_tile<double2, true, LD_INJECT_T, ST_PLAIN>(ta, np, B, cfg.full.nthr, cfg.full.lds, s);
    } else {
      TileArgs ta = tile_base(g, g.dc->tw64, cfg.cols);
      ta.in = ob; ta.out = ob; ta.eup = g.adn; ta.eup2 = g.aup; ta.eup_stride = nq; ta.active = g.mask2;
      launch_tile<double2, true, LD_INJECT_T, ST_PLAIN>(ta, np, B, cfg.cols.nthr, cfg.cols.lds, s);
      TileArgs tb = tile_base(g, g.dc->tw64, cfg.rows);
      tb.in = ob; tb.out = ob; tb.active = g.mask2;
      launch_tile<double2, true, LD_PLAIN, ST_PLAIN>(tb, np, B, cfg.rows.nthr, cfg.rows.lds, s);
    }
  }
  // lam: transposed coupled solve, lam0 = 0
  HIPCHK(hipMemsetAsync(g.x, 0, sizeof(double2) * n3 * B, s));
  HIPCHK(hipMemsetAsync(g.st, 0, sizeof(GState) * B, s));
  std::vector<double> tol(B, o.rtol);
  st = linear_solve<T>(g, o, all, tol, stats, 1, 1, s);
  if (!st.ok()) return st;
  launch_gradient(sh.N, g.tab, g.tab_stride, g.x, u, n3, grad, gstride, B, s);
  for (int b = 0; b < B; ++b) { stats[b].outer = 1; stats[b].mono = stats[b].rel_res; }
  HIPCHK(hipGetLastError());
  return Status();
}

Status adjoint_group(Group& g, const Opts& o, const double2* u, const double2* grad_orders, double2* grad,
                     std::vector<SolveStats>& stats, hipStream_t s) {
  if (g.prec == PSFD_MIXED) return adjoint_group_t<float2>(g, o, u, grad_orders, grad, g.sh.N, stats, s);
  return adjoint_group_t<double2>(g, o, u, grad_orders, grad, g.sh.N, stats, s);
}

}  // namespace psfd
