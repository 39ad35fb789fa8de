// Differential PSFD operator with a z-PML (Sec. 3: eqs. (6)-(8) and the
// preconditioner study): on an extended z grid of nz_ext planes, with the clip
// periodic in x and y,
//     A E = curl curl E - k_bg^2 E - V E,   V = k0^2 delta_eps on the contrast planes,
// every derivative pseudo-spectral (eq. (6)); along z, stretched inside the PML
// layers at both ends by 1 / (1 + i s(z)) (eq. (7)). The spectral-damping
// preconditioner D(k) = min(1, k_bg^2 / |k|^2) acts on the left.
//
// One apply is three kinds of launch over the field [3][nz_ext][ny][nx]:
//   transverse FFT of every plane (the tile kernels of the main path, plain
//   load and store), the z pencil below (curl curl - k_bg^2 in the transverse
//   spectrum, every z derivative by an LDS FFT along the pencil), and the
//   inverse transverse FFT; then y -= V x on the contrast planes. With the
//   damping, y goes once more through forward, pencil (D) and inverse passes.
#include "diff.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "fft_lds.hpp"
#include "gmres_host.hpp"

struct psfd_diff_plan {
  psfd_diff_problem p{};
  psfd::Problem base;        // validated copy (layers owned)
  psfd::Shape se;            // extended grid (nz = nz_ext)
  int device = 0;
  std::unique_ptr<psfd::Group> gb;  // tables of the absorber problem (orders, T_R, incidence), FP64 buffers
  double* zt = nullptr;      // [kappa_d (nz_ext)][kappa (nz_ext)][inv_s (2 nz_ext)]
  void* ws32 = nullptr;      // apply workspaces (3 N_ext values)
  void* ws64 = nullptr;
  void* plane = nullptr;     // 3 planes of the readout, complex128
  std::vector<void*> owned;
  ~psfd_diff_plan() {
    for (void* q : owned) (void)hipFree(q);
  }
};

namespace psfd {

namespace {

#define DCHK(call)                                     \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_status(e_, #call); \
  } while (0)

Status bad(int code, const std::string& m) {
  Status s;
  s.code = code;
  s.msg = m;
  return s;
}

PSFD_D double2 cexpi(double2 z) {  // exp(i z)
  const double e = exp(-z.y);
  double sn, cs;
  sincos(z.x, &sn, &cs);
  return make_double2(e * cs, e * sn);
}

template <class T> PSFD_D T mul_i(T a, double k) {  // i k a
  typedef typename real_of<T>::type R;
  T r;
  r.x = -(R)k * a.y;
  r.y = (R)k * a.x;
  return r;
}

constexpr int DMODE_CURL = 0, DMODE_DAMP = 1;
constexpr int PMAX = 4;   // pencil points per thread per component

struct DiffPencilArgs {
  int nx, ny, pe, log2pe, bx, nthr;
  void* w;                  // [3][pe][ny][nx] in place
  const double* kx;         // [nx] per-order x wavenumbers (with the Bloch shift)
  const double* ky;         // [ny]
  const double* zt;         // kappa_d [pe], kappa [pe], inv_s [pe] (complex)
  double kbg2;
  const void* tw;
};

// One block: bx consecutive kx columns of one ky row, all pe planes of the three
// components. Both modes fold in 1 / (Nx Ny) for the unnormalised transverse
// transforms around them. Sequences live interleaved in LDS (element z of sequence s at
// z * NS + s), so FFT butterflies run sequence-fastest.
template <class T, int MODE>
__global__ void k_diff_pencil(DiffPencilArgs a) {
  extern __shared__ unsigned char smem[];
  T* L = reinterpret_cast<T*>(smem);
  typedef typename real_of<T>::type R;
  const int bx = a.bx, pe = a.pe, nthr = a.nthr, tid = threadIdx.x;
  const int ky = blockIdx.x / (a.nx / bx);
  const int kx0 = (blockIdx.x % (a.nx / bx)) * bx;
  const long long nxny = (long long)a.nx * a.ny, cstride = nxny * pe;
  T* w = (T*)a.w;
  const T* tw = (const T*)a.tw;
  const double* kap_d = a.zt;
  const double* kap = a.zt + pe;
  const double2* inv_s = reinterpret_cast<const double2*>(a.zt + 2 * pe);
  const double kyv = a.ky[ky];
  const int npts = bx * pe;   // points per component
  const R inv_pe = (R)(1.0 / pe);
  // the transverse transforms on either side are unnormalised: 1 / (Nx Ny) here
  const R inv_t = (R)(1.0 / ((double)a.nx * a.ny));
  if (MODE == DMODE_DAMP) {
    // 3 bx sequences: FFT_z, multiply by min(1, k_bg^2 / |k|^2) / pe, inverse
    const int NS = 3 * bx;
    for (int f = tid; f < 3 * npts; f += nthr) {
      const int c = f / npts, r = f - c * npts, z = r / bx, col = r - z * bx;
      L[z * NS + c * bx + col] = w[c * cstride + (long long)z * nxny + (long long)ky * a.nx + kx0 + col];
    }
    __syncthreads();
    lds_fft<T, false, true>(L, a.log2pe, NS, 1, NS, tw, tid, nthr);
    for (int f = tid; f < 3 * npts; f += nthr) {
      const int l = f / NS, sq = f - l * NS, col = sq % bx;
      const double kxv = a.kx[kx0 + col];
      const double k2 = kxv * kxv + kyv * kyv + kap[l] * kap[l];
      const double d = k2 > a.kbg2 ? a.kbg2 / k2 : 1.0;
      L[f] = cscale(L[f], (R)(d / ((double)pe * a.nx * a.ny)));
    }
    __syncthreads();
    lds_fft<T, true, true>(L, a.log2pe, NS, 1, NS, tw, tid, nthr);
    for (int f = tid; f < 3 * npts; f += nthr) {
      const int c = f / npts, r = f - c * npts, z = r / bx, col = r - z * bx;
      w[c * cstride + (long long)z * nxny + (long long)ky * a.nx + kx0 + col] = L[z * NS + c * bx + col];
    }
    return;
  }
  // curl curl - k_bg^2: the pencil's points stay in registers; the two z
  // derivatives of each curl go through LDS (sequences x: 0..bx-1, y: bx..2bx-1)
  const int NS = 2 * bx;
  T ux[PMAX], uy[PMAX], uz[PMAX], cz[PMAX], dzv[PMAX];
#pragma unroll
  for (int i = 0; i < PMAX; ++i) {
    const int f = tid + i * nthr;
    if (f < npts) {
      const int z = f / bx, col = f - z * bx;
      const long long o = (long long)z * nxny + (long long)ky * a.nx + kx0 + col;
      ux[i] = w[o];
      uy[i] = w[cstride + o];
      uz[i] = w[2 * cstride + o];
    }
  }
  // D_z f = (1 / s(z)) IFFT_z(i kappa_d FFT_z f) of the two sequences in LDS
  auto dz_pair = [&]() {
    __syncthreads();
    lds_fft<T, false, true>(L, a.log2pe, NS, 1, NS, tw, tid, nthr);
    for (int f = tid; f < NS * pe; f += nthr) {
      const int l = f / NS;
      L[f] = mul_i(L[f], kap_d[l] * (double)inv_pe);
    }
    __syncthreads();
    lds_fft<T, true, true>(L, a.log2pe, NS, 1, NS, tw, tid, nthr);
  };
#pragma unroll
  for (int i = 0; i < PMAX; ++i) {
    const int f = tid + i * nthr;
    if (f < npts) {
      const int z = f / bx, col = f - z * bx;
      L[z * NS + col] = ux[i];
      L[z * NS + bx + col] = uy[i];
    }
  }
  dz_pair();
  // c = curl u; then the sequences take c_x, c_y for the second curl
  T cx[PMAX], cy[PMAX];
#pragma unroll
  for (int i = 0; i < PMAX; ++i) {
    const int f = tid + i * nthr;
    if (f < npts) {
      const int z = f / bx, col = f - z * bx;
      const double kxv = a.kx[kx0 + col];
      const double2 is = inv_s[z];
      const T dzx = cmul(L[z * NS + col], from_d<T>(is)), dzy = cmul(L[z * NS + bx + col], from_d<T>(is));
      cx[i] = csub(mul_i(uz[i], kyv), dzy);
      cy[i] = csub(dzx, mul_i(uz[i], kxv));
      cz[i] = csub(mul_i(uy[i], kxv), mul_i(ux[i], kyv));
      dzv[i] = csub(mul_i(cy[i], kxv), mul_i(cx[i], kyv));   // (curl c)_z
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PMAX; ++i) {
    const int f = tid + i * nthr;
    if (f < npts) {
      const int z = f / bx, col = f - z * bx;
      L[z * NS + col] = cx[i];
      L[z * NS + bx + col] = cy[i];
    }
  }
  dz_pair();
  const R kb2 = (R)a.kbg2;
#pragma unroll
  for (int i = 0; i < PMAX; ++i) {
    const int f = tid + i * nthr;
    if (f < npts) {
      const int z = f / bx, col = f - z * bx;
      const double kxv = a.kx[kx0 + col];
      const double2 is = inv_s[z];
      const T dcx = cmul(L[z * NS + col], from_d<T>(is)), dcy = cmul(L[z * NS + bx + col], from_d<T>(is));
      const T dx = csub(mul_i(cz[i], kyv), dcy);
      const T dy = csub(dcx, mul_i(cz[i], kxv));
      const long long o = (long long)z * nxny + (long long)ky * a.nx + kx0 + col;
      w[o] = cscale(csub(dx, cscale(ux[i], kb2)), inv_t);
      w[cstride + o] = cscale(csub(dy, cscale(uy[i], kb2)), inv_t);
      w[2 * cstride + o] = cscale(csub(dzv[i], cscale(uz[i], kb2)), inv_t);
    }
  }
}

// y[c][zc0 + k] -= k0^2 deps[k] x[c][zc0 + k] on the contrast planes
template <class T>
__global__ void k_diff_vx(const T* __restrict__ deps, const T* __restrict__ x, T* __restrict__ y, long long plane,
                          long long nc, long long zoff, long long cstride, double k0sq) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nc) return;
  const long long c = e / nc, r = e - c * nc;
  const long long o = c * cstride + zoff * plane + r;
  typedef typename real_of<T>::type R;
  y[o] = csub(y[o], cscale(cmul(deps[r], x[o]), (R)k0sq));
}

// b = k0^2 deps e on the contrast planes (zero elsewhere, set beforehand); e is
// the source field on those planes ([3][ncz][ny][nx]), or, when e is null, the
// incident plane wave einc exp(-i beta0 z_k) (uniform over x and y: the
// envelope of the incident order 0) with z_k = (zc0 + k - z0 + 1/2) dz
__global__ void k_diff_rhs(const double2* __restrict__ deps, const double2* __restrict__ e, double2* __restrict__ b,
                           long long plane, int ncz, long long zoff, long long cstride, double k0sq, double2 ex,
                           double2 ey, double2 ez, double2 beta0, double zbase, double dz) {
  const long long nc = plane * ncz;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nc) return;
  const long long c = i / nc, r = i - c * nc;
  double2 src;
  if (e) {
    src = e[c * nc + r];
  } else {
    const double z = zbase + ((double)(r / plane) + 0.5) * dz;
    const double2 ph = cexpi(make_double2(-beta0.x * z, -beta0.y * z));
    src = cmul(c == 0 ? ex : (c == 1 ? ey : ez), ph);
  }
  b[c * cstride + zoff * plane + r] = cscale(cmul(deps[r], src), k0sq);
}

// Per-order amplitudes of a plane's transverse spectrum (3 planes, [3][ny][nx]):
// a_q = spec_q exp(-i beta_q dist) / (Nx Ny), zero on the orders the table drops
__global__ void k_diff_plane_orders(int nx, int ny, const double* __restrict__ tab, const double2* __restrict__ spec,
                                    double dist, double2* __restrict__ a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nx * ny) return;
  TabLayout L{nx, ny};
  const double keep = tab[L.off_keep() + q];
  const double2 beta = reinterpret_cast<const double2*>(tab + L.off_beta())[q];
  const double2 ph = cscale(cexpi(make_double2(-beta.x * dist, -beta.y * dist)), tab[TS_INVNXNY] * keep);
  const long long nq = (long long)nx * ny;
  for (int c = 0; c < 3; ++c) a[3LL * q + c] = cmul(spec[c * nq + q], ph);
}

template <class T>
__global__ void k_diff_cast(const double2* __restrict__ a, T* __restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = from_d<T>(a[e]);
}

// Block shape of the pencil: bx columns (power of two, <= 8, dividing nx) with
// 3 bx sequences of pe values within the FFT budget of <= 1024 threads and
// 96 KiB of LDS; threads enough for PMAX points each.
struct PencilCfg { int bx, nthr; size_t lds; };
PencilCfg pencil_cfg(int nx, int pe, size_t esz) {
  const int E = esz == 8 ? FftBudget<float2>::E : FftBudget<double2>::E;
  int bx = std::min(nx, 8);
  while (bx > 1 && (3 * bx * pe > E * 1024 || 3 * (size_t)bx * pe * esz > 96 * 1024 || bx * pe > PMAX * 1024)) bx /= 2;
  int nthr = std::max(64, (3 * bx * pe + E - 1) / E);
  nthr = std::max(nthr, (bx * pe + PMAX - 1) / PMAX);
  nthr = (nthr + 63) / 64 * 64;
  return PencilCfg{bx, std::min(nthr, 1024), 3 * (size_t)bx * pe * esz};
}

template <class T>
void launch_diff_pencil(const psfd_diff_plan& P, void* w, int mode, hipStream_t s) {
  const Shape& se = P.se;
  const size_t esz = sizeof(T);
  const PencilCfg c = pencil_cfg(se.nx, se.nz, esz);
  DiffPencilArgs a;
  a.nx = se.nx; a.ny = se.ny; a.pe = se.nz; a.log2pe = ilog2i(se.nz); a.bx = c.bx; a.nthr = c.nthr;
  a.w = w;
  TabLayout L{se.nx, se.ny};
  a.kx = P.gb->tab + L.off_kx();
  a.ky = P.gb->tab + L.off_ky();
  a.zt = P.zt;
  a.kbg2 = P.p.base.eps_bg * std::pow(2.0 * 3.14159265358979323846 / P.p.base.wavelength_nm, 2);
  a.tw = esz == 8 ? (const void*)P.gb->dc->tw32 : (const void*)P.gb->dc->tw64;
  dim3 grid((unsigned)(se.ny * (se.nx / c.bx)));
  auto go = [&](auto kern) {
    if (c.lds > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
    hipLaunchKernelGGL(kern, grid, dim3(c.nthr), c.lds, s, a);
  };
  if (mode == DMODE_DAMP) go(k_diff_pencil<T, DMODE_DAMP>);
  else go(k_diff_pencil<T, DMODE_CURL>);
}

// the transverse FFT of every plane of a [3][nz_ext][ny][nx] field (or of
// `nplanes` planes of a field of `sh`'s planes), plain load and store
template <class T, bool INV>
void transverse(const psfd_diff_plan& P, const Shape& sh, int nplanes, const void* in, void* out, hipStream_t s) {
  const XYCfg c = xy_config(sh, sizeof(T));
  const void* tw = sizeof(T) == 8 ? (const void*)P.gb->dc->tw32 : (const void*)P.gb->dc->tw64;
  auto base = [&](const TileShape& t) {
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = sh.nx; a.ny = sh.ny; a.nz = sh.nz;
    a.log2nx = ilog2i(sh.nx); a.log2ny = ilog2i(sh.ny);
    a.tx = t.tx; a.ty = t.ty; a.pitch = t.pitch;
    a.tiles_x = sh.nx / t.tx; a.tiles_y = sh.ny / t.ty;
    a.do_x = t.do_x; a.do_y = t.do_y;
    a.tab = P.gb->tab; a.tab_stride = P.gb->tab_stride;
    a.tw = tw;
    a.alpha = 0; a.gamma = 1;
    return a;
  };
  if (c.fused) {
    TileArgs a = base(c.full);
    a.in = vr(in); a.out = vr(out);
    launch_tile<T, INV, LD_PLAIN, ST_PLAIN>(a, nplanes, 1, c.full.nthr, c.full.lds, s);
  } else {
    // forward: rows then columns; inverse: columns then rows (either order is the 2-D DFT)
    TileArgs a = base(INV ? c.cols : c.rows);
    a.in = vr(in); a.out = vr(out);
    const TileShape& t1 = INV ? c.cols : c.rows;
    launch_tile<T, INV, LD_PLAIN, ST_PLAIN>(a, nplanes, 1, t1.nthr, t1.lds, s);
    TileArgs b2 = base(INV ? c.rows : c.cols);
    b2.in = vr(out); b2.out = vr(out);
    const TileShape& t2 = INV ? c.rows : c.cols;
    launch_tile<T, INV, LD_PLAIN, ST_PLAIN>(b2, nplanes, 1, t2.nthr, t2.lds, s);
  }
}

template <class T>
Status apply_t(psfd_diff_plan* P, const T* deps, const T* x, T* y, int precond, hipStream_t s) {
  const Shape& se = P->se;
  T* ws = (T*)(sizeof(T) == 8 ? P->ws32 : P->ws64);
  const int np = 3 * se.nz;
  transverse<T, false>(*P, se, np, x, ws, s);
  launch_diff_pencil<T>(*P, ws, DMODE_CURL, s);
  transverse<T, true>(*P, se, np, ws, y, s);
  const long long plane = se.nxny, nc = plane * P->p.ncz;
  const double k0 = 2.0 * 3.14159265358979323846 / P->p.base.wavelength_nm;
  hipLaunchKernelGGL(k_diff_vx<T>, dim3((unsigned)((3 * nc + 255) / 256)), dim3(256), 0, s, deps, x, y, plane, nc,
                     (long long)P->p.zc0, se.N, k0 * k0);
  if (precond == PSFD_PRECOND_DAMPING) {
    transverse<T, false>(*P, se, np, y, ws, s);
    launch_diff_pencil<T>(*P, ws, DMODE_DAMP, s);
    transverse<T, true>(*P, se, np, ws, y, s);
  }
  DCHK(hipGetLastError());
  return Status();
}

// D b in place on a complex128 field (the left preconditioning of the right-hand side)
Status damp64(psfd_diff_plan* P, double2* f, hipStream_t s) {
  const Shape& se = P->se;
  double2* ws = (double2*)P->ws64;
  transverse<double2, false>(*P, se, 3 * se.nz, f, ws, s);
  launch_diff_pencil<double2>(*P, ws, DMODE_DAMP, s);
  transverse<double2, true>(*P, se, 3 * se.nz, ws, f, s);
  DCHK(hipGetLastError());
  return Status();
}

// per-order amplitudes of the field e on plane k, carried `dist` away from the sources
Status read_plane(psfd_diff_plan* P, const double2* e, int k, double dist, double2* out, hipStream_t s) {
  const Shape& se = P->se;
  double2* pl = (double2*)P->plane;
  for (int c = 0; c < 3; ++c)
    DCHK(hipMemcpyAsync(pl + c * se.nxny, e + c * se.N + (long long)k * se.nxny, se.nxny * sizeof(double2),
                        hipMemcpyDeviceToDevice, s));
  Shape s1 = se;
  s1.nz = 1;
  transverse<double2, false>(*P, s1, 3, pl, pl, s);
  hipLaunchKernelGGL(k_diff_plane_orders, dim3((unsigned)((se.nxny + 255) / 256)), dim3(256), 0, s, se.nx, se.ny,
                     P->gb->tab, pl, dist, out);
  DCHK(hipGetLastError());
  return Status();
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

}  // namespace

Status diff_create(const psfd_diff_problem& p, psfd_diff_plan*& out) {
  auto P = std::make_unique<psfd_diff_plan>();
  P->p = p;
  Status st = validate_problem(&p.base, P->base);
  if (!st.ok()) return st;
  P->p.base.layers = nullptr;
  const int nz = p.base.nz;
  if (!pow2_in(p.nz_ext, 16, TW_MAX_N)) return bad(PSFD_ERR_UNSUPPORTED_SIZE, "nz_ext must be a power of two in [16, 1024]");
  if (p.form != PSFD_DIFF_BACKGROUND && p.form != PSFD_DIFF_FULL_DOMAIN)
    return bad(PSFD_ERR_INVALID_ARG, "form must be PSFD_DIFF_BACKGROUND or PSFD_DIFF_FULL_DOMAIN");
  if (p.form == PSFD_DIFF_BACKGROUND ? p.ncz != nz : p.ncz < nz)
    return bad(PSFD_ERR_INVALID_ARG, "the contrast planes must be the absorber (background form) or contain it");
  if (p.pml_cells < 0 || p.zc0 < p.pml_cells + 1 || p.zc0 + p.ncz + 1 > p.nz_ext - p.pml_cells)
    return bad(PSFD_ERR_INVALID_ARG, "the contrast planes and a readout plane on each side must lie outside the PML");
  if (!(p.pml_reflection > 0.0) || p.pml_reflection >= 1.0) P->p.pml_reflection = 1e-8;
  if (p.pml_order <= 0) P->p.pml_order = 3;
  DCHK(hipGetDevice(&P->device));
  Shape sb = shape_of(P->base.p);
  P->se = sb;
  P->se.nz = p.nz_ext;
  P->se.N = (long long)sb.nxny * p.nz_ext;
  P->se.n3 = 3 * P->se.N;
  std::vector<double> tab;
  st = build_table(P->base, tab);
  if (!st.ok()) return st;
  P->gb = std::make_unique<Group>();
  st = group_alloc(*P->gb, sb, 1, 1, PSFD_FP64);
  if (!st.ok()) return st;
  st = group_set_tables(*P->gb, 0, P->base, tab, nullptr);
  if (!st.ok()) return st;
  // z tables: kappa_d (z-Nyquist zeroed), kappa, 1 / s(z)
  const int pe = p.nz_ext;
  const double dz = p.base.t_nm / nz, kbg = 2.0 * 3.14159265358979323846 / p.base.wavelength_nm * std::sqrt(p.base.eps_bg);
  std::vector<double> zt(4 * (size_t)pe);
  const int npml = p.pml_cells, po = P->p.pml_order;
  const double Lp = npml * dz;
  const double smax = npml > 0 ? (po + 1) * std::log(1.0 / P->p.pml_reflection) / (2.0 * kbg * Lp) : 0.0;
  for (int k = 0; k < pe; ++k) {
    const int l = k < pe / 2 ? k : k - pe;
    const double kap = 2.0 * 3.14159265358979323846 * l / (pe * dz);
    zt[k] = l == -pe / 2 ? 0.0 : kap;
    zt[pe + k] = kap;
    double depth = -1.0;
    if (k < npml) depth = (npml - k - 0.5) * dz;
    else if (k >= pe - npml) depth = (k - (pe - npml) + 0.5) * dz;
    const double sg = depth >= 0.0 ? smax * std::pow(depth / Lp, po) : 0.0;
    // 1 / (1 + i sg)
    const double den = 1.0 + sg * sg;
    zt[2 * pe + 2 * k] = 1.0 / den;
    zt[2 * pe + 2 * k + 1] = -sg / den;
  }
  DCHK(hipMalloc((void**)&P->zt, zt.size() * sizeof(double)));
  P->owned.push_back(P->zt);
  DCHK(hipMemcpy(P->zt, zt.data(), zt.size() * sizeof(double), hipMemcpyHostToDevice));
  DCHK(hipMalloc(&P->plane, 3 * (size_t)sb.nxny * sizeof(double2)));
  P->owned.push_back(P->plane);
  DCHK(hipDeviceSynchronize());
  out = P.release();
  return Status();
}

void diff_destroy(psfd_diff_plan* p) { delete p; }

static Status ensure_ws(psfd_diff_plan* P, int dtype) {
  void*& w = dtype == PSFD_C64 ? P->ws32 : P->ws64;
  if (!w) {
    DCHK(hipMalloc(&w, (size_t)P->se.n3 * (dtype == PSFD_C64 ? 8 : 16)));
    P->owned.push_back(w);
  }
  return Status();
}

Status diff_apply(psfd_diff_plan* P, const void* deps, const void* x, void* y, int dtype, int precond, hipStream_t s) {
  if (precond != PSFD_PRECOND_NONE && precond != PSFD_PRECOND_DAMPING)
    return bad(PSFD_ERR_INVALID_ARG, "precond must be PSFD_PRECOND_NONE or PSFD_PRECOND_DAMPING");
  Status st = ensure_ws(P, dtype);
  if (!st.ok()) return st;
  if (dtype == PSFD_C64) return apply_t<float2>(P, (const float2*)deps, (const float2*)x, (float2*)y, precond, s);
  return apply_t<double2>(P, (const double2*)deps, (const double2*)x, (double2*)y, precond, s);
}

Status diff_solve(psfd_diff_plan* P, const void* deps_v, void* e_v, void* orders, const psfd_opts* opts, int precond,
                  psfd_info* info, hipStream_t s) {
  Opts o;
  Status st = make_opts(opts, o, 64);
  if (!st.ok()) return st;
  if (precond != PSFD_PRECOND_NONE && precond != PSFD_PRECOND_DAMPING)
    return bad(PSFD_ERR_INVALID_ARG, "precond must be PSFD_PRECOND_NONE or PSFD_PRECOND_DAMPING");
  if ((st = ensure_ws(P, PSFD_C128)).ok() && o.precision == PSFD_MIXED) st = ensure_ws(P, PSFD_C64);
  if (!st.ok()) return st;
  const Shape& se = P->se;
  Group& g = *P->gb;
  const Shape& sb = g.sh;
  const long long plane = se.nxny, nc = plane * P->p.ncz;
  const double2* deps = (const double2*)deps_v;
  double2* E = (double2*)e_v;
  const double k0 = 2.0 * 3.14159265358979323846 / P->p.base.wavelength_nm;
  const double dz = P->p.base.t_nm / sb.nz;
  const int z0 = P->p.zc0 + P->p.ncz - sb.nz;  // first absorber plane
  const long long nq = sb.nxny * 3;
  // FP32 contrast for the mixed-precision applies; b
  float2* deps32 = nullptr;
  double2* b = nullptr;
  struct Free {
    void* q[2];
    ~Free() { for (void* a : q) if (a) (void)hipFree(a); }
  } fr{{nullptr, nullptr}};
  DCHK(hipMalloc((void**)&b, (size_t)se.n3 * sizeof(double2)));
  fr.q[0] = b;
  if (o.precision == PSFD_MIXED) {
    DCHK(hipMalloc((void**)&deps32, (size_t)nc * sizeof(float2)));
    fr.q[1] = deps32;
    hipLaunchKernelGGL(k_diff_cast<float2>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, deps, deps32, nc);
  }
  ApplyFn A = [&](const void* x, void* y, int dt, hipStream_t q) {
    return diff_apply(P, dt == PSFD_C64 ? (const void*)deps32 : (const void*)deps, x, y, dt, precond, q);
  };
  HostGmres go;
  go.rtol = o.rtol;
  go.m = o.restart;
  go.max_iters = o.max_iters;
  go.precision = o.precision;
  go.warm = true;
  DCHK(hipMemsetAsync(E, 0, (size_t)se.n3 * sizeof(double2), s));
  psfd_info inf{};
  std::vector<int> one(1, 1);
  st = set_mask(g, g.mask2, one, s);
  if (!st.ok()) return st;
  // the incident wave's reflection E_up (no mask field yet); zero for the full domain
  DCHK(hipMemsetAsync(g.adn, 0, nq * sizeof(double2), s));
  DCHK(hipMemsetAsync(g.eup, 0, nq * sizeof(double2), s));
  const bool bg = P->p.form == PSFD_DIFF_BACKGROUND;
  if (bg) {
    st = reflect(g, g.eup, g.mask2, nullptr, s);
    if (!st.ok()) return st;
  }
  const int max_outer = bg ? std::max(1, o.max_outer) : 1;
  std::vector<double> change(1, 0.0);
  for (int outer = 1; outer <= max_outer; ++outer) {
    DCHK(hipMemsetAsync(b, 0, (size_t)se.n3 * sizeof(double2), s));
    if (bg) {
      inject(g, g.eup, g.e, g.mask2, s);  // e = E_inc + E_layer on the absorber planes
      hipLaunchKernelGGL(k_diff_rhs, dim3((unsigned)((3 * nc + 255) / 256)), dim3(256), 0, s, deps, g.e, b, plane,
                         P->p.ncz, (long long)P->p.zc0, se.N, k0 * k0, make_double2(0, 0), make_double2(0, 0),
                         make_double2(0, 0), make_double2(0, 0), 0.0, dz);
    } else {
      std::vector<double> h(TS_COUNT);
      DCHK(hipMemcpyAsync(h.data(), g.tab, sizeof(double) * TS_COUNT, hipMemcpyDeviceToHost, s));
      DCHK(hipStreamSynchronize(s));
      const double2 ex = make_double2(h[TS_EINC], h[TS_EINC + 1]), ey = make_double2(h[TS_EINC + 2], h[TS_EINC + 3]),
                    ez = make_double2(h[TS_EINC + 4], h[TS_EINC + 5]), b0 = make_double2(h[TS_BINC], h[TS_BINC + 1]);
      hipLaunchKernelGGL(k_diff_rhs, dim3((unsigned)((3 * nc + 255) / 256)), dim3(256), 0, s, deps,
                         (const double2*)nullptr, b, plane, P->p.ncz, (long long)P->p.zc0, se.N, k0 * k0, ex, ey, ez,
                         b0, (P->p.zc0 - z0) * dz, dz);
    }
    DCHK(hipGetLastError());
    if (precond == PSFD_PRECOND_DAMPING) {
      st = damp64(P, b, s);
      if (!st.ok()) return st;
    }
    psfd_info li{};
    st = gmres_host(se.n3, A, b, E, go, li, s);
    if (!st.ok()) return st;
    inf.iters += li.iters;
    inf.cycles += li.cycles;
    inf.rel_residual = li.rel_residual;
    inf.status = li.status;
    inf.outer_iters = outer;
    if (!bg) break;
    // downgoing mask field at z = 0 from the plane below the absorber; new E_up
    st = read_plane(P, E, z0 - 1, 0.5 * dz, g.adn, s);
    if (!st.ok()) return st;
    st = reflect(g, g.eup, g.mask2, &change, s);
    if (!st.ok()) return st;
    inf.outer_change = change[0];
    if (li.status != PSFD_OK || change[0] <= (o.outer_rtol > 0 ? o.outer_rtol : o.rtol)) break;
  }
  if (bg && inf.status == PSFD_OK && inf.outer_change > (o.outer_rtol > 0 ? o.outer_rtol : o.rtol))
    inf.status = PSFD_NOT_CONVERGED;
  if (orders) {
    // upgoing field above the absorber, referenced at z = T; plus E_up exp(i beta T)
    st = read_plane(P, E, z0 + sb.nz, 0.5 * dz, g.aup, s);
    if (!st.ok()) return st;
    if (!bg) DCHK(hipMemsetAsync(g.eup, 0, nq * sizeof(double2), s));
    launch_orders(sb.nx, sb.ny, g.tab, g.tab_stride, g.eup, g.aup, (double2*)orders, nq, 1, s);
    DCHK(hipGetLastError());
  }
  DCHK(hipStreamSynchronize(s));
  if (info) *info = inf;
  return Status();
}

}  // namespace psfd
