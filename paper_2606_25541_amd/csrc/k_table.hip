// Per-order tables of one instance, computed on the device in FP64: the
// z-wavenumber beta of every transverse Floquet order, exp(i beta L), the
// Nyquist keep mask and the reflection dyad T_R = r_s s s^T + r_p p+ p-^T of
// the layered stack (Sec. 2, background field; r_s and r_p from the recursive
// generalized reflection coefficient, r_s the E-field and r_p the H-field
// ratio). One thread per order; the recursion walks the stack from the
// substrate up, one interface at a time.
#include "kernels.hpp"

namespace psfd {

// principal square root, then the branch with Im >= 0 (Re >= 0 on the real axis):
// outgoing or decaying waves for the e^{-i omega t} convention
PSFD_D double2 kz_branch(double2 z) {
  const double a = z.x, b = z.y;
  const double r = hypot(a, b);
  double2 w;
  if (r == 0.0) {
    w.x = 0.0; w.y = 0.0;
  } else if (a >= 0.0) {
    const double t = sqrt(0.5 * (r + a));
    w.x = t; w.y = b / (2.0 * t);
  } else {
    const double t = sqrt(0.5 * (r - a));
    w.x = fabs(b) / (2.0 * t); w.y = copysign(t, b);
  }
  if (w.y < 0.0 || (w.y == 0.0 && w.x < 0.0)) { w.x = -w.x; w.y = -w.y; }
  return w;
}

PSFD_D double2 cexp_d(double2 z) {
  double s, c;
  sincos(z.y, &s, &c);
  const double m = exp(z.x);
  return make_double2(m * c, m * s);
}

// Fresnel coefficient of the interface between media i (above) and j (below)
PSFD_D double2 fresnel(bool tm, double2 ei, double2 ki, double2 ej, double2 kj) {
  if (!tm) return cdiv(csub(ki, kj), cadd(ki, kj));
  const double2 a = cmul(ej, ki), b = cmul(ei, kj);
  return cdiv(csub(a, b), cadd(a, b));
}

// Generalized reflection coefficient at the top of the stack for transverse
// wavenumber kt: R_i = (r_i + R_{i+1} ph) / (1 + r_i R_{i+1} ph), with
// ph = exp(2 i kz_{i+1} d_{i+1}), starting from the last interface.
// lay[0] ambient, lay[1..nl] layers (top first), lay[nl+1] substrate, each
// (eps_re, eps_im, thickness, 0).
PSFD_D double2 stack_r(bool tm, double k0sq, double kt2, const double4* __restrict__ lay, int nl) {
  double2 eb = make_double2(lay[nl + 1].x, lay[nl + 1].y);
  double2 kb = kz_branch(make_double2(k0sq * eb.x - kt2, k0sq * eb.y));
  double2 ea = make_double2(lay[nl].x, lay[nl].y);
  double2 ka = kz_branch(make_double2(k0sq * ea.x - kt2, k0sq * ea.y));
  double2 R = fresnel(tm, ea, ka, eb, kb);
  for (int i = nl - 1; i >= 0; --i) {
    // interface between layer i (above) and layer i+1 (below, thickness d)
    eb = ea; kb = ka;
    const double d = lay[i + 1].z;
    ea = make_double2(lay[i].x, lay[i].y);
    ka = kz_branch(make_double2(k0sq * ea.x - kt2, k0sq * ea.y));
    const double2 r = fresnel(tm, ea, ka, eb, kb);
    const double2 ph = cexp_d(make_double2(-2.0 * kb.y * d, 2.0 * kb.x * d));
    const double2 Rp = cmul(R, ph);
    R = cdiv(cadd(r, Rp), cadd(make_double2(1.0, 0.0), cmul(r, Rp)));
  }
  return R;
}

__global__ void __launch_bounds__(256) k_stack_table(int nx, int ny, double* __restrict__ tab,
                                                     const double4* __restrict__ lay, int nl, double k0sq,
                                                     double phi) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nx * ny) return;
  const int i = q % nx, j = q / nx;
  const TabLayout Lt{nx, ny};
  const double kbg = tab[TS_KBG], T = tab[TS_L];
  const double kx = tab[Lt.off_kx() + i], ky = tab[Lt.off_ky() + j];
  const double kt2 = kx * kx + ky * ky, kt = sqrt(kt2);
  const double2 b = kz_branch(make_double2(kbg * kbg - kt2, 0.0));
  double* beta = tab + Lt.off_beta();
  double* eibl = tab + Lt.off_eibl();
  double* keep = tab + Lt.off_keep();
  double* tr = tab + Lt.off_tr() + 18LL * q;
  double* mono = tab + Lt.off_mono() + 18LL * q;
  beta[2 * q] = b.x; beta[2 * q + 1] = b.y;
  const double2 e = cexp_d(make_double2(-b.y * T, b.x * T));
  eibl[2 * q] = e.x; eibl[2 * q + 1] = e.y;
  const bool nyq = (i == nx / 2) || (j == ny / 2);
  keep[q] = nyq ? 0.0 : 1.0;
  if (nyq) {
    for (int k = 0; k < 18; ++k) { tr[k] = 0.0; mono[k] = 0.0; }
    return;
  }
  // s = z x kt / |kt| (azimuth of the incidence at kt = 0); p+- = k+- x s / kbg
  double s0, s1;
  if (kt > 0.0) { s0 = -ky / kt; s1 = kx / kt; }
  else { s0 = -sin(phi); s1 = cos(phi); }
  // k+- x s with s = (s0, s1, 0), k+- = (kx, ky, +-b)
  const double ib = 1.0 / kbg;
  double2 pp[3], pm[3];
  pp[0] = cscale(cscale(b, -s1), ib);           // ky*0 - (+b) s1
  pp[1] = cscale(cscale(b, s0), ib);            // (+b) s0 - kx*0
  pp[2] = make_double2((kx * s1 - ky * s0) * ib, 0.0);
  pm[0] = cscale(pp[0], -1.0);
  pm[1] = cscale(pp[1], -1.0);
  pm[2] = pp[2];
  const double2 rs = stack_r(false, k0sq, kt2, lay, nl);
  const double2 rp = stack_r(true, k0sq, kt2, lay, nl);
  const double sv[3] = {s0, s1, 0.0};
  double2 T_R[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double2 t = cadd(cscale(rs, sv[r] * sv[c]), cmul(rp, cmul(pp[r], pm[c])));
      T_R[3 * r + c] = t;
      tr[2 * (3 * r + c)] = t.x;
      tr[2 * (3 * r + c) + 1] = t.y;
    }
  // M = T_R fac P-, fac = (i dz / 2 beta) / (Nx Ny), P- = I - k- k-^T / k_bg^2, k- = (kx, ky, -beta)
  const double2 fac = cscale(cdiv(make_double2(0.0, tab[TS_DZ]), make_double2(2.0 * b.x, 2.0 * b.y)), tab[TS_INVNXNY]);
  const double2 km[3] = {make_double2(kx, 0.0), make_double2(ky, 0.0), make_double2(-b.x, -b.y)};
  const double ik2 = 1.0 / (kbg * kbg);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      // (T_R P-)_{rc} = T_R,rc - sum_k T_R,rk km_k km_c / k_bg^2
      const double2 tk = cadd(cadd(cmul(T_R[3 * r], km[0]), cmul(T_R[3 * r + 1], km[1])), cmul(T_R[3 * r + 2], km[2]));
      const double2 m = cmul(fac, csub(T_R[3 * r + c], cscale(cmul(tk, km[c]), ik2)));
      mono[2 * (3 * r + c)] = m.x;
      mono[2 * (3 * r + c) + 1] = m.y;
    }
}

void launch_stack_table(int nx, int ny, double* tab, const double4* lay, int nl, double k0sq, double phi,
                        hipStream_t s) {
  const int n = nx * ny;
  k_stack_table<<<(n + 255) / 256, 256, 0, s>>>(nx, ny, tab, lay, nl, k0sq, phi);
}

}  // namespace psfd
