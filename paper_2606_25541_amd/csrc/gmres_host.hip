// Host-driven restarted GMRES (Saad & Schultz): classical Gram-Schmidt with the
// projections and ||w||^2 from one launch and the new norm by Pythagoras (a
// second pass where the update leaves less than `cancel` of the norm), Givens
// rotations and the small triangular solve on the host. Reductions run in a
// fixed order (block partials, then one block per sum), so a solve is
// deterministic.
#include "gmres_host.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <type_traits>
#include <vector>

namespace psfd {

namespace {

constexpr int KB = 256;      // threads per block
constexpr int KNB = 1024;    // blocks of a reduction pass
constexpr double ETA_MIXED = 1e-4;

#define GMCHK(call)                                    \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_status(e_, #call); \
  } while (0)

Status bad(int code, const char* m) {
  Status s;
  s.code = code;
  s.msg = m;
  return s;
}

// part[i * KNB + blk] = sum over the block's chunk of conj(V_i) w, i < nv (FP64 accumulation)
template <class TV, class TW>
__global__ void k_gm_dots(const TV* __restrict__ V, long long stride, const TW* __restrict__ w, long long n,
                          double2* __restrict__ part) {
  __shared__ double2 red[KB];
  const int i = blockIdx.y;
  const TV* v = V + i * stride;
  double2 acc = make_double2(0.0, 0.0);
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)KNB * KB) {
    const double2 a = to_d(v[e]), c = to_d(w[e]);
    acc.x += a.x * c.x + a.y * c.y;
    acc.y += a.x * c.y - a.y * c.x;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = KB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)i * KNB + blockIdx.x] = red[0];
}

// out[i] = sum of the KNB partials of i (one block per i, fixed order)
__global__ void k_gm_sum(const double2* __restrict__ part, double2* __restrict__ out) {
  __shared__ double2 red[KB];
  const int i = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int c = threadIdx.x; c < KNB; c += KB) acc = cadd(acc, part[(long long)i * KNB + c]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = KB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// w += sgn sum_{i < nv} coef[i] V_i (in FP64, stored in w's type)
template <class TW, class TV>
__global__ void k_gm_axpys(TW* __restrict__ w, const TV* __restrict__ V, long long stride,
                           const double2* __restrict__ coef, int nv, long long n, double sgn) {
  const long long e = (long long)blockIdx.x * KB + threadIdx.x;
  if (e >= n) return;
  double2 acc = to_d(w[e]);
  for (int i = 0; i < nv; ++i) {
    const double2 c = coef[i], v = to_d(V[i * stride + e]);
    acc.x += sgn * (c.x * v.x - c.y * v.y);
    acc.y += sgn * (c.x * v.y + c.y * v.x);
  }
  w[e] = from_d<TW>(acc);
}

// out = a + s c (s real)
__global__ void k_gm_comb(const double2* __restrict__ a, const double2* __restrict__ c, double s,
                          double2* __restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * KB + threadIdx.x;
  if (e < n) out[e] = make_double2(a[e].x + s * c[e].x, a[e].y + s * c[e].y);
}

// out = s a, converted to out's type (a may equal out)
template <class TA, class TO>
__global__ void k_gm_scale(const TA* a, double s, TO* out, long long n) {
  const long long e = (long long)blockIdx.x * KB + threadIdx.x;
  if (e < n) out[e] = from_d<TO>(cscale(to_d(a[e]), s));
}

template <class T>
Status gmres_t(long long n, const ApplyFn& A, const double2* B, double2* X, const HostGmres& o, psfd_info& inf,
               hipStream_t s) {
  typedef std::complex<double> cd;
  const bool f32 = sizeof(T) == 8;
  const int m = o.m;
  T* V = nullptr;
  double2 *w64 = nullptr, *r64 = nullptr, *part = nullptr, *hd = nullptr;
  struct Free {
    void* q[5];
    ~Free() { for (void* a : q) if (a) (void)hipFree(a); }
  } fr{{nullptr, nullptr, nullptr, nullptr, nullptr}};
  GMCHK(hipMalloc((void**)&V, (size_t)(m + 1) * n * sizeof(T)));
  fr.q[0] = V;
  GMCHK(hipMalloc((void**)&w64, (size_t)n * sizeof(double2)));
  fr.q[1] = w64;
  GMCHK(hipMalloc((void**)&r64, (size_t)n * sizeof(double2)));
  fr.q[2] = r64;
  GMCHK(hipMalloc((void**)&part, (size_t)KNB * (m + 1) * sizeof(double2)));
  fr.q[3] = part;
  GMCHK(hipMalloc((void**)&hd, (size_t)(m + 1) * sizeof(double2)));
  fr.q[4] = hd;
  const unsigned g1 = (unsigned)((n + KB - 1) / KB);
  const int dt = f32 ? PSFD_C64 : PSFD_C128;
  std::vector<cd> hv(m + 1);
  // hv[0..nv) = V_i^H x
  auto dots = [&](auto Vb, int nv, auto x) -> Status {
    typedef std::remove_cv_t<std::remove_pointer_t<decltype(Vb)>> TV;
    typedef std::remove_cv_t<std::remove_pointer_t<decltype(x)>> TX;
    hipLaunchKernelGGL((k_gm_dots<TV, TX>), dim3(KNB, nv), dim3(KB), 0, s, Vb, n, x, n, part);
    hipLaunchKernelGGL(k_gm_sum, dim3(nv), dim3(KB), 0, s, part, hd);
    GMCHK(hipGetLastError());
    GMCHK(hipMemcpyAsync(hv.data(), hd, nv * sizeof(double2), hipMemcpyDeviceToHost, s));
    GMCHK(hipStreamSynchronize(s));
    return Status();
  };
  // x += sgn sum_i c[i] V_i
  auto axpys = [&](auto x, const T* Vb, const std::vector<cd>& c, int nv, double sgn) -> Status {
    typedef std::remove_pointer_t<decltype(x)> TX;
    GMCHK(hipMemcpyAsync(hd, c.data(), nv * sizeof(double2), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((k_gm_axpys<TX, T>), dim3(g1), dim3(KB), 0, s, x, Vb, n, (const double2*)hd, nv, n, sgn);
    GMCHK(hipGetLastError());
    GMCHK(hipStreamSynchronize(s));  // c may change before the next call
    return Status();
  };
  auto norm = [&](auto x, double& out) -> Status {
    Status st = dots(x, 1, x);
    out = std::sqrt(std::max(hv[0].real(), 0.0));
    return st;
  };
  Status st;
  double bnorm = 0.0;
  if (!(st = norm(B, bnorm)).ok()) return st;
  if (!std::isfinite(bnorm)) return bad(PSFD_ERR_NONFINITE, "right-hand side is not finite");
  if (bnorm == 0.0) {
    GMCHK(hipMemsetAsync(X, 0, n * sizeof(double2), s));
    GMCHK(hipStreamSynchronize(s));
    inf.status = PSFD_OK;
    inf.rel_residual = 0.0;
    return Status();
  }
  double beta = bnorm, rel = 1.0;
  if (o.warm) {
    // r = b - A x0
    if (!(st = A(X, w64, PSFD_C128, s)).ok()) return st;
    hipLaunchKernelGGL(k_gm_comb, dim3(g1), dim3(KB), 0, s, B, w64, -1.0, r64, n);
    if (!(st = norm((const double2*)r64, beta)).ok()) return st;
    rel = beta / bnorm;
    if (!std::isfinite(rel)) return bad(PSFD_ERR_NONFINITE, "non-finite residual");
    inf.rel_residual = rel;
    if (rel <= o.rtol) {
      inf.status = PSFD_OK;
      GMCHK(hipStreamSynchronize(s));
      return Status();
    }
    hipLaunchKernelGGL((k_gm_scale<double2, T>), dim3(g1), dim3(KB), 0, s, r64, 1.0 / beta, V, n);
  } else {
    GMCHK(hipMemsetAsync(X, 0, n * sizeof(double2), s));
    hipLaunchKernelGGL((k_gm_scale<double2, T>), dim3(g1), dim3(KB), 0, s, B, 1.0 / beta, V, n);
  }
  std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), sn(m), h1(m + 1), y(m);
  std::vector<double> cs(m);
  auto Hij = [&](int i, int j) -> cd& { return H[(size_t)i * m + j]; };
  while (inf.iters < o.max_iters) {
    ++inf.cycles;
    std::fill(H.begin(), H.end(), cd(0.0));
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    const double stop = std::max(o.rtol * bnorm, f32 ? ETA_MIXED * beta : 0.0);
    int k = 0;
    for (int j = 0; j < m && inf.iters < o.max_iters; ++j) {
      // w = A v_j straight into slot j + 1; one launch gives V_{0..j}^H w and
      // ||w||^2; the norm after the update follows from Pythagoras, and a
      // cancellation (norm ratio below cancel) takes a second pass with a
      // computed norm
      T* wj = V + (j + 1) * n;
      if (!(st = A(V + j * n, wj, dt, s)).ok()) return st;
      if (!(st = dots((const T*)V, j + 2, (const T*)wj)).ok()) return st;
      const double w2 = hv[j + 1].real();
      double p2 = 0.0;
      for (int i = 0; i <= j; ++i) { h1[i] = hv[i]; Hij(i, j) = hv[i]; p2 += std::norm(hv[i]); }
      if (!(st = axpys(wj, V, h1, j + 1, -1.0)).ok()) return st;
      double hn = std::sqrt(std::max(w2 - p2, 0.0));
      if (!(hn >= o.cancel * std::sqrt(std::max(w2, 0.0)))) {
        if (!(st = dots((const T*)V, j + 1, (const T*)wj)).ok()) return st;
        for (int i = 0; i <= j; ++i) { h1[i] = hv[i]; Hij(i, j) += hv[i]; }
        if (!(st = axpys(wj, V, h1, j + 1, -1.0)).ok()) return st;
        if (!(st = norm((const T*)wj, hn)).ok()) return st;
      }
      if (!std::isfinite(hn) || !std::isfinite(w2)) return bad(PSFD_ERR_NONFINITE, "non-finite Krylov vector");
      Hij(j + 1, j) = hn;
      ++inf.iters;
      k = j + 1;
      for (int i = 0; i < j; ++i) {  // previous rotations
        const cd a = Hij(i, j), c2 = Hij(i + 1, j);
        Hij(i, j) = cs[i] * a + sn[i] * c2;
        Hij(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * c2;
      }
      const cd a = Hij(j, j);
      const double bb = hn, r = std::sqrt(std::norm(a) + bb * bb);
      if (r == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
      else if (std::abs(a) == 0.0) { cs[j] = 0.0; sn[j] = 1.0; }
      else { cs[j] = std::abs(a) / r; sn[j] = (a / std::abs(a)) * bb / r; }
      Hij(j, j) = cs[j] * a + sn[j] * bb;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      if (hn > 0.0) hipLaunchKernelGGL((k_gm_scale<T, T>), dim3(g1), dim3(KB), 0, s, wj, 1.0 / hn, wj, n);
      if (std::abs(g[j + 1]) <= stop || hn == 0.0) break;
    }
    for (int i = k - 1; i >= 0; --i) {  // back substitution
      cd acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= Hij(i, l) * y[l];
      y[i] = acc / Hij(i, i);
    }
    std::vector<cd> yk(y.begin(), y.begin() + k);
    if (!(st = axpys(X, V, yk, k, 1.0)).ok()) return st;
    // FP64 residual r = b - A x
    if (!(st = A(X, w64, PSFD_C128, s)).ok()) return st;
    hipLaunchKernelGGL(k_gm_comb, dim3(g1), dim3(KB), 0, s, B, w64, -1.0, r64, n);
    if (!(st = norm((const double2*)r64, beta)).ok()) return st;
    rel = beta / bnorm;
    if (!std::isfinite(rel)) return bad(PSFD_ERR_NONFINITE, "non-finite residual");
    if (rel <= o.rtol) { inf.status = PSFD_OK; break; }
    hipLaunchKernelGGL((k_gm_scale<double2, T>), dim3(g1), dim3(KB), 0, s, r64, 1.0 / beta, V, n);
  }
  inf.rel_residual = rel;
  inf.mono_residual = rel;
  GMCHK(hipGetLastError());
  GMCHK(hipStreamSynchronize(s));
  return Status();
}

}  // namespace

Status gmres_host(long long n, const ApplyFn& A, const double2* b, double2* x, const HostGmres& o, psfd_info& info,
                  hipStream_t s) {
  if (!(o.rtol > 0.0) || o.m < 1 || o.m > 64 || o.max_iters < 1)
    return bad(PSFD_ERR_INVALID_ARG, "need rtol > 0, 1 <= restart <= 64, max_iters >= 1");
  if (o.precision != PSFD_FP64 && o.precision != PSFD_MIXED)
    return bad(PSFD_ERR_INVALID_ARG, "precision must be PSFD_FP64 or PSFD_MIXED");
  info.status = PSFD_NOT_CONVERGED;
  return o.precision == PSFD_MIXED ? gmres_t<float2>(n, A, b, x, o, info, s) : gmres_t<double2>(n, A, b, x, o, info, s);
}

}  // namespace psfd
