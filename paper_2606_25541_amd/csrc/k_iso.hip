// Isolated-domain mode: the Lippmann-Schwinger operator of eq. (18) for a
// scatterer in free space, with the dyadic Green's function truncated to a ball
// of radius R (eqs. (13), (15)-(17)) and zero padding by 2 on all three axes.
//
// Precompute (FP64, once per plan): F[G_R] = A(k) I + B(k) k^ k^ sampled on a
// grid oversampled per axis (period P_a = o_a L_a, o_a the smallest power of two
// >= max(4, 1 + R / L_a), so that the images of the ball at multiples of P_a
// miss every offset |j| <= L_a the padded convolution meets), Nyquist planes
// zeroed; inverse DFT, restriction to the offsets [-n, n) per axis, forward
// DFT on the 2n grid: the 6 distinct entries of the symmetric 3 x 3 table per
// wavevector of the padded grid.
//
// Apply y = x - P IFFT(table . FFT(Z V x)), V = k0^2 delta_eps:
//   X_FWD  rows x[c][z][y][0:nx] times V, FFT of length 2nx (zero half not read)
//   Y_FWD  columns of length ny -> 2ny (zero half not read)
//   Z_MUL  per (ky, kx): FFT of the 3 components along z (nz -> 2nz), 3 x 3
//          table product, inverse FFT, first nz outputs kept
//   Y_INV  columns 2ny -> first ny
//   X_INV  rows 2nx -> first nx, y = x - w / (8 nx ny nz)
// The padded spectrum lives in W[3][nz][2ny][2nx]: rows z >= nz of the padded
// grid are zero before the z transform and not needed after it, so they are
// never stored.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <type_traits>
#include <vector>

#include "engine.hpp"
#include "fft_lds.hpp"
#include "gmres_host.hpp"
#include "iso.hpp"

using namespace psfd;

namespace {

constexpr int ISO_TW_MAX = 1024;  // longest line of the precompute

// Line batch of one pass: line l of the pass starts at
// ((l & (cin - 1)) * s_in + (l >> lcin) * s_out) in src and in dst (own mappings),
// its elements are es apart (src and dst alike).
struct IsoLines {
  const void* src;
  void* dst;
  const void* xin;         // X_INV: the input x (y = x - scale w)
  const void* deps;        // X_FWD: delta_eps [nz][ny][nx], same type as x
  double vscale;           // X_FWD: k0^2
  long long nlines;
  int ln, lload, lstore;   // log2 of the FFT length, of the elements read and stored per line
  int lb, llb;             // lines per block (and log2)
  long long es;
  int lcin_s, lcin_d;
  long long sin_s, sout_s, sin_d, sout_d;
  int lvmod;               // X_FWD: delta_eps row of line l: l & (2^lvmod - 1)
  double scale;
  const void* tw;
};

enum { LN_PLAIN = 0, LN_VLOAD = 1, LN_AXPY = 2 };

// values per thread in the FFT passes of a line block (8 complex values: no
// spills in either precision; the block has (lines x length) / 8 threads)
constexpr int LFE = 8;

PSFD_D long long line_base(long long l, int lcin, long long s_in, long long s_out) {
  return (l & ((1LL << lcin) - 1)) * s_in + (l >> lcin) * s_out;
}

// One block: lb lines. SFL (strided lines, es != 1): consecutive threads take
// consecutive lines at one element (adjacent in memory), and the lines are
// interleaved in LDS; otherwise consecutive threads take consecutive elements
// of one line.
template <class T, bool INV, int MODE, bool SFL, bool ZIN, bool ZOUT>
__global__ void k_iso_lines(IsoLines a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  long long blk = blockIdx.x;
  if (MODE == LN_VLOAD) {
    // the three component blocks of one row group read the same delta_eps
    // rows: consecutive ids of an XCD's run take components 0, 1, 2 of one
    // group (the pass has 3 nz ny lines, so 3 divides the block count)
    const unsigned nb = gridDim.x, q = xcd_order(blockIdx.x, nb);
    blk = (long long)(q % 3u) * (nb / 3u) + q / 3u;
  }
  const long long l0 = blk << a.llb;
  const int n = 1 << a.ln;
  const T* src = (const T*)a.src;
  const int nld = (1 << a.lload) << a.llb;
  for (int idx = tid; idx < nld; idx += nthr) {
    int li, e;
    if (SFL) { li = idx & (a.lb - 1); e = idx >> a.llb; }
    else { li = idx >> a.lload; e = idx & ((1 << a.lload) - 1); }
    const long long l = l0 + li;
    T v = src[line_base(l, a.lcin_s, a.sin_s, a.sout_s) + e * a.es];
    if (MODE == LN_VLOAD) {
      const T d = ((const T*)a.deps)[((l & ((1LL << a.lvmod) - 1)) << a.lload) + e];
      v = cmul(v, cscale(d, (typename real_of<T>::type)a.vscale));
    }
    lds[SFL ? (e << a.llb) + li : (li << a.ln) + e] = v;
  }
  __syncthreads();
  if (SFL) lds_fft<T, INV, true, LFE, ZIN, ZOUT>(lds, a.ln, a.lb, 1, a.lb, (const T*)a.tw, tid, nthr);
  else lds_fft<T, INV, false, LFE, ZIN, ZOUT>(lds, a.ln, a.lb, n, 1, (const T*)a.tw, tid, nthr);
  T* dst = (T*)a.dst;
  const T* xin = (const T*)a.xin;
  typedef typename real_of<T>::type R;
  const R sc = (R)a.scale;
  const int nst = (1 << a.lstore) << a.llb;
  for (int idx = tid; idx < nst; idx += nthr) {
    int li, e;
    if (SFL) { li = idx & (a.lb - 1); e = idx >> a.llb; }
    else { li = idx >> a.lstore; e = idx & ((1 << a.lstore) - 1); }
    const long long l = l0 + li;
    const long long o = line_base(l, a.lcin_d, a.sin_d, a.sout_d) + e * a.es;
    const T w = cscale(lds[SFL ? (e << a.llb) + li : (li << a.ln) + e], sc);
    dst[o] = MODE == LN_AXPY ? csub(xin[o], w) : w;
  }
}

// Z_MUL: a block takes lb adjacent kx of one ky, all three
// components: 3 lb sequences of length 2nz interleaved in LDS.
struct IsoZ {
  void* w;
  const void* table;   // pencil-major: block (ky, kx / lb), then [nz + 1][6][lb] (kz <= nz); entries xx, yy, zz, xy, xz, yz
  int lnz, lnx2;       // log2 nz, log2 2nx
  int lb, llb;
  long long plane;     // 2ny 2nx
  long long n8;        // 8 nx ny nz
  const void* tw;
};

// Each thread owns the table products of points tid + i nthr (i < ZPT) and
// loads their six table entries before the forward z FFT, so that the loads
// are in flight while the FFT runs; points beyond ZPT nthr (not met by the
// launch shapes used) load theirs after it.
// (ZPT: 2 points per thread in FP32; none in FP64, where the prefetched
// entries and the FFT registers do not fit together without spills)
template <class T> struct Zpt { static constexpr int v = sizeof(T) == 8 ? 2 : 0; };
// values per thread in the z FFT passes (the block has at least els / ZFE threads)
constexpr int ZFE = 8;

template <class T>
PSFD_D void zmul_point(T* f, int lb, const T t[6]) {
  const T f0 = f[0], f1 = f[lb], f2 = f[2 * lb];
  f[0] = cadd(cadd(cmul(t[0], f0), cmul(t[3], f1)), cmul(t[4], f2));
  f[lb] = cadd(cadd(cmul(t[3], f0), cmul(t[1], f1)), cmul(t[5], f2));
  f[2 * lb] = cadd(cadd(cmul(t[4], f0), cmul(t[5], f1)), cmul(t[2], f2));
}

template <class T>
PSFD_D void zmul_entries(const T* tb, int kz, int li, int nz, int lb, T t[6]) {
  const bool up = kz > nz;
  const T* q = tb + (up ? 2 * nz - kz : kz) * 6 * lb + li;
#pragma unroll
  for (int k = 0; k < 6; ++k) t[k] = q[k * lb];
  if (up) {
    t[4].x = -t[4].x; t[4].y = -t[4].y;
    t[5].x = -t[5].x; t[5].y = -t[5].y;
  }
}

template <class T>
__global__ void k_iso_zmul(IsoZ a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nz = 1 << a.lnz, lb = a.lb, nsq = 3 * lb, npts = 2 * nz * lb;
  // logical block (ky, kx / lb) in XCD order: the blocks of adjacent kx runs
  // fill the two halves of the same 128-byte lines of W, so they are kept on
  // one L2 (else each XCD fetches the whole line for its half)
  const unsigned nbx = gridDim.x;
  const unsigned lid = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y);
  const long long col = ((long long)(lid / nbx) << a.lnx2) + ((long long)(lid % nbx) << a.llb);
  // this block's table entries: one contiguous run of (nz + 1) 6 lb values,
  // point (kz, li) entry k at (kz * 6 + k) * lb + li for kz <= nz; a point
  // kz > nz takes kz' = 2nz - kz, with xz and yz negated (the table is even in
  // kz, those two entries odd)
  const T* tb = (const T*)a.table + ((long long)lid * (nz + 1) * 6 * lb);
  constexpr int ZPT = Zpt<T>::v;
  T tt[ZPT > 0 ? ZPT : 1][6];
#pragma unroll
  for (int i = 0; i < ZPT; ++i) {
    const int p = tid + i * nthr;
    if (p < npts) zmul_entries(tb, p >> a.llb, p & (lb - 1), nz, lb, tt[i]);
  }
  T* w = (T*)a.w;
  for (int idx = tid; idx < nz * nsq; idx += nthr) {
    const int li = idx & (lb - 1), r = idx >> a.llb;
    const int iz = r / 3, c = r - 3 * iz;
    lds[iz * nsq + c * lb + li] = w[(long long)(c * nz + iz) * a.plane + col + li];
  }
  __syncthreads();
  lds_fft<T, false, true, ZFE, true, false>(lds, a.lnz + 1, nsq, 1, nsq, (const T*)a.tw, tid, nthr);
#pragma unroll
  for (int i = 0; i < ZPT; ++i) {
    const int p = tid + i * nthr;
    if (p < npts) zmul_point(lds + (p >> a.llb) * nsq + (p & (lb - 1)), lb, tt[i]);
  }
  for (int p = tid + ZPT * nthr; p < npts; p += nthr) {
    T t[6];
    zmul_entries(tb, p >> a.llb, p & (lb - 1), nz, lb, t);
    zmul_point(lds + (p >> a.llb) * nsq + (p & (lb - 1)), lb, t);
  }
  __syncthreads();
  lds_fft<T, true, true, ZFE, false, true>(lds, a.lnz + 1, nsq, 1, nsq, (const T*)a.tw, tid, nthr);
  for (int idx = tid; idx < nz * nsq; idx += nthr) {
    const int li = idx & (lb - 1), r = idx >> a.llb;
    const int iz = r / 3, c = r - 3 * iz;
    w[(long long)(c * nz + iz) * a.plane + col + li] = lds[iz * nsq + c * lb + li];
  }
}

// The same pass with the shape fixed at compile time (FFT length 2^LZ2, LB
// columns, NT threads): every global load of a thread is issued before its
// first LDS write, the twiddles are staged in LDS so that no FFT pass waits on
// the vector-memory counter of the table entries in flight, and the FFT index
// arithmetic folds to constants.
template <class T, int LZ2, int LB, int NT>
__global__ void __launch_bounds__(NT) k_iso_zmul_ct(IsoZ a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  constexpr int NZ = 1 << (LZ2 - 1), NSQ = 3 * LB, NPTS = 2 * NZ * LB, LLB = LB == 8 ? 3 : LB == 4 ? 2 : 1;
  constexpr int NV = NZ * NSQ / NT;  // data values per thread
  static_assert(NV * NT == NZ * NSQ && (1 << LLB) == LB, "z pass split");
  T* twl = lds + (2 * NZ) * NSQ;
  const int tid = threadIdx.x;
  const unsigned nbx = gridDim.x;
  const unsigned lid = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y);
  const long long col = ((long long)(lid / nbx) << a.lnx2) + ((long long)(lid % nbx) << LLB);
  const T* tb = (const T*)a.table + ((long long)lid * (NZ + 1) * 6 * LB);
  const T* twg = (const T*)a.tw + 2 * NZ;
  const T tw0 = twg[tid & (2 * NZ - 1)];
  __builtin_amdgcn_sched_barrier(0);
  const T* w = (const T*)a.w;
  T v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int idx = tid + k * NT, li = idx & (LB - 1), r = idx >> LLB;
    const int iz = r / 3, c = r - 3 * iz;
    v[k] = w[(long long)(c * NZ + iz) * a.plane + col + li];
  }
  constexpr int ZPT = Zpt<T>::v;
  T tt[ZPT > 0 ? ZPT : 1][6];
#pragma unroll
  for (int i = 0; i < ZPT; ++i) {
    const int pt = tid + i * NT;
    if (pt < NPTS) zmul_entries(tb, pt >> LLB, pt & (LB - 1), NZ, LB, tt[i]);
  }
  if (tid < 2 * NZ) twl[tid] = tw0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int idx = tid + k * NT, li = idx & (LB - 1), r = idx >> LLB;
    const int iz = r / 3, c = r - 3 * iz;
    lds[iz * NSQ + c * LB + li] = v[k];
  }
  __syncthreads();
  typedef FftCT<LZ2, NSQ, 1, NSQ, NT> D;
  lds_fft_tab<T, false, true, ZFE, D, true, false>(lds, D(), twl, tid);
#pragma unroll
  for (int i = 0; i < ZPT; ++i) {
    const int pt = tid + i * NT;
    if (pt < NPTS) zmul_point(lds + (pt >> LLB) * NSQ + (pt & (LB - 1)), LB, tt[i]);
  }
  for (int pt = tid + ZPT * NT; pt < NPTS; pt += NT) {
    T t[6];
    zmul_entries(tb, pt >> LLB, pt & (LB - 1), NZ, LB, t);
    zmul_point(lds + (pt >> LLB) * NSQ + (pt & (LB - 1)), LB, t);
  }
  __syncthreads();
  lds_fft_tab<T, true, true, ZFE, D, false, true>(lds, D(), twl, tid);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int idx = tid + k * NT, li = idx & (LB - 1), r = idx >> LLB;
    const int iz = r / 3, c = r - 3 * iz;
    v[k] = lds[iz * NSQ + c * LB + li];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int idx = tid + k * NT, li = idx & (LB - 1), r = idx >> LLB;
    const int iz = r / 3, c = r - 3 * iz;
    ((T*)a.w)[(long long)(c * NZ + iz) * a.plane + col + li] = v[k];
  }
}

// ---------------------------------------------------------------------------
// Precompute kernels (FP64).

// constants of F[G_R] (windowed kernel section, eqs. (15)-(17), with h(k; R)
// carrying R^2 and A(0) the factor 4 pi)
struct IsoSample {
  double2* g;             // [6][M0][M1][M2]
  int l0, l1, l2;         // log2 M per axis (z, y, x)
  double dk0, dk1, dk2;   // 2 pi / (M_a h_a)
  double2 kbg, kbg2, inv_kbg2, e, at0, atkb, gp;
  double R;
};

// j1(x) / x; series below 1e-3 (limit 1/3)
PSFD_D double j1x(double x) {
  if (fabs(x) < 1e-3) { const double x2 = x * x; return 1.0 / 3.0 - x2 / 30.0 + x2 * x2 / 840.0; }
  double sn, cs;
  sincos(x, &sn, &cs);
  return (sn / x - cs) / (x * x);
}

__global__ void k_iso_sample(IsoSample a) {
  const long long tot = 1LL << (a.l0 + a.l1 + a.l2);
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int M0 = 1 << a.l0, M1 = 1 << a.l1, M2 = 1 << a.l2;
  const int i2 = (int)(idx & (M2 - 1)), i1 = (int)((idx >> a.l2) & (M1 - 1)), i0 = (int)(idx >> (a.l1 + a.l2));
  double2 out[6];
  for (int c = 0; c < 6; ++c) out[c] = make_double2(0.0, 0.0);
  if (i0 != M0 / 2 && i1 != M1 / 2 && i2 != M2 / 2) {
    const double kz = (i0 < M0 / 2 ? i0 : i0 - M0) * a.dk0;
    const double ky = (i1 < M1 / 2 ? i1 : i1 - M1) * a.dk1;
    const double kx = (i2 < M2 / 2 ? i2 : i2 - M2) * a.dk2;
    const double k = sqrt(kx * kx + ky * ky + kz * kz);
    double2 F;
    if (k == 0.0) {
      F = a.at0;
    } else {
      const double2 den = make_double2(a.kbg2.x - k * k, a.kbg2.y);
      if (sqrt(cabs2(den)) < 1e-10 * sqrt(cabs2(a.kbg2))) {
        F = a.atkb;
      } else {
        double sn, cs;
        sincos(k * a.R, &sn, &cs);
        // e (cos kR - i (k_bg / k) sin kR) - 1
        const double2 t = make_double2(cs + a.kbg.y / k * sn, -a.kbg.x / k * sn);
        F = cdiv(csub(cmul(a.e, t), make_double2(1.0, 0.0)), den);
      }
    }
    const double2 h = cmul(cscale(a.gp, j1x(k * a.R)), a.inv_kbg2);
    const double2 A = cadd(F, h);
    double2 B = make_double2(0.0, 0.0);
    double u[3] = {0.0, 0.0, 0.0};
    if (k != 0.0) {
      B = csub(csub(make_double2(-F.x, -F.y), cscale(h, 3.0)), a.inv_kbg2);
      u[0] = kx / k; u[1] = ky / k; u[2] = kz / k;
    }
    out[0] = cadd(A, cscale(B, u[0] * u[0]));
    out[1] = cadd(A, cscale(B, u[1] * u[1]));
    out[2] = cadd(A, cscale(B, u[2] * u[2]));
    out[3] = cscale(B, u[0] * u[1]);
    out[4] = cscale(B, u[0] * u[2]);
    out[5] = cscale(B, u[1] * u[2]);
  }
  for (int c = 0; c < 6; ++c) a.g[c * tot + idx] = out[c];
}

// offsets [-n, n) of the oversampled inverse DFT, in FFT order on the 2n grid,
// times `scale`: index j < n comes from j, j >= n from j + M - 2n
__global__ void k_iso_restrict(const double2* __restrict__ g, double2* __restrict__ t, int lz, int ly, int lx, int l0,
                               int l1, int l2, double scale) {
  const long long per = 8LL << (lz + ly + lx);
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 6 * per) return;
  const int c = (int)(idx / per);
  const long long r = idx - c * per;
  const int j2 = (int)(r & ((2 << lx) - 1)), j1 = (int)((r >> (lx + 1)) & ((2 << ly) - 1)),
            j0 = (int)(r >> (lx + ly + 2));
  const int s0 = j0 < (1 << lz) ? j0 : j0 + (1 << l0) - (2 << lz);
  const int s1 = j1 < (1 << ly) ? j1 : j1 + (1 << l1) - (2 << ly);
  const int s2 = j2 < (1 << lx) ? j2 : j2 + (1 << l2) - (2 << lx);
  const long long src = (((long long)c << (l0 + l1 + l2)) + ((long long)s0 << (l1 + l2)) + ((long long)s1 << l2) + s2);
  t[idx] = cscale(g[src], scale);
}

// the table in the z-pencil order of the apply: for block (ky, kb) of lb
// adjacent kx, [nz + 1][6][lb] (kz = 0 .. nz), from the natural [6][2nz][2ny][2nx]
template <class T>
__global__ void k_iso_pencil_table(const double2* __restrict__ nat, T* __restrict__ out, int lz, int ly, int lx,
                                   int llb) {
  const long long n8 = 8LL << (lz + ly + lx);
  const int nz1 = (1 << lz) + 1;
  const long long tot = 6LL * nz1 * (4LL << (ly + lx));
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int lb = 1 << llb;
  const int li = (int)(idx & (lb - 1));
  const long long r = idx >> llb;
  const int k = (int)(r % 6);
  const long long r2 = r / 6;
  const int kz = (int)(r2 % nz1);
  const long long blk = r2 / nz1;                 // ky * (2nx / lb) + kb
  const int nkb = (2 << lx) >> llb;
  const long long ky = blk / nkb, kb = blk - ky * nkb;
  const long long src = k * n8 + (((long long)kz << (ly + 1)) + ky) * (2LL << lx) + (kb << llb) + li;
  out[idx] = from_d<T>(nat[src]);
}

// zero the offset plane jz = -nz (index nz on the 2n grid) of the samples
// [6][2nz][2ny][2nx]: it couples no two voxels of the box, and without it the
// samples are even (xx, yy, zz, xy) or odd (xz, yz) in jz
__global__ void k_iso_zero_zplane(double2* __restrict__ k, int lz, int ly, int lx) {
  const long long pl = 4LL << (ly + lx);
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 6 * pl) return;
  const long long c = idx / pl, e = idx - c * pl;
  k[c * (8LL << (lz + ly + lx)) + ((long long)1 << lz) * pl + e] = make_double2(0.0, 0.0);
}

constexpr int KB = 256;      // threads per block of the elementwise kernels

// out = s a, converted to out's type (a may equal out)
template <class TA, class TO>
__global__ void k_iso_scale(const TA* a, double s, TO* out, long long n) {
  const long long e = (long long)blockIdx.x * KB + threadIdx.x;
  if (e < n) out[e] = from_d<TO>(cscale(to_d(a[e]), s));
}

int ilog2_exact(long long v) {
  int r = 0;
  while ((1LL << r) < v) ++r;
  return (1LL << r) == v ? r : -1;
}

}  // namespace

// ---------------------------------------------------------------------------
struct psfd_iso_plan {
  psfd_iso_problem p{};
  int n[3] = {0, 0, 0};    // z, y, x
  int ln[3] = {0, 0, 0};
  int over[3] = {0, 0, 0};
  double R = 0.0, k0 = 0.0;
  int device = 0;
  double2* tab64 = nullptr;  // [6][2nz][2ny][2nx]
  double2* ptab64 = nullptr; // tab64 in the z-pencil order of the FP64 apply
  float2* ptab32 = nullptr;  // FP32 rounding, in the z-pencil order of the FP32 apply
  double2* tw64 = nullptr;   // tw[m + i] = exp(-2 pi i i / m), m = 2 .. ISO_TW_MAX
  float2* tw32 = nullptr;
  void* work[2] = {nullptr, nullptr};  // W [3][nz][2ny][2nx] per dtype (C64, C128)
  ~psfd_iso_plan() {
    for (void* q : {(void*)tab64, (void*)ptab64, (void*)ptab32, (void*)tw64, (void*)tw32, work[0], work[1]})
      if (q) (void)hipFree(q);
  }
};

namespace psfd {

namespace {

#define ISOCHK(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_status(e_, #call); \
  } while (0)

Status bad(int code, const char* m) { Status s; s.code = code; s.msg = m; return s; }

// lines per block and threads of a line pass of FFT length 2^ln over nlines lines
void line_shape(int ln, long long nlines, int e, int& lb, int& nthr) {
  lb = std::max(1, std::min(16, 4096 >> ln));
  while (nlines % lb) lb >>= 1;
  const int els = lb << ln;
  nthr = std::min(1024, std::max(64, (els / e + 63) / 64 * 64));
}

template <class T, bool INV, int MODE, bool SFL, bool ZIN, bool ZOUT>
Status run_lines(IsoLines a, hipStream_t s) {
  int lb, nthr;
  line_shape(a.ln, a.nlines, LFE, lb, nthr);
  a.lb = lb;
  a.llb = ilog2_exact(lb);
  if (MODE == LN_VLOAD && (a.nlines / lb) % 3) return bad(PSFD_ERR_UNSUPPORTED_SIZE, "row pass needs three component blocks per group");
  const size_t bytes = ((size_t)lb << a.ln) * sizeof(T);
  auto fn = k_iso_lines<T, INV, MODE, SFL, ZIN, ZOUT>;
  if (bytes > 65536) ISOCHK(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  hipLaunchKernelGGL(fn, dim3((unsigned)(a.nlines / lb)), dim3(nthr), bytes, s, a);
  return Status();
}

// in-place unnormalised 3-D FFT of C components [C][2^l0][2^l1][2^l2], FP64
template <bool INV>
Status fft3_c(double2* d, int C, int l0, int l1, int l2, const double2* tw, hipStream_t s) {
  const long long M2 = 1LL << l2, M12 = 1LL << (l1 + l2), M = 1LL << (l0 + l1 + l2);
  IsoLines a{};
  a.src = d; a.dst = d; a.tw = tw; a.scale = 1.0;
  // axis x: contiguous lines
  a.nlines = (long long)C << (l0 + l1); a.ln = a.lload = a.lstore = l2; a.es = 1;
  a.lcin_s = a.lcin_d = 0; a.sin_s = a.sin_d = 0; a.sout_s = a.sout_d = M2;
  Status st = run_lines<double2, INV, LN_PLAIN, false, false, false>(a, s);
  if (!st.ok()) return st;
  // axis y: lines (c, i0, i2), inner index i2
  a.nlines = (long long)C << (l0 + l2); a.ln = a.lload = a.lstore = l1; a.es = M2;
  a.lcin_s = a.lcin_d = l2; a.sin_s = a.sin_d = 1; a.sout_s = a.sout_d = M12;
  st = run_lines<double2, INV, LN_PLAIN, true, false, false>(a, s);
  if (!st.ok()) return st;
  // axis z: lines (c, i1, i2), inner index i1 M2 + i2
  a.nlines = (long long)C << (l1 + l2); a.ln = a.lload = a.lstore = l0; a.es = M12;
  a.lcin_s = a.lcin_d = l1 + l2; a.sin_s = a.sin_d = 1; a.sout_s = a.sout_d = M;
  return run_lines<double2, INV, LN_PLAIN, true, false, false>(a, s);
}

template <class T> T* tw_of(psfd_iso_plan* p);
template <> double2* tw_of<double2>(psfd_iso_plan* p) { return p->tw64; }
template <> float2* tw_of<float2>(psfd_iso_plan* p) { return p->tw32; }
template <class T> const T* tab_of(psfd_iso_plan* p);
template <> const double2* tab_of<double2>(psfd_iso_plan* p) { return p->ptab64; }
template <> const float2* tab_of<float2>(psfd_iso_plan* p) { return p->ptab32; }

// adjacent kx per z-pencil block: at most the cap below, the three padded z
// sequences of all of them within 64 KB of LDS and at most ZFE values per
// thread of 1024
static int env_int_iso(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

template <class T> int z_lb(int nz, int nx) {
  // measured at 128 x 128 x 64 (widths 16, 8, 4): 8 in FP32, 4 in FP64 (more
  // blocks per CU to cover the FFT barriers); PSFD_ISO_ZLB overrides (sweeps)
  static const int cap = [] {
    const char* e = std::getenv("PSFD_ISO_ZLB");
    const int dflt = sizeof(T) == 8 ? 8 : 4;
    const int v = e ? std::atoi(e) : dflt;
    return v >= 1 && v <= 16 && (v & (v - 1)) == 0 ? v : dflt;
  }();
  int lb = std::min(cap, 2 * nx);
  while (lb > 1 && ((long long)2 * nz * 3 * lb * (long long)sizeof(T) > 65536 || 2 * nz * 3 * lb > ZFE * 1024))
    lb >>= 1;
  return lb;
}

// stage -1: the whole apply; 0 .. 4: X_FWD, Y_FWD, Z_MUL, Y_INV, X_INV
template <class T>
Status apply_t(psfd_iso_plan* p, const T* deps, const T* x, T* y, T* W, int stage, hipStream_t s) {
  const int lz = p->ln[0], ly = p->ln[1], lx = p->ln[2];
  const long long nx = 1LL << lx, ny = 1LL << ly, nz = 1LL << lz;
  const long long plane = 4 * nx * ny, nrow = 3 * nz * ny;
  const T* tw = tw_of<T>(p);
  Status st;
  IsoLines a{};
  a.tw = tw;
  a.scale = 1.0;
  if (stage < 0 || stage == 0) {  // rows of x times V -> W rows y < ny, all 2nx
    IsoLines b = a;
    b.src = x; b.dst = W; b.deps = deps; b.vscale = p->k0 * p->k0;
    b.nlines = nrow; b.ln = lx + 1; b.lload = lx; b.lstore = lx + 1; b.es = 1;
    b.lcin_s = 0; b.sin_s = 0; b.sout_s = nx;
    b.lcin_d = ly; b.sin_d = 2 * nx; b.sout_d = plane;
    b.lvmod = lz + ly;
    st = run_lines<T, false, LN_VLOAD, false, true, false>(b, s);
    if (!st.ok()) return st;
  }
  if (stage < 0 || stage == 1) {  // columns y < ny -> 2ny
    IsoLines b = a;
    b.src = W; b.dst = W;
    b.nlines = 3 * nz * 2 * nx; b.ln = ly + 1; b.lload = ly; b.lstore = ly + 1; b.es = 2 * nx;
    b.lcin_s = b.lcin_d = lx + 1; b.sin_s = b.sin_d = 1; b.sout_s = b.sout_d = plane;
    st = run_lines<T, false, LN_PLAIN, true, true, false>(b, s);
    if (!st.ok()) return st;
  }
  if (stage < 0 || stage == 2) {
    IsoZ z{};
    z.w = W; z.table = tab_of<T>(p); z.lnz = lz; z.lnx2 = lx + 1;
    z.lb = z_lb<T>((int)nz, (int)nx);
    z.llb = ilog2_exact(z.lb);
    z.plane = plane; z.n8 = 8 * nx * ny * nz; z.tw = tw;
    const int els = (int)(2 * nz) * 3 * z.lb;
    const int npts = (int)(2 * nz) * z.lb;
    const int pre = Zpt<T>::v ? (npts / std::max(1, Zpt<T>::v) + 63) / 64 * 64 : 64;
    const int nthr = std::min(1024, std::max({64, (els / ZFE + 63) / 64 * 64, pre}));
    if (els > ZFE * nthr) return bad(PSFD_ERR_UNSUPPORTED_SIZE, "z pencil tile exceeds the FFT budget");
    const size_t bytes = (size_t)els * sizeof(T);
    const dim3 grid((unsigned)(2 * nx / z.lb), (unsigned)(2 * ny));
    // compile-time shapes for the 64-plane grids at the measured block widths
    constexpr int LBC = sizeof(T) == 8 ? 8 : 4, NTC = sizeof(T) == 8 ? 512 : 192;
    if (lz == 6 && z.lb == LBC && nthr == NTC && env_int_iso("PSFD_ISO_ZCT", 1)) {
      auto fc = k_iso_zmul_ct<T, 7, LBC, NTC>;
      const size_t bc = bytes + (size_t)128 * sizeof(T);
      if (bc > 65536) ISOCHK(hipFuncSetAttribute((const void*)fc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bc));
      hipLaunchKernelGGL(fc, grid, dim3(NTC), bc, s, z);
    } else {
      auto fn = k_iso_zmul<T>;
      if (bytes > 65536) ISOCHK(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
      hipLaunchKernelGGL(fn, grid, dim3(nthr), bytes, s, z);
    }
  }
  if (stage < 0 || stage == 3) {  // columns 2ny -> first ny
    IsoLines b = a;
    b.src = W; b.dst = W;
    b.nlines = 3 * nz * 2 * nx; b.ln = ly + 1; b.lload = ly + 1; b.lstore = ly; b.es = 2 * nx;
    b.lcin_s = b.lcin_d = lx + 1; b.sin_s = b.sin_d = 1; b.sout_s = b.sout_d = plane;
    st = run_lines<T, true, LN_PLAIN, true, false, true>(b, s);
    if (!st.ok()) return st;
  }
  if (stage < 0 || stage == 4) {  // rows 2nx -> first nx, y = x - w / (8 n)
    IsoLines b = a;
    b.src = W; b.dst = y; b.xin = x;
    b.nlines = nrow; b.ln = lx + 1; b.lload = lx + 1; b.lstore = lx; b.es = 1;
    b.lcin_s = ly; b.sin_s = 2 * nx; b.sout_s = plane;
    b.lcin_d = 0; b.sin_d = 0; b.sout_d = nx;
    b.scale = 1.0 / (8.0 * (double)(nx * ny * nz));
    st = run_lines<T, true, LN_AXPY, false, false, true>(b, s);
    if (!st.ok()) return st;
  }
  ISOCHK(hipGetLastError());
  return Status();
}

}  // namespace

Status iso_create(const psfd_iso_problem& pr, psfd_iso_plan*& out) {
  out = nullptr;
  const int nn[3] = {pr.nz, pr.ny, pr.nx};
  const double hh[3] = {pr.dz_nm, pr.dy_nm, pr.dx_nm};
  for (int a = 0; a < 3; ++a) {
    if (nn[a] < 2 || nn[a] > 128 || ilog2_exact(nn[a]) < 0)
      return bad(PSFD_ERR_UNSUPPORTED_SIZE, "nx, ny, nz must be powers of two in [2, 128]");
    if (!(hh[a] > 0.0) || !std::isfinite(hh[a])) return bad(PSFD_ERR_INVALID_ARG, "voxel sizes must be positive");
  }
  if (!(pr.wavelength_nm > 0.0)) return bad(PSFD_ERR_INVALID_ARG, "wavelength must be positive");
  if (!(pr.eps_bg_re > 0.0) || !(pr.eps_bg_im >= 0.0))
    return bad(PSFD_ERR_INVALID_ARG, "eps_bg needs Re > 0 and Im >= 0");
  std::unique_ptr<psfd_iso_plan> p(new psfd_iso_plan());
  p->p = pr;
  double L2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    p->n[a] = nn[a];
    p->ln[a] = ilog2_exact(nn[a]);
    L2 += (nn[a] * hh[a]) * (nn[a] * hh[a]);
  }
  p->R = pr.radius_nm > 0.0 ? pr.radius_nm : std::sqrt(L2);
  if (!std::isfinite(p->R)) return bad(PSFD_ERR_INVALID_ARG, "radius must be finite");
  int lo[3];
  for (int a = 0; a < 3; ++a) {
    int f = 4;
    while (f < 1.0 + p->R / (nn[a] * hh[a]) && f * nn[a] <= ISO_TW_MAX) f *= 2;
    if (f * nn[a] > ISO_TW_MAX) return bad(PSFD_ERR_UNSUPPORTED_SIZE, "window radius needs a precompute grid beyond 1024 per axis");
    p->over[a] = f;
    lo[a] = ilog2_exact((long long)f * nn[a]);
  }
  ISOCHK(hipGetDevice(&p->device));
  // twiddles of every length up to ISO_TW_MAX, in FP64 (FP32 rounded from them)
  std::vector<double2> tw(2 * ISO_TW_MAX);
  std::vector<float2> tw32(2 * ISO_TW_MAX);
  for (int m = 2; m <= ISO_TW_MAX; m <<= 1)
    for (int i = 0; i < m; ++i) {
      const double ang = 2.0 * M_PI * i / m;
      tw[m + i] = make_double2(std::cos(ang), -std::sin(ang));
    }
  for (size_t i = 0; i < tw.size(); ++i) tw32[i] = to_f(tw[i]);
  ISOCHK(hipMalloc((void**)&p->tw64, tw.size() * sizeof(double2)));
  ISOCHK(hipMalloc((void**)&p->tw32, tw32.size() * sizeof(float2)));
  ISOCHK(hipMemcpy(p->tw64, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
  ISOCHK(hipMemcpy(p->tw32, tw32.data(), tw32.size() * sizeof(float2), hipMemcpyHostToDevice));
  // kernel constants
  typedef std::complex<double> cd;
  const double k0 = 2.0 * M_PI / pr.wavelength_nm;
  p->k0 = k0;
  const cd kbg = k0 * std::sqrt(cd(pr.eps_bg_re, pr.eps_bg_im));
  const double R = p->R;
  const cd I1(0.0, 1.0);
  const cd e = std::exp(I1 * kbg * R);
  const cd kbg2 = kbg * kbg;
  const cd at0 = (e * (1.0 - I1 * R * kbg) - 1.0) / kbg2;
  const cd atkb = I1 * R / (2.0 * kbg) - I1 / (2.0 * kbg2) * e * std::sin(kbg * R);
  const cd gp = e * (I1 * kbg * R - 1.0);
  auto d2 = [](cd v) { return make_double2(v.real(), v.imag()); };
  const long long Mtot = 1LL << (lo[0] + lo[1] + lo[2]);
  const long long n8 = 8LL * nn[0] * nn[1] * nn[2];
  double2* g = nullptr;
  ISOCHK(hipMalloc((void**)&g, 6 * Mtot * sizeof(double2)));
  struct Free { double2* q; ~Free() { if (q) (void)hipFree(q); } } fg{g};
  ISOCHK(hipMalloc((void**)&p->tab64, 6 * n8 * sizeof(double2)));
  const long long nhalf = 6LL * (nn[0] + 1) * 4 * nn[1] * nn[2];  // pencil tables: kz = 0 .. nz
  ISOCHK(hipMalloc((void**)&p->ptab64, nhalf * sizeof(double2)));
  ISOCHK(hipMalloc((void**)&p->ptab32, nhalf * sizeof(float2)));
  double2* kev = nullptr;
  ISOCHK(hipMalloc((void**)&kev, 6 * n8 * sizeof(double2)));
  struct Free2 { double2* q; ~Free2() { if (q) (void)hipFree(q); } } fk{kev};
  IsoSample smp{};
  smp.g = g; smp.l0 = lo[0]; smp.l1 = lo[1]; smp.l2 = lo[2];
  smp.dk0 = 2.0 * M_PI / ((double)(1 << lo[0]) * hh[0]);
  smp.dk1 = 2.0 * M_PI / ((double)(1 << lo[1]) * hh[1]);
  smp.dk2 = 2.0 * M_PI / ((double)(1 << lo[2]) * hh[2]);
  smp.kbg = d2(kbg); smp.kbg2 = d2(kbg2); smp.inv_kbg2 = d2(1.0 / kbg2); smp.e = d2(e);
  smp.at0 = d2(at0); smp.atkb = d2(atkb); smp.gp = d2(gp); smp.R = R;
  hipStream_t s = 0;
  hipLaunchKernelGGL(k_iso_sample, dim3((unsigned)((Mtot + 255) / 256)), dim3(256), 0, s, smp);
  ISOCHK(hipGetLastError());
  Status st = fft3_c<true>(g, 6, lo[0], lo[1], lo[2], p->tw64, s);
  if (!st.ok()) return st;
  hipLaunchKernelGGL(k_iso_restrict, dim3((unsigned)((6 * n8 + 255) / 256)), dim3(256), 0, s, g, p->tab64,
                     p->ln[0], p->ln[1], p->ln[2], lo[0], lo[1], lo[2], 1.0 / (double)Mtot);
  ISOCHK(hipGetLastError());
  // the samples with the offset plane jz = -nz zeroed: the same operator, a
  // table even / odd in kz (the apply reads kz <= nz only)
  ISOCHK(hipMemcpyAsync(kev, p->tab64, 6 * n8 * sizeof(double2), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_iso_zero_zplane, dim3((unsigned)((6 * n8 / (2 * nn[0]) + 255) / 256)), dim3(256), 0, s, kev,
                     p->ln[0], p->ln[1], p->ln[2]);
  ISOCHK(hipGetLastError());
  st = fft3_c<false>(kev, 6, p->ln[0] + 1, p->ln[1] + 1, p->ln[2] + 1, p->tw64, s);
  if (!st.ok()) return st;
  st = fft3_c<false>(p->tab64, 6, p->ln[0] + 1, p->ln[1] + 1, p->ln[2] + 1, p->tw64, s);
  if (!st.ok()) return st;
  hipLaunchKernelGGL(k_iso_pencil_table<double2>, dim3((unsigned)((nhalf + 255) / 256)), dim3(256), 0, s, kev,
                     p->ptab64, p->ln[0], p->ln[1], p->ln[2], ilog2_exact(z_lb<double2>(nn[0], nn[2])));
  hipLaunchKernelGGL(k_iso_pencil_table<float2>, dim3((unsigned)((nhalf + 255) / 256)), dim3(256), 0, s, kev,
                     p->ptab32, p->ln[0], p->ln[1], p->ln[2], ilog2_exact(z_lb<float2>(nn[0], nn[2])));
  ISOCHK(hipGetLastError());
  ISOCHK(hipStreamSynchronize(s));
  out = p.release();
  return Status();
}

void iso_destroy(psfd_iso_plan* p) { delete p; }

static Status iso_work(psfd_iso_plan* p, int dtype, void*& W) {
  const int i = dtype == PSFD_C64 ? 0 : 1;
  if (!p->work[i]) {
    const size_t esz = dtype == PSFD_C64 ? sizeof(float2) : sizeof(double2);
    ISOCHK(hipMalloc(&p->work[i], 12ULL * p->n[0] * p->n[1] * p->n[2] * esz));
  }
  W = p->work[i];
  return Status();
}

Status iso_apply(psfd_iso_plan* p, const void* deps, const void* x, void* y, int dtype, int stage, hipStream_t s) {
  if (dtype != PSFD_C64 && dtype != PSFD_C128) return bad(PSFD_ERR_INVALID_ARG, "dtype must be PSFD_C64 or PSFD_C128");
  if (stage < -1 || stage > 4) return bad(PSFD_ERR_INVALID_ARG, "stage must be -1 .. 4");
  int dev = 0;
  ISOCHK(hipGetDevice(&dev));
  if (dev != p->device) return bad(PSFD_ERR_INVALID_ARG, "plan belongs to another device");
  void* W = nullptr;
  Status st = iso_work(p, dtype, W);
  if (!st.ok()) return st;
  if (dtype == PSFD_C64)
    return apply_t<float2>(p, (const float2*)deps, (const float2*)x, (float2*)y, (float2*)W, stage, s);
  return apply_t<double2>(p, (const double2*)deps, (const double2*)x, (double2*)y, (double2*)W, stage, s);
}

Status iso_table(psfd_iso_plan* p, void* d_table, int32_t* over, double* radius, hipStream_t s) {
  if (d_table)
    ISOCHK(hipMemcpyAsync(d_table, p->tab64, 48ULL * p->n[0] * p->n[1] * p->n[2] * sizeof(double2),
                          hipMemcpyDeviceToDevice, s));
  if (over)
    for (int a = 0; a < 3; ++a) over[a] = p->over[a];
  if (radius) *radius = p->R;
  return Status();
}


// GMRES(m) on y = x - K(V x) from x0 = 0 (the host-driven solver of
// gmres_host.hip): in mixed precision the basis and the applies are FP32 (an
// FP32 copy of the contrast is made for the call) and every restart starts
// from the FP64 residual. PSFD_ISO_CANCEL overrides the norm ratio below which
// Gram-Schmidt takes a second pass (1/sqrt(2)), so that a test can force it.
Status iso_solve(psfd_iso_plan* p, const void* deps, const void* b, void* u, double rtol, int m, int max_iters,
                 int precision, psfd_info* info, hipStream_t s) {
  if (!(rtol > 0.0) || m < 1 || m > 64 || max_iters < 1)
    return bad(PSFD_ERR_INVALID_ARG, "need rtol > 0, 1 <= restart <= 64, max_iters >= 1");
  if (precision != PSFD_FP64 && precision != PSFD_MIXED)
    return bad(PSFD_ERR_INVALID_ARG, "precision must be PSFD_FP64 or PSFD_MIXED");
  int dev = 0;
  ISOCHK(hipGetDevice(&dev));
  if (dev != p->device) return bad(PSFD_ERR_INVALID_ARG, "plan belongs to another device");
  const long long N = (long long)p->n[0] * p->n[1] * p->n[2];
  float2* depsT = nullptr;
  struct Free {
    void* q;
    ~Free() { if (q) (void)hipFree(q); }
  } fr{nullptr};
  if (precision == PSFD_MIXED) {
    ISOCHK(hipMalloc((void**)&depsT, (size_t)N * sizeof(float2)));
    fr.q = depsT;
    hipLaunchKernelGGL((k_iso_scale<double2, float2>), dim3((unsigned)((N + KB - 1) / KB)), dim3(KB), 0, s,
                       (const double2*)deps, 1.0, depsT, N);
    ISOCHK(hipGetLastError());
  }
  ApplyFn A = [&](const void* x, void* y, int dt, hipStream_t q) {
    return iso_apply(p, dt == PSFD_C64 ? (const void*)depsT : deps, x, y, dt, -1, q);
  };
  HostGmres o;
  o.rtol = rtol;
  o.m = m;
  o.max_iters = max_iters;
  o.precision = precision;
  if (const char* e = std::getenv("PSFD_ISO_CANCEL")) o.cancel = std::atof(e);
  psfd_info inf{};
  inf.outer_iters = 1;
  Status st = gmres_host(3 * N, A, (const double2*)b, (double2*)u, o, inf, s);
  if (info) *info = inf;
  return st;
}

}  // namespace psfd
