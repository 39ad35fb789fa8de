// Operator-apply kernels of the discrete Lippmann-Schwinger system (eq. (18)):
//   transverse FFT tiles  (contrast multiply V x fused into the forward load,
//                          axpy y = alpha x + gamma w fused into the inverse store),
//   z-pencil kernel       (zero-padded z-FFT, dyadic windowed Green's function
//                          F[G_L](k) evaluated on the fly, inverse z-FFT),
// plus the per-order background-field kernels of the outer loop (eqs. (8)-(9)):
// plane-wave readouts of the mask field, reflection by T_R, order amplitudes.
#include <cstdio>
#include <cstdlib>

#include "kernels.hpp"
#include "fft_lds.hpp"
#include "givens.hpp"

namespace psfd {

PSFD_D double2 cexp_i(double2 z) {  // exp(i z)
  double e = exp(-z.y);
  double sn, cs;
  sincos(z.x, &sn, &cs);
  return make_double2(e * cs, e * sn);
}

// -------------------------------------------------------------------------
// Transverse FFT tile kernel
// -------------------------------------------------------------------------
template <class T, bool INV, int LD, int ST>
__global__ void __launch_bounds__(1024) k_tile(TileArgs a) {
  extern __shared__ double2 smem_d[];
  T* lds = reinterpret_cast<T*>(smem_d);
  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;
  const int tiles = a.tiles_x * a.tiles_y;
  const int plane = blockIdx.x / tiles;
  const int tile = blockIdx.x - plane * tiles;
  const int z = plane % a.nz;
  const int c = plane / a.nz;
  const int tx = a.tx, ty = a.ty, nxa = a.nx, pitch = a.pitch;
  const int nthr = blockDim.x;
  const int ltx = ilog2i(a.tx);
  const int x0 = (tile % a.tiles_x) * tx;
  const int y0 = (tile / a.tiles_x) * ty;
  const long long nxny = (long long)a.nx * a.ny;
  const long long poff = (long long)plane * nxny;
  const int tid = threadIdx.x;
  const int ntile = tx * ty;
  const T* in = vref<T>(a.in, b) + poff;
  const T* aux = (LD == LD_VXE || ST == ST_AXPBY) ? vref<T>(a.aux, b) + poff : nullptr;
  const T* vol = (LD == LD_VX || LD == LD_VXE) ? vref<T>(a.vol, b) + (long long)z * nxny : nullptr;
  const double* tab = a.tab + (long long)b * a.tab_stride;
  typedef typename real_of<T>::type R;
  const R k0sq = (R)tab[TS_K0SQ];
  // A thread handles elements tid + k nthr, k < KT (the launch keeps tx ty <= KT nthr).
  // Global loads are issued in groups of KG before their LDS writes (the loop
  // would otherwise wait on every load), within the register budget of the FFT.
  constexpr int KT = FftBudget<T>::E;
  constexpr int KG = 8;
  // in-plane offset of element i (32-bit: a plane holds at most 2^16 elements)
  auto off_of = [&](int i) -> int { return (y0 + (i >> ltx)) * nxa + (x0 + (i & (tx - 1))); };
  // scale of the input on load (the newest Arnoldi vector is kept unnormalised),
  // folded into the contrast factor
  const R ks = k0sq * ((LD == LD_VX && a.in_scale) ? (R)a.in_scale[(long long)b * a.scale_stride] : (R)1);
  if (LD == LD_PLAIN || LD == LD_VX) {
#pragma unroll 1
    for (int g = 0; g < KT; g += KG) {
      T va[KG], vb[KG];
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        // unconditional loads (clamped index): a load under a branch would be waited
        // for before the next one is issued
        const int i = min(tid + (g + k) * nthr, ntile - 1);
        const int o = off_of(i);
        va[k] = in[o];
        if (LD == LD_VX) vb[k] = vol[o];
      }
#pragma unroll
      for (int k = 0; k < KG; ++k) {
        const int i = tid + (g + k) * nthr;
        if (i < ntile) {
          const T x = va[k];
          const T v = LD == LD_VX ? cscale(cmul(vb[k], x), ks) : x;
          lds[(i >> ltx) * pitch + (i & (tx - 1))] = v;
        }
      }
    }
  }
  for (int i = tid; i < ntile && LD != LD_PLAIN && LD != LD_VX; i += nthr) {
    int yy = i >> ltx, xx = i & (tx - 1);
    long long o = (long long)(y0 + yy) * a.nx + (x0 + xx);
    T v;
    if (LD == LD_PLAIN) {
      v = in[o];
    } else if (LD == LD_VX) {
      v = cscale(cmul(vol[o], in[o]), k0sq);
    } else if (LD == LD_VXE) {
      v = cscale(cmul(vol[o], cadd(in[o], aux[o])), k0sq);
    } else if (LD == LD_INJECT_T) {
      // transposed plane-wave readouts: position o carries order q = -o with
      // b_dn,q exp(i beta_q z) + b_up,q exp(i beta_q (T - z))
      TabLayout L{a.nx, a.ny};
      const int io = (int)(o % a.nx), jo = (int)(o / a.nx);
      const long long q = (long long)((a.ny - jo) & (a.ny - 1)) * a.nx + ((a.nx - io) & (a.nx - 1));
      const double zk = (z + 0.5) * tab[TS_DZ], Tt = tab[TS_T];
      const double2 bq = reinterpret_cast<const double2*>(tab + L.off_beta())[q];
      const double2* bdn = a.eup + (long long)b * a.eup_stride;
      const double2* bup = a.eup2 + (long long)b * a.eup_stride;
      double2 val = cadd(cmul(bdn[q * 3 + c], cexp_i(make_double2(bq.x * zk, bq.y * zk))),
                         cmul(bup[q * 3 + c], cexp_i(make_double2(bq.x * (Tt - zk), bq.y * (Tt - zk)))));
      v = from_d<T>(val);
    } else {
      // spectrum of the layered field on plane z: E_up,q exp(i beta_q z)
      // plus the incident wave in its order, E_inc exp(-i beta_inc z)
      TabLayout L{a.nx, a.ny};
      const double zk = (z + 0.5) * tab[TS_DZ];
      const double2* beta = reinterpret_cast<const double2*>(tab + L.off_beta());
      const double2* eup = a.eup + (long long)b * a.eup_stride;
      double2 bq = beta[o];
      double2 ph = cexp_i(make_double2(bq.x * zk, bq.y * zk));
      double2 val = cmul(eup[o * 3 + c], ph);
      if (o == (long long)tab[TS_INCQ]) {
        double2 bi = make_double2(tab[TS_BINC], tab[TS_BINC + 1]);
        double2 pi = cexp_i(make_double2(-bi.x * zk, -bi.y * zk));
        double2 ei = make_double2(tab[TS_EINC + 2 * c], tab[TS_EINC + 2 * c + 1]);
        val = cadd(val, cmul(ei, pi));
      }
      v = from_d<T>(val);
    }
    lds[yy * pitch + xx] = v;
  }
  __syncthreads();
  const T* tw = reinterpret_cast<const T*>(a.tw);
  // sequence-fastest butterflies (consecutive lanes take consecutive rows or
  // columns at the same butterfly)
  if (!INV) {
    if (a.do_x) lds_fft<T, false, true>(lds, a.log2nx, ty, pitch, 1, tw, tid, nthr);
    if (a.do_y) lds_fft<T, false, true>(lds, a.log2ny, tx, 1, pitch, tw, tid, nthr);
  } else {
    if (a.do_y) lds_fft<T, true, true>(lds, a.log2ny, tx, 1, pitch, tw, tid, nthr);
    if (a.do_x) lds_fft<T, true, true>(lds, a.log2nx, ty, pitch, 1, tw, tid, nthr);
  }
  T* out = vref<T>(a.out, b) + poff;
  const R al = (R)a.alpha, ga = (R)a.gamma;
#pragma unroll 1
  for (int g = 0; g < KT; g += KG) {
    T xa[KG];
    if (ST == ST_AXPBY) {
#pragma unroll
      for (int k = 0; k < KG; ++k) xa[k] = aux[off_of(min(tid + (g + k) * nthr, ntile - 1))];
    }
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const int i = tid + (g + k) * nthr;
      if (i < ntile) {
        T v = lds[(i >> ltx) * pitch + (i & (tx - 1))];
        if (ST == ST_AXPBY) {
          v.x = al * xa[k].x + ga * v.x;
          v.y = al * xa[k].y + ga * v.y;
        }
        out[off_of(i)] = v;
      }
    }
  }
}

// dynamic LDS above the default limit needs the per-kernel opt-in
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// -------------------------------------------------------------------------
// Square-plane kernel: one N x N plane (N = 2^LN) per block with the shapes
// fixed at compile time, for the contrast-multiply + forward and the inverse +
// axpy stages of the fused transverse FFT. Every global load of a thread,
// including the axpy operand of the store, is issued at the start. The
// twiddles sit in LDS so that their reads never wait on the vector-memory
// counter of those loads. Rows are transformed first in both directions (the
// 2-D transform is separable).
// -------------------------------------------------------------------------
__host__ __device__ constexpr int plane_threads(int ln) { return (1 << (2 * ln)) / 8 < 1024 ? (1 << (2 * ln)) / 8 : 1024; }
__host__ __device__ constexpr size_t plane_lds(int ln, size_t esz) {
  return ((size_t)(1 << ln) * ((1 << ln) + 1) + (1 << ln)) * esz;
}

// The Gram-Schmidt update of column j - 1 over one plane of slot j, in place:
// wv (the plane's KT values per thread of slot j, element tid + k NT at poff)
// becomes w - sum_{i<j} h_i s_i slot_i and is stored back to slot j (vb then
// receives the plane's contrast values from vol), and the
// plane's ||slot_j||^2 goes to part[b * planes + plane]. h_i = s_i <slot_i, w>
// from the projection partials, each summed as the update kernel sums it (lane
// l takes partials l, l + 64, ... in order, then the wavefront sum), so every
// block gets the same coefficients bit for bit; the block of plane 0 stores h
// and ||w||^2 before the update for the Givens step.
template <class T, int KT, int NT>
PSFD_D void plane_update(const TileArgs& a, int cnt, T (&wv)[KT], T (&vb)[KT], const T* vol, T* slot, int b,
                         int plane, long long poff) {
  constexpr int NW = NT / 64, NBD = DotBlocks<float2>::value, PL = NBD / 64;
  typedef typename real_of<T>::type R;
  __shared__ double2 hsum[MAXM + 1];
  __shared__ T hc[MAXM];
  __shared__ double nred[NW];
  const UpdateTask& u = a.up;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  GState& S = u.st[b];
  const T* sb = reinterpret_cast<const T*>(u.V) + (long long)b * u.bsv + poff;
  // the slot scales and the projection partials are requested together (w is
  // already on its way); then one slot per pass
  const double scv = S.sc[min(tid, MAXM)];
  const double2* pb = u.dpart + (long long)b * PSTR * NBD;
  for (int i = wave; i <= cnt; i += NW) {
    double2 pv[PL];
#pragma unroll
    for (int k = 0; k < PL; ++k) pv[k] = pb[(long long)i * NBD + lane + 64 * k];
    double2 t = make_double2(0, 0);
#pragma unroll
    for (int k = 0; k < PL; ++k) t = cadd(t, pv[k]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      t.x += __shfl_xor(t.x, off, 64);
      t.y += __shfl_xor(t.y, off, 64);
    }
    if (lane == 0) hsum[i] = t;
  }
  __syncthreads();
  if (tid < cnt) {
    hc[tid] = from_d<T>(cscale(hsum[tid], scv * scv));
    if (plane == 0) S.h[tid] = cscale(hsum[tid], scv);
  } else if (tid == cnt && plane == 0) {
    S.wn2_in = hsum[cnt].x;
  }
  __syncthreads();
  for (int i = 0; i < cnt; ++i) {
    const T* si = sb + (long long)i * u.ldv;
    T p[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) p[k] = si[tid + k * NT];
    const T h = hc[i];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      wv[k].x -= h.x * p[k].x - h.y * p[k].y;
      wv[k].y -= h.x * p[k].y + h.y * p[k].x;
    }
  }
  // the contrast values, loaded only now (fewer live registers in the loop
  // above); their latency overlaps the stores and the norm reduction
#pragma unroll
  for (int k = 0; k < KT; ++k) vb[k] = vol[tid + k * NT];
  R nn = 0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    slot[tid + k * NT] = wv[k];
    nn += wv[k].x * wv[k].x + wv[k].y * wv[k].y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nn += __shfl_xor(nn, off, 64);
  if (lane == 0) nred[wave] = (double)nn;
  __syncthreads();
  if (tid == 0) {
    double t = nred[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) t += nred[w];
    u.part[(long long)b * (3 * a.nz) + plane] = make_double2(t, 0.0);
  }
}

// Gram-Schmidt projections of one plane of the new Arnoldi vector w (its KT
// values per thread in wv, element tid + k NT of the plane at poff): partial
// <slot_i, w> for i = 0..j and ||w||^2, summed in the vector precision within a
// wavefront and in FP64 across the wavefronts in a fixed order, stored as this
// plane's partial of the projection pass; partial indices no plane owns get zeros.
template <class T, int KT, int NT>
PSFD_D void plane_dots(const TileArgs& a, const T (&wv)[KT], int b, int plane, long long poff) {
  constexpr int NW = NT / 64, NBD = DotBlocks<float2>::value;
  extern __shared__ double2 smem_d[];
  double2* red = smem_d;  // [PSTR][NW]; the plane's LDS is free after the barrier
  const DotTask& d = a.dt;
  const int cnt = (d.jh >= 0 ? d.jh : d.st[b].j) + 1;
  const T* vb = reinterpret_cast<const T*>(d.V) + (long long)b * d.bsv + poff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto wsum = [](T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v.x += __shfl_xor(v.x, off, 64);
      v.y += __shfl_xor(v.y, off, 64);
    }
    return v;
  };
  __syncthreads();
  // two slots per pass, their loads issued together (the second index clamped)
  for (int i0 = 0; i0 < cnt; i0 += 2) {
    const int i1 = min(i0 + 1, cnt - 1);
    const T* s0 = vb + (long long)i0 * d.ldv;
    const T* s1 = vb + (long long)i1 * d.ldv;
    T p0[KT], p1[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      p0[k] = s0[tid + k * NT];
      p1[k] = s1[tid + k * NT];
    }
    T a0 = cmake<T>(0, 0), a1 = cmake<T>(0, 0);
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      a0.x += p0[k].x * wv[k].x + p0[k].y * wv[k].y;
      a0.y += p0[k].x * wv[k].y - p0[k].y * wv[k].x;
      a1.x += p1[k].x * wv[k].x + p1[k].y * wv[k].y;
      a1.y += p1[k].x * wv[k].y - p1[k].y * wv[k].x;
    }
    a0 = wsum(a0);
    a1 = wsum(a1);
    if (lane == 0) {
      red[i0 * NW + wave] = to_d(a0);
      if (i0 + 1 < cnt) red[(i0 + 1) * NW + wave] = to_d(a1);
    }
  }
  T nn = cmake<T>(0, 0);
#pragma unroll
  for (int k = 0; k < KT; ++k) nn.x += wv[k].x * wv[k].x + wv[k].y * wv[k].y;
  nn = wsum(nn);
  if (lane == 0) red[cnt * NW + wave] = to_d(nn);
  __syncthreads();
  if (tid <= cnt) {
    double2 t = red[tid * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) t = cadd(t, red[tid * NW + w]);
    double2* pp = d.part + ((long long)b * PSTR + tid) * NBD;
    pp[plane] = t;
    for (int q = plane + 3 * a.nz; q < NBD; q += 3 * a.nz) pp[q] = make_double2(0, 0);
  }
  // the update of this column is now pending (read by the next step's kernels)
  if (plane == 0 && tid == 0) d.st[b].pend = 1;
}

template <class T, bool INV, int LD, int ST, int LN>
__global__ void __launch_bounds__(plane_threads(LN)) k_plane(TileArgs a) {
  constexpr int N = 1 << LN, P = N + 1, NT = plane_threads(LN);
  constexpr int KT = N * N / NT;  // elements per thread
  static_assert(KT * NT == N * N, "plane split");
  extern __shared__ double2 smem_d[];
  T* lds = reinterpret_cast<T*>(smem_d);
  T* twl = lds + N * P;
  const int b = blockIdx.y;
  constexpr bool UPD = LD == LD_UPD_VX || LD == LD_UPD_SLOT;  // Gram-Schmidt update on load
  constexpr bool VX = LD == LD_VX || UPD;                     // contrast multiply on load
  // a GivensTask takes the extra last block of the grid
  if (LD == LD_VX && a.gv.st && blockIdx.x == gridDim.x - 1) {
    givens_task(a.gv.st, a.gv.run, a.gv.part, a.gv.nblk, b);
    return;
  }
  if (a.active && !a.active[b]) return;
  const int plane = blockIdx.x;
  const int z = plane % a.nz;
  const long long poff = (long long)plane * N * N;
  const int tid = threadIdx.x;
  const T* in = vref<T>(a.in, b) + poff;
  // LD_UPD_VX: the update of column cnt - 1 on slot cnt; per instance (up.j < 0)
  // only with a pending update, and at up.j = 0 not at all: then the plain
  // scaled load of the slot (by S.inv_norm, as LD_VX with in_scale)
  int cnt = LD == LD_UPD_VX ? a.up.j : 0;
  bool upd = LD == LD_UPD_VX;
  if constexpr (LD == LD_UPD_SLOT) {
    if (a.up.j >= 0) {
      cnt = a.up.j;
      upd = cnt > 0;  // step 0 of a cycle: the plain scaled load
    } else {
      const GState& S = a.up.st[b];
      const int pend = S.pend, js = S.j;
      upd = pend != 0;
      cnt = js + 1;
      in = reinterpret_cast<const T*>(a.up.V) + (long long)b * a.up.bsv + (long long)(upd ? js + 1 : js) * a.up.ldv +
           poff;
    }
  }
  const T* vol = VX ? vref<T>(a.vol, b) + (long long)z * N * N : nullptr;
  const T* aux = ST == ST_AXPBY ? vref<T>(a.aux, b) + poff : nullptr;
  typedef typename real_of<T>::type R;
  const T* twg = reinterpret_cast<const T*>(a.tw) + N;
  // element i = tid + k NT is (row i >> LN, column i & (N - 1)), plane offset i
  const T tw0 = twg[tid & (N - 1)];
  // keep the twiddle load ahead of the data loads: its LDS write below then waits
  // for it alone
  __builtin_amdgcn_sched_barrier(0);
  T va[KT], vb[VX ? KT : 1], xa[ST == ST_AXPBY ? KT : 1];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    va[k] = in[tid + k * NT];
    if (LD == LD_VX) vb[k] = vol[tid + k * NT];
  }
  if (ST == ST_AXPBY) {
#pragma unroll
    for (int k = 0; k < KT; ++k) xa[k] = aux[tid + k * NT];
  }
  // the Gram-Schmidt update of the previous column on slot j before its transform
  if constexpr (UPD) {
    if (LD == LD_UPD_VX || upd) {
      plane_update<T, KT, NT>(a, cnt, va, vb, vol, const_cast<T*>(in), b, plane, poff);
    } else {
#pragma unroll
      for (int k = 0; k < KT; ++k) vb[k] = vol[tid + k * NT];
    }
  }
  const double* tab = a.tab + (long long)b * a.tab_stride;
  const R k0sq = (R)tab[TS_K0SQ];
  // scale of the input on load (the newest Arnoldi vector is kept unnormalised),
  // folded into the contrast factor: from in_scale, or with a GivensTask from
  // the norm partials the task itself sums (bitwise the same value); LD_UPD_VX
  // leaves the vector unscaled (the pencil kernel scales it)
  R scl = (R)1;
  if (LD == LD_VX && a.gv.st) scl = (R)inv_norm_of(norm_from_partials(a.gv.part + (long long)b * a.gv.nblk, a.gv.nblk));
  else if (LD == LD_VX && a.in_scale) scl = (R)a.in_scale[(long long)b * a.scale_stride];
  else if (LD == LD_UPD_SLOT && !upd) scl = (R)a.up.st[b].inv_norm;
  const R ks = k0sq * scl;
  if (tid < N) twl[tid] = tw0;
  auto put = [&](int k) {
    const int i = tid + k * NT;
    const T x = va[k];
    const T v = VX ? cscale(cmul(vb[VX ? k : 0], x), ks) : x;
    lds[(i >> LN) * P + (i & (N - 1))] = v;
  };
  typedef FftCT<LN, N, P, 1, NT> Rows;
  typedef FftCT<LN, N, 1, P, NT> Cols;
#pragma unroll
  for (int k = 0; k < KT; ++k) put(k);
  __syncthreads();
  // sequence-fastest butterflies: consecutive lanes take consecutive rows (or
  // columns), so with the odd pitch every LDS access of a pass is conflict-free
  lds_fft_tab<T, INV, true, KT, Rows, false, false, 4>(lds, Rows(), twl, tid);
  // the column transform's last pass leaves its results in registers: its
  // butterfly b = tid + i NT (column b mod N, index t = b / N) forms rows
  // t + PL j of that column, i.e. plane elements tid + (i + KJ j) NT, which are
  // this thread's own store elements k = i + KJ j
  T res[KT];
  lds_fft_tab_regout<T, INV, true, KT, Cols, false, 4>(lds, Cols(), twl, tid, res);
  constexpr int LRL = (LN - 1) % 4 + 1, RL = 1 << LRL, NBL = KT / RL, PL = N / RL, KJ = PL * N / NT;
  static_assert(LN >= 4 && NBL * RL == KT && KJ * NT == PL * N && KJ == NBL, "plane last pass");
  T* out = vref<T>(a.out, b) + poff;
  const R al = (R)a.alpha, ga = (R)a.gamma;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int kj = k / KJ, ki = k - kj * KJ;  // k = ki + KJ kj: butterfly ki, output kj
    T v = res[ki * RL + kj];
    if (ST == ST_AXPBY) {
      const T xv = xa[ST == ST_AXPBY ? k : 0];
      v.x = al * xv.x + ga * v.x;
      v.y = al * xv.y + ga * v.y;
    }
    out[tid + k * NT] = v;
    if (ST == ST_DOTS) va[k] = v;
  }
  if constexpr (ST == ST_DOTS) plane_dots<T, KT, NT>(a, va, b, plane, poff);
}

// -------------------------------------------------------------------------
// Quarter-plane kernels (N x N planes, N = 128, and 256 in FP32; operator
// apply). The transverse transform of a plane is split four ways over y: block
// q of a plane takes the rows y = 4 r + q (r < N / 4), transforms them along x
// (N points) and along r (N / 4 points), and stores the quarter spectrum times
// its twiddle, Y'_q(ky', kx) = W_N^(q ky') Y_q(ky', kx), ky' < N / 4. The full
// spectrum is the radix-4 decimation-in-time combine
//   X(ky' + (N / 4) m, kx) = sum_q W4^(q m) Y'_q(ky', kx),
// a twiddle-free 4-point DFT that the z-pencil kernel takes on load. Back the
// same way: the pencil stores Z'_q = sum_m W4^(-q m) X(ky' + (N / 4) m), and
// block q multiplies by W_N^(-q ky') and transforms along r and x back to the
// rows y = 4 r + q. At N = 128, four blocks per plane (768 at 192 planes) keep
// every CU busy with three resident blocks whose loads and FFT passes overlap;
// one block per plane leaves 64 of 256 CUs idle and runs each CU's load,
// transform and store one after the other. At N = 256 (FP32) a quarter plane
// is one block per CU, and the transform is one pass through HBM where the
// row and column strips take two.
// Layout between the kernels, per plane: the four quarter spectra interleaved
// in 32-byte pieces, (q, ky', kx) at qp_index<N>(ky', kx, q), so that the 16
// values a pencil block takes at one (component, z) form one 128-byte line.
// -------------------------------------------------------------------------
// threads of a quarter-plane block: 16 values each in FP32 (rows of 128 by radix
// 16 and 8, of 256 by 16 and 16), 8 in FP64 (radix 8, 8 and 2); the column
// passes take radix 8, then 4 (N / 4 = 32) or 8 (N / 4 = 64)
template <class T, int LN> struct QpShape {
  static constexpr int N = 1 << LN, ROWS = N / 4;
  static constexpr int NT = sizeof(T) == 16 ? 512 : (LN == 7 ? 256 : 1024), KT = ROWS * N / NT;
  static constexpr int LRM_ROWS = sizeof(T) == 8 ? 4 : 3;
  static constexpr int LRL = (LN - 3) % 3 + 1, RL = 1 << LRL;  // last column pass: radix RL
};
__host__ __device__ constexpr size_t qplane_lds(int ln, size_t esz) {
  return ((size_t)((1 << ln) / 4) * ((1 << ln) + 1) + (1 << ln) + (1 << ln) / 4) * esz;
}
template <int N> PSFD_D int qp_index(int kyq, int kx, int q) { return kyq * (4 * N) + (kx >> 2) * 16 + 4 * q + (kx & 3); }

template <class T, bool INV, int LD, int ST, int LN>
__global__ void __launch_bounds__((QpShape<T, LN>::NT)) k_qplane(TileArgs a) {
  typedef QpShape<T, LN> S;
  constexpr int N = S::N, QP_ROWS = S::ROWS, P = N + 1, NT = S::NT, KT = S::KT, TS = NT / N;
  static_assert(KT * NT == QP_ROWS * N && NT % N == 0, "quarter-plane thread split");
  static_assert(!INV || LD == LD_PLAIN, "inverse: plain load");
  static_assert(INV || (LD == LD_VX && ST == ST_PLAIN), "forward: contrast multiply, plain store");
  extern __shared__ double2 smem_d[];
  T* lds = reinterpret_cast<T*>(smem_d);
  T* twl = lds + QP_ROWS * P;  // W_N^k, k < N
  T* twl32 = twl + N;          // W_(N/4)^k = W_N^(4 k), k < N / 4
  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;
  // block order: with 8 | nz, XCD x (= hw mod 8) takes the planes z = x mod 8 of
  // all three components and their four quarters, so the three blocks that read
  // one contrast plane share an L2, and so do the four that write (or read) one
  // 128-byte line of the layout
  int plane, q;
  {
    const int hw = blockIdx.x;
    if ((a.nz & 7) == 0) {
      const int xc = hw & 7, i = hw >> 3, t = i >> 2, c = t % 3, zz = t / 3;
      q = i & 3;
      plane = c * a.nz + xc + 8 * zz;
    } else {
      plane = hw >> 2;
      q = hw & 3;
    }
  }
  const int z = plane % a.nz;
  const long long poff = (long long)plane * N * N;
  const int tid = threadIdx.x;
  typedef typename real_of<T>::type R;
  const T* twg = reinterpret_cast<const T*>(a.tw) + N;
  const T tw0 = twg[tid & (N - 1)];
  const T tw1 = twg[(tid & (QP_ROWS - 1)) * 4];
  // the twiddle loads ahead of the data loads: their LDS writes wait for them alone
  __builtin_amdgcn_sched_barrier(0);
  const T* in = vref<T>(a.in, b) + poff;
  const T* vol = INV ? nullptr : vref<T>(a.vol, b) + (long long)z * N * N;
  const T* aux = ST == ST_AXPBY ? vref<T>(a.aux, b) + poff : nullptr;
  // the column transform's last pass (radix RL, stride PL = N / 4 / RL = 8)
  // leaves its results in registers: butterfly i of the thread (column
  // s = tid mod N, index t = tid / N + (NT / N) i) forms rows r = t + PL j of
  // that column
  constexpr int RL = S::RL, PL = QP_ROWS / RL, NBL = KT / RL;
  static_assert(PL == 8 && NBL * RL == KT, "quarter-plane last column pass");
  T va[KT], vb[INV ? 1 : KT], xa[ST == ST_AXPBY ? KT : 1];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = tid + k * NT, r = i >> LN, x = i & (N - 1);
    if constexpr (!INV) {
      va[k] = in[(4 * r + q) * N + x];
      vb[k] = vol[(4 * r + q) * N + x];
    } else {
      va[k] = in[qp_index<N>(r, x, q)];
    }
  }
  if constexpr (ST == ST_AXPBY) {
#pragma unroll
    for (int i = 0; i < NBL; ++i)
#pragma unroll
      for (int j = 0; j < RL; ++j) {
        const int r = (tid >> LN) + TS * i + PL * j, x = tid & (N - 1);
        xa[i * RL + j] = aux[(4 * r + q) * N + x];
      }
  }
  const double* tab = a.tab + (long long)b * a.tab_stride;
  R ks = (R)1;
  if constexpr (!INV) ks = (R)tab[TS_K0SQ] * (a.in_scale ? (R)a.in_scale[(long long)b * a.scale_stride] : (R)1);
  if (tid < N) twl[tid] = tw0;
  if (tid < QP_ROWS) twl32[tid] = tw1;
  // the inverse multiplies by W128^(-q ky') on the way into LDS
  if constexpr (INV) __syncthreads();
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = tid + k * NT, r = i >> LN;
    T v;
    if constexpr (INV) v = cmulc(va[k], twl[q * r]);
    else v = cscale(cmul(vb[k], va[k]), ks);
    lds[r * P + (i & (N - 1))] = v;
  }
  __syncthreads();
  typedef FftCT<LN, QP_ROWS, P, 1, NT> Rows;  // N / 4 rows of N points
  typedef FftCT<LN - 2, N, 1, P, NT> Cols;     // N columns of N / 4 points
  lds_fft_tab<T, INV, true, KT, Rows, false, false, S::LRM_ROWS>(lds, Rows(), twl, tid);
  T res[KT];
  lds_fft_tab_regout<T, INV, true, KT, Cols, false, 3>(lds, Cols(), twl32, tid, res);
  T* out = vref<T>(a.out, b) + poff;
  const R al = (R)a.alpha, ga = (R)a.gamma;
#pragma unroll
  for (int i = 0; i < NBL; ++i)
#pragma unroll
    for (int j = 0; j < RL; ++j) {
      const int r = (tid >> LN) + TS * i + PL * j, x = tid & (N - 1);
      T v = res[i * RL + j];
      if constexpr (!INV) {
        out[qp_index<N>(r, x, q)] = cmul(v, twl[q * r]);
      } else {
        if constexpr (ST == ST_AXPBY) {
          const T xv = xa[ST == ST_AXPBY ? i * RL + j : 0];
          v.x = al * xv.x + ga * v.x;
          v.y = al * xv.y + ga * v.y;
        }
        out[(4 * r + q) * N + x] = v;
      }
    }
}


template <class T, bool INV, int LD, int ST>
void launch_qplane(const TileArgs& a, int nplanes, int nbatch, hipStream_t s) {
  const bool ok = a.nx == a.ny && (a.nx == 128 || (a.nx == 256 && sizeof(T) == 8));
  if (!ok || a.gv.st || nplanes != 3 * a.nz) {
    std::fprintf(stderr, "psfd: internal error: quarter-plane launch on an unsupported shape\n");
    std::abort();
  }
  auto go = [&](auto kern, int ln, int nt) {
    const size_t l = qplane_lds(ln, sizeof(T));
    allow_lds(reinterpret_cast<const void*>(kern), l);
    hipLaunchKernelGGL(kern, dim3(4 * nplanes, nbatch), dim3(nt), l, s, a);
  };
  if constexpr (sizeof(T) == 8) {
    if (a.nx == 256) return go(k_qplane<T, INV, LD, ST, 8>, 8, QpShape<T, 8>::NT);
  }
  go(k_qplane<T, INV, LD, ST, 7>, 7, QpShape<T, 7>::NT);
}
template void launch_qplane<float2, false, LD_VX, ST_PLAIN>(const TileArgs&, int, int, hipStream_t);
template void launch_qplane<float2, true, LD_PLAIN, ST_PLAIN>(const TileArgs&, int, int, hipStream_t);
template void launch_qplane<float2, true, LD_PLAIN, ST_AXPBY>(const TileArgs&, int, int, hipStream_t);
template void launch_qplane<double2, false, LD_VX, ST_PLAIN>(const TileArgs&, int, int, hipStream_t);
template void launch_qplane<double2, true, LD_PLAIN, ST_PLAIN>(const TileArgs&, int, int, hipStream_t);
template void launch_qplane<double2, true, LD_PLAIN, ST_AXPBY>(const TileArgs&, int, int, hipStream_t);

// -------------------------------------------------------------------------
// Strip kernel: for square N x N planes too large for LDS, the x-FFT of
// TY = 4096 / N full rows (ROWS) or the y-FFT of 16 full columns of one plane,
// with the shapes fixed at compile time; 8 elements per thread, twiddles in
// LDS, every global load of a thread issued before its LDS writes.
// -------------------------------------------------------------------------
template <int LN, bool ROWS> struct StripShape {
  static constexpr int N = 1 << LN;
  static constexpr int TX = ROWS ? N : 16, TY = ROWS ? 4096 / N : N, LTX = ROWS ? LN : 4;
  static constexpr int P = TX + 1, ELEM = TX * TY, KT = 8, NT = ELEM / KT;
  static constexpr int TILES = ROWS ? N / TY : N / 16;
};
template <int LN, bool ROWS> __host__ constexpr size_t strip_lds(size_t esz) {
  return ((size_t)StripShape<LN, ROWS>::TY * StripShape<LN, ROWS>::P + StripShape<LN, ROWS>::N) * esz;
}

template <class T, bool INV, int LD, int ST, int LN, bool ROWS>
__global__ void __launch_bounds__(512) k_strip(TileArgs a) {
  typedef StripShape<LN, ROWS> S;
  constexpr int N = S::N, TX = S::TX, TY = S::TY, LTX = S::LTX, P = S::P, KT = S::KT, NT = S::NT;
  extern __shared__ double2 smem_d[];
  T* lds = reinterpret_cast<T*>(smem_d);
  T* twl = lds + TY * P;
  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;
  const int plane = blockIdx.x / S::TILES, tile = blockIdx.x % S::TILES;
  const int z = plane % a.nz;
  const int x0 = ROWS ? 0 : tile * TX, y0 = ROWS ? tile * TY : 0;
  const long long poff = (long long)plane * N * N;
  const int tid = threadIdx.x;
  const T* in = vref<T>(a.in, b) + poff;
  const T* vol = LD == LD_VX ? vref<T>(a.vol, b) + (long long)z * N * N : nullptr;
  const T* aux = ST == ST_AXPBY ? vref<T>(a.aux, b) + poff : nullptr;
  typedef typename real_of<T>::type R;
  auto off_of = [&](int i) -> int { return (y0 + (i >> LTX)) * N + (x0 + (i & (TX - 1))); };
  const T tw0 = reinterpret_cast<const T*>(a.tw)[N + (tid & (N - 1))];
  __builtin_amdgcn_sched_barrier(0);
  T va[KT], vb[LD == LD_VX ? KT : 1], xa[ST == ST_AXPBY ? KT : 1];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int o = off_of(tid + k * NT);
    va[k] = in[o];
    if (LD == LD_VX) vb[k] = vol[o];
  }
  if (ST == ST_AXPBY) {
#pragma unroll
    for (int k = 0; k < KT; ++k) xa[k] = aux[off_of(tid + k * NT)];
  }
  const double* tab = a.tab + (long long)b * a.tab_stride;
  const R k0sq = (R)tab[TS_K0SQ];
  // scale of the input on load (the newest Arnoldi vector is kept unnormalised),
  // folded into the contrast factor
  const R ks = k0sq * ((LD == LD_VX && a.in_scale) ? (R)a.in_scale[(long long)b * a.scale_stride] : (R)1);
  static_assert(NT >= N, "one twiddle per thread");
  if (tid < N) twl[tid] = tw0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = tid + k * NT;
    const T x = va[k];
    const T v = LD == LD_VX ? cscale(cmul(vb[LD == LD_VX ? k : 0], x), ks) : x;
    lds[(i >> LTX) * P + (i & (TX - 1))] = v;
  }
  __syncthreads();
  // sequence-fastest butterflies (conflict-free LDS accesses through the odd pitch)
  if constexpr (ROWS) lds_fft_tab<T, INV, true, KT, FftCT<LN, TY, P, 1, NT>>(lds, FftCT<LN, TY, P, 1, NT>(), twl, tid);
  else lds_fft_tab<T, INV, true, KT, FftCT<LN, 16, 1, P, NT>>(lds, FftCT<LN, 16, 1, P, NT>(), twl, tid);
  T* out = vref<T>(a.out, b) + poff;
  const R al = (R)a.alpha, ga = (R)a.gamma;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int i = tid + k * NT;
    T v = lds[(i >> LTX) * P + (i & (TX - 1))];
    if (ST == ST_AXPBY) {
      const T xv = xa[ST == ST_AXPBY ? k : 0];
      v.x = al * xv.x + ga * v.x;
      v.y = al * xv.y + ga * v.y;
    }
    out[off_of(i)] = v;
  }
}

// fused square planes of 64 x 64 (and 128 x 128 in FP32) with plain or
// contrast-multiply loads take the square-plane kernel; the row and column
// passes of square 128 x 128 and 256 x 256 planes take the strip kernel
// log2 of the plane side when launch_tile runs the square-plane kernel (fused
// transverse FFT of full N x N planes in LDS: 64^2, and 128^2 in FP32), else 0
static int plane_ln(const TileArgs& a, size_t esz) {
  const bool sq = a.do_x && a.do_y && a.tx == a.nx && a.ty == a.ny && a.nx == a.ny;
  if (sq && a.nx == 64) return 6;
  if (sq && a.nx == 128 && esz == 8) return 7;
  return 0;
}
bool tile_is_plane(const TileArgs& a, size_t esz) { return plane_ln(a, esz) != 0; }
bool tile_takes_update(const TileArgs& a, size_t esz) { return esz == 8 && plane_ln(a, esz) != 0; }
bool tile_takes_dots(const TileArgs& a, size_t esz) {
  return esz == 8 && plane_ln(a, esz) != 0 && 3 * a.nz <= DotBlocks<float2>::value;
}

// The Givens task and norm_from_partials need blocks of at least GIVENS_THREADS
// threads (their partial sums are spread over that many lanes). Every launch that
// passes a GivensTask (or the update task, whose blocks sum the same partials) is
// gated on that by its caller; a launch that breaks the rule would sum unwritten
// LDS words, so it stops the process instead of computing a wrong result.
[[noreturn]] static void givens_block_too_small(const char* kern, int nthr) {
  std::fprintf(stderr, "psfd: internal error: %s launched with a Givens task in blocks of %d threads (< %d)\n",
               kern, nthr, GIVENS_THREADS);
  std::abort();
}

template <class T, bool INV, int LD, int ST>
void launch_tile(const TileArgs& a, int nplanes, int nbatch, int nthr, size_t lds, hipStream_t s) {
  dim3 grid(nplanes * a.tiles_x * a.tiles_y, nbatch);
  auto plane = [&](auto kern, int ln) {
    const size_t l = plane_lds(ln, sizeof(T));
    allow_lds(reinterpret_cast<const void*>(kern), l);
    dim3 g2 = grid;
    if (LD == LD_VX && a.gv.st) g2.x += 1;  // the GivensTask block
    if ((a.gv.st || LD == LD_UPD_VX || LD == LD_UPD_SLOT) && plane_threads(ln) < GIVENS_THREADS)
      givens_block_too_small("k_plane", plane_threads(ln));
    hipLaunchKernelGGL(kern, g2, dim3(plane_threads(ln)), l, s, a);
  };
  if constexpr (ST == ST_DOTS) {
    // only the FP32 square planes (64 x 64, 128 x 128) store with the projections
    if constexpr (sizeof(T) == 8) {
      if (tile_takes_dots(a, sizeof(T))) {
        if (plane_ln(a, sizeof(T)) == 6) return plane(k_plane<T, INV, LD, ST, 6>, 6);
        return plane(k_plane<T, INV, LD, ST, 7>, 7);
      }
    }
    return;
  } else if constexpr (LD == LD_UPD_VX || LD == LD_UPD_SLOT) {
    // only the FP32 square planes (64 x 64, 128 x 128) load with the update
    if constexpr (sizeof(T) == 8) {
      if (tile_takes_update(a, sizeof(T))) {
        if (plane_ln(a, sizeof(T)) == 6) return plane(k_plane<T, INV, LD, ST, 6>, 6);
        return plane(k_plane<T, INV, LD, ST, 7>, 7);
      }
    }
    return;
  } else if constexpr (LD == LD_PLAIN || LD == LD_VX) {
    const int ln = plane_ln(a, sizeof(T));
    if (ln == 6) return plane(k_plane<T, INV, LD, ST, 6>, 6);
    if constexpr (sizeof(T) == 8)
      if (ln == 7) return plane(k_plane<T, INV, LD, ST, 7>, 7);
    // strips of square planes: rows (TY = 4096 / N full rows) or 16-column strips
    auto strip = [&](auto kern, int nt, size_t l) {
      allow_lds(reinterpret_cast<const void*>(kern), l);
      hipLaunchKernelGGL(kern, grid, dim3(nt), l, s, a);
    };
    const bool square = a.nx == a.ny && (a.nx == 128 || a.nx == 256);
    const bool rows = square && a.do_x && !a.do_y && a.tx == a.nx && a.ty == 4096 / a.nx;
    const bool cols = square && !a.do_x && a.do_y && a.tx == 16 && a.ty == a.ny;
    if (rows && a.nx == 128)
      return strip(k_strip<T, INV, LD, ST, 7, true>, StripShape<7, true>::NT, strip_lds<7, true>(sizeof(T)));
    if (rows && a.nx == 256)
      return strip(k_strip<T, INV, LD, ST, 8, true>, StripShape<8, true>::NT, strip_lds<8, true>(sizeof(T)));
    if (cols && a.nx == 128)
      return strip(k_strip<T, INV, LD, ST, 7, false>, StripShape<7, false>::NT, strip_lds<7, false>(sizeof(T)));
    if (cols && a.nx == 256)
      return strip(k_strip<T, INV, LD, ST, 8, false>, StripShape<8, false>::NT, strip_lds<8, false>(sizeof(T)));
  }
  allow_lds(reinterpret_cast<const void*>(&k_tile<T, INV, LD, ST>), lds);
  hipLaunchKernelGGL((k_tile<T, INV, LD, ST>), grid, dim3(nthr), lds, s, a);
}

template void launch_tile<float2, false, LD_VX, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<float2, false, LD_PLAIN, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<float2, true, LD_PLAIN, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<float2, true, LD_PLAIN, ST_AXPBY>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<float2, true, LD_PLAIN, ST_DOTS>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<float2, false, LD_UPD_VX, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<float2, false, LD_UPD_SLOT, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, false, LD_VX, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, false, LD_PLAIN, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, true, LD_PLAIN, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, true, LD_PLAIN, ST_AXPBY>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, false, LD_VXE, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, true, LD_INJECT, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);
template void launch_tile<double2, true, LD_INJECT_T, ST_PLAIN>(const TileArgs&, int, int, int, size_t, hipStream_t);

// -------------------------------------------------------------------------
// z-pencil kernel: pad, FFT_z, dyadic kernel, IFFT_z, restrict
// -------------------------------------------------------------------------

// z-windowed scalar factor F = (s e^{i beta L} - 1) / (beta^2 - kappa^2), with the
// removable resonance kappa = +-beta taken by its Taylor series.
PSFD_D double2 window_factor(double2 beta, double2 eibl, double kap, double L, double s) {
  double2 num = make_double2(s * eibl.x - 1.0, s * eibl.y);
  double ak = fabs(kap);
  double ur = (beta.x - ak) * L, ui = beta.y * L;
  if (ur * ur + ui * ui < 1e-12) {
    // L (i - u/2 - i u^2/6) / (beta + |kappa|)
    double2 u = make_double2(ur, ui);
    double2 u2 = cmul(u, u);
    double2 ser = make_double2(-0.5 * u.x + u2.y / 6.0, 1.0 - 0.5 * u.y - u2.x / 6.0);
    ser = cscale(ser, L);
    return cdiv(ser, make_double2(beta.x + ak, beta.y));
  }
  double2 den = make_double2(beta.x * beta.x - beta.y * beta.y - kap * kap, 2.0 * beta.x * beta.y);
  return cdiv(num, den);
}

// exp(i beta z) in the working precision. FP64: direct. FP32: the phase is
// reduced modulo 2 pi in FP64 and the sine, cosine and decay taken in FP32.
template <class T> PSFD_D T phase_exp(double2 beta, double z);
template <> PSFD_D double2 phase_exp<double2>(double2 beta, double z) {
  return cexp_i(make_double2(beta.x * z, beta.y * z));
}
template <> PSFD_D float2 phase_exp<float2>(double2 beta, double z) {
  const double th = beta.x * z;
  const double red = th - 6.283185307179586 * rint(th * 0.15915494309189535);
  float sn, cs;
  sincosf((float)red, &sn, &cs);
  const float m = expf((float)(-beta.y * z));
  return make_float2(m * cs, m * sn);
}

// F scale for one (order, kappa) point: the denominator beta^2 - kappa^2 and the
// numerator s e^{i beta L} - 1 are formed in FP64 (the cancellation is there);
// their quotient is taken in the working precision. Near the resonance
// kappa = +-beta the series of window_factor is used.
template <class T>
PSFD_D T window_factor_fast(double2 beta, double2 beta2, double2 num, double kap, double L, double s, double scale) {
  const double ak = fabs(kap);
  const double ur = (beta.x - ak) * L, ui = beta.y * L;
  if (ur * ur + ui * ui < 1e-12) {
    const double2 e = make_double2(s * (num.x + 1.0), s * (num.y));  // e^{i beta L}
    return from_d<T>(cscale(window_factor(beta, e, kap, L, s), scale));
  }
  const double2 den = make_double2(beta2.x - kap * kap, beta2.y);
  const T n = from_d<T>(make_double2(num.x * scale, num.y * scale));
  const T d = from_d<T>(den);
  typedef typename real_of<T>::type R;
  // FP32: hardware reciprocal (1 ulp, far inside the single-precision error of the
  // apply); |den|^2 stays normal outside the resonance window of the series above
  R inv;
  if constexpr (sizeof(R) == 4) inv = __builtin_amdgcn_rcpf(d.x * d.x + d.y * d.y);
  else inv = (R)1 / (d.x * d.x + d.y * d.y);
  T r;
  r.x = (n.x * d.x + n.y * d.y) * inv;
  r.y = (n.y * d.x - n.x * d.y) * inv;
  return r;
}

// LDS layout of a pencil block: element z of sequence (c, kxl) at z * LS + c * bx + kxl
// (sequences interleaved, LS = 3 bx), so every FFT pass, the kernel multiply and
// the global load/store touch consecutive LDS words across a wavefront.
// At most 8 values per thread in the pencil FFTs (the launch gives 3 bx pz / 8
// threads, at most 768), which halves the register arrays of the FP32 passes.
// Threads of a pencil block with bx columns and padded length 2^LPZ: at most 8
// values per thread in the FFT passes, at least four readout partial sums per
// sequence (the host's pencil_threads gives the same count).
__host__ __device__ constexpr int pencil_threads_ct(int lpz, int bx) {
  return (3 * bx * (1 << lpz) / 8 + 63) / 64 * 64 > (12 * bx + 63) / 64 * 64 ? (3 * bx * (1 << lpz) / 8 + 63) / 64 * 64
                                                                            : (12 * bx + 63) / 64 * 64;
}

// Quarter-spectrum combine of the pencil (quarter-plane layout): a 4-point DFT
// across the four lanes of a quad, lane q holding input q. Its radix-2 stages
// pair lanes q, q ^ 2 and then q, q ^ 1 through DPP quad permutations
// (partner + sign * own). Forward: lane q receives X_brev(q) =
// sum_p W4^(p brev(q)) Y_p (brev: the 2-bit reversal); inverse: lane q holds
// X_brev(q) and receives Z_q = sum_m W4^(-q m) X_m.
// (every source lane of a quad permutation is valid, so no old value is needed)
template <int CTRL> PSFD_D float quad_perm_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
// a double moves as its two 32-bit halves
template <int CTRL> PSFD_D double quad_perm_f(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL, class T> PSFD_D T quad_bfly(T v, typename real_of<T>::type sg) {
  T r;
  r.x = quad_perm_f<CTRL>(v.x) + sg * v.x;
  r.y = quad_perm_f<CTRL>(v.y) + sg * v.y;
  return r;
}
constexpr int DPP_QUAD_SWAP2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int DPP_QUAD_SWAP1 = 0xB1;  // quad_perm [1, 0, 3, 2]
template <class T> PSFD_D T quad_dft4(T v, int q, bool inv) {
  typedef typename real_of<T>::type R;
  const R s2 = q < 2 ? (R)1 : (R)-1, s1 = (q & 1) ? (R)-1 : (R)1;
  T r;
  if (!inv) {
    v = quad_bfly<DPP_QUAD_SWAP2>(v, s2);
    if (q == 3) { r.x = v.y; r.y = -v.x; v = r; }  // times -i
    return quad_bfly<DPP_QUAD_SWAP1>(v, s1);
  }
  v = quad_bfly<DPP_QUAD_SWAP1>(v, s1);
  if (q == 3) { r.x = -v.y; r.y = v.x; v = r; }  // times +i
  return quad_bfly<DPP_QUAD_SWAP2>(v, s2);
}
// pencil column c of a quarter-layout block: kx = kx0 + c / 4 and quarter
// q = c mod 4 on load (position 4 q + c / 4 of the block's 16-value piece), row
// ky' + (ny / 4) brev(q) after the combine
PSFD_D int qp_pos(int c) { return ((c & 3) << 2) | (c >> 2); }
PSFD_D int brev2(int q) { return ((q & 1) << 1) | (q >> 1); }

// LPZ > 0: BXC columns and padded length 2^LPZ fixed at compile time (the FFT
// index arithmetic folds to constants); LPZ = 0: shapes from the arguments.
// YQ: the workspace holds the quarter-plane layout (see k_qplane): a block
// takes 4 kx of the quarter-spectrum row ky' in its 4 quarters, which the
// combine on load turns into the 16 columns kx0 + kx, ky' + (ny / 4) m, and
// the inverse combine on store back into quarters.
template <class T, int LPZ, int BXC, bool YQ>
__global__ void __launch_bounds__(768) k_pencil(PencilArgs a) {
  extern __shared__ double2 smem_d[];
  T* lds = reinterpret_cast<T*>(smem_d);
  typedef typename real_of<T>::type R;
  const int b = blockIdx.y;
  // a GivensTask takes the extra last block of the grid; by_pend: only for the
  // instances with a pending update
  const bool gvb = a.gv.st && (!a.gv.by_pend || a.gv.st[b].pend);
  if (a.gv.st && blockIdx.x == gridDim.x - 1) {
    if (gvb) givens_task(a.gv.st, a.gv.run, a.gv.part, a.gv.nblk, b);
    return;
  }
  if (a.active && !a.active[b]) return;
  const int bx = LPZ ? BXC : a.bx, pz = LPZ ? (1 << LPZ) : a.pz, nz = pz / 2, nx = a.nx, ny = a.ny;
  static_assert(!YQ || (LPZ > 0 && BXC == 16), "quarter layout: compile-time pencils");
  const int ky = blockIdx.x / a.nblk_x;  // YQ: the quarter-spectrum row ky'
  const int kx0 = (blockIdx.x - ky * a.nblk_x) * (YQ ? 4 : bx);
  const int tid = threadIdx.x, nthr = LPZ ? pencil_threads_ct(LPZ, BXC) : (int)blockDim.x;
  const int LS = 3 * bx;
  const int lbx = LPZ ? (BXC == 16 ? 4 : BXC == 8 ? 3 : 2) : ilog2i(bx);
  T* w = vref<T>(a.w, b);
  // The data half (z < nz) is LDS elements [0, nz LS): i = z LS + c bx + kxl, at
  // most 4 per thread (3 pz bx <= 8 nthr). Loads are unconditional (clamped index)
  // and all issued before the LDS writes; the padded half (z >= nz) is not stored.
  const int nval = nz * LS;
  // compile-time shapes: nthr is a multiple of LS, so element i = tid + k nthr
  // of a thread keeps its component c0 and column ck and moves zstep planes per
  // k; its global offset (32-bit: a field has fewer than 2^31 elements) then
  // advances by a constant
  constexpr bool CT = LPZ > 0;
  static_assert(!CT || ((BXC == 16 || BXC == 8 || BXC == 4) && pencil_threads_ct(LPZ, BXC) % (3 * BXC) == 0),
                "pencil thread split");
  const int ck = tid & (bx - 1);
  const int zstep = CT ? nthr / LS : 0;
  const int c0 = CT ? (tid >> lbx) % 3 : 0, z0 = CT ? tid / LS : 0;
  const int goff0 = YQ ? (c0 * nz + z0) * ny * nx + ky * 4 * nx + kx0 * 4 + qp_pos(ck)
                      : ((c0 * nz + z0) * ny + ky) * nx + kx0 + ck,
            gstep = zstep * ny * nx;
  // compile-time shapes: the data stays in registers, where the forward
  // transform's first pass and the readout partial sums take it (elements
  // z0 + k zstep of sequence (c0, ck) are exactly that pass's inputs)
  T buf[4];
  {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (CT) {
        buf[k] = w[goff0 + min(k, (nval - 1 - tid) / nthr) * gstep];
      } else {
        const int i = min(tid + k * nthr, nval - 1);
        const int kxl = i & (bx - 1), rest = i >> lbx;
        const int c = rest % 3, z = rest / 3;
        buf[k] = w[((long long)(c * nz + z) * ny + ky) * nx + kx0 + kxl];
      }
    }
    // the quarter spectra of the thread's quad become its 4 columns' spectra
    // (the 16 lanes of a quad group share their component and planes)
    if constexpr (YQ) {
#pragma unroll
      for (int k = 0; k < 4; ++k) buf[k] = quad_dft4<T>(buf[k], tid & 3, false);
    }
    if constexpr (!CT) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = tid + k * nthr;
        if (i < nval) lds[i] = buf[k];
      }
    }
  }
  // the padded half is never read: the first forward pass treats it as zero
  const double* tab = a.tab + (long long)b * a.tab_stride;
  TabLayout L{nx, ny};
  // LDS after the data: the phase factors of the stack response, the window
  // factors F(|l|) of the kernel multiply, E_up [bx][3] in the working
  // precision, the readout partial sums, the order constants [bx][7] and the
  // twiddles of length pz (compile-time shapes)
  const PencilLds lo(pz, bx, nthr, (int)sizeof(T));
  char* lb = reinterpret_cast<char*>(smem_d);
  T* ab = reinterpret_cast<T*>(lb + lo.fac);
  T* ftab = reinterpret_cast<T*>(lb + lo.win);
  T* eupT = reinterpret_cast<T*>(lb + lo.eup);
  double2* part = reinterpret_cast<double2*>(lb + lo.part);
  double2* ptab = reinterpret_cast<double2*>(lb + lo.ptab);
  T* twl = reinterpret_cast<T*>(lb + lo.twl);
  // the norm partials' wavefront sums (the scale of a GivensTask's input)
  __shared__ double2 gsw[GIVENS_THREADS / 64];
  // order of column kxl (the transposed operator reads the kernel at the negated order)
  auto order_of = [&](int kxl, int& mq, int& nq) {
    if constexpr (YQ) {
      mq = kx0 + (kxl >> 2); nq = ky + (ny >> 2) * brev2(kxl & 3);
    } else {
      mq = kx0 + kxl; nq = ky;
    }
    if (a.transpose) { mq = (nx - mq) & (nx - 1); nq = (ny - nq) & (ny - 1); }
  };
  if (LPZ > 0 && tid < pz) twl[tid] = reinterpret_cast<const T*>(a.tw)[pz + tid];
  // the stack response's row r of M (or of M^T) for column kxl, thread tid =
  // r bx + kxl < 3 bx: requested now, so that its latency overlaps the data
  // loads instead of following the readout's barriers
  double2 mrow[3];
  if (a.reflect && tid < 3 * bx) {
    const int kxl = tid % bx, r = tid / bx;
    int mq, nq;
    order_of(kxl, mq, nq);
    const double2* M = reinterpret_cast<const double2*>(tab + L.off_mono()) + 9LL * (nq * nx + mq);
#pragma unroll
    for (int c = 0; c < 3; ++c) mrow[c] = a.transpose ? M[3 * c + r] : M[3 * r + c];
  }
  if (tid < bx) {
    int mq, nq;
    order_of(tid, mq, nq);
    const int q = nq * nx + mq;
    const double ikb = 1.0 / tab[TS_KBG];
    const double2 bq = reinterpret_cast<const double2*>(tab + L.off_beta())[q];
    const double2 e = reinterpret_cast<const double2*>(tab + L.off_eibl())[q];
    const double sik = tab[TS_SCALE] * ikb * ikb;
    ptab[tid * 7 + 0] = bq;
    ptab[tid * 7 + 1] = cmul(bq, bq);
    ptab[tid * 7 + 2] = make_double2(e.x - 1.0, e.y);    // s e^{i beta L} - 1 at s = +1
    ptab[tid * 7 + 3] = make_double2(-e.x - 1.0, -e.y);  // and at s = -1
    ptab[tid * 7 + 4] = make_double2(tab[L.off_kx() + mq] * ikb, tab[L.off_ky() + nq] * ikb);
    // the keep flag, and kappa / k_bg (the same for every column: one FP64
    // division here instead of one per wavefront)
    ptab[tid * 7 + 5] = make_double2(tab[L.off_keep() + q], tab[TS_KAPPA] / tab[TS_KBG]);
    ptab[tid * 7 + 6] = make_double2(e.x * sik, e.y * sik);  // e^{i beta L} scale / k_bg^2 (zz term at s = +1)
  }
  // Layered-stack response of this block's orders (monolithic coupling):
  // E_up,q = M_q sum_k exp(i beta_q z_k) f_q(z_k), M_q = T_R (i dz / 2 beta) P- / (Nx Ny)
  // from the table, added back as E_up,q exp(i beta_q z_k) on every plane. The
  // transposed operator uses the negated order and M_q^T. The phases
  // exp(i beta z_k), z_k = (k + 1/2) dz, are products of two factors, k = Q a + c:
  // exp(i beta (c + 1/2) dz) exp(i beta Q a dz); the NF = Q + nz / Q factors of a
  // column are tabulated, and every use forms the same product.
  const int Q = nz < 8 ? nz : 8, NF = Q + nz / Q;
  auto phase_at = [&](int z, int kxl) { return cmul(ab[(z % Q) * bx + kxl], ab[(Q + z / Q) * bx + kxl]); };
  if (a.reflect) {
    const double2* tb = reinterpret_cast<const double2*>(tab + L.off_beta());
    const double dz = tab[TS_DZ];
    for (int i = tid; i < NF * bx; i += nthr) {
      const int kxl = i % bx, f = i / bx;
      int mq, nq;
      order_of(kxl, mq, nq);
      const double2 bq = tb[nq * nx + mq];
      ab[f * bx + kxl] = phase_exp<T>(bq, f < Q ? (f + 0.5) * dz : (double)(Q * (f - Q)) * dz);
    }
  }
  // with a GivensTask the input is the new Arnoldi vector unscaled: its scale,
  // from the norm partials the task sums (bitwise the same value), multiplies
  // the output (every step of the kernel is linear in its input)
  if (gvb) norm_wave_sums(a.gv.part + (long long)b * a.gv.nblk, a.gv.nblk, gsw);
  __syncthreads();
  // the first wavefront forms the scale (FP64 square root and division) for
  // the block; the others read it at the store, many barriers later
  __shared__ R sclw;
  if (gvb && tid < 64) {
    const R sc = (R)inv_norm_of(norm_total(gsw));
    if (tid == 0) sclw = sc;
  }
  // readout partial sums over z: thread (ch, sq) takes planes ch, ch + nch, ...
  // (read before the forward transform's first barrier, summed after its last)
  const int nch = nthr / LS;
  T ph4[4];  // compile-time shapes: the phases of the thread's planes z0 + k zstep, kept for the store
  if (a.reflect && tid < nch * LS) {
    const int sq = tid % LS, ch = tid / LS;
    const int kxl = sq & (bx - 1);
    T acc = cmake<T>(0, 0);
    if constexpr (CT) {
      // (ch, sq) = (z0, tid mod LS): this thread's own data, planes z0 + k zstep
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ph4[k] = phase_at(ch + k * nch, kxl);
        acc = cadd(acc, cmul(ph4[k], buf[k]));
      }
    } else {
      for (int z = ch; z < nz; z += nch) acc = cadd(acc, cmul(phase_at(z, kxl), lds[z * LS + sq]));
    }
    part[tid] = to_d(acc);
  }
  // window factors F(|l|) of every column (F is even in l): the FP64 work of the
  // kernel multiply once per |l| instead of once per point
  {
    const double Lw = tab[TS_L], kap_u = tab[TS_KAPPA], scale = tab[TS_SCALE];
    for (int i = tid; i < (pz / 2 + 1) * bx; i += nthr) {
      const int kxl = i % bx, la = i / bx;
      const double2* pt7 = ptab + kxl * 7;
      const bool odd = (la & 1) != 0;
      ftab[la * bx + kxl] =
          window_factor_fast<T>(pt7[0], pt7[1], pt7[odd ? 3 : 2], kap_u * la, Lw, odd ? -1.0 : 1.0, scale);
    }
  }
  const T* tw = reinterpret_cast<const T*>(a.tw);
  typedef FftCT<LPZ, 3 * BXC, 1, 3 * BXC, pencil_threads_ct(LPZ, BXC)> ZCT;
  if constexpr (LPZ > 0) {
    // radix 8 first, from the registers (its inputs t + pz/8 j, j < 4, of
    // sequence tid mod LS, t = tid / LS, are buf[j]), then the last pass
    static_assert(LPZ == 6 || LPZ == 7, "pencil lengths with a register first pass");
    stockham_pass_regin<T, 8, false, true, 8, ZCT, true>(lds, ZCT(), tid, buf);
    __syncthreads();
    if constexpr (LPZ == 7) pass_r<T, false, true, 8, ZCT, false, false, 16>(lds, ZCT(), 3, twl, tid, false, true);
    else pass_r<T, false, true, 8, ZCT, false, false, 8>(lds, ZCT(), 3, twl, tid, false, true);
  } else {
    lds_fft<T, false, true, 8, true, false>(lds, a.log2pz, LS, 1, LS, tw, tid, nthr);
  }
  // the readout of sequence tid: its partial sums in order (slot 0 is its own,
  // which no other thread reads)
  if (a.reflect && tid < LS) {
    double2 v = make_double2(0, 0);
    for (int ch = 0; ch < nch; ++ch) v = cadd(v, part[ch * LS + tid]);
    part[tid] = v;
  }

  // the points of a thread all lie in its column ck (nthr is a multiple of bx):
  // its order constants are read once, in the working precision
  const int npt = bx * pz;
  const double2* pc = ptab + ck * 7;
  const bool keep_c = pc[5].x != 0.0;
  const R kxk = (R)pc[4].x, kyk = (R)pc[4].y;
  const T tz0 = from_d<T>(pc[6]);  // e^{i beta L} scale / k_bg^2 (zz term at s = +1)
  const R kzr = (R)pc[5].y;  // kappa_l / k_bg = l kzr
  for (int pt = tid; pt < npt; pt += nthr) {
    const int l = pt >> lbx;
    int ls = (l < pz / 2) ? l : l - pz;
    const bool nyqz = (ls == -pz / 2);
    const int lq = a.transpose ? -ls : ls;
    T* p0 = lds + l * LS + 0 * bx + ck;
    T* p1 = p0 + bx;
    T* p2 = p0 + 2 * bx;
    if (!keep_c) {
      *p0 = cmake<T>(0, 0); *p1 = cmake<T>(0, 0); *p2 = cmake<T>(0, 0);
      continue;
    }
    const bool odd = (lq & 1) != 0;
    const T F = ftab[(lq < 0 ? -lq : lq) * bx + ck];
    T tz = tz0;  // s e^{i beta L} scale / k_bg^2 with s = (-1)^l
    if (odd) { tz.x = -tz.x; tz.y = -tz.y; }
    const R kzk = (R)lq * kzr;
    T v0 = *p0, v1 = *p1, v2 = *p2;
    T dxy; dxy.x = kxk * v0.x + kyk * v1.x; dxy.y = kxk * v0.y + kyk * v1.y;
    T o0, o1, o2;
    if (!nyqz) {
      T d; d.x = dxy.x + kzk * v2.x; d.y = dxy.y + kzk * v2.y;
      o0.x = v0.x - kxk * d.x; o0.y = v0.y - kxk * d.y;
      o1.x = v1.x - kyk * d.x; o1.y = v1.y - kyk * d.y;
      o2.x = v2.x - kzk * d.x; o2.y = v2.y - kzk * d.y;
    } else {
      o0.x = v0.x - kxk * dxy.x; o0.y = v0.y - kxk * dxy.y;
      o1.x = v1.x - kyk * dxy.x; o1.y = v1.y - kyk * dxy.y;
      R f = (R)1 - kzk * kzk;
      o2.x = f * v2.x; o2.y = f * v2.y;
    }
    *p0 = cmul(F, o0);
    *p1 = cmul(F, o1);
    *p2 = csub(cmul(F, o2), cmul(tz, v2));
  }
  __syncthreads();
  if (a.reflect && tid < 3 * bx) {
    // row r of M (or of M^T) times the summed readouts of column kxl (read at
    // the store, after the inverse transform's barriers)
    const int kxl = tid % bx, r = tid / bx;
    double2 o = make_double2(0, 0);
#pragma unroll
    for (int c = 0; c < 3; ++c) o = cadd(o, cmul(mrow[c], part[c * bx + kxl]));
    eupT[kxl * 3 + r] = from_d<T>(o);
  }
  const int nst = 3 * nz * bx;
  if constexpr (CT) {
    // the inverse transform's last pass leaves the kept half in registers, and
    // the thread that forms output t + 16 j of sequence s stores it: last pass
    // of radix R (8 for pz = 128, 4 for pz = 64) has stride pz / R = 16 and
    // 8 / R butterflies b = tid + i nthr per thread, b = t LS + s
    T out[4];
    lds_fft_tab_regout<T, true, true, 8, ZCT, true, 4>(lds, ZCT(), twl, tid, out);
    const R scl = gvb ? sclw : (R)1;
    constexpr int RL = LPZ == 7 ? 8 : 4, NBL = 8 / RL, PL = (1 << LPZ) / RL;
    static_assert(LPZ == 6 || LPZ == 7, "pencil lengths with a register last pass");
    // output plane t + PL j of butterfly i is the thread's loaded plane z0 + k zstep,
    // k = i + j PL / zstep (t = z0 + i zstep): its phase is ph4[k]
    constexpr int ZST = pencil_threads_ct(LPZ, BXC) / (3 * BXC);
    static_assert(PL % ZST == 0 && (NBL - 1) + (RL / 2 - 1) * (PL / ZST) < 4, "store planes are the loaded planes");
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
      const int bfl = tid + i * nthr, t = bfl / LS, sq = bfl - t * LS;
      const int c = sq >> lbx, kxl = sq & (bx - 1);
      const T e = eupT[kxl * 3 + c];
#pragma unroll
      for (int j = 0; j < RL / 2; ++j) {
        const int z = t + PL * j;
        T v = out[i * (RL / 2) + j];
        if (a.reflect) v = cadd(v, cmul(e, ph4[i + j * (PL / ZST)]));
        if (gvb) v = cscale(v, scl);
        if constexpr (YQ) {
          // back to quarter spectra across the quad (kxl = tid mod 16)
          v = quad_dft4<T>(v, kxl & 3, true);
          w[(c * nz + z) * ny * nx + ky * 4 * nx + kx0 * 4 + qp_pos(kxl)] = v;
        } else {
          w[((c * nz + z) * ny + ky) * nx + kx0 + kxl] = v;
        }
      }
    }
  } else {
    lds_fft<T, true, true, 8, false, true>(lds, a.log2pz, LS, 1, LS, tw, tid, nthr);
    const R scl = gvb ? sclw : (R)1;
    for (int i = tid; i < nst; i += nthr) {
      const int kxl = i & (bx - 1);
      const int rest = i >> lbx;
      const int c = rest % 3;
      const int z = rest / 3;
      T v = lds[z * LS + c * bx + kxl];
      if (a.reflect) v = cadd(v, cmul(eupT[kxl * 3 + c], phase_at(z, kxl)));
      if (gvb) v = cscale(v, scl);
      w[((long long)(c * nz + z) * ny + ky) * nx + kx0 + kxl] = v;
    }
  }
}

template <class T>
void launch_pencil(const PencilArgs& a, int nbatch, int nthr, size_t lds, hipStream_t s) {
  // + the GivensTask block; the quarter layout has ny / 4 block rows
  dim3 grid(a.nblk_x * (a.yq ? a.ny / 4 : a.ny) + (a.gv.st ? 1 : 0), nbatch);
  if (a.gv.st && nthr < GIVENS_THREADS) givens_block_too_small("k_pencil", nthr);
  auto go = [&](auto kern) {
    allow_lds(reinterpret_cast<const void*>(kern), lds);
    hipLaunchKernelGGL(kern, grid, dim3(nthr), lds, s, a);
  };
  if (a.yq) {
    if (a.bx == 16 && a.pz == 128 && nthr == pencil_threads_ct(7, 16)) return go(k_pencil<T, 7, 16, true>);
    if (a.bx == 16 && a.pz == 64 && nthr == pencil_threads_ct(6, 16)) return go(k_pencil<T, 6, 16, true>);
    std::fprintf(stderr, "psfd: internal error: quarter-plane pencil on an unsupported shape\n");
    std::abort();
  }
  if (a.bx == 16 && a.pz == 128 && nthr == pencil_threads_ct(7, 16)) return go(k_pencil<T, 7, 16, false>);
  if (a.bx == 16 && a.pz == 64 && nthr == pencil_threads_ct(6, 16)) return go(k_pencil<T, 6, 16, false>);
  go(k_pencil<T, 0, 16, false>);
}
template void launch_pencil<float2>(const PencilArgs&, int, int, size_t, hipStream_t);
template void launch_pencil<double2>(const PencilArgs&, int, int, size_t, hipStream_t);

// the operator apply's shapes that take the quarter-plane kernels and the
// quarter-layout pencil (FP32 128 x 128 planes, compile-time pencil)
bool qplane_shape(int nx, int ny, int nz, int pz, int bx, int nthr, size_t esz) {
  return nx == ny && (nx == 128 || (nx == 256 && esz == 8)) && nz > 0 && bx == 16 &&
         ((pz == 128 && nthr == pencil_threads_ct(7, 16)) || (pz == 64 && nthr == pencil_threads_ct(6, 16)));
}

// -------------------------------------------------------------------------
// Per-order kernels of the background-field outer loop (FP64)
// -------------------------------------------------------------------------
__global__ void k_readout(int nx, int ny, int nz, VecRef spec, const double* tab_all, long long tab_stride,
                          double2* adn_all, double2* aup_all, long long ostride, const int* active) {
  const int b = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int nxny = nx * ny;
  if (q >= nxny || (active && !active[b])) return;
  const double* tab = tab_all + (long long)b * tab_stride;
  TabLayout L{nx, ny};
  const double2* f = vref<double2>(spec, b);
  const double2 beta = reinterpret_cast<const double2*>(tab + L.off_beta())[q];
  const double dz = tab[TS_DZ], T = tab[TS_T], kbg = tab[TS_KBG];
  double2 dn[3] = {{0, 0}, {0, 0}, {0, 0}}, up[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int k = 0; k < nz; ++k) {
    const double zk = (k + 0.5) * dz;
    double2 pd = cexp_i(make_double2(beta.x * zk, beta.y * zk));
    double2 pu = cexp_i(make_double2(beta.x * (T - zk), beta.y * (T - zk)));
    for (int c = 0; c < 3; ++c) {
      double2 v = f[((long long)c * nz + k) * nxny + q];
      dn[c] = cadd(dn[c], cmul(pd, v));
      up[c] = cadd(up[c], cmul(pu, v));
    }
  }
  double2* adn = adn_all + (long long)b * ostride + 3LL * q;
  double2* aup = aup_all + (long long)b * ostride + 3LL * q;
  if (tab[L.off_keep() + q] == 0.0) {
    for (int c = 0; c < 3; ++c) { adn[c] = make_double2(0, 0); aup[c] = make_double2(0, 0); }
    return;
  }
  // factor i dz / (2 beta) / (Nx Ny)
  double2 fac = cdiv(make_double2(0.0, dz * tab[TS_INVNXNY]), make_double2(2.0 * beta.x, 2.0 * beta.y));
  const double kx = tab[L.off_kx() + (q % nx)], ky = tab[L.off_ky() + (q / nx)];
  const double ik2 = 1.0 / (kbg * kbg);
  for (int dir = 0; dir < 2; ++dir) {
    double2* acc = dir == 0 ? dn : up;
    // P = I - k k^T / kbg^2 with k = (kx, ky, -+beta) (bilinear)
    double2 kz = dir == 0 ? make_double2(-beta.x, -beta.y) : beta;
    double2 kv[3] = {make_double2(kx, 0), make_double2(ky, 0), kz};
    double2 d = cadd(cadd(cmul(kv[0], acc[0]), cmul(kv[1], acc[1])), cmul(kv[2], acc[2]));
    double2 o[3];
    for (int c = 0; c < 3; ++c) o[c] = cmul(fac, csub(acc[c], cscale(cmul(kv[c], d), ik2)));
    double2* dst = dir == 0 ? adn : aup;
    for (int c = 0; c < 3; ++c) dst[c] = o[c];
  }
}

void launch_readout(int nx, int ny, int nz, VecRef spec, const double* tab, long long tab_stride,
                    double2* adn, double2* aup, long long ostride, const int* active, int nbatch, hipStream_t s) {
  int nxny = nx * ny;
  dim3 grid((nxny + 255) / 256, nbatch);
  hipLaunchKernelGGL(k_readout, grid, dim3(256), 0, s, nx, ny, nz, spec, tab, tab_stride, adn, aup, ostride, active);
}

__global__ void k_reflect(int nx, int ny, const double* tab_all, long long tab_stride, const double2* adn_all,
                          double2* eup_all, long long ostride, double* part, const int* active) {
  __shared__ double sd[256], sn[256];
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int nxny = nx * ny;
  const double* tab = tab_all + (long long)b * tab_stride;
  TabLayout L{nx, ny};
  double d2 = 0, n2 = 0;
  if (q < nxny) {
    const double2* adn = adn_all + (long long)b * ostride + 3LL * q;
    double2* eup = eup_all + (long long)b * ostride + 3LL * q;
    double2 e[3] = {adn[0], adn[1], adn[2]};
    if (q == (int)tab[TS_INCQ])
      for (int c = 0; c < 3; ++c) e[c] = cadd(e[c], make_double2(tab[TS_EINC + 2 * c], tab[TS_EINC + 2 * c + 1]));
    const double2* tr = reinterpret_cast<const double2*>(tab + L.off_tr()) + 9LL * q;
    for (int i = 0; i < 3; ++i) {
      double2 v = cadd(cadd(cmul(tr[3 * i], e[0]), cmul(tr[3 * i + 1], e[1])), cmul(tr[3 * i + 2], e[2]));
      d2 += cabs2(csub(v, eup[i]));
      n2 += cabs2(v);
      eup[i] = v;
    }
  }
  sd[threadIdx.x] = d2;
  sn[threadIdx.x] = n2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) { sd[threadIdx.x] += sd[threadIdx.x + st]; sn[threadIdx.x] += sn[threadIdx.x + st]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((long long)b * gridDim.x + blockIdx.x) * 2] = sd[0];
    part[((long long)b * gridDim.x + blockIdx.x) * 2 + 1] = sn[0];
  }
}

void launch_reflect(int nx, int ny, const double* tab, long long tab_stride, const double2* adn,
                    double2* eup, long long ostride, double* part, int nblk, const int* active, int nbatch,
                    hipStream_t s) {
  dim3 grid(nblk, nbatch);
  hipLaunchKernelGGL(k_reflect, grid, dim3(256), 0, s, nx, ny, tab, tab_stride, adn, eup, ostride, part, active);
}

__global__ void k_adjoint_source(int nx, int ny, const double* tab_all, long long tab_stride, const double2* g_all,
                                 double2* bdn_all, double2* bup_all, long long ostride) {
  const int b = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nx * ny) return;
  const double* tab = tab_all + (long long)b * tab_stride;
  TabLayout L{nx, ny};
  const long long o = (long long)b * ostride + 3LL * q;
  double2* bdn = bdn_all + o;
  double2* bup = bup_all + o;
  if (tab[L.off_keep() + q] == 0.0) {
    for (int i = 0; i < 3; ++i) { bdn[i] = make_double2(0, 0); bup[i] = make_double2(0, 0); }
    return;
  }
  const double2 beta = reinterpret_cast<const double2*>(tab + L.off_beta())[q];
  const double T = tab[TS_T], dz = tab[TS_DZ], kbg = tab[TS_KBG];
  const double2 fac = cscale(cdiv(make_double2(0.0, dz), make_double2(2.0 * beta.x, 2.0 * beta.y)), tab[TS_INVNXNY]);
  const double2 ph = cexp_i(make_double2(beta.x * T, beta.y * T));
  const double2* tr = reinterpret_cast<const double2*>(tab + L.off_tr()) + 9LL * q;
  // c = conj(G): the cotangent in the convention dL/dRe a + i dL/dIm a
  double2 c[3], v[3], t[3];
  for (int i = 0; i < 3; ++i) c[i] = make_double2(g_all[o + i].x, -g_all[o + i].y);
  for (int i = 0; i < 3; ++i) v[i] = cmul(ph, c[i]);
  for (int r = 0; r < 3; ++r) t[r] = cadd(cadd(cmul(tr[r], v[0]), cmul(tr[3 + r], v[1])), cmul(tr[6 + r], v[2]));
  const double ik2 = 1.0 / (kbg * kbg);
  const double kx = tab[L.off_kx() + (q % nx)], ky = tab[L.off_ky() + (q / nx)];
  for (int dir = 0; dir < 2; ++dir) {
    const double2* in = dir == 0 ? t : c;
    double2 kz = dir == 0 ? make_double2(-beta.x, -beta.y) : beta;
    double2 kv[3] = {make_double2(kx, 0), make_double2(ky, 0), kz};
    double2 d = cadd(cadd(cmul(kv[0], in[0]), cmul(kv[1], in[1])), cmul(kv[2], in[2]));
    double2* dst = dir == 0 ? bdn : bup;
    for (int i = 0; i < 3; ++i) dst[i] = cmul(fac, csub(in[i], cscale(cmul(kv[i], d), ik2)));
  }
}

void launch_adjoint_source(int nx, int ny, const double* tab, long long tab_stride, const double2* c,
                           double2* bdn, double2* bup, long long ostride, int nbatch, hipStream_t s) {
  dim3 grid((nx * ny + 255) / 256, nbatch);
  hipLaunchKernelGGL(k_adjoint_source, grid, dim3(256), 0, s, nx, ny, tab, tab_stride, c, bdn, bup, ostride);
}

__global__ void k_gradient(long long N, const double* tab_all, long long tab_stride, const double2* lam_all,
                           const double2* u_all, long long n3stride, double2* grad_all, long long gstride) {
  const int b = blockIdx.y;
  const double k0sq = tab_all[(long long)b * tab_stride + TS_K0SQ];
  const double2* lam = lam_all + (long long)b * n3stride;
  const double2* u = u_all + (long long)b * n3stride;
  double2* g = grad_all + (long long)b * gstride;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (long long)gridDim.x * blockDim.x) {
    double2 t = make_double2(0, 0);
    for (int c = 0; c < 3; ++c) t = cadd(t, cmul(lam[c * N + r], u[c * N + r]));
    g[r] = make_double2(k0sq * t.x, -k0sq * t.y);
  }
}

void launch_gradient(long long N, const double* tab, long long tab_stride, const double2* lam, const double2* u,
                     long long n3stride, double2* grad, long long gstride, int nbatch, hipStream_t s) {
  int nb = (int)((N + 255) / 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_gradient, dim3(nb, nbatch), dim3(256), 0, s, N, tab, tab_stride, lam, u, n3stride, grad, gstride);
}

__global__ void k_orders(int nx, int ny, const double* tab_all, long long tab_stride, const double2* eup_all,
                         const double2* aup_all, double2* ord_all, long long ostride) {
  const int b = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nx * ny) return;
  const double* tab = tab_all + (long long)b * tab_stride;
  TabLayout L{nx, ny};
  double2 beta = reinterpret_cast<const double2*>(tab + L.off_beta())[q];
  double T = tab[TS_T];
  double2 ph = cexp_i(make_double2(beta.x * T, beta.y * T));
  const long long o = (long long)b * ostride + 3LL * q;
  for (int c = 0; c < 3; ++c) ord_all[o + c] = cadd(cmul(eup_all[o + c], ph), aup_all[o + c]);
}

void launch_orders(int nx, int ny, const double* tab, long long tab_stride, const double2* eup,
                   const double2* aup, double2* orders, long long ostride, int nbatch, hipStream_t s) {
  dim3 grid((nx * ny + 255) / 256, nbatch);
  hipLaunchKernelGGL(k_orders, grid, dim3(256), 0, s, nx, ny, tab, tab_stride, eup, aup, orders, ostride);
}

}  // namespace psfd
