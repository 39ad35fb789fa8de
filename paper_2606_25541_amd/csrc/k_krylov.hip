// Krylov kernels of restarted GMRES (Saad & Schultz) with classical Gram-Schmidt
// (one pass; severe cancellation ends the cycle): multi-dot products of the basis
// against the new vector, fused update + norm, the Givens step of the new Hessenberg column,
// back substitution, the solution update and the device-side cycle control.
// Vector data may be FP32 or FP64; per-thread and per-wavefront partial sums
// are in the vector precision, every sum across wavefronts and blocks is in
// FP64 and in a fixed order (bitwise reproducible, independent of the batch).
#include "krylov.hpp"
#include "givens.hpp"
#include "../../include/psfd.h"

namespace psfd {

static constexpr int KB = 256;  // threads per block of the vector kernels
static_assert(KB == GIVENS_THREADS, "the update-final block is the Givens task's block");
static constexpr int VG = 4;    // basis vectors loaded together in the Gram-Schmidt passes
// threads per block of the projection pass: its accumulators fill 66 registers
// in FP32 (1024 threads fit) and 132 in FP64 (512 threads); DotBlocks<T> blocks
// per instance keep the thread count the same
template <class T> struct DotThreads { static constexpr int value = sizeof(T) == 8 ? 1024 : 512; };

PSFD_D double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum of cnt (<= MAXM + 1) complex values held per thread; thread 0..
// of the block end with the totals in sm_out (LDS), valid after the call.
template <int NV>
PSFD_D void block_sum(double2 (&acc)[NV], int cnt, double2* sm /*[KB/64][NV]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < cnt) {
      double re = wave_sum(acc[i].x), im = wave_sum(acc[i].y);
      if (lane == 0) sm[wave * NV + i] = make_double2(re, im);
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double2 t = sm[threadIdx.x];
    for (int wv = 1; wv < KB / 64; ++wv) t = cadd(t, sm[wv * NV + threadIdx.x]);
    sm[threadIdx.x] = t;
  }
  __syncthreads();
}

// block-wide sums in the vector precision (wave shuffles), combined across the
// waves of the block in FP64; totals land in sm[0..cnt)
template <class T> PSFD_D T wave_sum_c(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

template <class T, int NV, int NW = KB / 64>
PSFD_D void block_sum_c(T (&acc)[NV], int cnt, double2* sm /*[NW][NV]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < cnt) {
      T r = wave_sum_c(acc[i]);
      if (lane == 0) sm[wave * NV + i] = to_d(r);
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double2 t = sm[threadIdx.x];
    for (int wv = 1; wv < NW; ++wv) t = cadd(t, sm[wv * NV + threadIdx.x]);
    sm[threadIdx.x] = t;
  }
  __syncthreads();
}

// element pairs: FP32 complex bases are read two at a time (16-byte loads)
template <class T> struct Pair { T a, b; };
template <class T> PSFD_D Pair<T> ld2(const T* p, long long e2) {
  Pair<T> r;
  if constexpr (sizeof(T) == 8) {
    const float4 v = reinterpret_cast<const float4*>(p)[e2];
    r.a = make_float2(v.x, v.y);
    r.b = make_float2(v.z, v.w);
  } else {
    r.a = p[2 * e2];
    r.b = p[2 * e2 + 1];
  }
  return r;
}
template <class T> PSFD_D void st2(T* p, long long e2, Pair<T> v) {
  if constexpr (sizeof(T) == 8) {
    reinterpret_cast<float4*>(p)[e2] = make_float4(v.a.x, v.a.y, v.b.x, v.b.y);
  } else {
    p[2 * e2] = v.a;
    p[2 * e2 + 1] = v.b;
  }
}
// acc += conj(v) w
template <class T> PSFD_D void cfma_conj(T& acc, T v, T w) {
  acc.x += v.x * w.x + v.y * w.y;
  acc.y += v.x * w.y - v.y * w.x;
}

// Classical Gram-Schmidt, projections: per-block partial sums of h_i = <v_i, w>
// (i <= j) and of ||w||^2 for the new vector w = v_{j+1}, stored value-major
// (part[b][i][block]) for the update kernel, whose blocks each sum them. n must
// be even (fields are 3 nx ny nz complex with nx >= 4).
template <class T>
__global__ void __launch_bounds__(DotThreads<T>::value) k_dots(const T* V, long long ldv, long long bsv, long long n,
                                                               GState* st, const int* run, double2* part, int jh) {
  constexpr int KBD = DotThreads<T>::value;
  __shared__ double2 sm[(KBD / 64) * (MAXM + 1)];
  const int b = blockIdx.y;
  // the flag and the Krylov index are read together (one memory latency); a
  // caller whose instances all stand at the same step passes it as jh >= 0
  const int rb = run[b], jd = jh >= 0 ? jh : st[b].j;
  asm volatile("" ::"s"(rb), "s"(jd));
  if (!rb) return;
  const int cnt = jd + 1;
  const T* Vb = V + (long long)b * bsv;
  const T* wb = Vb + (long long)cnt * ldv;
  T acc[MAXM + 1];
#pragma unroll
  for (int i = 0; i < MAXM + 1; ++i) acc[i] = cmake<T>(0, 0);
  const long long n2 = n >> 1;
  for (long long e = (long long)blockIdx.x * KBD + threadIdx.x; e < n2; e += (long long)gridDim.x * KBD) {
    const Pair<T> wv = ld2(wb, e);
    // basis vectors in groups of VG: the loads of a group are unconditional
    // (index clamped to the last vector) so that they are all in flight together
#pragma unroll
    for (int i0 = 0; i0 < MAXM; i0 += VG) {
      if (i0 < cnt) {
        Pair<T> v[VG];
#pragma unroll
        for (int u = 0; u < VG; ++u) v[u] = ld2(Vb + (long long)min(i0 + u, cnt - 1) * ldv, e);
#pragma unroll
        for (int u = 0; u < VG; ++u) {
          if (i0 + u < cnt) {
            cfma_conj(acc[i0 + u], v[u].a, wv.a);
            cfma_conj(acc[i0 + u], v[u].b, wv.b);
          }
        }
      }
    }
    // ||w||^2 in the slot after the last dot
#pragma unroll
    for (int i = 1; i < MAXM + 1; ++i)
      if (i == cnt) acc[i].x += wv.a.x * wv.a.x + wv.a.y * wv.a.y + wv.b.x * wv.b.x + wv.b.y * wv.b.y;
  }
  block_sum_c<T, MAXM + 1, KBD / 64>(acc, cnt + 1, sm);
  if ((int)threadIdx.x <= cnt)
    part[((long long)b * PSTR + threadIdx.x) * gridDim.x + blockIdx.x] = sm[threadIdx.x];
}

template <class T>
void krylov_dots(const T* V, long long ldv, long long bsv, long long n, GState* st, const int* run,
                 double2* part, int nbatch, hipStream_t s, int jh) {
  hipLaunchKernelGGL((k_dots<T>), dim3(DotBlocks<T>::value, nbatch), dim3(DotThreads<T>::value), 0, s, V, ldv, bsv, n,
                     st, run, part, jh);
}

// ---------------------------------------------------------------------------
// Classical Gram-Schmidt, update: w -= sum_{i<=j} h_i v_i, with per-block
// partial sums of ||w||^2 afterwards.
template <class T>
__global__ void __launch_bounds__(KB) k_update(T* V, long long ldv, long long bsv, long long n, GState* st,
                                               const int* run, const double2* dpart, double2* part, int jh) {
  __shared__ double2 sm[(KB / 64) * 1];
  __shared__ double2 hsum[MAXM + 2];
  __shared__ T hs[MAXM + 1];
  const int b = blockIdx.y;
  const int rb = run[b], jd = jh >= 0 ? jh : st[b].j;
  asm volatile("" ::"s"(rb), "s"(jd));
  if (!rb) return;
  const int cnt = jd + 1;
  // slot scale of this thread's projection (v_i = sc_i slot_i, sc real)
  const double scv = st[b].sc[min((int)threadIdx.x, MAXM)];
  // projections: every block sums the DotBlocks<T> partials of k_dots itself, in
  // a fixed order (wave w takes values w, w + 4, ...; lane l partials l, l + 64,
  // ...). The loads of up to RU values per wave are issued together (clamped
  // value index), so the sum waits for one memory latency.
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NBD = DotBlocks<T>::value, PL = NBD / 64, NW = KB / 64;
    constexpr int RU = 12 / PL > 0 ? 12 / PL : 1;
    const double2* pb = dpart + (long long)b * PSTR * NBD;
    for (int i0 = wave; i0 <= cnt; i0 += NW * RU) {
      double2 pv[RU][PL];
#pragma unroll
      for (int r = 0; r < RU; ++r) {
        const int i = min(i0 + r * NW, cnt);
#pragma unroll
        for (int k = 0; k < PL; ++k) pv[r][k] = pb[(long long)i * NBD + lane + 64 * k];
      }
#pragma unroll
      for (int r = 0; r < RU; ++r) {
        if (i0 + r * NW <= cnt) {
          double2 t = make_double2(0, 0);
#pragma unroll
          for (int k = 0; k < PL; ++k) t = cadd(t, pv[r][k]);
          t.x = wave_sum(t.x);
          t.y = wave_sum(t.y);
          if (lane == 0) hsum[i0 + r * NW] = t;
        }
      }
    }
  }
  __syncthreads();
  GState& S = st[b];
  // h_i = <v_i, w> = sc_i <slot_i, w>; w -= sum_i h_i v_i = sum_i (h_i sc_i) slot_i
  if ((int)threadIdx.x < cnt) hs[threadIdx.x] = from_d<T>(cscale(hsum[threadIdx.x], scv * scv));
  if (blockIdx.x == 0) {
    // the projections and ||w||^2 before the update
    const int i = threadIdx.x;
    if (i < cnt) S.h[i] = cscale(hsum[i], scv);
    else if (i == cnt) S.wn2_in = hsum[i].x;
  }
  __syncthreads();
  T* Vb = V + (long long)b * bsv;
  T* wb = Vb + (long long)cnt * ldv;
  T nn[1] = {cmake<T>(0, 0)};
  const long long n2 = n >> 1;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n2; e += (long long)gridDim.x * KB) {
    T a0 = cmake<T>(0, 0), a1 = cmake<T>(0, 0);
    Pair<T> wv = ld2(wb, e);
#pragma unroll
    for (int i0 = 0; i0 < MAXM; i0 += VG) {
      if (i0 < cnt) {
        Pair<T> v[VG];
#pragma unroll
        for (int u = 0; u < VG; ++u) v[u] = ld2(Vb + (long long)min(i0 + u, cnt - 1) * ldv, e);
#pragma unroll
        for (int u = 0; u < VG; ++u) {
          if (i0 + u < cnt) {
            const T h = hs[i0 + u];
            a0.x += h.x * v[u].a.x - h.y * v[u].a.y;
            a0.y += h.x * v[u].a.y + h.y * v[u].a.x;
            a1.x += h.x * v[u].b.x - h.y * v[u].b.y;
            a1.y += h.x * v[u].b.y + h.y * v[u].b.x;
          }
        }
      }
    }
    wv.a.x -= a0.x; wv.a.y -= a0.y;
    wv.b.x -= a1.x; wv.b.y -= a1.y;
    st2(wb, e, wv);
    nn[0].x += wv.a.x * wv.a.x + wv.a.y * wv.a.y + wv.b.x * wv.b.x + wv.b.y * wv.b.y;
  }
  block_sum_c<T, 1>(nn, 1, sm);
  if (threadIdx.x == 0) part[((long long)b * gridDim.x + blockIdx.x)] = sm[0];
}

// the Givens step of the newest column (see givens_task), one block per instance
__global__ void __launch_bounds__(KB) k_update_final(GState* st, int* run, const double2* part, int nblk) {
  givens_task(st, run, part, nblk, blockIdx.x);
}

void krylov_givens(GState* st, int* run, const double2* part, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(k_update_final, dim3(nbatch), dim3(KB), 0, s, st, run, part, RED_BLOCKS);
}

// the Givens step of the last column from its projections alone (see
// krylov_givens_proj); the partials are summed as k_update sums them. Every
// thread of the block calls it (the condition is uniform over the block).
PSFD_D void givens_proj_block(GState* st, int* run, const double2* dpart, int jh) {
  __shared__ double2 hsum[MAXM + 2];
  __shared__ double wn2s;
  const int b = blockIdx.x;
  const int rb = run[b], jd = jh >= 0 ? jh : st[b].j, mb = st[b].m;
  asm volatile("" ::"s"(rb), "s"(jd), "s"(mb));
  // jh < 0 (instances at different steps): only those at the last column
  if (!rb || (jh < 0 && jd != mb - 1)) return;
  const int cnt = jd + 1;
  const double scv = st[b].sc[min((int)threadIdx.x, MAXM)];
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NBD = DotBlocks<float2>::value, PL = NBD / 64, NW = KB / 64;
    const double2* pb = dpart + (long long)b * PSTR * NBD;
    for (int i = wave; i <= cnt; i += NW) {
      double2 pv[PL];
#pragma unroll
      for (int k = 0; k < PL; ++k) pv[k] = pb[(long long)i * NBD + lane + 64 * k];
      double2 t = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < PL; ++k) t = cadd(t, pv[k]);
      t.x = wave_sum(t.x);
      t.y = wave_sum(t.y);
      if (lane == 0) hsum[i] = t;
    }
  }
  __syncthreads();
  // h_i = sc_i <slot_i, w>; ||w - V h||^2 = ||w||^2 - sum |h_i|^2 in a fixed order
  const double2 hv = (int)threadIdx.x < cnt ? cscale(hsum[threadIdx.x], scv) : make_double2(0, 0);
  GState& S = st[b];
  if ((int)threadIdx.x < cnt) S.h[threadIdx.x] = hv;
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int i = 0; i < cnt; ++i) {
      const double2 h = cscale(hsum[i], st[b].sc[i]);
      a += h.x * h.x + h.y * h.y;
    }
    const double w2 = hsum[cnt].x;
    S.wn2_in = w2;
    wn2s = w2 - a > 0.0 ? w2 - a : 0.0;
  }
  __syncthreads();
  givens_impl<true>(st, run, nullptr, 0, b, hv, hsum[cnt].x, wn2s);
}

__global__ void __launch_bounds__(KB) k_givens_proj(GState* st, int* run, const double2* dpart, int jh) {
  givens_proj_block(st, run, dpart, jh);
}

void krylov_givens_proj(GState* st, int* run, const double2* dpart, int nbatch, hipStream_t s, int jh) {
  hipLaunchKernelGGL(k_givens_proj, dim3(nbatch), dim3(KB), 0, s, st, run, dpart, jh);
}

template <class T>
void krylov_update(T* V, long long ldv, long long bsv, long long n, GState* st, int* run,
                   const double2* dpart, double2* part, int nbatch, hipStream_t s, int jh, bool givens) {
  hipLaunchKernelGGL((k_update<T>), dim3(RED_BLOCKS, nbatch), dim3(KB), 0, s, V, ldv, bsv, n, st, (const int*)run,
                     dpart, part, jh);
  if (givens) krylov_givens(st, run, part, nbatch, s);
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// back substitution y = R^{-1} g on the upper triangle of the rotated
// Hessenberg matrix; the block stages R and g in LDS so that the single-thread
// recurrence reads no global memory
PSFD_D void solve_small_block(GState* st, const int* mask) {
  __shared__ double2 R[MAXM][MAXM], gl[MAXM + 1], yl[MAXM], cl[MAXM + 1], snl[MAXM];
  __shared__ double csl[MAXM];
  const int b = blockIdx.x;
  if (mask && !mask[b]) return;
  GState& S = st[b];
  const int k = S.ncols;
  for (int e = threadIdx.x; e < k * k; e += KB) {
    const int i = e / k, c = e - i * k;
    if (c >= i) R[i][c] = S.H[i][c];
  }
  if ((int)threadIdx.x <= k) gl[threadIdx.x] = S.g[threadIdx.x];
  if ((int)threadIdx.x < k) { csl[threadIdx.x] = S.cs[threadIdx.x]; snl[threadIdx.x] = S.sn[threadIdx.x]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double2 t = gl[i];
      for (int c = i + 1; c < k; ++c) t = csub(t, cmul(R[i][c], yl[c]));
      yl[i] = cdiv(t, R[i][i]);
    }
  }
  if (threadIdx.x == 1) {
    // r = V_{k+1} (beta e_1 - Hbar y) = V_{k+1} Q^H (g_k e_k): undo the rotations
    // G_i = [[cs, sn], [-conj(sn), cs]], last first, on g_k e_k
    for (int i = 0; i < k; ++i) cl[i] = make_double2(0, 0);
    cl[k] = gl[k];
    for (int i = k - 1; i >= 0; --i) {
      const double2 a = cl[i], c = cl[i + 1], sn = snl[i];
      const double cs = csl[i];
      cl[i] = csub(cscale(a, cs), cmul(sn, c));
      cl[i + 1] = cadd(cmul(make_double2(sn.x, -sn.y), a), cscale(c, cs));
    }
  }
  __syncthreads();
  // as coefficients of the slots, which hold v_i / sc_i
  if ((int)threadIdx.x < k) S.y[threadIdx.x] = cscale(yl[threadIdx.x], S.sc[threadIdx.x]);
  if ((int)threadIdx.x <= k) {
    double2 c = cscale(cl[threadIdx.x], S.sc[threadIdx.x]);
    // slot k still holds w = v_k / sc_k + sum_{i<k} h_i v_i: fold the update in
    if (k > 0 && S.raw_last == k && (int)threadIdx.x < k) {
      const double2 ck = cscale(cl[k], S.sc[k]);
      c = csub(c, cscale(cmul(ck, S.h[threadIdx.x]), S.sc[threadIdx.x]));
    }
    S.cres[threadIdx.x] = c;
  }
}

__global__ void __launch_bounds__(KB) k_solve_small(GState* st, const int* mask) { solve_small_block(st, mask); }

void krylov_solve_small(GState* st, const int* mask, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_small, dim3(nbatch), dim3(KB), 0, s, st, mask);
}

// the last column's Givens step from its projections, then the back
// substitution, in one launch (the block's barrier orders the state it writes
// before the reads of the second part)
__global__ void __launch_bounds__(KB) k_givens_proj_solve(GState* st, int* run, const double2* dpart, int jh,
                                                          const int* mask) {
  givens_proj_block(st, run, dpart, jh);
  __syncthreads();
  solve_small_block(st, mask);
}

void krylov_givens_proj_solve(GState* st, int* run, const double2* dpart, const int* mask, int nbatch, hipStream_t s,
                              int jh) {
  hipLaunchKernelGGL(k_givens_proj_solve, dim3(nbatch), dim3(KB), 0, s, st, run, dpart, jh, mask);
}

template <class T, class TX>
__global__ void __launch_bounds__(KB) k_lincomb_res(T* V, long long ldv, long long bsv, TX* x, long long bsx,
                                                    long long n, GState* st, const int* mask, const int* rec,
                                                    double* part) {
  __shared__ double2 ys[MAXM], cr[MAXM + 1], sm[KB / 64];
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const int k = st[b].ncols;
  const bool dor = rec[b] != 0;
  if ((int)threadIdx.x < k) ys[threadIdx.x] = st[b].y[threadIdx.x];
  if ((int)threadIdx.x <= k) cr[threadIdx.x] = st[b].cres[threadIdx.x];
  __syncthreads();
  if (k == 0) return;
  T* Vb = V + (long long)b * bsv;
  TX* xb = x + (long long)b * bsx;
  double2 acc[1] = {make_double2(0, 0)};
  const int nv = dor ? k + 1 : k;  // slots read: the cycle's basis, and slot k for the residual
  // basis vectors in groups of LG with unconditional (clamped) loads, all in
  // flight together with the x load: one group for the 9 slots of an FP32
  // GMRES(8) restart, groups of 8 for FP64 slots (the faster width for each,
  // as measured).
  // The group loop stays rolled: unrolled, the compiler keeps every coefficient
  // of the LDS tables in registers across the element loop (hundreds of VGPRs,
  // one wavefront per SIMD); rolled, each group reads its coefficients at use.
  constexpr int LG = sizeof(T) == 8 ? 9 : 8;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
    double2 sx = make_double2(0, 0), sr = make_double2(0, 0);
    const double2 xv = to_d(xb[e]);
#pragma unroll 1
    for (int i0 = 0; i0 < nv; i0 += LG) {
      T v[LG];
#pragma unroll
      for (int u = 0; u < LG; ++u) v[u] = Vb[(long long)min(i0 + u, nv - 1) * ldv + e];
#pragma unroll
      for (int u = 0; u < LG; ++u) {
        const int i = i0 + u;
        if (i < k) sx = cadd(sx, cmul(ys[i], to_d(v[u])));
        if (dor && i < nv) sr = cadd(sr, cmul(cr[i], to_d(v[u])));
      }
    }
    xb[e] = from_d<TX>(cadd(xv, sx));
    if (dor) {
      Vb[e] = from_d<T>(sr);
      acc[0].x += sr.x * sr.x + sr.y * sr.y;
    }
  }
  if (!dor) return;
  block_sum<1>(acc, 1, sm);
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = sm[0].x;
}

template <class T, class TX>
void krylov_lincomb_res(T* V, long long ldv, long long bsv, TX* x, long long bsx, long long n, GState* st,
                        const int* mask, const int* rec, double* part, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL((k_lincomb_res<T, TX>), dim3(LIN_BLOCKS, nbatch), dim3(KB), 0, s, V, ldv, bsv, x, bsx, n, st,
                     mask, rec, part);
}

__global__ void k_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                        double cancel_thr, const int* mask, int* run) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0 || (mask && !mask[b])) return;  // other instances keep their state
  GState& S = st[b];
  const double rn = sqrt(rnorm2[b]);
  S.j = 0;
  S.pend = 0;
  S.m = m;
  S.cancel_thr = cancel_thr;
  S.ncols = 0;
  S.beta = rn;
  S.g[0] = make_double2(rn, 0.0);
  for (int i = 1; i <= MAXM; ++i) S.g[i] = make_double2(0, 0);
  double t = eta * rn;
  S.target = abs_target[b] > t ? abs_target[b] : t;
  S.res = rn;
  S.conv = 0;
  S.inv_norm = rn > 0.0 ? 1.0 / rn : 0.0;  // v_0 holds r unnormalised; the first apply scales it
  S.sc[0] = S.inv_norm;
  const bool go = rn > abs_target[b] && rn > 0.0 && rn == rn;
  S.stop = go ? 0 : 1;
  run[b] = go ? 1 : 0;
}

__global__ void k_solve_init(GState* st, const double* bnorm2, const double* rtol, double* abs_target, int max_iters,
                             const int* act) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0 || !act[b]) return;
  GState& S = st[b];
  S.bnorm = sqrt(bnorm2[b]);
  abs_target[b] = rtol[b] * S.bnorm;
  S.iter_limit = S.iters + max_iters;
  S.cycles = 0;
  S.status = PSFD_OK;
  S.rel_res = 0.0;
}

void krylov_solve_init(GState* st, const double* bnorm2, const double* rtol, double* abs_target, int max_iters,
                       const int* act, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_init, dim3(nbatch), dim3(64), 0, s, st, bnorm2, rtol, abs_target, max_iters, act);
}

// sum of the nblk partials of instance b, fixed order (thread t adds partials
// t, t + KB, ..., then a fixed block tree); every thread of a KB-thread block
// calls it and gets the total
PSFD_D double sum_partials(const double* part, int nblk, int b) {
  __shared__ double2 sm[KB / 64];
  double t = 0;
  for (int k = threadIdx.x; k < nblk; k += KB) t += part[(long long)b * nblk + k];
  double2 acc[1] = {make_double2(t, 0.0)};
  block_sum<1>(acc, 1, sm);
  return sm[0].x;
}

// fp64 = false: this restart has no b - A x (the launch sequence left it out);
// an instance that asked for one keeps its request and starts no cycle
PSFD_D void cycle_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                        double cancel_thr, int every, int* act, int* tres, int* rres, int* run, int* cyc, int b,
                        bool fp64 = true) {
  cyc[b] = 0;
  run[b] = 0;
  const bool was_true = tres[b] != 0;
  tres[b] = 0;
  rres[b] = 0;
  if (!act[b]) return;
  if (was_true && !fp64) {
    tres[b] = 1;
    return;
  }
  GState& S = st[b];
  const double rn = sqrt(rnorm2[b]);
  if (!(rn == rn) || isinf(rn)) { S.status = PSFD_ERR_NONFINITE; act[b] = 0; return; }
  const bool met = rn <= abs_target[b] || S.bnorm == 0.0;
  const bool limit = S.iters >= S.iter_limit;
  if (was_true) {
    S.rel_res = S.bnorm > 0 ? rn / S.bnorm : 0.0;
    if (met) { act[b] = 0; return; }
    if (limit) { S.status = PSFD_NOT_CONVERGED; act[b] = 0; return; }
  } else if (met || limit) {
    tres[b] = 1;  // decide on b - A x at the next restart, without a cycle now
    return;
  }
  S.j = 0;
  S.pend = 0;
  S.m = m;
  S.cancel_thr = cancel_thr;
  S.ncols = 0;
  S.beta = rn;
  S.g[0] = make_double2(rn, 0.0);
  for (int i = 1; i <= MAXM; ++i) S.g[i] = make_double2(0, 0);
  const double t = eta * rn;
  S.target = abs_target[b] > t ? abs_target[b] : t;
  S.res = rn;
  S.conv = 0;
  S.stop = 0;
  S.inv_norm = 1.0 / rn;  // v_0 holds r unnormalised; the first apply scales it
  S.sc[0] = S.inv_norm;
  S.cycles += 1;
  S.since_true = was_true ? 0 : S.since_true + 1;
  const bool next_true = S.since_true + 1 >= every || rn <= 2.0 * abs_target[b];
  tres[b] = next_true ? 1 : 0;
  rres[b] = next_true ? 0 : 1;
  cyc[b] = 1;
  run[b] = 1;
}

__global__ void k_cycle_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                              double cancel_thr, int every, int* act, int* tres, int* rres, int* run, int* cyc) {
  if (threadIdx.x == 0) cycle_start(st, rnorm2, abs_target, eta, m, cancel_thr, every, act, tres, rres, run, cyc,
                                    blockIdx.x);
}

// the same, with ||r||^2 summed here from the partials of b - A x (tpart,
// RED_BLOCKS per instance) or of the basis residual (lpart, LIN_BLOCKS), in the
// order of k_sum_part, and stored to rnorm2. fp64: whether b - A x was formed
// at this restart (see cycle_start). With host (host memory mapped for the
// device) the instance's flags are also written there.
__global__ void __launch_bounds__(KB) k_cycle_start_sum(GState* st, double* rnorm2, const double* tpart,
                                                        const double* lpart, const double* abs_target, double eta,
                                                        int m, double cancel_thr, int every, int* act, int* tres,
                                                        int* rres, int* run, int* cyc, int fp64, HostFlags* host) {
  const int b = blockIdx.x;
  const int t = tres[b], r = rres[b];
  const bool have = (t && fp64) || (!t && r);
  if (have) {
    const double n2 = t ? sum_partials(tpart, RED_BLOCKS, b) : sum_partials(lpart, LIN_BLOCKS, b);
    if (threadIdx.x == 0) rnorm2[b] = n2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cycle_start(st, rnorm2, abs_target, eta, m, cancel_thr, every, act, tres, rres, run, cyc, b, fp64 != 0);
    if (host) {
      host[b].act = act[b];
      host[b].want = tres[b];
      if (have && act[b]) {
        host[b].ratio = abs_target[b] > 0.0 ? sqrt(rnorm2[b]) / abs_target[b] : 0.0;
        host[b].cycles = st[b].cycles;
      }
    }
  }
}

void krylov_cycle_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                        double cancel_thr, int every, int* act, int* tres, int* rres, int* run, int* cyc,
                        int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_start, dim3(nbatch), dim3(64), 0, s, st, rnorm2, abs_target, eta, m, cancel_thr, every,
                     act, tres, rres, run, cyc);
}

void krylov_cycle_start_sum(GState* st, double* rnorm2, const double* tpart, const double* lpart,
                            const double* abs_target, double eta, int m, double cancel_thr, int every, int* act,
                            int* tres, int* rres, int* run, int* cyc, int nbatch, hipStream_t s, HostFlags* host,
                            bool fp64) {
  hipLaunchKernelGGL(k_cycle_start_sum, dim3(nbatch), dim3(KB), 0, s, st, rnorm2, tpart, lpart, abs_target, eta, m,
                     cancel_thr, every, act, tres, rres, run, cyc, fp64 ? 1 : 0, host);
}



void krylov_start(GState* st, const double* rnorm2, const double* abs_target, double eta, int m,
                  double cancel_thr, const int* mask, int* run, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(k_start, dim3(nbatch), dim3(64), 0, s, st, rnorm2, abs_target, eta, m, cancel_thr, mask, run);
}

// ---------------------------------------------------------------------------
template <class TO, class TX, class TY>
__global__ void __launch_bounds__(KB) k_axpby(TO* out, const TX* x, const TY* y, double a, double c, long long n,
                                              long long bs, const int* mask) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const long long o = (long long)b * bs;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
    double2 xv = to_d(x[o + e]);
    double2 r = make_double2(a * xv.x, a * xv.y);
    if (y) { double2 yv = to_d(y[o + e]); r.x += c * yv.x; r.y += c * yv.y; }
    out[o + e] = from_d<TO>(r);
  }
}

template <class TO, class TX, class TY>
void vec_axpby(TO* out, const TX* x, const TY* y, double a, double c, long long n, long long bstride,
               const int* mask, int nbatch, hipStream_t s) {
  int nb = (int)((n + KB - 1) / KB);
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL((k_axpby<TO, TX, TY>), dim3(nb, nbatch), dim3(KB), 0, s, out, x, y, a, c, n, bstride, mask);
}

template <class T>
__global__ void __launch_bounds__(KB) k_norm2(const T* x, long long n, long long bs, double* part, const int* mask) {
  __shared__ double2 sm[KB / 64];
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const T* xb = x + (long long)b * bs;
  double2 acc[1] = {make_double2(0, 0)};
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
    double2 v = to_d(xb[e]);
    acc[0].x += v.x * v.x + v.y * v.y;
  }
  block_sum<1>(acc, 1, sm);
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = sm[0].x;
}

__global__ void __launch_bounds__(KB) k_sum_part(const double* part, int nblk, double* out, const int* mask) {
  const int b = blockIdx.x;
  if (mask && !mask[b]) return;
  const double t = sum_partials(part, nblk, b);
  if (threadIdx.x == 0) out[b] = t;
}

void krylov_sum_norm(const double* part, double* n2, const int* mask, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_part, dim3(nbatch), dim3(KB), 0, s, part, LIN_BLOCKS, n2, mask);
}

template <class T>
void vec_norm2(const T* x, long long n, long long bstride, double* part, double* out, const int* mask,
               int nbatch, hipStream_t s) {
  hipLaunchKernelGGL((k_norm2<T>), dim3(RED_BLOCKS, nbatch), dim3(KB), 0, s, x, n, bstride, part, mask);
  hipLaunchKernelGGL(k_sum_part, dim3(nbatch), dim3(KB), 0, s, (const double*)part, RED_BLOCKS, out, mask);
}

template <class T>
__global__ void __launch_bounds__(KB) k_diff2(const T* x, const T* y, long long n, long long bs, double* part) {
  __shared__ double2 sm[(KB / 64) * 2];
  const int b = blockIdx.y;
  const T* xb = x + (long long)b * bs;
  const T* yb = y + (long long)b * bs;
  double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
    double2 u = to_d(xb[e]), v = to_d(yb[e]);
    double2 d = csub(u, v);
    acc[0].x += d.x * d.x + d.y * d.y;
    acc[1].x += u.x * u.x + u.y * u.y;
  }
  block_sum<2>(acc, 2, sm);
  if (threadIdx.x == 0) {
    part[((long long)b * gridDim.x + blockIdx.x) * 2] = sm[0].x;
    part[((long long)b * gridDim.x + blockIdx.x) * 2 + 1] = sm[1].x;
  }
}

// the two sums of k_diff2's partials, fixed order
__global__ void __launch_bounds__(KB) k_sum_part2(const double* part, int nblk, double* out) {
  __shared__ double2 sm[(KB / 64) * 2];
  const int b = blockIdx.x;
  double t0 = 0, t1 = 0;
  for (int k = threadIdx.x; k < nblk; k += KB) {
    t0 += part[((long long)b * nblk + k) * 2];
    t1 += part[((long long)b * nblk + k) * 2 + 1];
  }
  double2 acc[2] = {make_double2(t0, 0.0), make_double2(t1, 0.0)};
  block_sum<2>(acc, 2, sm);
  if (threadIdx.x == 0) {
    out[2 * b] = sm[0].x;
    out[2 * b + 1] = sm[1].x;
  }
}

template <class T>
void vec_diff2(const T* x, const T* y, long long n, long long bstride, double* part, double* out,
               int nbatch, hipStream_t s) {
  hipLaunchKernelGGL((k_diff2<T>), dim3(RED_BLOCKS, nbatch), dim3(KB), 0, s, x, y, n, bstride, part);
  hipLaunchKernelGGL(k_sum_part2, dim3(nbatch), dim3(KB), 0, s, (const double*)part, RED_BLOCKS, out);
}

// r = b - Ax in FP64 with per-block partial sums of ||r||^2, stored only as the
// unnormalised first basis vector v0 in the working precision
template <class T>
__global__ void __launch_bounds__(KB) k_resid(const double2* bv, const double2* ax, T* v0, long long n, long long bs,
                                              long long bsv, double* part, const int* mask) {
  __shared__ double2 sm[KB / 64];
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const double2* bb = bv + (long long)b * bs;
  const double2* ab = ax + (long long)b * bs;
  T* vb = v0 + (long long)b * bsv;
  double2 acc[1] = {make_double2(0, 0)};
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < n; e += (long long)gridDim.x * KB) {
    const double2 r = csub(bb[e], ab[e]);
    vb[e] = from_d<T>(r);
    acc[0].x += r.x * r.x + r.y * r.y;
  }
  block_sum<1>(acc, 1, sm);
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = sm[0].x;
}

template <class T>
void krylov_residual(const double2* bv, const double2* ax, T* v0, long long n, long long bs, long long bsv,
                     double* part, double* n2, const int* mask, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL((k_resid<T>), dim3(RED_BLOCKS, nbatch), dim3(KB), 0, s, bv, ax, v0, n, bs, bsv, part, mask);
  hipLaunchKernelGGL(k_sum_part, dim3(nbatch), dim3(KB), 0, s, (const double*)part, RED_BLOCKS, n2, mask);
}

template <class T>
void krylov_residual_parts(const double2* bv, const double2* ax, T* v0, long long n, long long bs, long long bsv,
                           double* part, const int* mask, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL((k_resid<T>), dim3(RED_BLOCKS, nbatch), dim3(KB), 0, s, bv, ax, v0, n, bs, bsv, part, mask);
}

// ---- instantiations ----------------------------------------------------------
#define INST_T(T)                                                                                       \
  template void krylov_dots<T>(const T*, long long, long long, long long, GState*, const int*,           \
                               double2*, int, hipStream_t, int);                                        \
  template void krylov_update<T>(T*, long long, long long, long long, GState*, int*,                     \
                                 const double2*, double2*, int, hipStream_t, int, bool);                \
  template void vec_norm2<T>(const T*, long long, long long, double*, double*, const int*, int,          \
                             hipStream_t);                                                              \
  template void krylov_residual<T>(const double2*, const double2*, T*, long long, long long, long long,  \
                                   double*, double*, const int*, int, hipStream_t);                     \
  template void krylov_residual_parts<T>(const double2*, const double2*, T*, long long, long long,      \
                                         long long, double*, const int*, int, hipStream_t);             \
  template void vec_diff2<T>(const T*, const T*, long long, long long, double*, double*, int, hipStream_t);
INST_T(float2)
INST_T(double2)
template void krylov_lincomb_res<float2, double2>(float2*, long long, long long, double2*, long long, long long,
                                                  GState*, const int*, const int*, double*, int, hipStream_t);
template void krylov_lincomb_res<double2, double2>(double2*, long long, long long, double2*, long long, long long,
                                                   GState*, const int*, const int*, double*, int, hipStream_t);
template void vec_axpby<double2, double2, double2>(double2*, const double2*, const double2*, double, double,
                                                   long long, long long, const int*, int, hipStream_t);
template void vec_axpby<float2, double2, double2>(float2*, const double2*, const double2*, double, double,
                                                  long long, long long, const int*, int, hipStream_t);
template void vec_axpby<double2, float2, float2>(double2*, const float2*, const float2*, double, double,
                                                 long long, long long, const int*, int, hipStream_t);
template void vec_axpby<float2, float2, float2>(float2*, const float2*, const float2*, double, double,
                                                long long, long long, const int*, int, hipStream_t);

}  // namespace psfd
