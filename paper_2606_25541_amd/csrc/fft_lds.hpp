// Radix-2/4/8 Stockham FFT passes on data staged in LDS.
//
// A batch of `nseq` sequences of power-of-two length n lives in LDS; element j
// of sequence s sits at lds[s * sstride + j * estride]. Each pass of radix R
// gives every thread up to E / R butterflies: the thread reads its R inputs
// (spaced n / R apart) into registers, the workgroup synchronises, then it
// applies the twiddles exp(-+2 pi i j k / (p R)), a register DFT of size R and
// writes the outputs in self-sorting (Stockham) order. The pass works in place
// because every read of the pass precedes the barrier. Requires
// n * nseq <= E * nthreads (E = 16 for FP32, 8 for FP64).
//
// Twiddles come from a table built on the host in FP64: tw[n + i] =
// exp(-2 pi i i / n) for every power of two n (so the table of length n
// starts at offset n).
#pragma once
#include "common.hpp"

namespace psfd {

template <class T, bool INV> PSFD_D void dft2(T& a, T& b) {
  T t = a; a = cadd(t, b); b = csub(t, b);
}

template <class T, bool INV> PSFD_D void dft4(T& x0, T& x1, T& x2, T& x3) {
  T a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = cmul_mi<T, INV>(csub(x1, x3));
  x0 = cadd(a0, a2); x2 = csub(a0, a2); x1 = cadd(a1, a3); x3 = csub(a1, a3);
}

// multiply by exp(-+2 pi i k / 8)
template <class T, bool INV, int K> PSFD_D T w8(T a) {
  typedef typename real_of<T>::type R;
  const R h = (R)0.70710678118654752440;
  if (K == 0) return a;
  if (K == 2) return cmul_mi<T, INV>(a);
  T r;
  if (K == 1) {  // (1 -+ i)/sqrt2
    if (!INV) { r.x = h * (a.x + a.y); r.y = h * (a.y - a.x); }
    else      { r.x = h * (a.x - a.y); r.y = h * (a.y + a.x); }
  } else {       // K == 3: (-1 -+ i)/sqrt2
    if (!INV) { r.x = h * (a.y - a.x); r.y = -h * (a.x + a.y); }
    else      { r.x = -h * (a.x + a.y); r.y = h * (a.x - a.y); }
  }
  return r;
}

template <class T, bool INV> PSFD_D void dft8(T* x) {
  // even / odd split: X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
  T e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  T o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  o1 = w8<T, INV, 1>(o1); o2 = w8<T, INV, 2>(o2); o3 = w8<T, INV, 3>(o3);
  x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1); x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2); x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3); x[7] = csub(e3, o3);
}

template <class T, int R, bool INV> PSFD_D void dft_r(T* u) {
  if (R == 2) dft2<T, INV>(u[0], u[1]);
  else if (R == 4) dft4<T, INV>(u[0], u[1], u[2], u[3]);
  else dft8<T, INV>(u);
}

// Shape of a batch of sequences in LDS: length 2^ln(), ns() sequences, element
// j of sequence s at s * ss() + j * es(), nt() threads. FftRT carries run-time
// values; FftCT fixes them at compile time, which turns every LDS address of a
// butterfly into one register plus immediate offsets and removes the integer
// multiplies of the index arithmetic.
struct FftRT {
  int log2n, nseq, sstride, estride, nthreads;
  PSFD_D int ln() const { return log2n; }
  PSFD_D int ns() const { return nseq; }
  PSFD_D int ss() const { return sstride; }
  PSFD_D int es() const { return estride; }
  PSFD_D int nt() const { return nthreads; }
};
template <int LN, int NS, int SS, int ES, int NT> struct FftCT {
  PSFD_D static constexpr int ln() { return LN; }
  PSFD_D static constexpr int ns() { return NS; }
  PSFD_D static constexpr int ss() { return SS; }
  PSFD_D static constexpr int es() { return ES; }
  PSFD_D static constexpr int nt() { return NT; }
};

// Butterfly b of a pass -> (sequence s, butterfly t within the sequence).
// SF (sequence-fastest): consecutive threads take consecutive sequences at the
// same butterfly index, the conflict-free mapping when sequences are
// interleaved in LDS (sstride 1); otherwise consecutive threads take
// consecutive butterflies of one sequence. b / nseq goes through a float
// reciprocal (exact for b < 2^22 and nseq <= 4096).
template <bool SF>
PSFD_D void bfly_index(int b, int log2nr, int nseq, float inv_nseq, int& s, int& t) {
  if (SF) { t = (int)(((float)b + 0.5f) * inv_nseq); s = b - t * nseq; }
  else { s = b >> log2nr; t = b & ((1 << log2nr) - 1); }
}

// twiddles w^j (j = 1..R-1) of one butterfly from w^1, w^2, w^4 (table reads) and
// single products for the others, so each value carries at most one rounding
// more than the table
template <class T, int R, bool INV>
PSFD_D void twiddle_apply(T* u, const T* __restrict__ tw, int step) {
  if (R == 2) {
    const T w1 = tw[step];
    u[1] = INV ? cmulc(u[1], w1) : cmul(u[1], w1);
  } else if (R == 4) {
    const T w1 = tw[step], w2 = tw[2 * step];
    const T w3 = cmul(w1, w2);
    u[1] = INV ? cmulc(u[1], w1) : cmul(u[1], w1);
    u[2] = INV ? cmulc(u[2], w2) : cmul(u[2], w2);
    u[3] = INV ? cmulc(u[3], w3) : cmul(u[3], w3);
  } else {
    const T w1 = tw[step], w2 = tw[2 * step], w4 = tw[4 * step];
    const T w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
    const T w[8] = {w1, w1, w2, w3, w4, w5, w6, w7};
#pragma unroll
    for (int j = 1; j < 8; ++j) u[j] = INV ? cmulc(u[j], w[j]) : cmul(u[j], w[j]);
  }
}

// Per-thread element budget of a pass (16 FP32 / 8 FP64 complex values) and the
// largest radix: radix-8 butterflies keep a 1024-thread workgroup inside its 128
// registers per lane; a radix-16 butterfly with its twiddles does not.
template <class T> struct FftBudget {
  static constexpr int E = sizeof(T) == 8 ? 16 : 8;
  static constexpr int LRMAX = 3;
};

template <class T, int R, bool INV, bool SF, int E, class D>
__device__ __forceinline__ void stockham_pass(T* lds, const D& d, int log2p, const T* __restrict__ tw, int tid) {
  constexpr int NB = E >= R ? E / R : 1;  // E < R: one butterfly on the first threads
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  const int log2nr = d.ln() - LR;
  const int nr = 1 << log2nr;
  const int nbt = d.ns() << log2nr;
  const int nthr = d.nt();
  const float inv_nseq = 1.0f / (float)d.ns();
  T u[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    int b = tid + i * nthr;
    if (b < nbt) {
      int s, t;
      bfly_index<SF>(b, log2nr, d.ns(), inv_nseq, s, t);
      const T* base = lds + s * d.ss() + t * d.es();
#pragma unroll
      for (int j = 0; j < R; ++j) u[i][j] = base[j * nr * d.es()];
    }
  }
  __syncthreads();
  const int p = 1 << log2p;
  const int tsh = d.ln() - log2p - LR;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    int b = tid + i * nthr;
    if (b < nbt) {
      int s, t;
      bfly_index<SF>(b, log2nr, d.ns(), inv_nseq, s, t);
      int k = t & (p - 1);
      int step = k << tsh;
      if (k != 0) twiddle_apply<T, R, INV>(u[i], tw, step);
      dft_r<T, R, INV>(u[i]);
      T* base = lds + s * d.ss() + ((t - k) * R + k) * d.es();
#pragma unroll
      for (int j = 0; j < R; ++j) base[j * p * d.es()] = u[i][j];
    }
  }
  __syncthreads();
}

// Full FFT of the batch described by d (unnormalised; INV uses the +i sign).
// All threads of the workgroup must call it. With a compile-time shape the pass
// sequence unrolls and log2p is a constant in every pass.
// tw: the twiddle table of this length, tw[i] = exp(-2 pi i i / n), i < n
// (global memory or LDS).
template <class T, bool INV, bool SF, int E, class D>
__device__ __forceinline__ void lds_fft_tab(T* lds, const D& d, const T* __restrict__ tw, int tid) {
  constexpr int LRM = FftBudget<T>::LRMAX;
#pragma unroll
  for (int log2p = 0; log2p < d.ln();) {
    const int rem = d.ln() - log2p;
    const int lr = rem >= LRM ? LRM : rem;
    if (lr == 3) stockham_pass<T, 8, INV, SF, E>(lds, d, log2p, tw, tid);
    else if (lr == 2) stockham_pass<T, 4, INV, SF, E>(lds, d, log2p, tw, tid);
    else stockham_pass<T, 2, INV, SF, E>(lds, d, log2p, tw, tid);
    log2p += lr;
  }
}

// tw_all: the table of every length (tw_all[n + i] = exp(-2 pi i i / n))
template <class T, bool INV, bool SF, int E, class D>
__device__ __forceinline__ void lds_fft_d(T* lds, const D& d, const T* __restrict__ tw_all, int tid) {
  lds_fft_tab<T, INV, SF, E>(lds, d, tw_all + (1 << d.ln()), tid);
}

// Run-time shape: nseq sequences of length 2^log2n, element j of sequence s at
// s * sstride + j * estride.
template <class T, bool INV, bool SF = false, int E = FftBudget<T>::E>
__device__ __forceinline__ void lds_fft(T* lds, int log2n, int nseq, int sstride, int estride,
                        const T* __restrict__ tw_all, int tid, int nthr) {
  lds_fft_d<T, INV, SF, E>(lds, FftRT{log2n, nseq, sstride, estride, nthr}, tw_all, tid);
}

}  // namespace psfd
