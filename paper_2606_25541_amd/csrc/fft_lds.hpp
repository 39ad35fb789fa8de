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

// multiply by exp(-+2 pi i k / 16) for k = 1, 3 (the other odd powers follow by
// symmetry); cos(pi/8) and sin(pi/8)
template <class T, bool INV, int K> PSFD_D T w16(T a) {
  typedef typename real_of<T>::type R;
  const R c = (R)0.92387953251128675613, sn = (R)0.38268343236508977173;
  // exp(-i pi/8) = c - i s, exp(-3 i pi/8) = s - i c (conjugates for INV)
  const R wr = K == 1 ? c : sn, wi = INV ? (K == 1 ? sn : c) : -(K == 1 ? sn : c);
  T r;
  r.x = a.x * wr - a.y * wi;
  r.y = a.x * wi + a.y * wr;
  return r;
}

// 16-point DFT as 4 x 4: DFT4 over n1 of x[4 n1 + n2], twiddle W16^(n2 k1),
// DFT4 over n2; output k1 + 4 k2 in natural order. dft16_tail: the twiddles
// and the second DFT4s, from the first stage's y[4 n2 + k1].
template <class T, bool INV> PSFD_D void dft16_tail(T* y, T* x) {
  // W16^(n2 k1): n2 = 1: k1 = 1, 2, 3 -> W^1, W^2, W^3; n2 = 2: W^2, W^4, W^6; n2 = 3: W^3, W^6, W^9
  y[5] = w16<T, INV, 1>(y[5]);
  y[6] = w8<T, INV, 1>(y[6]);
  y[7] = w16<T, INV, 3>(y[7]);
  y[9] = w8<T, INV, 1>(y[9]);
  y[10] = cmul_mi<T, INV>(y[10]);
  y[11] = w8<T, INV, 3>(y[11]);
  y[13] = w16<T, INV, 3>(y[13]);
  y[14] = w8<T, INV, 3>(y[14]);
  {  // W16^9 = -W16^1
    T t = w16<T, INV, 1>(y[15]);
    t.x = -t.x; t.y = -t.y;
    y[15] = t;
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    T a = y[k1], b = y[4 + k1], c = y[8 + k1], d = y[12 + k1];
    dft4<T, INV>(a, b, c, d);
    x[k1] = a; x[k1 + 4] = b; x[k1 + 8] = c; x[k1 + 12] = d;
  }
}
template <class T, bool INV> PSFD_D void dft16(T* x) {
  T y[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T a = x[n2], b = x[4 + n2], c = x[8 + n2], d = x[12 + n2];
    dft4<T, INV>(a, b, c, d);
    y[4 * n2 + 0] = a; y[4 * n2 + 1] = b; y[4 * n2 + 2] = c; y[4 * n2 + 3] = d;
  }
  dft16_tail<T, INV>(y, x);
}

template <class T, int R, bool INV> PSFD_D void dft_r(T* u) {
  if (R == 2) dft2<T, INV>(u[0], u[1]);
  else if (R == 4) dft4<T, INV>(u[0], u[1], u[2], u[3]);
  else if (R == 8) dft8<T, INV>(u);
  else dft16<T, INV>(u);
}

// DFT of size R whose inputs R/2 .. R-1 are zero (first pass over a sequence
// zero-padded to twice its length): only the non-zero half is read.
template <class T, int R, bool INV> PSFD_D void dft_r_half(T* u) {
  if (R == 2) {
    u[1] = u[0];
  } else if (R == 4) {
    const T a = u[0], b = u[1];
    const T c = cmul_mi<T, INV>(b);
    u[0] = cadd(a, b); u[2] = csub(a, b); u[1] = cadd(a, c); u[3] = csub(a, c);
  } else if (R == 16) {
    // dft16 with x[8..15] = 0: each first-stage DFT4 takes (x[n2], x[4 + n2], 0, 0)
    T y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const T a = u[n2], b = u[4 + n2], c = cmul_mi<T, INV>(b);
      y[4 * n2 + 0] = cadd(a, b); y[4 * n2 + 2] = csub(a, b);
      y[4 * n2 + 1] = cadd(a, c); y[4 * n2 + 3] = csub(a, c);
    }
    dft16_tail<T, INV>(y, u);
  } else {
    // even part (x0, x2, 0, 0) and odd part (x1, x3, 0, 0) as 4-point DFTs
    const T x0 = u[0], x1 = u[1], x2 = u[2], x3 = u[3];
    const T e0 = cadd(x0, x2), e2 = csub(x0, x2), ex = cmul_mi<T, INV>(x2);
    const T e1 = cadd(x0, ex), e3 = csub(x0, ex);
    const T o0 = cadd(x1, x3), o2 = csub(x1, x3), ox = cmul_mi<T, INV>(x3);
    T o1 = cadd(x1, ox), o3 = csub(x1, ox);
    o1 = w8<T, INV, 1>(o1);
    const T o2w = w8<T, INV, 2>(o2);
    o3 = w8<T, INV, 3>(o3);
    u[0] = cadd(e0, o0); u[4] = csub(e0, o0);
    u[1] = cadd(e1, o1); u[5] = csub(e1, o1);
    u[2] = cadd(e2, o2w); u[6] = csub(e2, o2w);
    u[3] = cadd(e3, o3); u[7] = csub(e3, o3);
  }
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
  } else if (R == 8) {
    const T w1 = tw[step], w2 = tw[2 * step], w4 = tw[4 * step];
    const T w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
    const T w[8] = {w1, w1, w2, w3, w4, w5, w6, w7};
#pragma unroll
    for (int j = 1; j < 8; ++j) u[j] = INV ? cmulc(u[j], w[j]) : cmul(u[j], w[j]);
  } else {
    // radix 16: every power read from the table (an LDS table in the kernels
    // that use this radix)
#pragma unroll
    for (int j = 1; j < 16; ++j) {
      const T w = tw[j * step];
      u[j] = INV ? cmulc(u[j], w) : cmul(u[j], w);
    }
  }
}

// Per-thread element budget of a pass (16 FP32 / 8 FP64 complex values) and the
// largest radix: radix-8 butterflies keep a 1024-thread workgroup inside its 128
// registers per lane; a radix-16 butterfly with its twiddles does not.
template <class T> struct FftBudget {
  static constexpr int E = sizeof(T) == 8 ? 16 : 8;
  static constexpr int LRMAX = 3;
};

// ZIN (first pass only): the second half of every sequence is zero and is
// neither read nor needed in LDS. ZOUT (last pass only): only the first half of
// every sequence is stored.
template <class T, int R, bool INV, bool SF, int E, class D, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void stockham_pass(T* lds, const D& d, int log2p, const T* __restrict__ tw, int tid) {
  constexpr int NB = E >= R ? E / R : 1;  // E < R: one butterfly on the first threads
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
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
      for (int j = 0; j < (ZIN ? R / 2 : R); ++j) u[i][j] = base[j * nr * d.es()];
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
      if (ZIN) {
        dft_r_half<T, R, INV>(u[i]);  // first pass: p = 1, no twiddles
      } else {
        if (k != 0) twiddle_apply<T, R, INV>(u[i], tw, step);
        dft_r<T, R, INV>(u[i]);
      }
      T* base = lds + s * d.ss() + ((t - k) * R + k) * d.es();
      // last pass: output j of butterfly t lands at t + j n / R, in the first half for j < R / 2
#pragma unroll
      for (int j = 0; j < (ZOUT ? R / 2 : R); ++j) base[j * p * d.es()] = u[i][j];
    }
  }
  __syncthreads();
}

// Full FFT of the batch described by d (unnormalised; INV uses the +i sign).
// All threads of the workgroup must call it. With a compile-time shape the pass
// sequence unrolls and log2p is a constant in every pass.
// tw: the twiddle table of this length, tw[i] = exp(-2 pi i i / n), i < n
// (global memory or LDS).
// ZIN: every sequence is zero in its second half (which need not be set in
// LDS); ZOUT: only the first half of every result is needed (the second half
// of LDS is left unspecified).
// LRM: largest radix as log2 (3: radix 8, 4: radix 16 with every twiddle read
// from the table). The passes take the largest radix first.
template <class T, bool INV, bool SF, int E, class D, bool ZIN, bool ZOUT, int R>
__device__ __forceinline__ void pass_r(T* lds, const D& d, int log2p, const T* __restrict__ tw, int tid,
                                       bool first, bool last) {
  if (ZIN && first) stockham_pass<T, R, INV, SF, E, D, true, false>(lds, d, log2p, tw, tid);
  else if (ZOUT && last) stockham_pass<T, R, INV, SF, E, D, false, true>(lds, d, log2p, tw, tid);
  else stockham_pass<T, R, INV, SF, E, D, false, false>(lds, d, log2p, tw, tid);
}

template <class T, bool INV, bool SF, int E, class D, bool ZIN = false, bool ZOUT = false,
          int LRM = FftBudget<T>::LRMAX>
__device__ __forceinline__ void lds_fft_tab(T* lds, const D& d, const T* __restrict__ tw, int tid) {
#pragma unroll
  for (int log2p = 0; log2p < d.ln();) {
    const int rem = d.ln() - log2p;
    const int lr = rem >= LRM ? LRM : rem;
    const bool first = log2p == 0, last = lr == rem;
    if (LRM >= 4 && lr == 4) pass_r<T, INV, SF, E, D, ZIN, ZOUT, 16>(lds, d, log2p, tw, tid, first, last);
    else if (lr == 3) pass_r<T, INV, SF, E, D, ZIN, ZOUT, 8>(lds, d, log2p, tw, tid, first, last);
    else if (lr == 2) pass_r<T, INV, SF, E, D, ZIN, ZOUT, 4>(lds, d, log2p, tw, tid, first, last);
    else pass_r<T, INV, SF, E, D, ZIN, ZOUT, 2>(lds, d, log2p, tw, tid, first, last);
    log2p += lr;
  }
}

// First pass (p = 1, no twiddles) of a transform whose inputs are already in
// registers: in[i NI + j] is element t + j nr of the sequence of butterfly
// b = tid + i nt (sequence s, index t < nr = n / R), for j < NI, NI = R / 2
// with ZIN (the second half of every sequence is zero), else R. The outputs
// go to LDS in Stockham order; the caller synchronises before the next pass.
template <class T, int R, bool INV, bool SF, int E, class D, bool ZIN>
__device__ __forceinline__ void stockham_pass_regin(T* lds, const D& d, int tid, const T* in) {
  constexpr int NB = E >= R ? E / R : 1;
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  constexpr int NI = ZIN ? R / 2 : R;
  const int log2nr = d.ln() - LR;
  const int nbt = d.ns() << log2nr;
  const int nthr = d.nt();
  const float inv_nseq = 1.0f / (float)d.ns();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * nthr;
    if (b < nbt) {
      int s, t;
      bfly_index<SF>(b, log2nr, d.ns(), inv_nseq, s, t);
      T u[R];
#pragma unroll
      for (int j = 0; j < NI; ++j) u[j] = in[i * NI + j];
      if (ZIN) dft_r_half<T, R, INV>(u);
      else dft_r<T, R, INV>(u);
      T* base = lds + s * d.ss() + t * R * d.es();
#pragma unroll
      for (int j = 0; j < R; ++j) base[j * d.es()] = u[j];
    }
  }
}

// Last pass of lds_fft_tab with its outputs left in registers instead of LDS:
// out[i NO + j] is output t + j p of butterfly b = tid + i nt (sequence s,
// index t < p = n / R, p the stride of the last pass), for j < NO, NO = R / 2
// with HALF (only the first half of every sequence is kept, as ZOUT), else R.
// It only reads LDS, so it has no barrier; the caller consumes out directly.
template <class T, int R, bool INV, bool SF, int E, class D, bool HALF>
__device__ __forceinline__ void stockham_pass_regout(const T* lds, const D& d, int log2p, const T* __restrict__ tw,
                                                     int tid, T* out) {
  constexpr int NO = HALF ? R / 2 : R;
  constexpr int NB = E >= R ? E / R : 1;
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  const int log2nr = d.ln() - LR;
  const int nr = 1 << log2nr;
  const int nbt = d.ns() << log2nr;
  const int nthr = d.nt();
  const float inv_nseq = 1.0f / (float)d.ns();
  const int p = 1 << log2p;
  const int tsh = d.ln() - log2p - LR;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = tid + i * nthr;
    if (b < nbt) {
      int s, t;
      bfly_index<SF>(b, log2nr, d.ns(), inv_nseq, s, t);
      const T* base = lds + s * d.ss() + t * d.es();
      T u[R];
#pragma unroll
      for (int j = 0; j < R; ++j) u[j] = base[j * nr * d.es()];
      const int k = t & (p - 1);
      if (k != 0) twiddle_apply<T, R, INV>(u, tw, k << tsh);
      dft_r<T, R, INV>(u);
#pragma unroll
      for (int j = 0; j < NO; ++j) out[i * NO + j] = u[j];
    }
  }
}

// lds_fft_tab (compile-time shapes) whose last pass returns its results (the
// first half of every sequence with HALF) in registers (stockham_pass_regout)
// instead of storing them.
template <class T, bool INV, bool SF, int E, class D, bool HALF, int LRM = FftBudget<T>::LRMAX>
__device__ __forceinline__ void lds_fft_tab_regout(T* lds, const D& d, const T* __restrict__ tw, int tid, T* out) {
#pragma unroll
  for (int log2p = 0; log2p < d.ln();) {
    const int rem = d.ln() - log2p;
    const int lr = rem >= LRM ? LRM : rem;
    const bool first = log2p == 0;
    if (lr == rem) {
      // (radix 16 only where LRM allows it: out holds E / 2 values with HALF, E without)
      if (lr == 4) {
        if constexpr (LRM >= 4) stockham_pass_regout<T, 16, INV, SF, E, D, HALF>(lds, d, log2p, tw, tid, out);
      } else if (lr == 3) {
        stockham_pass_regout<T, 8, INV, SF, E, D, HALF>(lds, d, log2p, tw, tid, out);
      } else if (lr == 2) stockham_pass_regout<T, 4, INV, SF, E, D, HALF>(lds, d, log2p, tw, tid, out);
      else stockham_pass_regout<T, 2, INV, SF, E, D, HALF>(lds, d, log2p, tw, tid, out);
    } else if (LRM >= 4 && lr == 4) {
      pass_r<T, INV, SF, E, D, false, false, 16>(lds, d, log2p, tw, tid, first, false);
    } else if (lr == 3) {
      pass_r<T, INV, SF, E, D, false, false, 8>(lds, d, log2p, tw, tid, first, false);
    } else if (lr == 2) {
      pass_r<T, INV, SF, E, D, false, false, 4>(lds, d, log2p, tw, tid, first, false);
    } else {
      pass_r<T, INV, SF, E, D, false, false, 2>(lds, d, log2p, tw, tid, first, false);
    }
    log2p += lr;
  }
}

// tw_all: the table of every length (tw_all[n + i] = exp(-2 pi i i / n))
template <class T, bool INV, bool SF, int E, class D, bool ZIN = false, bool ZOUT = false,
          int LRM = FftBudget<T>::LRMAX>
__device__ __forceinline__ void lds_fft_d(T* lds, const D& d, const T* __restrict__ tw_all, int tid) {
  lds_fft_tab<T, INV, SF, E, D, ZIN, ZOUT, LRM>(lds, d, tw_all + (1 << d.ln()), tid);
}

// Run-time shape: nseq sequences of length 2^log2n, element j of sequence s at
// s * sstride + j * estride.
template <class T, bool INV, bool SF = false, int E = FftBudget<T>::E, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void lds_fft(T* lds, int log2n, int nseq, int sstride, int estride,
                        const T* __restrict__ tw_all, int tid, int nthr) {
  lds_fft_d<T, INV, SF, E, FftRT, ZIN, ZOUT>(lds, FftRT{log2n, nseq, sstride, estride, nthr}, tw_all, tid);
}

}  // namespace psfd
