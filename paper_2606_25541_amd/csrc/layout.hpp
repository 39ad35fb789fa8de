// Per-instance FP64 table layout and vector addressing shared by kernels and host code.
#pragma once
#include "common.hpp"

namespace psfd {

// Scalars at the head of every per-instance table (indices into the double array).
enum TabScalar {
  TS_KBG = 0,        // background wavenumber k_bg
  TS_L = 1,          // window half-length L = T (absorber thickness)
  TS_DZ = 2,         // plane spacing dz
  TS_KAPPA = 3,      // 2 pi / (Pz dz): z-wavenumber step of the padded grid
  TS_SCALE = 4,      // 1 / (Nx Ny Pz): inverse 3-D FFT normalisation folded into the kernel
  TS_K0SQ = 5,       // k0^2, the factor of V = k0^2 delta_eps
  TS_INCQ = 6,       // flat index of the incident order
  TS_EINC = 8,       // incident polarisation vector (3 complex: 6 doubles)
  TS_BINC = 14,      // beta of the incident order (complex)
  TS_T = 16,         // absorber thickness T (z of the top surface)
  TS_INVNXNY = 17,   // 1 / (Nx Ny)
  TS_ST = 18,        // sin(theta) cos(phi), sin(theta) sin(phi) of the incidence (2 doubles)
  TS_COUNT = 32
};

struct TabLayout {
  int nx, ny;
  __host__ __device__ long long off_kx() const { return TS_COUNT; }
  __host__ __device__ long long off_ky() const { return TS_COUNT + nx; }
  __host__ __device__ long long off_beta() const { return TS_COUNT + nx + ny; }
  __host__ __device__ long long off_eibl() const { return off_beta() + 2LL * nx * ny; }
  __host__ __device__ long long off_keep() const { return off_eibl() + 2LL * nx * ny; }
  __host__ __device__ long long off_tr() const { return off_keep() + 1LL * nx * ny; }
  // stack response of an order in the coupled operator: M_q = T_R (i dz / 2 beta) P- / (Nx Ny),
  // P- = I - k- k-^T / k_bg^2 with k- = (kx, ky, -beta); 3x3 complex, row-major
  __host__ __device__ long long off_mono() const { return off_tr() + 18LL * nx * ny; }
  __host__ __device__ long long size() const { return off_mono() + 18LL * nx * ny; }
};

// A vector of one instance: base + b * bstride + j * jstride elements, where j is
// idx[b * idx_stride] + joff when idx is set (device-side Krylov index, e.g. the
// j field of a GState array) and joff otherwise.
struct VecRef {
  void* base;
  long long bstride;
  long long jstride;
  const int* idx;
  int idx_stride;
  int joff;
};

template <class T> PSFD_D T* vref(const VecRef& r, int b) {
  long long j = r.idx ? (long long)(r.idx[(long long)b * r.idx_stride] + r.joff) : (long long)r.joff;
  return (T*)r.base + (long long)b * r.bstride + j * r.jstride;
}

inline VecRef vr(const void* p, long long bstride = 0) {
  VecRef r; r.base = const_cast<void*>(p); r.bstride = bstride; r.jstride = 0; r.idx = nullptr; r.idx_stride = 0; r.joff = 0;
  return r;
}

}  // namespace psfd
