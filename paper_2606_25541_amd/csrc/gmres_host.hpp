// Restarted GMRES with the Hessenberg system and Givens rotations on the host,
// for operators whose applies cost far more than a host round trip per step
// (the isolated-domain operator, the differential PSFD operator).
#pragma once
#include <functional>

#include "engine.hpp"

namespace psfd {

// y = A x for device vectors of n complex values of `dtype` (PSFD_C64 or PSFD_C128).
using ApplyFn = std::function<Status(const void* x, void* y, int dtype, hipStream_t s)>;

struct HostGmres {
  double rtol = 1e-8;   // stop at ||b - A x|| <= rtol ||b||
  int m = 30;           // restart length, 1..64
  int max_iters = 1000; // Arnoldi steps
  int precision = PSFD_FP64;  // PSFD_MIXED: FP32 basis and applies (A called with PSFD_C64)
  double cancel = 0.70710678118654752;  // second Gram-Schmidt pass below this norm ratio
  bool warm = false;    // x holds the initial guess (else x0 = 0)
};

// Solves A x = b (b, x: complex128 device vectors of n values, x must not alias b).
// Every restart starts from the FP64 residual b - A x (A called with PSFD_C128),
// x accumulates in FP64; with an FP32 basis a cycle also ends once it has
// reduced the residual estimate 1e4-fold. info: iters, cycles, rel_residual,
// status PSFD_OK or PSFD_NOT_CONVERGED.
Status gmres_host(long long n, const ApplyFn& A, const double2* b, double2* x, const HostGmres& o, psfd_info& info,
                  hipStream_t s);

}  // namespace psfd
