// Isolated-domain mode (spherical window, padding by 2 on all axes): plan with
// the precomputed kernel table, and the operator apply.
#pragma once
#include "engine.hpp"

struct psfd_iso_plan;

namespace psfd {

Status iso_create(const psfd_iso_problem& p, psfd_iso_plan*& out);
void iso_destroy(psfd_iso_plan* p);
// stage -1: the whole apply; 0 .. 4 one of its passes (timing)
Status iso_apply(psfd_iso_plan* p, const void* deps, const void* x, void* y, int dtype, int stage, hipStream_t s);
// GMRES(m) on the isolated operator (precision PSFD_FP64 or PSFD_MIXED);
// info->status PSFD_OK or PSFD_NOT_CONVERGED
Status iso_solve(psfd_iso_plan* p, const void* deps, const void* b, void* u, double rtol, int m, int max_iters,
                 int precision, psfd_info* info, hipStream_t s);
Status iso_table(psfd_iso_plan* p, void* d_table, int32_t* over, double* radius, hipStream_t s);

}  // namespace psfd
