// Differential PSFD operator with a z-PML (the comparison solver of the
// preconditioner study) and its background-field and full-domain solves.
#pragma once
#include "engine.hpp"

struct psfd_diff_plan;

namespace psfd {

Status diff_create(const psfd_diff_problem& p, psfd_diff_plan*& out);
void diff_destroy(psfd_diff_plan* p);
// y = A x (precond PSFD_PRECOND_NONE) or D A x (PSFD_PRECOND_DAMPING); deps: the
// contrast planes [ncz][ny][nx], x, y: [3][nz_ext][ny][nx], all of dtype
Status diff_apply(psfd_diff_plan* p, const void* deps, const void* x, void* y, int dtype, int precond, hipStream_t s);
Status diff_solve(psfd_diff_plan* p, const void* deps, void* e, void* orders, const psfd_opts* opts, int precond,
                  psfd_info* info, hipStream_t s);

}  // namespace psfd
