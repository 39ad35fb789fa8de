// Batched solves and the continuous-batching solve server.
#pragma once
#include "engine.hpp"

namespace psfd {

Status solve_batch(int n, const psfd_problem* probs, const psfd_opts* opts, const void* const* d_deps,
                   void* const* d_emask, void* const* d_orders, psfd_info* info, hipStream_t s);
void release_cached_groups();

Status server_create(size_t hbm_budget, int max_slots, const psfd_opts* opts, psfd_server** out);
Status server_submit(psfd_server* srv, const psfd_problem* prob, const psfd_opts* opts, const void* d_deps,
                     void* d_emask, void* d_orders, uint64_t* ticket);
Status server_poll(psfd_server* srv, uint64_t ticket, int* done, psfd_info* info, double* latency_s);
Status server_destroy(psfd_server* srv);

}  // namespace psfd
