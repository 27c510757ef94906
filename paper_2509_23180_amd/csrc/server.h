// Request server: continuous batching of solves at GMRES-cycle granularity.
#pragma once

#include "runtime.h"

struct fds_server;

namespace fds {
fds_server* server_create(size_t budget, int max_slots);
void server_destroy(fds_server* s);
fds_status server_submit(fds_server* s, fds_plan* plan, const double* rhs, const double* bc,
                         double* x, double tol, hipStream_t stream, uint64_t* ticket);
fds_status server_poll(fds_server* s, uint64_t ticket, fds_result* res);
fds_status server_wait_any(fds_server* s, int64_t timeout_us, uint64_t* ticket, fds_result* res);
void server_stats(fds_server* s, fds_server_stats* out);
}  // namespace fds
