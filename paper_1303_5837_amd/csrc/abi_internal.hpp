// Library-internal entry points shared by the C ABI and the request server.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/caqr.h"

namespace caqr {

// Device bytes a least-squares solve of an m-by-n problem needs for its
// factors (tau, signs and compact-WY T of every panel), when lent to it.
size_t ls_workspace_bytes(int64_t m, int64_t n);

// Least-squares solve with validated arguments on the handle's stream.  With
// ws (ls_workspace_bytes bytes of device memory, 256-byte aligned) the solve
// allocates and frees no device memory for its factors; without, it
// allocates its own.  With tickets (zeroed counters, as many as the
// factorization's trees need) the panel loop uses them instead of the
// handle's and runs on the handle's stream alone; with status (two words of
// device memory) the solution check writes there instead of the handle's.
// Returns after the solve has finished (it reads back the status words).
caqr_status_t ls_solve_ws(caqr_handle_t h, int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B,
                          int64_t ldb, void *ws, caqr_ls_info_t *info, unsigned *tickets = nullptr,
                          int64_t *status = nullptr);

// Mixed-precision least-squares solve (validated arguments, n > 64): A only
// read; solutions in B(0:n, :).  Allocates its workspace.
caqr_status_t ls_solve_mixed(caqr_handle_t h, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                             double *B, int64_t ldb, const caqr_ls_opts_t &o, caqr_ls_info_t *info);

// Pre-size the handle's ticket counters (device-tree synchronization).
caqr_status_t reserve_tickets(caqr_handle_t h, size_t counters);

}  // namespace caqr
