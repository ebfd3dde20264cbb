// Fixed-count stationary solves enqueued without a host round trip (not part
// of the C-ABI): the time step's pressure solves, whose cycle count is fixed
// in advance, so every decision the synchronous finish takes on the host
// (where the iterate ends, a zero right-hand side) is taken on the device.
#pragma once

#include "mg_internal.h"

namespace nn4mg {

// Bytes of the solve-state header one solve copies to the host.
size_t solve_header_bytes();

// Enqueue on the hierarchy's stream, with nothing waited for on the host:
// `cycles` V-cycles of A x = b from x (as nn4mg_solve with fixed_cycles),
// the finish on the device and an asynchronous copy of the solve-state header
// into host_hdr (pinned host memory of solve_header_bytes()).  EINVAL for
// singular, FCG or batched hierarchies, which keep the synchronous solve.
int solve_fixed_enqueue(nn4mg_t H, const double *b, double *x, int cycles, void *host_hdr);

// Once the stream has passed the header copy: NN4MG_OK or NN4MG_EBREAKDOWN,
// and the final relative residual.
int solve_fixed_result(const void *host_hdr, double *relres);

// x = 0 if the state's right-hand-side norm is zero; else, when direct
// (direct finest form), x = t if the state's cycle count is odd.
hipError_t launch_finish_fixed(double *x, const double *t, size_t n, const SolveState *st, int direct,
                               hipStream_t s);

}  // namespace nn4mg
