// Solver internals shared by the C ABI (pcheb.hip) and the serving engine
// (serve.hip).  All work is enqueued on the given stream for a range of solve
// slots of one handle; slots iterate independently (each has its own scalars
// and stop flag) and the work of a slot does not depend on the others.
#pragma once

#include "handle.hpp"

namespace pcheb {

Handle* create_handle(const pcheb_operator* A, const pcheb_params* p, hipStream_t stream);
void destroy_handle(Handle* h);
size_t footprint_bytes(const pcheb_operator* A, const pcheb_params* p, int32_t nrhs);
const char* last_error_cstr();

// Workspace for at least `cap` slots (frees and reallocates the workspace);
// the slot states are cleared on `stream`.
void ensure_workspace(Handle& h, int cap, hipStream_t stream);

// Fresh scalars for the slots (tolerance, iteration limit, flexible beta).
void solver_init_states(Handle& h, Slots sl, double tol, int maxit, int flexible, hipStream_t s);
// Mark running slots finished so launches over a wider range skip them.
void solver_retire(Handle& h, Slots sl, hipStream_t s);
// r = b - A x (or x = 0, r = b), the first preconditioner application and gamma.
void solver_start(Handle& h, Slots sl, const double* b, int64_t ldb, double* x, int64_t ldx, bool x0_given,
                  int flexible, hipStream_t s);
// Capture the graph of two PCG iterations of the slots now (otherwise the first
// solver_iteration_pairs call with these arguments does).
void solver_prepare_graph(Handle& h, Slots sl, double* x, int64_t ldx, int flexible);
// `pairs` x two PCG iterations of the slots, replayed from a HIP graph.
void solver_iteration_pairs(Handle& h, Slots sl, double* x, int64_t ldx, int pairs, int flexible, hipStream_t s);
// Two PCG iterations of the slots, launched directly (no graph); under a
// LaunchRecorder this records the launches of an iteration pair.
void solver_iterations_direct(Handle& h, Slots sl, double* x, int64_t ldx, int flexible, hipStream_t s);
// z = P_k r for one vector pair (slot 0 of the workspace).
void solver_apply(Handle& h, const double* r, double* z, hipStream_t s);
// True residual of the slots (norms into their scalars).
void solver_finish(Handle& h, Slots sl, const double* b, int64_t ldb, const double* x, int64_t ldx, hipStream_t s);
// Statistics of one slot from its scalars.
void fill_stats(const Handle& h, const DevState& st, uint32_t flags, pcg_stats* out);

}  // namespace pcheb
