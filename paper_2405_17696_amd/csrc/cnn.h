// Interface between the Krylov driver and the encoder-solver network module.
#pragma once
#include "internal.h"

namespace helm {

// Make sure the encoder context of (net, op) is current (runs the encoder if
// needed) and the workspaces of an nrhs-vector application exist.  slot: one
// set of workspaces per slot, for applications in flight at the same time.
int cnn_prepare(cnn_net* net, const helm_op* op, int nrhs, hipStream_t s, int slot = 0);
// e = SolverNet(scale_r * r) / scale_r for nrhs vectors of op's grid (c64, or c128
// when wide != 0), skipping RHS whose state is inactive.  scale_r comes from
// fscale[(rhs0 + r) * fstride] (may be null: 1).  fallback: e = 0 for a RHS
// whose network output is not finite.  slot as in cnn_prepare.
int cnn_apply_masked(cnn_net* net, const helm_op* op, const void* r, const double* fscale, int fstride, void* e,
                     int nrhs, const RhsState* st, int rhs0, int wide, hipStream_t s, bool fallback = false,
                     int slot = 0);
// Drop any encoder context cached on op.
void cnn_release_cache(helm_op* op);

}  // namespace helm
