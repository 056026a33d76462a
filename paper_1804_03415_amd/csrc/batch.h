// Batched eig_leftmost over independent decompositions (see batch.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include "handle.h"
#include "mmdeig.h"

namespace mmd {

void leftmost_batched(int B, mmd_handle* const* hs, const int* nev, double tol,
                      const eig_opts& o, double* const* evals, double* const* evecs,
                      eig_stats* st, hipStream_t caller);

}  // namespace mmd
