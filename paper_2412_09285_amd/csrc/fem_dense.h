// Dense-W MaxCut step (fem_dense.hip): launcher and tile constants.  Not part
// of the public ABI.
#pragma once

#include "fem_internal.h"

namespace fem {

// rows of W (and of the state) per workgroup; a dense problem's tiles are
// exactly these row blocks, and its matrix is zero-padded to a multiple
constexpr int DENSE_ROWS = 64;
// replicas per workgroup
constexpr int DENSE_COLS = 64;

// One explicit-gradient MaxCut step with phi = W m formed by matrix-core
// products: float32 marginals use the float32 MFMA, bfloat16 marginals the
// bfloat16 MFMA on a bfloat16 copy of W (exact by construction, see
// fem_maxcut_create_dense).  Grid: (n_tiles, ceil(R / DENSE_COLS)).
hipError_t launch_dense_step(const Problem& p, int dtype, bool en, bool nt, int n_tiles, const StepArgs& a,
                             hipStream_t st);

}  // namespace fem
