// Dense-W MaxCut step (fem_dense.hip): launcher and tile constants.  Not part
// of the public ABI.
#pragma once

#include "fem_internal.h"

namespace fem {

// rows of W (and of the state) per workgroup; a dense problem's tiles are
// exactly these row blocks
constexpr int DENSE_ROWS = 64;
// replicas per workgroup
constexpr int DENSE_COLS = 64;
// W and the int8 digit planes are zero-padded to a multiple of this many
// columns (the K block of the int8 kernel)
constexpr int DENSE_LD_ALIGN = 128;

// replica rows of each int8 digit plane of the marginal copy
inline int dense_rows_padded(int R) { return (R + DENSE_COLS - 1) / DENSE_COLS * DENSE_COLS; }

// One explicit-gradient MaxCut step with phi = W m formed by matrix-core
// products: exact int32 products of int8 weights and the four int8 digit
// planes of the fixed-point marginals when the problem holds dense_w8 (W
// integral, |W| <= 127), FP64 products of the float32 W and marginals
// otherwise.  Float32 marginal type only.  Grid: (n_tiles, ceil(R / 64)).
hipError_t launch_dense_step(const Problem& p, int dtype, bool en, bool nt, int n_tiles, const StepArgs& a,
                             hipStream_t st);
// the digit planes of the marginals of a.h into a.marg_nxt (int8 path)
hipError_t launch_dense_i8_init(const Problem& p, const StepArgs& a, hipStream_t st);

}  // namespace fem
