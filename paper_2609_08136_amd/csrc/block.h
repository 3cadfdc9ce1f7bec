// Declarations of the block PCG kernels (block.hip).
#pragma once

#include "nys_internal.h"

namespace nys {

// largest block (columns per group) the block kernels take
int block_max_s();

// For each group g < groups, on the n x s column block at columns g s .. g s + s - 1 of
// row-major n x (groups s) matrices with leading dimension ld, and C_g the s x s matrix
// at C + g s s (row-major, device):
//   mode 0: Out += A C_g;  mode 1: Out -= A C_g;  mode 2: Out = Zs + A C_g
template <class TA, class TO>
int32_t blk_apply(int mode, const TA *A, const double *C, int s, int groups, int ld, TO *Out, const TO *Zs,
                  int64_t n, hipStream_t st);

}  // namespace nys
