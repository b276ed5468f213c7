// Small device helpers shared by the kernel sources of the batched
// contingency PCG library.
#pragma once

#include "gpcg_internal.h"

namespace gpcg {
namespace {

template <int S>
__device__ __forceinline__ double col_sum(double v) {
    // butterfly over the R lanes of one column; every lane gets the same
    // bits because each addition is commutative
#pragma unroll
    for (int off = S; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ bool in_interval(int v, int lo, int hi) { return v >= lo && v < hi; }

}  // namespace
}  // namespace gpcg
