// Kernels of the split-precision MFMA contraction: elasticity, fp32 operands.
#include "internal.hpp"
#include "split.hpp"

namespace fe {

template <int CELL, int P, int NQP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_split_elasticity_fp32(SplitArgs a)
{
    extern __shared__ char lds_bytes[];
    split_kernel_body<ELASTICITY, CELL, SPLIT_FP32, P, NQP>(a, lds_bytes);
}

template <int CELL, int P>
static hipError_t go(int nqp, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (nqp == 8) hipLaunchKernelGGL((k_split_elasticity_fp32<CELL, P, 8>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    else if (nqp == 16) hipLaunchKernelGGL((k_split_elasticity_fp32<CELL, P, 16>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    else hipLaunchKernelGGL((k_split_elasticity_fp32<CELL, P, 32>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    return hipGetLastError();
}

// (cell, degree) pairs whose element matrix fits one 32x32 tile
hipError_t launch_split_elasticity_fp32(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (cell == TRI) {
        if (p == 1) return go<TRI, 1>(nqp, a, grid, lds, s);
        if (p == 2) return go<TRI, 2>(nqp, a, grid, lds, s);
        if (p == 3) return go<TRI, 3>(nqp, a, grid, lds, s);
        return go<TRI, 4>(nqp, a, grid, lds, s);
    }
    if (cell == TET) return p == 1 ? go<TET, 1>(nqp, a, grid, lds, s) : go<TET, 2>(nqp, a, grid, lds, s);
    return go<PRISM, 1>(nqp, a, grid, lds, s);
}

}  // namespace fe
