// Kernels of the split-precision MFMA contraction (elasticity, hyperelastic).
#include "internal.hpp"
#include "split.hpp"

namespace fe {

template <int FORM, int CELL, int PREC, int NQP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_split(SplitArgs a)
{
    extern __shared__ char lds_bytes[];
    split_kernel_body<FORM, CELL, PREC, NQP>(a, lds_bytes);
}

template <int FORM, int CELL, int PREC>
static hipError_t go(int nqp, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (nqp == 8) hipLaunchKernelGGL((k_split<FORM, CELL, PREC, 8>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    else if (nqp == 16) hipLaunchKernelGGL((k_split<FORM, CELL, PREC, 16>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    else hipLaunchKernelGGL((k_split<FORM, CELL, PREC, 32>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    return hipGetLastError();
}

template <int FORM, int PREC>
static hipError_t go_cell(int cell, int nqp, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (cell == TRI) return go<FORM, TRI, PREC>(nqp, a, grid, lds, s);
    if (cell == TET) return go<FORM, TET, PREC>(nqp, a, grid, lds, s);
    return go<FORM, PRISM, PREC>(nqp, a, grid, lds, s);
}

hipError_t launch_split(int form, int cell, int prec, int nqp, const SplitArgs& a, int grid, size_t lds,
                        hipStream_t s)
{
    if (form == ELASTICITY)
        return prec == SPLIT_FP32 ? go_cell<ELASTICITY, SPLIT_FP32>(cell, nqp, a, grid, lds, s)
                                  : go_cell<ELASTICITY, SPLIT_BF16X3>(cell, nqp, a, grid, lds, s);
    return prec == SPLIT_FP32 ? go_cell<HYPERELASTIC, SPLIT_FP32>(cell, nqp, a, grid, lds, s)
                              : go_cell<HYPERELASTIC, SPLIT_BF16X3>(cell, nqp, a, grid, lds, s);
}

}  // namespace fe
