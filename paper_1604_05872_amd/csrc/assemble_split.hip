// Kernels of the split-precision MFMA contraction (elasticity, hyperelastic).
#include "internal.hpp"
#include "split.hpp"

namespace fe {

template <int FORM, int CELL, int PREC, int NKB>
__global__ __launch_bounds__(256) void k_split(SplitArgs a)
{
    extern __shared__ double lds[];
    constexpr int D = cell_dim(CELL);
    double* sTab = lds + SPLIT_WAVES * SPLIT_WAVE_DOUBLES;
    const int ntab = a.nq * a.ns * D;
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) sTab[i] = a.dphi[i];
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * SPLIT_WAVES; base < a.E; base += (int64_t)gridDim.x * SPLIT_WAVES)
        split_step<FORM, CELL, PREC, NKB>(a, base, lds, sTab);
}

template <int FORM, int CELL, int PREC>
static hipError_t go(int nkb, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (nkb == 1) hipLaunchKernelGGL((k_split<FORM, CELL, PREC, 1>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    else if (nkb == 2) hipLaunchKernelGGL((k_split<FORM, CELL, PREC, 2>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    else hipLaunchKernelGGL((k_split<FORM, CELL, PREC, 4>), dim3(grid), dim3(SPLIT_BLOCK), lds, s, a);
    return hipGetLastError();
}

template <int FORM, int PREC>
static hipError_t go_cell(int cell, int nkb, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (cell == TRI) return go<FORM, TRI, PREC>(nkb, a, grid, lds, s);
    if (cell == TET) return go<FORM, TET, PREC>(nkb, a, grid, lds, s);
    return go<FORM, PRISM, PREC>(nkb, a, grid, lds, s);
}

hipError_t launch_split(int form, int cell, int prec, int nkb, const SplitArgs& a, int grid, size_t lds,
                        hipStream_t s)
{
    if (form == ELASTICITY)
        return prec == SPLIT_FP32 ? go_cell<ELASTICITY, SPLIT_FP32>(cell, nkb, a, grid, lds, s)
                                  : go_cell<ELASTICITY, SPLIT_BF16X3>(cell, nkb, a, grid, lds, s);
    return prec == SPLIT_FP32 ? go_cell<HYPERELASTIC, SPLIT_FP32>(cell, nkb, a, grid, lds, s)
                              : go_cell<HYPERELASTIC, SPLIT_BF16X3>(cell, nkb, a, grid, lds, s);
}

}  // namespace fe
