// Kernels of the pre-evaluated contraction (mass, Helmholtz).
#include "internal.hpp"
#include "preeval.hpp"

namespace fe {

template <int FORM, int CELL, int MM>
__global__ __launch_bounds__(512) void k_preeval(PreevalArgs a)
{
    extern __shared__ double lds[];
    for (int64_t t = blockIdx.x; t * a.chunk < a.E; t += gridDim.x) preeval_tile<FORM, CELL, MM>(a, t * a.chunk, lds);
}

template <int FORM, int CELL>
static hipError_t go(const PreevalArgs& a, int block, int grid, hipStream_t s)
{
    const size_t lds = preeval_lds_bytes(FORM, CELL, a.chunk);
    hipLaunchKernelGGL((k_preeval<FORM, CELL, preeval_mm(FORM)>), dim3(grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_preeval(int form, int cell, const PreevalArgs& a, int block, int grid, hipStream_t s)
{
    if (form == MASS) {
        if (cell == TRI) return go<MASS, TRI>(a, block, grid, s);
        if (cell == TET) return go<MASS, TET>(a, block, grid, s);
        return go<MASS, PRISM>(a, block, grid, s);
    }
    if (cell == TRI) return go<HELMHOLTZ, TRI>(a, block, grid, s);
    if (cell == TET) return go<HELMHOLTZ, TET>(a, block, grid, s);
    return go<HELMHOLTZ, PRISM>(a, block, grid, s);
}

}  // namespace fe
