// Kernels of the sharing-eliminated float64 quadrature, form elasticity.
#include "internal.hpp"
#include "quad.hpp"

namespace fe {

template <int FORM, int CELL, int KB>
__global__ __launch_bounds__(256) void k_quad_elasticity(QuadArgs a)
{
    extern __shared__ double lds[];
    for (int64_t t = blockIdx.x; t * a.eb < a.E; t += gridDim.x) quad_tile<FORM, CELL, KB>(a, t * a.eb, lds);
}

template <int CELL, int KB>
static hipError_t go(const QuadArgs& a, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_quad_elasticity<ELASTICITY, CELL, KB>), dim3(grid), dim3(QUAD_BLOCK), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_quad_elasticity(int cell, int kb, const QuadArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (cell == TRI) return kb == 3 ? go<TRI, 3>(a, grid, lds, s) : go<TRI, 5>(a, grid, lds, s);
    if (cell == TET) return kb == 4 ? go<TET, 4>(a, grid, lds, s) : go<TET, 5>(a, grid, lds, s);
    return kb == 3 ? go<PRISM, 3>(a, grid, lds, s) : go<PRISM, 5>(a, grid, lds, s);
}

}  // namespace fe
