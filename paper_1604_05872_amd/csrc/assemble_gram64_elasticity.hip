// Kernels of the float64 matrix-core contraction: elasticity.
#include "gram64.hpp"
#include "internal.hpp"

namespace fe {

template <int CELL, int P, int NQP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gram64_elasticity(SplitArgs a)
{
    extern __shared__ char lds_bytes[];
    gram64_kernel_body<ELASTICITY, CELL, P, NQP>(a, lds_bytes);
}

template <int CELL, int P>
static hipError_t go(int nqp, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    switch (nqp) {
    case 4: hipLaunchKernelGGL((k_gram64_elasticity<CELL, P, 4>), dim3(grid), dim3(256), lds, s, a); break;
    case 8: hipLaunchKernelGGL((k_gram64_elasticity<CELL, P, 8>), dim3(grid), dim3(256), lds, s, a); break;
    case 16: hipLaunchKernelGGL((k_gram64_elasticity<CELL, P, 16>), dim3(grid), dim3(256), lds, s, a); break;
    case 28: hipLaunchKernelGGL((k_gram64_elasticity<CELL, P, 28>), dim3(grid), dim3(256), lds, s, a); break;
    case 32: hipLaunchKernelGGL((k_gram64_elasticity<CELL, P, 32>), dim3(grid), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// (cell, degree) pairs whose element matrix fits one 32x32 tile
hipError_t launch_gram64_elasticity(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds, hipStream_t s)
{
    if (cell == TRI) {
        if (p == 1) return go<TRI, 1>(nqp, a, grid, lds, s);
        if (p == 2) return go<TRI, 2>(nqp, a, grid, lds, s);
        if (p == 3) return go<TRI, 3>(nqp, a, grid, lds, s);
        if (p == 4) return go<TRI, 4>(nqp, a, grid, lds, s);
        return hipErrorInvalidValue;
    }
    if (cell == TET) {
        if (p == 1) return go<TET, 1>(nqp, a, grid, lds, s);
        if (p == 2) return go<TET, 2>(nqp, a, grid, lds, s);
        return hipErrorInvalidValue;
    }
    if (p == 1) return go<PRISM, 1>(nqp, a, grid, lds, s);
    return hipErrorInvalidValue;
}

}  // namespace fe
