// Kernels of the pre-evaluated contraction (mass, Helmholtz).
#include <algorithm>
#include <map>
#include <mutex>

#include "internal.hpp"
#include "preeval.hpp"

namespace fe {

template <int FORM, int CELL, int MM>
__global__ __launch_bounds__(512) void k_preeval(PreevalArgs a)
{
    extern __shared__ double lds[];
    for (int64_t t = blockIdx.x; t * a.chunk < a.E; t += gridDim.x) preeval_tile<FORM, CELL, MM>(a, t * a.chunk, lds);
}

template <int FORM, int CELL, int MM>
__global__ __launch_bounds__(512) void k_preeval_stream(PreevalArgs a)
{
    extern __shared__ double lds[];
    preeval_stream<FORM, CELL, MM>(a, lds);
}

// Resident blocks per CU of one streaming instantiation (cached).  chunk of
// the arguments: elements per visit (a multiple of epi), 0 = automatic.
template <int FORM, int CELL, int MM>
static int stream_occupancy(int block, size_t lds)
{
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({block, lds});
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_preeval_stream<FORM, CELL, MM>, block, lds) !=
            hipSuccess ||
        n < 1)
        n = 1;
    cache[{block, lds}] = n;
    return n;
}

template <int FORM, int CELL, int MM>
static hipError_t go_stream(const PreevalArgs& a, int block, int max_per_cu, int cus, hipStream_t s)
{
    const size_t lds = preeval_stream_lds_bytes(FORM, CELL, block, a.epi);
    const int per_cu = std::min(max_per_cu, stream_occupancy<FORM, CELL, MM>(block, lds));
    const int64_t steps = (a.E + a.epi - 1) / a.epi;
    const int64_t resident = (int64_t)cus * per_cu;
    PreevalArgs b = a;
    if (b.chunk == 0) {
        // visits of about 256 KiB of output, while every resident block
        // still gets at least four of them
        const int64_t bytes = (int64_t)a.epi * a.nn * 8;
        int64_t t = std::max<int64_t>(1, (256 * 1024 + bytes / 2) / bytes);
        t = std::min<int64_t>(t, std::max<int64_t>(1, steps / (4 * resident)));
        b.chunk = (int)t * a.epi;
    }
    const int64_t visits = (steps + b.chunk / a.epi - 1) / (b.chunk / a.epi);
    const int grid = (int)std::min<int64_t>(visits, resident);
    hipLaunchKernelGGL((k_preeval_stream<FORM, CELL, MM>), dim3(grid), dim3(block), lds, s, b);
    return hipGetLastError();
}

template <int FORM, int CELL>
static hipError_t stream_mm(const PreevalArgs& a, int block, int max_per_cu, int cus, hipStream_t s)
{
    const int mm = preeval_stream_mm(FORM, a.epi * a.nn, block);
    if (mm == 4) return go_stream<FORM, CELL, 4>(a, block, max_per_cu, cus, s);
    if (mm == 8) return go_stream<FORM, CELL, 8>(a, block, max_per_cu, cus, s);
    if constexpr (FORM == MASS)
        if (mm == 16) return go_stream<FORM, CELL, 16>(a, block, max_per_cu, cus, s);
    return hipErrorInvalidValue;
}

hipError_t launch_preeval_stream(int form, int cell, const PreevalArgs& a, int block, int max_per_cu, int cus,
                                 hipStream_t s)
{
    if (form == MASS) {
        if (cell == TRI) return stream_mm<MASS, TRI>(a, block, max_per_cu, cus, s);
        if (cell == TET) return stream_mm<MASS, TET>(a, block, max_per_cu, cus, s);
        return stream_mm<MASS, PRISM>(a, block, max_per_cu, cus, s);
    }
    if (cell == TRI) return stream_mm<HELMHOLTZ, TRI>(a, block, max_per_cu, cus, s);
    if (cell == TET) return stream_mm<HELMHOLTZ, TET>(a, block, max_per_cu, cus, s);
    return stream_mm<HELMHOLTZ, PRISM>(a, block, max_per_cu, cus, s);
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
