// Global assembly into compressed sparse rows.
//
// Sec. 2 splits assembly into a local step (the element matrices) and a
// global step that adds every element matrix into the matrix of the
// continuous space, A_ij = a(phi_i, phi_j), at the global numbers of the
// element's DOFs; Sec. 7.1 times the two together.
//
// Pattern (fe_csr_create), built on the device:
//   1. validate the global numbers (in range, distinct within an element);
//   2. count the (element, local DOF) pairs of every global row, scan the
//      counts, fill each row's list of pairs e*n + j and sort it;
//   3. per row, gather the global numbers of its elements, sort them and
//      drop repeats: the row's columns (one pass for the lengths, a scan,
//      one pass for the columns);
//   4. the position table pos[e][j][k]: where column dofs[e][k] sits within
//      row dofs[e][j].
// Insertion (fe_csr_insert): one wavefront per row accumulates the row in
// LDS, adding the contributions of the row's elements in increasing element
// order, then stores it with contiguous writes.  Each stored value is the
// element-order sum of its contributions, so it does not depend on the launch
// and equals a sequential element-order sum bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "felocal.h"
#include "internal.hpp"

namespace fe {
namespace {

constexpr int CSR_WAVE = 64;
// LDS words (int32) of the per-row candidate list: (elements of the row) * n
constexpr int CSR_MAX_CANDIDATES = 8192;
constexpr int CSR_MAX_N = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_TILE = SCAN_ITEMS * SCAN_BLOCK;

// ---------------------------------------------------------------------------
// Exclusive scan of n counts into out[0..n] (out[n] = total)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const T* __restrict__ in, int64_t n,
                                                           int64_t* __restrict__ out, int64_t* __restrict__ sums)
{
    __shared__ int64_t s[SCAN_BLOCK];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + i;
        v[i] = idx < n ? (int64_t)in[idx] : 0;
        run += v[i];
    }
    s[t] = run;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        const int64_t x = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    int64_t ex = s[t] - run;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        const int64_t idx = base + i;
        if (idx <= n) out[idx] = ex;
        ex += v[i];
    }
    if (t == SCAN_BLOCK - 1) sums[blockIdx.x] = s[t];
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_add(int64_t* __restrict__ out, int64_t n,
                                                         const int64_t* __restrict__ offs)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    const int64_t o = offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++)
        if (base + i <= n) out[base + i] += o;
}

// out[0..n]: the logical input has n + 1 items, the last one zero, so that
// out[n] receives the total.
template <typename T>
hipError_t scan_exclusive(const T* in, int64_t n, int64_t* out, hipStream_t s)
{
    const int64_t tiles = (n + 1 + SCAN_TILE - 1) / SCAN_TILE;
    int64_t* sums = nullptr;
    hipError_t e = hipMalloc(&sums, sizeof(int64_t) * (size_t)(2 * tiles + 1));
    if (e != hipSuccess) return e;
    int64_t* sums_ex = sums + tiles;
    k_scan_tiles<T><<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, n, out, sums);
    e = hipGetLastError();
    if (e == hipSuccess && tiles > 1) {
        e = scan_exclusive<int64_t>(sums, tiles, sums_ex, s);
        if (e == hipSuccess) {
            k_scan_add<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(out, n, sums_ex);
            e = hipGetLastError();
        }
    }
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(sums);
    return e != hipSuccess ? e : e2;
}

// ---------------------------------------------------------------------------
// Pattern construction
// ---------------------------------------------------------------------------

// bit 0: a number out of range; bit 1: a number repeated within an element
__global__ void k_csr_validate(int64_t pairs, int n, const int32_t* __restrict__ dofs, int64_t N,
                               int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pairs) return;
    const int32_t d = dofs[i];
    if (d < 0 || (int64_t)d >= N) {
        atomicOr(bad, 1);
        return;
    }
    const int64_t e0 = i - i % n;
    for (int64_t k = i + 1; k < e0 + n; k++)
        if (dofs[k] == d) atomicOr(bad, 2);
}

__global__ void k_csr_count(int64_t pairs, const int32_t* __restrict__ dofs, uint32_t* __restrict__ cnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < pairs) atomicAdd(&cnt[dofs[i]], 1u);
}

__global__ void k_csr_fill(int64_t pairs, const int32_t* __restrict__ dofs, const int64_t* __restrict__ pair_ptr,
                           uint32_t* __restrict__ cursor, uint32_t* __restrict__ list)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pairs) return;
    const int32_t d = dofs[i];
    const uint32_t slot = atomicAdd(&cursor[d], 1u);
    list[pair_ptr[d] + slot] = (uint32_t)i;
}

// Each row's pair list in increasing order (so increasing element); also the
// largest list.  Lists are short (the elements around one node).
__global__ void k_csr_sort_pairs(int64_t N, const int64_t* __restrict__ pair_ptr, uint32_t* __restrict__ list,
                                 uint32_t* __restrict__ stats)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const int64_t a = pair_ptr[r], b = pair_ptr[r + 1];
    for (int64_t i = a + 1; i < b; i++) {
        const uint32_t v = list[i];
        int64_t j = i - 1;
        while (j >= a && list[j] > v) {
            list[j + 1] = list[j];
            j--;
        }
        list[j + 1] = v;
    }
    atomicMax(&stats[0], (uint32_t)(b - a));
}

// One 64-thread block per row (grid-stride).  The candidate columns of the
// row (the global numbers of all its elements) are sorted in LDS by a
// bitonic network; the distinct ones are the row's columns.
//   WRITE = 0: row_len[r] = number of columns, stats[1] = the largest
//   WRITE = 1: cols[row_ptr[r] ...] = columns, and pos[e*n + j][k] = index of
//              column dofs[e][k] within the row, for every pair (e, j) of r
template <int WRITE>
__global__ __launch_bounds__(CSR_WAVE) void k_csr_rows(int64_t N, int n, const int32_t* __restrict__ dofs,
                                                       const int64_t* __restrict__ pair_ptr,
                                                       const uint32_t* __restrict__ list,
                                                       uint32_t* __restrict__ row_len,
                                                       const int64_t* __restrict__ row_ptr,
                                                       int32_t* __restrict__ cols, uint16_t* __restrict__ pos,
                                                       uint32_t* __restrict__ stats, int cap)
{
    extern __shared__ int32_t sm[];
    int32_t* key = sm;          // [cap]
    int32_t* uniq = sm + cap;   // [cap] (WRITE only)
    const int t = threadIdx.x;
    const unsigned long long below = (1ull << t) - 1ull;
    for (int64_t r = blockIdx.x; r < N; r += gridDim.x) {
        const int64_t p0 = pair_ptr[r];
        const int m = (int)(pair_ptr[r + 1] - p0) * n;
        int P = CSR_WAVE;
        while (P < m) P <<= 1;
        for (int f = t; f < P; f += CSR_WAVE) {
            int32_t v = INT_MAX;
            if (f < m) {
                const int s = f / n;
                const uint32_t ej = list[p0 + s];
                v = dofs[(int64_t)(ej / (uint32_t)n) * n + (f - s * n)];
            }
            key[f] = v;
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = t; i < P; i += CSR_WAVE) {
                    const int l = i ^ j;
                    if (l > i) {
                        const int32_t a = key[i], b = key[l];
                        if ((a > b) == ((i & k) == 0)) {
                            key[i] = b;
                            key[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        int count = 0;
        for (int i0 = 0; i0 < m; i0 += CSR_WAVE) {
            const int i = i0 + t;
            const bool first = i < m && (i == 0 || key[i] != key[i - 1]);
            const unsigned long long bal = __ballot(first);
            if (WRITE && first) {
                const int idx = count + __popcll(bal & below);
                uniq[idx] = key[i];
                cols[row_ptr[r] + idx] = key[i];
            }
            count += __popcll(bal);
        }
        if (!WRITE) {
            if (t == 0) {
                row_len[r] = (uint32_t)count;
                atomicMax(&stats[1], (uint32_t)count);
            }
        } else {
            __syncthreads();
            for (int f = t; f < m; f += CSR_WAVE) {
                const int s = f / n;
                const int k = f - s * n;
                const uint32_t ej = list[p0 + s];
                const int32_t c = dofs[(int64_t)(ej / (uint32_t)n) * n + k];
                int lo = 0, hi = count;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (uniq[mid] < c) lo = mid + 1; else hi = mid;
                }
                pos[(int64_t)ej * n + k] = (uint16_t)lo;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Insertion
// ---------------------------------------------------------------------------

constexpr int INSERT_BATCH = 8;      // elements whose loads are in flight together
constexpr int INSERT_ROWS = 16;      // consecutive rows per visit of a block

// One 64-thread block per visit of INSERT_ROWS consecutive rows.  Blocks are
// renumbered so that consecutive visits run on one XCD (workgroups are dealt
// to the 8 XCDs in turn), which keeps the element-matrix lines shared by
// neighbouring rows in one L2.  KPL = entries of an element row per lane.
template <int KPL>
__global__ __launch_bounds__(CSR_WAVE) void k_csr_insert(int64_t N, int n, const int64_t* __restrict__ row_ptr,
                                                         const int64_t* __restrict__ pair_ptr,
                                                         const uint32_t* __restrict__ list,
                                                         const uint16_t* __restrict__ pos,
                                                         const double* __restrict__ A, double* __restrict__ vals)
{
    extern __shared__ double acc[];
    const int t = threadIdx.x;
    const int G = gridDim.x;
    const int b = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    for (int64_t r0 = (int64_t)b * INSERT_ROWS; r0 < N; r0 += (int64_t)G * INSERT_ROWS) {
        const int64_t r1 = r0 + INSERT_ROWS < N ? r0 + INSERT_ROWS : N;
        for (int64_t r = r0; r < r1; r++) {
            const int64_t rp = row_ptr[r];
            const int len = (int)(row_ptr[r + 1] - rp);
            for (int i = t; i < len; i += CSR_WAVE) acc[i] = 0.0;
            __syncthreads();
            const int64_t p0 = pair_ptr[r];
            const int c = (int)(pair_ptr[r + 1] - p0);
            for (int s0 = 0; s0 < c; s0 += INSERT_BATCH) {
                double v[INSERT_BATCH][KPL];
                int q[INSERT_BATCH][KPL];
#pragma unroll
                for (int u = 0; u < INSERT_BATCH; u++) {
                    if (s0 + u < c) {
                        const int64_t base = (int64_t)list[p0 + s0 + u] * n;
#pragma unroll
                        for (int kk = 0; kk < KPL; kk++) {
                            const int k = t + CSR_WAVE * kk;
                            if (k < n) {
                                v[u][kk] = A[base + k];
                                q[u][kk] = pos[base + k];
                            }
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < INSERT_BATCH; u++) {
                    if (s0 + u < c) {
#pragma unroll
                        for (int kk = 0; kk < KPL; kk++) {
                            const int k = t + CSR_WAVE * kk;
                            if (k < n) acc[q[u][kk]] += v[u][kk];
                        }
                        // the next element may add to the same entries from other lanes
                        __syncthreads();
                    }
                }
            }
            for (int i = t; i < len; i += CSR_WAVE) vals[rp + i] = acc[i];
            __syncthreads();
        }
    }
}

template <int KPL>
hipError_t launch_insert(int64_t N, int n, const int64_t* row_ptr, const int64_t* pair_ptr, const uint32_t* list,
                         const uint16_t* pos, const double* A, double* vals, size_t lds, hipStream_t s)
{
    static int per_cu[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    int occ = dev >= 0 && dev < 64 ? per_cu[dev] : 0;
    if (occ == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_csr_insert<KPL>, CSR_WAVE, lds) != hipSuccess ||
            occ <= 0)
            occ = 8;
        if (dev >= 0 && dev < 64) per_cu[dev] = occ;
    }
    const int64_t visits = (N + INSERT_ROWS - 1) / INSERT_ROWS;
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > visits) grid = visits;
    if (grid < 1) grid = 1;
    k_csr_insert<KPL><<<(unsigned)grid, CSR_WAVE, lds, s>>>(N, n, row_ptr, pair_ptr, list, pos, A, vals);
    return hipGetLastError();
}

}  // namespace
}  // namespace fe

struct fe_csr {
    int64_t E = 0, N = 0, nnz = 0;
    int n = 0, max_row = 0, max_pairs = 0;
    int64_t* row_ptr = nullptr;    // [N + 1]
    int32_t* cols = nullptr;       // [nnz]
    int64_t* pair_ptr = nullptr;   // [N + 1]
    uint32_t* list = nullptr;      // [E * n] pairs e * n + j of each row, increasing
    uint16_t* pos = nullptr;       // [E * n * n]
};

static void csr_free(fe_csr* c)
{
    if (!c) return;
    (void)hipFree(c->row_ptr);
    (void)hipFree(c->cols);
    (void)hipFree(c->pair_ptr);
    (void)hipFree(c->list);
    (void)hipFree(c->pos);
    delete c;
}

extern "C" int fe_csr_create(int64_t n_elems, int n, const int32_t* cell_dofs, int64_t n_rows, void* stream,
                             fe_csr_t** out)
{
    using namespace fe;
    if (!out) return FE_EINVAL;
    *out = nullptr;
    if (n_elems < 0 || n < 1 || n_rows < 0 || (n_elems > 0 && !cell_dofs)) return FE_EINVAL;
    if (n > CSR_MAX_N || n_rows >= INT32_MAX || (uint64_t)n_elems * (uint64_t)n >= (1ull << 32))
        return FE_ENOTSUP;
    hipStream_t s = (hipStream_t)stream;
    fe_csr* c = new fe_csr();
    c->E = n_elems;
    c->n = n;
    c->N = n_rows;
    const int64_t pairs = n_elems * n;
    uint32_t* cnt = nullptr;     // [N] counts, then cursors, then row lengths
    uint32_t* stats = nullptr;   // [0] largest pair list, [1] longest row; [2] validation flags
    hipError_t e = hipSuccess;
    auto fail = [&](int code) {
        (void)hipFree(cnt);
        (void)hipFree(stats);
        csr_free(c);
        return code;
    };
    auto hip_fail = [&](hipError_t err, const char* where) { return fail(set_hip_error(err, where)); };
    const size_t Nb = (size_t)(n_rows > 0 ? n_rows : 1);
    if (hipMalloc(&c->row_ptr, sizeof(int64_t) * (Nb + 1)) != hipSuccess ||
        hipMalloc(&c->pair_ptr, sizeof(int64_t) * (Nb + 1)) != hipSuccess ||
        hipMalloc(&c->list, sizeof(uint32_t) * (size_t)(pairs > 0 ? pairs : 1)) != hipSuccess ||
        hipMalloc(&c->pos, sizeof(uint16_t) * (size_t)(pairs > 0 ? pairs * n : 1)) != hipSuccess ||
        hipMalloc(&cnt, sizeof(uint32_t) * Nb) != hipSuccess || hipMalloc(&stats, sizeof(uint32_t) * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FE_ENOMEM);
    }
    const unsigned TB = 256;
    const unsigned pblocks = (unsigned)((pairs + TB - 1) / TB);
    const unsigned rblocks = (unsigned)((n_rows + TB - 1) / TB);
    uint32_t h_stats[4] = {0, 0, 0, 0};
    if ((e = hipMemsetAsync(stats, 0, sizeof(uint32_t) * 4, s)) != hipSuccess) return hip_fail(e, "csr init");
    if (pairs > 0) {
        k_csr_validate<<<pblocks, TB, 0, s>>>(pairs, n, cell_dofs, n_rows, (int*)(stats + 2));
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "csr validate");
        if ((e = hipMemcpyAsync(h_stats, stats, sizeof(h_stats), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "csr validate");
        if (h_stats[2] != 0) return fail(FE_EINVAL);
    }
    // pairs of each row
    if ((e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * Nb, s)) != hipSuccess) return hip_fail(e, "csr count");
    if (pairs > 0) {
        k_csr_count<<<pblocks, TB, 0, s>>>(pairs, cell_dofs, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "csr count");
    }
    if ((e = scan_exclusive<uint32_t>(cnt, n_rows, c->pair_ptr, s)) != hipSuccess) return hip_fail(e, "csr scan");
    if ((e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * Nb, s)) != hipSuccess) return hip_fail(e, "csr fill");
    if (pairs > 0) {
        k_csr_fill<<<pblocks, TB, 0, s>>>(pairs, cell_dofs, c->pair_ptr, cnt, c->list);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "csr fill");
    }
    if (n_rows > 0) {
        k_csr_sort_pairs<<<rblocks, TB, 0, s>>>(n_rows, c->pair_ptr, c->list, stats);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "csr sort");
    }
    if ((e = hipMemcpyAsync(h_stats, stats, sizeof(h_stats), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "csr sort");
    c->max_pairs = (int)h_stats[0];
    const int64_t cand = (int64_t)c->max_pairs * n;
    if (cand > CSR_MAX_CANDIDATES) return fail(FE_ENOTSUP);
    int cap = CSR_WAVE;
    while (cap < cand) cap <<= 1;
    // columns: lengths, scan, then columns and positions
    int grid = device_cus() * 16;
    if (n_rows < grid) grid = (int)(n_rows > 0 ? n_rows : 1);
    if (n_rows > 0) {
        k_csr_rows<0><<<grid, CSR_WAVE, sizeof(int32_t) * cap, s>>>(n_rows, n, cell_dofs, c->pair_ptr, c->list, cnt,
                                                                   nullptr, nullptr, nullptr, stats, cap);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "csr row lengths");
    }
    if ((e = scan_exclusive<uint32_t>(cnt, n_rows, c->row_ptr, s)) != hipSuccess) return hip_fail(e, "csr scan");
    int64_t nnz = 0;
    if ((e = hipMemcpyAsync(&nnz, c->row_ptr + n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(h_stats, stats, sizeof(h_stats), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "csr row lengths");
    c->nnz = nnz;
    c->max_row = (int)h_stats[1];
    if (hipMalloc(&c->cols, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FE_ENOMEM);
    }
    if (n_rows > 0) {
        k_csr_rows<1><<<grid, CSR_WAVE, 2 * sizeof(int32_t) * cap, s>>>(n_rows, n, cell_dofs, c->pair_ptr, c->list,
                                                                       nullptr, c->row_ptr, c->cols, c->pos, stats,
                                                                       cap);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "csr columns");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "csr columns");
    (void)hipFree(cnt);
    (void)hipFree(stats);
    *out = c;
    return FE_OK;
}

extern "C" int fe_csr_info(const fe_csr_t* c, int64_t* n_rows, int64_t* nnz, int* max_row_len)
{
    if (!c) return FE_EINVAL;
    if (n_rows) *n_rows = c->N;
    if (nnz) *nnz = c->nnz;
    if (max_row_len) *max_row_len = c->max_row;
    return FE_OK;
}

extern "C" int fe_csr_pattern(const fe_csr_t* c, int64_t* row_ptr, int32_t* col_idx, void* stream)
{
    if (!c || !row_ptr || (c->nnz > 0 && !col_idx)) return FE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(row_ptr, c->row_ptr, sizeof(int64_t) * (size_t)(c->N + 1),
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && c->nnz > 0)
        e = hipMemcpyAsync(col_idx, c->cols, sizeof(int32_t) * (size_t)c->nnz, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? FE_OK : fe::set_hip_error(e, "fe_csr_pattern");
}

extern "C" int fe_csr_insert(const fe_csr_t* c, const double* local_A, double* values, void* stream)
{
    using namespace fe;
    if (!c || (c->nnz > 0 && (!local_A || !values))) return FE_EINVAL;
    if (c->nnz == 0) return FE_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = sizeof(double) * (size_t)(c->max_row > 0 ? c->max_row : 1);
    const int kpl = (c->n + CSR_WAVE - 1) / CSR_WAVE;
    hipError_t e;
    switch (kpl) {
    case 1: e = launch_insert<1>(c->N, c->n, c->row_ptr, c->pair_ptr, c->list, c->pos, local_A, values, lds, s); break;
    case 2: e = launch_insert<2>(c->N, c->n, c->row_ptr, c->pair_ptr, c->list, c->pos, local_A, values, lds, s); break;
    default:
        e = launch_insert<4>(c->N, c->n, c->row_ptr, c->pair_ptr, c->list, c->pos, local_A, values, lds, s);
        break;
    }
    return e == hipSuccess ? FE_OK : set_hip_error(e, "fe_csr_insert");
}

extern "C" int fe_csr_destroy(fe_csr_t* c)
{
    if (!c) return FE_EINVAL;
    (void)hipDeviceSynchronize();
    csr_free(c);
    return FE_OK;
}
