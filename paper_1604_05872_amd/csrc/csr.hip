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
//   4. the position table: for the t-th pair (e, j) of the row lists (rows in
//      order, each row's pairs in increasing element order), pos[t][k] is
//      where column dofs[e][k] sits within row dofs[e][j].  The insertion
//      reads it in that order, one contiguous stream.
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
#include "csr.hpp"
#include "internal.hpp"

namespace fe {
namespace {

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

// LDS sizes of the insertion: for rr = 1, 2, 4, ..., 32 the longest run of
// rr consecutive rows starting at a multiple of rr (entries), and the most
// element pairs of a visit of VISIT_ROWS rows.
__global__ void k_csr_round_stats(int64_t N, const int64_t* __restrict__ row_ptr,
                                  const int64_t* __restrict__ pair_ptr, int visit_rows,
                                  uint32_t* __restrict__ stats)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int l = 0; l < CSR_RR_LEVELS; l++) {
        const int64_t rr = (int64_t)1 << l;
        if (r % rr == 0) {
            const int64_t e = r + rr < N ? r + rr : N;
            atomicMax(&stats[l], (uint32_t)(row_ptr[e] - row_ptr[r]));
        }
    }
    if (r % visit_rows == 0) {
        const int64_t e = r + visit_rows < N ? r + visit_rows : N;
        atomicMax(&stats[CSR_RR_LEVELS], (uint32_t)(pair_ptr[e] - pair_ptr[r]));
    }
}

// One 64-thread block per row (grid-stride).  The candidate columns of the
// row (the global numbers of all its elements) are sorted in LDS by a
// bitonic network; the distinct ones are the row's columns.
//   WRITE = 0: row_len[r] = number of columns, stats[1] = the largest
//   WRITE = 1: cols[row_ptr[r] ...] = columns, and pos[t][k] = index of column
//              dofs[e][k] within the row, for every pair t = (e, j) of r
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
                pos[(p0 + s) * n + k] = (uint16_t)lo;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Insertion
// ---------------------------------------------------------------------------


// W lanes per row (a power of two, at least n / KPL; W < 64 puts 64 / W rows
// side by side in the wavefront), KPL entries of an element row per lane, IL
// rows interleaved per lane group so that their loads are in flight together,
// B elements per row per batch of loads.  A round covers RR = (64 / W) * IL
// consecutive rows, whose values are one contiguous LDS region: zeroed, then
// accumulated element by element in increasing element order (the rows of a
// round are disjoint, and a barrier separates two elements of one row), then
// stored with contiguous writes.  Blocks are renumbered so that consecutive
// visits run on one XCD (workgroups are dealt to the 8 XCDs in turn), which
// keeps the element-matrix lines shared by neighbouring rows in one L2.
template <int W, int KPL, int IL, int B>
__global__ __launch_bounds__(CSR_WAVE) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_csr_insert(int64_t N, int n, const int64_t* __restrict__ row_ptr,
                                                         const int64_t* __restrict__ pair_ptr,
                                                         const uint32_t* __restrict__ list,
                                                         const uint16_t* __restrict__ pos,
                                                         const double* __restrict__ A, double* __restrict__ vals,
                                                         int round_cap)
{
    constexpr int SUB = CSR_WAVE / W;
    constexpr int RR = SUB * IL;
    static_assert(VISIT_ROWS % RR == 0, "a visit is whole rounds");
    extern __shared__ double smem[];
    double* acc = smem;                                             // [round_cap] values of a round
    uint32_t* seg = reinterpret_cast<uint32_t*>(smem + round_cap);  // the visit's element lists
    const int t = threadIdx.x;
    const int g = t / W;
    const int kl = t % W;
    const int G = gridDim.x;
    const int b = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    for (int64_t v0 = (int64_t)b * VISIT_ROWS; v0 < N; v0 += (int64_t)G * VISIT_ROWS) {
        const int nv = (int)(N - v0 < VISIT_ROWS ? N - v0 : VISIT_ROWS);
        int64_t my_rp = 0, my_pp = 0;
        if (t <= nv) {
            my_rp = row_ptr[v0 + t];
            my_pp = pair_ptr[v0 + t];
        }
        const int64_t P0 = __shfl(my_pp, 0);
        const int np = (int)(__shfl(my_pp, nv) - P0);
        for (int i = t; i < np; i += CSR_WAVE) seg[i] = list[P0 + i];
        __syncthreads();
        for (int r0 = 0; r0 < nv; r0 += RR) {
            const int nr = nv - r0 < RR ? nv - r0 : RR;
            const int64_t vb = __shfl(my_rp, r0);
            const int V = (int)(__shfl(my_rp, r0 + nr) - vb);
            for (int i = t; i < V; i += CSR_WAVE) acc[i] = 0.0;
            int off[IL], cnt[IL], lp[IL];
            int cmax = 0;
#pragma unroll
            for (int i = 0; i < IL; i++) {
                const int li = r0 + g * IL + i;   // < VISIT_ROWS
                const int64_t rp = __shfl(my_rp, li);
                const int64_t pp = __shfl(my_pp, li);
                const int64_t pe = __shfl(my_pp, li + 1);
                const bool ok = g * IL + i < nr;
                off[i] = ok ? (int)(rp - vb) : 0;
                cnt[i] = ok ? (int)(pe - pp) : 0;
                lp[i] = (int)(pp - P0);
                cmax = cnt[i] > cmax ? cnt[i] : cmax;
            }
            for (int o = CSR_WAVE / 2; o > 0; o >>= 1) {
                const int x = __shfl_xor(cmax, o);
                cmax = x > cmax ? x : cmax;
            }
            __syncthreads();
            for (int s0 = 0; s0 < cmax; s0 += B) {
                // Loads are unconditional so that none sits in a branch and
                // all of them are in flight together: a slot past a row's
                // last element re-reads that element (a row without elements
                // reads the visit's first), a lane past n re-reads entry
                // n - 1, so the extra reads hit lines the wavefront loads anyway.
                double v[IL][B][KPL];
                int q[IL][B][KPL];
#pragma unroll
                for (int i = 0; i < IL; i++)
#pragma unroll
                    for (int u = 0; u < B; u++) {
                        const int sl = s0 + u < cnt[i] ? lp[i] + s0 + u : cnt[i] > 0 ? lp[i] + cnt[i] - 1 : 0;
                        const uint32_t ej = np > 0 ? seg[sl] : 0u;
                        const uint64_t base = (uint64_t)ej * (uint32_t)n;
                        const uint64_t pbase = (uint64_t)(np > 0 ? P0 + sl : 0) * (uint32_t)n;
#pragma unroll
                        for (int kk = 0; kk < KPL; kk++) {
                            const int k = kl + W * kk < n ? kl + W * kk : n - 1;
                            v[i][u][kk] = A[base + k];
                            q[i][u][kk] = pos[pbase + k];
                        }
                    }
#pragma unroll
                for (int u = 0; u < B; u++) {
#pragma unroll
                    for (int i = 0; i < IL; i++)
                        if (s0 + u < cnt[i]) {
#pragma unroll
                            for (int kk = 0; kk < KPL; kk++) {
                                const int k = kl + W * kk;
                                if (k < n) acc[off[i] + q[i][u][kk]] += v[i][u][kk];
                            }
                        }
                    // the next element of a row may add to the same entries from other lanes
                    __syncthreads();
                }
            }
            for (int i = t; i < V; i += CSR_WAVE) vals[vb + i] = acc[i];
            __syncthreads();
        }
    }
}

template <int W, int KPL, int IL, int B>
hipError_t launch_insert(int64_t N, int n, const int64_t* row_ptr, const int64_t* pair_ptr, const uint32_t* list,
                         const uint16_t* pos, const double* A, double* vals, int round_cap, int visit_pairs,
                         hipStream_t s)
{
    const size_t lds = insert_lds(round_cap, visit_pairs);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_csr_insert<W, KPL, IL, B>, CSR_WAVE, lds) !=
            hipSuccess ||
        occ <= 0)
        occ = 8;
    const int64_t visits = (N + VISIT_ROWS - 1) / VISIT_ROWS;
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid > visits) grid = visits;
    if (grid < 1) grid = 1;
    k_csr_insert<W, KPL, IL, B><<<(unsigned)grid, CSR_WAVE, lds, s>>>(N, n, row_ptr, pair_ptr, list, pos, A, vals,
                                                                       round_cap);
    return hipGetLastError();
}

}  // namespace
}  // namespace fe

void fe::csr_free(fe_csr* c)
{
    if (!c) return;
    (void)hipFree(c->row_ptr);
    (void)hipFree(c->cols);
    (void)hipFree(c->pair_ptr);
    (void)hipFree(c->list);
    (void)hipFree(c->pos);
    (void)hipFree(c->geo);
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
    {
        uint32_t h_round[CSR_RR_LEVELS + 1] = {0};
        uint32_t* d_round = nullptr;
        if (hipMalloc(&d_round, sizeof(h_round)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FE_ENOMEM);
        }
        e = hipMemsetAsync(d_round, 0, sizeof(h_round), s);
        if (e == hipSuccess && n_rows > 0) {
            k_csr_round_stats<<<rblocks, TB, 0, s>>>(n_rows, c->row_ptr, c->pair_ptr, VISIT_ROWS, d_round);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(h_round, d_round, sizeof(h_round), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(d_round);
        if (e != hipSuccess) return hip_fail(e, "csr round sizes");
        for (int l = 0; l < CSR_RR_LEVELS; l++) c->round_len[l] = (int)h_round[l];
        c->visit_pairs = (int)h_round[CSR_RR_LEVELS];
    }
    if (insert_lds(c->round_len[0], c->visit_pairs) > device_lds_per_block()) return fail(FE_ENOTSUP);
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
    hipError_t e;
    // rows side by side need LDS for each; one row per round always fits (checked at creation)
    // one row per lane group up to n = 64 (measured on MI355X: Helmholtz tet
    // P3 1.51 -> 1.32 ms, P4 4.43 -> 4.03 ms against two interleaved rows)
    const int W = c->n <= 4 ? 4 : c->n <= 8 ? 8 : c->n <= 16 ? 16 : c->n <= 32 ? 32 : 64;
    const int IL = c->n <= 64 || c->n > 128 ? 1 : 2;
    int level = 0;
    while ((1 << level) < CSR_WAVE / W * IL) level++;
    const int vp = c->visit_pairs > 0 ? c->visit_pairs : 1;
    const int cap = c->round_len[level] > 0 ? c->round_len[level] : 1;
    const int cap1 = c->round_len[0] > 0 ? c->round_len[0] : 1;
#define FE_INSERT(W, KPL, IL, B, CAP) \
    launch_insert<W, KPL, IL, B>(c->N, c->n, c->row_ptr, c->pair_ptr, c->list, c->pos, local_A, values, CAP, vp, s)
    if (insert_lds(cap, vp) > device_lds_per_block()) {
        if (c->n <= 64) e = FE_INSERT(64, 1, 1, 4, cap1);
        else if (c->n <= 128) e = FE_INSERT(64, 2, 1, 4, cap1);
        else e = FE_INSERT(64, 4, 1, 4, cap1);
    } else if (c->n <= 4) e = FE_INSERT(4, 1, 1, 8, cap);
    else if (c->n <= 8) e = FE_INSERT(8, 1, 1, 8, cap);
    else if (c->n <= 16) e = FE_INSERT(16, 1, 1, 8, cap);
    else if (c->n <= 32) e = FE_INSERT(32, 1, 1, 4, cap);
    else if (c->n <= 64) e = FE_INSERT(64, 1, 1, 4, cap);
    else if (c->n <= 128) e = FE_INSERT(64, 2, 2, 4, cap);
    else e = FE_INSERT(64, 4, 1, 4, cap);
#undef FE_INSERT
    return e == hipSuccess ? FE_OK : set_hip_error(e, "fe_csr_insert");
}

extern "C" int fe_csr_destroy(fe_csr_t* c)
{
    if (!c) return FE_EINVAL;
    (void)hipDeviceSynchronize();
    fe::csr_free(c);
    return FE_OK;
}
