// Pre-evaluated linear elasticity (Sec. 3.3 with the coefficient expansion
// of Sec. 4.2): the Lame fields are P1, lambda(X) = sum_l lambda_l psi_l(X)
// and likewise mu, so with g_{j,c} = sum_a K[a][c] dphi_{j,a} every
// monomial's coefficient is a polynomial and the reduction over points
// hoists into reference tables
//     T_{l,a,b}[j][k] = sum_q W_q psi_l(X_q) dphi_{q,j,a} dphi_{q,k,b}
// (iota = n_c = the P1 basis size, rho = d^2 per table set).  Block (c, e)
// of the element matrix is then
//     A[(c,j),(e,k)] = sum_{l,a,b} C^{ce}_{l,a,b} T_{l,a,b}[j][k],
//     C^{ce}_{l,a,b} = |det J| (lambda_l K_ac K_be + mu_l K_ae K_bc
//                               + delta_ce mu_l (K K^T)_ab):
// one dense product of a (16 elements) x (n_c d^2) coefficient matrix with
// the table matrix per block, on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64).  A workgroup takes a 16-element tile: it forms
// the coefficient rows of all d^2 blocks in LDS, then its wavefronts split
// the 16-entry column groups, each group's table values (read through the
// L2; the planner admits the tables only when they fit T_H) feeding the
// d^2 blocks as independent accumulator chains.
#include <algorithm>
#include <mutex>

#include "device_common.hpp"
#include "internal.hpp"

namespace fe {

typedef double v4d_e __attribute__((ext_vector_type(4)));
typedef unsigned u2_e __attribute__((ext_vector_type(2)));
// buffer resource word 3 on gfx950: a raw (stride 0) byte buffer whose
// accesses are range-checked against num_records; stores beyond it are
// dropped
constexpr int BUFFER_WORD3 = 0x00020000;

namespace {

// wavefronts per workgroup: eight on prisms, whose coefficient rows are the
// largest to form and whose units hold the most column groups (prism P4
// 1.79 -> 1.65 ms on MI355X), four elsewhere (eight are slower there)
__host__ __device__ constexpr int pe_waves(int cell) { return cell == PRISM ? 8 : 4; }

// T[((l * d + a) * d + b)][j * ns + k]
__global__ void k_elast_tables(int nq, int ns, int d, int nc, const double* __restrict__ W,
                               const double* __restrict__ psi, const double* __restrict__ dphi, double* __restrict__ T)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nn = ns * ns, nt = nc * d * d;
    if (tid >= (int64_t)nt * nn) return;
    const int t = (int)(tid / nn), jk = (int)(tid % nn), j = jk / ns, k = jk % ns;
    const int l = t / (d * d), a = (t / d) % d, b = t % d;
    double x = 0.0;
    for (int q = 0; q < nq; ++q)
        x = fma(W[q] * psi[q * nc + l], dphi[(q * ns + j) * d + a] * dphi[(q * ns + k) * d + b], x);
    T[tid] = x;
}

struct ElastArgs {
    const double* coords;
    const double* coeff;   // [E][2][nc]: lambda, then mu, at the vertices
    double* out;           // [E][n][n]
    int* status;
    const double* T;       // [nt][ns * ns]
    int64_t E;
    int ns;
    int parts;             // column-group ranges per tile (units = tiles x parts)
};

template <int CELL>
__global__ __launch_bounds__(64 * pe_waves(CELL)) __attribute__((amdgpu_waves_per_eu(2))) void k_preeval_elast(ElastArgs a)
{
    constexpr int PE_WAVES = pe_waves(CELL);
    constexpr int D = cell_dim(CELL), NC = cell_nv(CELL), NVD = NC * D;
    constexpr int NT = NC * D * D, NTP = (NT + 7) / 8 * 8, NB = D * D, NK = NTP / 4;
    // coefficient rows [block][element][(l, a, b)], rows NTP + 1 doubles apart
    // so that the 16 rows of an operand read fall in distinct LDS banks
    constexpr int LDA = NTP + 1;
    __shared__ double sA[NB * 16 * LDA];
    __shared__ double sG[16 * 12];           // K [9], |det J|, flag
    __shared__ double sL[16 * 2 * NC];       // Lame nodal values
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    const int ns = a.ns, nn = ns * ns, n = D * ns;
    const int64_t ntiles = (a.E + 15) / 16;
    const int ncb = (nn + 15) / 16;
    const int parts = a.parts;                 // column-group ranges per tile
    const int64_t units = ntiles * parts;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t tile = u / parts;
        const int part = (int)(u - tile * parts);
        const int64_t e0 = tile * 16;
        const int ne = a.E - e0 < 16 ? (int)(a.E - e0) : 16;
        // geometry and Lame values of the tile's elements
        if (tid < 16) {
            double K[3][3], adet;
            int bad = 0;
            if (tid < ne) {
                double v[NVD];
#pragma unroll
                for (int i = 0; i < NVD; ++i) v[i] = a.coords[(e0 + tid) * NVD + i];
                bad = affine_map<CELL>(v, K, adet);
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int q = 0; q < 3; ++q) K[r][q] = 0.0;
                adet = 0.0;
            }
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int q = 0; q < D; ++q) sG[tid * 12 + r * 3 + q] = K[r][q];
            sG[tid * 12 + 9] = adet;
            sG[tid * 12 + 10] = bad ? 1.0 : 0.0;
            // the tile's first unit reports flagged elements
            if (bad && part == 0 && a.status) atomicAdd(a.status, 1);
        }
        for (int i = tid; i < 16 * 2 * NC; i += blockDim.x) sL[i] = i < ne * 2 * NC ? a.coeff[e0 * 2 * NC + i] : 0.0;
        __syncthreads();
        // coefficient rows C^{c e2}[e][(l, a, b)] of every block, zero-padded to NTP
        for (int i = tid; i < NB * 16 * NTP; i += blockDim.x) {
            const int blk = i / (16 * NTP), r = i - blk * 16 * NTP, e = r / NTP, t = r - e * NTP;
            const int at = (blk * 16 + e) * LDA + t;
            const int c = blk / D, e2 = blk - c * D;
            double x = 0.0;
            if (t < NT) {
                const int l = t / (D * D), aa = (t / D) % D, b = t % D;
                const double* K = sG + e * 12;
                const double lam = sL[e * 2 * NC + l], mu = sL[e * 2 * NC + NC + l];
                x = lam * (K[aa * 3 + c] * K[b * 3 + e2]) + mu * (K[aa * 3 + e2] * K[b * 3 + c]);
                if (c == e2) {
                    double g = 0.0;
#pragma unroll
                    for (int m = 0; m < D; ++m) g = fma(K[aa * 3 + m], K[b * 3 + m], g);
                    x = fma(mu, g, x);
                }
                x *= K[9];
            }
            sA[at] = x;
        }
        __syncthreads();
        // the tile's output as a buffer of ne element matrices (byte records)
        const int nn_e = n * n;
        const __amdgpu_buffer_rsrc_t out_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            a.out + e0 * (int64_t)nn_e, 0, (int)((unsigned)ne * (unsigned)nn_e * 8u), BUFFER_WORD3);
        bool bad_row[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bad_row[r] = sG[(kq + 4 * r) * 12 + 10] != 0.0;
        // this unit's column groups, wavefront w taking every PE_WAVES-th; a
        // group's table values feed all NB blocks, loaded one group ahead
        const int cb_lo = (int)((int64_t)ncb * part / parts), cb_hi = (int)((int64_t)ncb * (part + 1) / parts);
        double bv[NK];
        auto load_b = [&](int cb) {
            const int col = 16 * cb + i16;
            const int colc = col < nn ? col : nn - 1;   // in-range table column for padding lanes
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                const int k = 4 * kk + kq;
                bv[kk] = k < NT ? a.T[(size_t)k * nn + colc] : 0.0;
            }
        };
        if (cb_lo + w < cb_hi) load_b(cb_lo + w);
        for (int cb = cb_lo + w; cb < cb_hi; cb += PE_WAVES) {
            double bc[NK];
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) bc[kk] = bv[kk];
            if (cb + PE_WAVES < cb_hi) load_b(cb + PE_WAVES);
            // blocks in groups of D (D independent accumulator chains per
            // group, few registers live), each group stored before the next
            const int col = 16 * cb + i16;
            const int j = col < nn ? col / ns : 0, k = col < nn ? col - (col / ns) * ns : 0;
#pragma unroll 1
            for (int c = 0; c < D; ++c) {
                v4d_e acc[D];
#pragma unroll
                for (int e2 = 0; e2 < D; ++e2) acc[e2] = (v4d_e){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < NK; ++kk)
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2)
                        acc[e2] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            sA[((c * D + e2) * 16 + i16) * LDA + 4 * kk + kq], bc[kk], acc[e2], 0, 0, 0);
                // lane holds elements kq + 4 r, entry col = (j, k) of blocks
                // (c, e2).  Every store is issued: a lane past the block or an
                // element past the tile addresses beyond the tile's records,
                // and the buffer unit drops it
#pragma unroll
                for (int e2 = 0; e2 < D; ++e2) {
                    const unsigned off = (unsigned)((c * ns + j) * n + e2 * ns + k);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const unsigned byte = col < nn ? (unsigned)((kq + 4 * r) * nn_e + off) * 8u : 0x80000000u;
                        const double v = bad_row[r] ? __builtin_nan("") : acc[e2][r];
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_e, v), out_rsrc, byte, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Row-staged variant for triangles and tetrahedra with n_s >= 16 (a
// 16-entry column group then touches at most two rows of a block).  A unit is (16-element tile, block row c): the
// workgroup forms the coefficient rows of blocks (c, e2), e2 < d, and its
// four wavefronts split the n_s rows j into contiguous bands.  A wavefront
// walks its band's (j, k) entries 16 at a time (any 16 table columns serve as
// one MFMA column group, so only a band's last group is partial), writes the
// d blocks' results into its own LDS row buffer [16 elements][n], and as soon
// as row (c, j) is complete stores it for the 16 elements: per element one
// contiguous run of n doubles, and consecutive rows of the band follow each
// other in memory, so the L2 receives whole lines from one wavefront instead
// of 128-byte pieces from several.
template <int CELL>
__global__ __launch_bounds__(256) void k_preeval_elast_rows(ElastArgs a)
{
    constexpr int D = cell_dim(CELL), NC = cell_nv(CELL), NVD = NC * D;
    constexpr int NT = NC * D * D, NTP = (NT + 7) / 8 * 8, NK = NTP / 4;
    constexpr int LDA = NTP + 1;
    extern __shared__ double lds_rows[];
    const int ns = a.ns, nn = ns * ns, n = D * ns, ldr = n | 1;
    double* sA = lds_rows;                       // [D][16][LDA] blocks (c, e2)
    double* sG = sA + D * 16 * LDA;              // [16][12] K, |det J|, flag
    double* sL = sG + 16 * 12;                   // [16][2 NC] Lame nodal values
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    double* slot = sL + 16 * 2 * NC + (size_t)w * 16 * ldr;   // [16][ldr] this wavefront's row
    const int64_t ntiles = (a.E + 15) / 16;
    const int64_t units = ntiles * D;
    const int jA = ns * w / 4, jB = ns * (w + 1) / 4;
    const int f0 = jA * ns, f1 = jB * ns;        // the band's (j, k) entries
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t tile = u / D;
        const int c = (int)(u - tile * D);
        const int64_t e0 = tile * 16;
        const int ne = a.E - e0 < 16 ? (int)(a.E - e0) : 16;
        if (tid < 16) {
            double K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, adet = 0.0;
            int bad = 0;
            if (tid < ne) {
                double v[NVD];
#pragma unroll
                for (int i = 0; i < NVD; ++i) v[i] = a.coords[(e0 + tid) * NVD + i];
                bad = affine_map<CELL>(v, K, adet);
                // the tile's first unit reports flagged elements
                if (bad && c == 0 && a.status) atomicAdd(a.status, 1);
            }
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q) sG[tid * 12 + r * 3 + q] = K[r][q];
            sG[tid * 12 + 9] = adet;
            sG[tid * 12 + 10] = bad ? 1.0 : 0.0;
        }
        for (int i = tid; i < 16 * 2 * NC; i += blockDim.x) sL[i] = i < ne * 2 * NC ? a.coeff[e0 * 2 * NC + i] : 0.0;
        __syncthreads();
        // coefficient rows C^{c e2}[e][(l, a, b)] of the unit's blocks, zero-padded to NTP
        for (int i = tid; i < D * 16 * NTP; i += blockDim.x) {
            const int e2 = i / (16 * NTP), r = i - e2 * 16 * NTP, e = r / NTP, t = r - e * NTP;
            double x = 0.0;
            if (t < NT) {
                const int l = t / (D * D), aa = (t / D) % D, b = t % D;
                const double* K = sG + e * 12;
                const double lam = sL[e * 2 * NC + l], mu = sL[e * 2 * NC + NC + l];
                x = lam * (K[aa * 3 + c] * K[b * 3 + e2]) + mu * (K[aa * 3 + e2] * K[b * 3 + c]);
                if (c == e2) {
                    double g = 0.0;
#pragma unroll
                    for (int m = 0; m < D; ++m) g = fma(K[aa * 3 + m], K[b * 3 + m], g);
                    x = fma(mu, g, x);
                }
                x *= K[9];
            }
            sA[(e2 * 16 + e) * LDA + t] = x;
        }
        __syncthreads();
        // row (c, j) of the tile's elements, from the row buffer
        auto flush = [&](int j) {
            double* o = a.out + e0 * (int64_t)n * n + (int64_t)(c * ns + j) * n;
            int e = 0, m = lane;
            while (m >= n) {
                m -= n;
                ++e;
            }
            for (; e < ne;) {
                const double v = sG[e * 12 + 10] != 0.0 ? __builtin_nan("") : slot[e * ldr + m];
                store_out(o + (int64_t)e * n * n + m, v, 0);
                m += 64;
                while (m >= n) {
                    m -= n;
                    ++e;
                }
            }
        };
        double bv[NK];
        auto load_b = [&](int f) {
            const int col = f + i16;
            const int colc = col < f1 ? col : f1 - 1;   // in-range table column for padding lanes
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                const int k = 4 * kk + kq;
                bv[kk] = k < NT ? a.T[(size_t)k * nn + colc] : 0.0;
            }
        };
        if (f0 < f1) load_b(f0);
        int jcur = jA;
        for (int f = f0; f < f1; f += 16) {
            double bc[NK];
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) bc[kk] = bv[kk];
            if (f + 16 < f1) load_b(f + 16);
            v4d_e acc[D];
#pragma unroll
            for (int e2 = 0; e2 < D; ++e2) acc[e2] = (v4d_e){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < NK; ++kk)
#pragma unroll
                for (int e2 = 0; e2 < D; ++e2)
                    acc[e2] = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[(e2 * 16 + i16) * LDA + 4 * kk + kq], bc[kk],
                                                                   acc[e2], 0, 0, 0);
            // lane holds elements kq + 4 r, entry col = (j, k) of blocks (c, e2)
            const int col = f + i16;
            const bool valid = col < f1;
            const int j = valid ? col / ns : -1, k = valid ? col - (col / ns) * ns : 0;
            if (j == jcur) {
#pragma unroll
                for (int e2 = 0; e2 < D; ++e2)
#pragma unroll
                    for (int r = 0; r < 4; ++r) slot[(kq + 4 * r) * ldr + e2 * ns + k] = acc[e2][r];
            }
            const int flast = (f + 16 < f1 ? f + 16 : f1) - 1;
            if (flast >= (jcur + 1) * ns - 1) {
                // row jcur is complete: store it, then the group's entries of the next row
                wave_sync();
                flush(jcur);
                wave_sync();
                ++jcur;
                if (j == jcur) {
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2)
#pragma unroll
                        for (int r = 0; r < 4; ++r) slot[(kq + 4 * r) * ldr + e2 * ns + k] = acc[e2][r];
                }
            }
        }
        __syncthreads();
    }
}

// raise the kernel's dynamic LDS limit to `bytes` once per (device, cell)
// (a host-side attribute, so it is also safe while a stream is captured)
hipError_t allow_dynamic_lds(const void* fn, int cell, size_t bytes)
{
    static std::mutex mu;
    static size_t done[64][3] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) return e != hipSuccess ? e : hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (done[dev][cell] >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done[dev][cell] = bytes;
    return e;
}

size_t preeval_elast_rows_lds_bytes(int cell, int ns)
{
    const int d = cell_dim(cell), nc = cell_nv(cell), nt = nc * d * d, ntp = (nt + 7) / 8 * 8;
    const int n = d * ns, ldr = n | 1;
    return sizeof(double) * ((size_t)d * 16 * (ntp + 1) + 16 * 12 + 16 * 2 * (size_t)nc + (size_t)4 * 16 * ldr);
}

}  // namespace

hipError_t launch_elast_tables(int nq, int ns, int d, int nc, const double* W, const double* psi, const double* dphi,
                               double* T, hipStream_t s)
{
    const int64_t n = (int64_t)nc * d * d * ns * ns;
    hipLaunchKernelGGL(k_elast_tables, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, nq, ns, d, nc, W, psi, dphi,
                       T);
    return hipGetLastError();
}

hipError_t launch_preeval_elast(int cell, const double* coords, const double* coeff, double* out, int* status,
                                const double* T, int64_t E, int ns, int grid_per_cu, int cus, hipStream_t s)
{
    ElastArgs a;
    a.coords = coords;
    a.coeff = coeff;
    a.out = out;
    a.status = status;
    a.T = T;
    a.E = E;
    a.ns = ns;
    if (ns >= 16 && cell != PRISM) {
        // row-staged kernel: a workgroup per (tile, block row), as many
        // resident per CU as the LDS holds, at most grid_per_cu
        const size_t lds = preeval_elast_rows_lds_bytes(cell, ns);
        const int by_lds = std::max(1, (int)(device_lds_per_cu() / lds));
        const int64_t units = (E + 15) / 16 * cell_dim(cell);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)cus * std::min(grid_per_cu, by_lds)));
        a.parts = 1;
        const void* fn = cell == TRI ? (const void*)k_preeval_elast_rows<TRI>
                       : cell == TET ? (const void*)k_preeval_elast_rows<TET>
                                     : (const void*)k_preeval_elast_rows<PRISM>;
        hipError_t e = allow_dynamic_lds(fn, cell, lds);
        if (e != hipSuccess) return e;
        if (cell == TRI) hipLaunchKernelGGL((k_preeval_elast_rows<TRI>), dim3(grid), dim3(256), lds, s, a);
        else if (cell == TET) hipLaunchKernelGGL((k_preeval_elast_rows<TET>), dim3(grid), dim3(256), lds, s, a);
        else hipLaunchKernelGGL((k_preeval_elast_rows<PRISM>), dim3(grid), dim3(256), lds, s, a);
        return hipGetLastError();
    }
    // a workgroup per (tile, column-group range).  A tile's ranges are
    // consecutive units, so they run at the same time: splitting a large
    // tile into ranges of about 20 column groups narrows the span of output
    // that the grid writes at once, and the L2 merges more of its partial
    // lines before they are evicted (tet P4 1.89 -> 1.60 ms, prism P4
    // 2.20 -> 1.75 ms on MI355X).  Small problems split their tiles so that
    // every CU gets two units.
    const int64_t tiles = (E + 15) / 16;
    const int64_t want = (int64_t)cus * 2;
    const int ncb = (ns * ns + 15) / 16;
    const int by_width = std::min(16, (ncb + 19) / 20);
    const int by_count = (int)std::max<int64_t>(1, std::min<int64_t>(4, (want + tiles - 1) / tiles));
    a.parts = std::max(1, std::min(ncb, std::max(by_width, by_count)));
    const int64_t units = tiles * a.parts;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)cus * grid_per_cu));
    if (cell == TRI) hipLaunchKernelGGL((k_preeval_elast<TRI>), dim3(grid), dim3(64 * pe_waves(TRI)), 0, s, a);
    else if (cell == TET) hipLaunchKernelGGL((k_preeval_elast<TET>), dim3(grid), dim3(64 * pe_waves(TET)), 0, s, a);
    else hipLaunchKernelGGL((k_preeval_elast<PRISM>), dim3(grid), dim3(64 * pe_waves(PRISM)), 0, s, a);
    return hipGetLastError();
}

int preeval_elast_grid_per_cu(int cell, int ns)
{
    // row-staged kernel (n_s >= 16): as many as the LDS holds.  Column-group
    // kernel: wide element matrices (48 or more column groups) run best with
    // one resident workgroup per CU, narrow ones with two (measured on MI355X)
    if (ns >= 16 && cell != PRISM) return 8;
    return (ns * ns + 15) / 16 >= 48 ? 1 : 2;
}

}  // namespace fe
