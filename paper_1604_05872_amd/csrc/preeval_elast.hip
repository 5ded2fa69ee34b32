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
// (v_mfma_f64_16x16x4_f64).  The unit of work is (16-element tile, block):
// a wavefront forms the tile's coefficients of its block in its own LDS area
// and sweeps the block's 16-entry column groups; the tables are read
// through the L2 (the planner admits them only when they fit T_H).
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace fe {

typedef double v4d_e __attribute__((ext_vector_type(4)));

namespace {

constexpr int PE_WAVES = 4;

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
};

template <int CELL>
__global__ __launch_bounds__(64 * PE_WAVES) void k_preeval_elast(ElastArgs a)
{
    constexpr int D = cell_dim(CELL), NC = cell_nv(CELL), NVD = NC * D;
    constexpr int NT = NC * D * D, NTP = (NT + 7) / 8 * 8, NB = D * D;
    __shared__ double sA[PE_WAVES][16 * NTP];       // the unit's coefficient rows
    __shared__ double sG[PE_WAVES][16 * 12];        // K [9], |det J|, flag
    __shared__ double sL[PE_WAVES][16 * 2 * NC];    // Lame nodal values
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    const int ns = a.ns, nn = ns * ns, n = D * ns;
    const int64_t ntiles = (a.E + 15) / 16;
    const int64_t units = ntiles * NB;
    const int ncb = (nn + 15) / 16;
    double* A = sA[w];
    double* G = sG[w];
    double* L = sL[w];
    for (int64_t u = (int64_t)blockIdx.x * PE_WAVES + w; u < units; u += (int64_t)gridDim.x * PE_WAVES) {
        const int64_t tile = u / NB;
        const int blk = (int)(u - tile * NB), c = blk / D, e2 = blk - c * D;
        const int64_t e0 = tile * 16;
        const int ne = a.E - e0 < 16 ? (int)(a.E - e0) : 16;
        // geometry and Lame values of the tile's elements
        if (lane < 16) {
            double K[3][3], adet;
            int bad = 0;
            if (lane < ne) {
                double v[NVD];
#pragma unroll
                for (int i = 0; i < NVD; ++i) v[i] = a.coords[(e0 + lane) * NVD + i];
                bad = affine_map<CELL>(v, K, adet);
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int s = 0; s < 3; ++s) K[r][s] = 0.0;
                adet = 0.0;
            }
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int s = 0; s < D; ++s) G[lane * 12 + r * 3 + s] = K[r][s];
            G[lane * 12 + 9] = adet;
            G[lane * 12 + 10] = bad ? 1.0 : 0.0;
            // one unit per tile reports flagged elements
            if (bad && blk == 0 && a.status) atomicAdd(a.status, 1);
        }
        for (int i = lane; i < 16 * 2 * NC; i += 64) L[i] = i < ne * 2 * NC ? a.coeff[e0 * 2 * NC + i] : 0.0;
        wave_sync();
        // coefficient rows C^{c e2}[e][(l, a, b)], zero-padded to NTP
        for (int i = lane; i < 16 * NTP; i += 64) {
            const int e = i / NTP, t = i - e * NTP;
            double x = 0.0;
            if (t < NT) {
                const int l = t / (D * D), aa = (t / D) % D, b = t % D;
                const double* K = G + e * 12;
                const double lam = L[e * 2 * NC + l], mu = L[e * 2 * NC + NC + l];
                x = lam * (K[aa * 3 + c] * K[b * 3 + e2]) + mu * (K[aa * 3 + e2] * K[b * 3 + c]);
                if (c == e2) {
                    double g = 0.0;
#pragma unroll
                    for (int m = 0; m < D; ++m) g = fma(K[aa * 3 + m], K[b * 3 + m], g);
                    x = fma(mu, g, x);
                }
                x *= K[9];
            }
            A[i] = x;
        }
        wave_sync();
        const bool bad_row[4] = {G[(kq + 0) * 12 + 10] != 0.0, G[(kq + 4) * 12 + 10] != 0.0,
                                 G[(kq + 8) * 12 + 10] != 0.0, G[(kq + 12) * 12 + 10] != 0.0};
        // the block's entries in 16-entry column groups, NG at a time (2 NG
        // independent accumulator chains; prisms, whose coefficient rows are
        // longer, take one group to keep two wavefronts per SIMD); a step's
        // table values are loaded together, one step ahead of its products
        constexpr int NK = NTP / 4, NG = CELL == PRISM ? 1 : 2;
        double bv[NG][NK];
        auto load_b = [&](int cb) {
#pragma unroll
            for (int h = 0; h < NG; ++h) {
                const int col = 16 * (cb + h) + i16;
                const int colc = col < nn ? col : nn - 1;   // in-range table column for padding lanes
#pragma unroll
                for (int kk = 0; kk < NK; ++kk) {
                    const int k = 4 * kk + kq;
                    bv[h][kk] = k < NT ? a.T[(size_t)k * nn + colc] : 0.0;
                }
            }
        };
        auto store_group = [&](int col, const v4d_e& x0, const v4d_e& x1) {
            // lane holds elements kq + 4 r, entry col = (j, k) of block (c, e2)
            if (col < nn) {
                const int j = col / ns, k = col - (col / ns) * ns;
                const int64_t off = (int64_t)(c * ns + j) * n + e2 * ns + k;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = kq + 4 * r;
                    if (row < ne) {
                        const double v = bad_row[r] ? __builtin_nan("") : x0[r] + x1[r];
                        store_out(a.out + (e0 + row) * (int64_t)(n * n) + off, v, 0);
                    }
                }
            }
        };
        load_b(0);
        for (int cb = 0; cb < ncb; cb += NG) {
            double bc[NG][NK];
#pragma unroll
            for (int h = 0; h < NG; ++h)
#pragma unroll
                for (int kk = 0; kk < NK; ++kk) bc[h][kk] = bv[h][kk];
            if (cb + NG < ncb) load_b(cb + NG);
            v4d_e acc[2 * NG];
#pragma unroll
            for (int i = 0; i < 2 * NG; ++i) acc[i] = (v4d_e){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                const double av = A[i16 * NTP + 4 * kk + kq];
#pragma unroll
                for (int h = 0; h < NG; ++h)
                    acc[2 * h + (kk & 1)] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(av, bc[h][kk], acc[2 * h + (kk & 1)], 0, 0, 0);
            }
#pragma unroll
            for (int h = 0; h < NG; ++h)   // a group past the block stores nothing
                store_group(16 * (cb + h) + i16, acc[2 * h], acc[2 * h + 1]);
        }
        wave_sync();
    }
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
    const int d = cell_dim(cell);
    const int64_t units = (E + 15) / 16 * d * d;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((units + PE_WAVES - 1) / PE_WAVES,
                                                                 (int64_t)cus * grid_per_cu));
    if (cell == TRI) hipLaunchKernelGGL((k_preeval_elast<TRI>), dim3(grid), dim3(64 * PE_WAVES), 0, s, a);
    else if (cell == TET) hipLaunchKernelGGL((k_preeval_elast<TET>), dim3(grid), dim3(64 * PE_WAVES), 0, s, a);
    else hipLaunchKernelGGL((k_preeval_elast<PRISM>), dim3(grid), dim3(64 * PE_WAVES), 0, s, a);
    return hipGetLastError();
}

}  // namespace fe
