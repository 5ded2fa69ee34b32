// Pre-evaluated contraction with nf pre-multiplying coefficient functions
// (mass and Helmholtz, the experiment matrix of Sec. 7.1).
//
// With f_i = sum_l f_il phi_l in the test/trial space, Algorithm 2 expands
// the coefficient product out of the reduction:
//     prod_i f_i(X) = sum_{S} C_S prod_{l in S} phi_l(X)
// over the multisets S of nf basis indices (iota = C(n_s + nf - 1, nf) of
// them, the increase factor of Sec. 4.2), with the symmetrised coefficient
//     C_S = sum over the distinct orderings (l_1..l_nf) of S of prod_i f_il_i.
// The reference tensors become R[(r, S)][j][k] = sum_q W_q prod_{l in S}
// phi_l(X_q) B_r[j][k](X_q) (B_0 = phi_j phi_k; B_r, r >= 1, the gradient
// products of the nf = 0 tables), and per element
//     A_e[jk] = sum_{r,S} G'_r(e) C_S(e) R[(r,S)][jk],
// one dense product of an element-by-(r,S) matrix with the table matrix: on
// the FP64 matrix cores (v_mfma_f64_16x16x4_f64), a tile of 16 elements per
// wavefront against 16-entry column blocks of the tables, which are read
// through the L2 (the planner admits them only when they fit T_H).
#include <algorithm>

#include "internal.hpp"
#include "preeval.hpp"

namespace fe {

typedef double v4d_c __attribute__((ext_vector_type(4)));

// R[(r * iota + c)][j * nb + k]; r = 0 the weighted mass table, r >= 1 the
// weighted gradient tables (aa, then ab + ba for a < b), nr of them.
__global__ void k_coef_tables(int nq, int nb, int d, int nf, int iota, int nr, const double* __restrict__ W,
                              const double* __restrict__ phi, const double* __restrict__ dphi,
                              const int* __restrict__ combos, double* __restrict__ R)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nn = nb * nb;
    if (tid >= (int64_t)iota * nn) return;
    const int c = (int)(tid / nn), jk = (int)(tid % nn), j = jk / nb, k = jk % nb;
    double m = 0.0, K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < nq; ++q) {
        double w = W[q];
        for (int i = 0; i < nf; ++i) w *= phi[q * nb + combos[c * nf + i]];
        m += w * phi[q * nb + j] * phi[q * nb + k];
        if (nr > 1)
            for (int a = 0; a < d; ++a) {
                const double wa = w * dphi[(q * nb + j) * d + a];
                for (int b = 0; b < d; ++b) K[a][b] += wa * dphi[(q * nb + k) * d + b];
            }
    }
    R[(size_t)c * nn + jk] = m;
    if (nr > 1) {
        for (int a = 0; a < d; ++a) R[((size_t)(1 + a) * iota + c) * nn + jk] = K[a][a];
        int r = 1 + d;
        for (int a = 0; a < d; ++a)
            for (int b = a + 1; b < d; ++b) R[((size_t)(r++) * iota + c) * nn + jk] = K[a][b] + K[b][a];
    }
}

// symmetrised coefficient product C_S of one element (f: [nf][nb])
__device__ __forceinline__ double coef_product(const double* f, int nb, int nf, const int* S)
{
    if (nf == 1) return f[S[0]];
    if (nf == 2) {
        const int a = S[0], b = S[1];
        const double v = f[a] * f[nb + b] + f[b] * f[nb + a];
        return a == b ? 0.5 * v : v;
    }
    const int a = S[0], b = S[1], c = S[2];
    const double* f0 = f;
    const double* f1 = f + nb;
    const double* f2 = f + 2 * nb;
    double v = f0[a] * (f1[b] * f2[c] + f1[c] * f2[b]) + f0[b] * (f1[a] * f2[c] + f1[c] * f2[a]) +
               f0[c] * (f1[a] * f2[b] + f1[b] * f2[a]);
    // each distinct ordering appears (multiplicities)! times among the 6
    const int mult = (a == b && b == c) ? 6 : (a == b || b == c || a == c) ? 2 : 1;
    return v / mult;
}

struct CoefArgs {
    const double* coords;
    const double* coeff;   // [E][nf][nb]
    double* out;           // [E][nn]
    int* status;
    const double* R;       // [nt][nn]
    const int* combos;     // [iota][nf], sorted multisets
    int64_t E;
    int nb, nn, nf, iota, nt, ntp;   // ntp: nt rounded up to a multiple of 8
    int r_lo, r_hi;        // geometry-tensor entries (monomials) evaluated here
    int accumulate;        // add to out instead of overwriting it
};

template <int FORM, int CELL>
__global__ __launch_bounds__(64) void k_preeval_coef(CoefArgs a)
{
    constexpr int NR = preeval_nt<FORM, CELL>();          // geometry tensor entries
    constexpr int NVD = cell_nv(CELL) * cell_dim(CELL);
    extern __shared__ double lds[];
    const int ntp = a.ntp, nb = a.nb, nn = a.nn, nf = a.nf, iota = a.iota;
    double* sA = lds;                       // [16][ntp]  rows of the element matrix
    double* sGeo = sA + 16 * ntp;           // [16][NR]
    double* sCf = sGeo + 16 * NR;           // [16][nf][nb]
    const int lane = threadIdx.x, i16 = lane & 15, kq = lane >> 4;
    const int64_t ntiles = (a.E + 15) / 16;
    const int nblk = (nn + 15) / 16;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t e0 = t * 16;
        const int ne = a.E - e0 < 16 ? (int)(a.E - e0) : 16;
        // geometry tensors G'(e) and the coefficient DOFs of the tile
        if (lane < 16) {
            double c[NR];
            if (lane < ne) {
                double v[NVD];
#pragma unroll
                for (int k = 0; k < NVD; ++k) v[k] = a.coords[(e0 + lane) * NVD + k];
                if (preeval_coeffs<FORM, CELL>(v, c)) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) c[r] = __builtin_nan("");
                    if (a.status) atomicAdd(a.status, 1);
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) c[r] = 0.0;
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) sGeo[lane * NR + r] = c[r];
        }
        const int ncf = nf * nb;
        for (int i = lane; i < 16 * ncf; i += 64) sCf[i] = i < ne * ncf ? a.coeff[e0 * ncf + i] : 0.0;
        __syncthreads();
        // A[e][(r, S)] = G'_r(e) C_S(e) for r in [r_lo, r_hi), zero-padded to ntp
        for (int idx = lane; idx < 16 * iota; idx += 64) {
            const int e = idx / iota, c = idx - (idx / iota) * iota;
            const double cs = coef_product(sCf + e * ncf, nb, nf, a.combos + c * nf);
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r >= a.r_lo && r < a.r_hi) sA[e * ntp + (r - a.r_lo) * iota + c] = sGeo[e * NR + r] * cs;
        }
        for (int idx = lane; idx < 16 * (ntp - a.nt); idx += 64) {
            const int e = idx / (ntp - a.nt);
            sA[e * ntp + a.nt + (idx - e * (ntp - a.nt))] = 0.0;
        }
        __syncthreads();
        // out tile [16 elements][16 entries] per column block, two accumulators
        for (int cb = 0; cb < nblk; ++cb) {
            const int col = 16 * cb + i16;
            const bool cvalid = col < nn;
            v4d_c acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
            for (int kb = 0; kb < ntp / 4; kb += 2) {
                const int k0 = 4 * kb + kq, k1 = k0 + 4;
                const double a0 = sA[i16 * ntp + k0], a1 = sA[i16 * ntp + k1];
                const double* Rr = a.R + (size_t)a.r_lo * iota * nn;   // tables of the evaluated monomials
                const double b0 = (cvalid && k0 < a.nt) ? Rr[(size_t)k0 * nn + col] : 0.0;
                const double b1 = (cvalid && k1 < a.nt) ? Rr[(size_t)k1 * nn + col] : 0.0;
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
            }
            // lane holds rows kq + 4 r (elements), column col (entry)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = kq + 4 * r;
                if (row < ne && cvalid) {
                    double* o = a.out + (e0 + row) * nn + col;
                    const double v = acc0[r] + acc1[r];
                    if (a.accumulate) *o += v;
                    else store_out(o, v, 0);
                }
            }
        }
        __syncthreads();
    }
}

size_t preeval_coef_lds_bytes(int form, int cell, int ntp, int nf, int nb)
{
    return ((size_t)16 * ntp + (size_t)16 * n_tables(form, cell) + (size_t)16 * nf * nb) * sizeof(double);
}

hipError_t launch_coef_tables(int nq, int nb, int d, int nf, int iota, int nr, const double* W, const double* phi,
                              const double* dphi, const int* combos, double* R, hipStream_t s)
{
    const int64_t n = (int64_t)iota * nb * nb;
    hipLaunchKernelGGL(k_coef_tables, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, nq, nb, d, nf, iota, nr, W,
                       phi, dphi, combos, R);
    return hipGetLastError();
}

hipError_t launch_preeval_coef(int form, int cell, const double* coords, const double* coeff, double* out,
                               int* status, const double* R, const int* combos, int64_t E, int nb, int nf,
                               int iota, int grid_per_cu, int cus, hipStream_t s, int r_lo, int r_hi, int accumulate)
{
    CoefArgs a;
    a.coords = coords;
    a.coeff = coeff;
    a.out = out;
    a.status = status;
    a.R = R;
    a.combos = combos;
    a.E = E;
    a.nb = nb;
    a.nn = nb * nb;
    a.nf = nf;
    a.iota = iota;
    a.r_lo = r_lo;
    a.r_hi = r_hi < 0 ? n_tables(form, cell) : r_hi;
    a.accumulate = accumulate;
    a.nt = (a.r_hi - a.r_lo) * iota;
    a.ntp = (a.nt + 7) / 8 * 8;
    const size_t lds = preeval_coef_lds_bytes(form, cell, a.ntp, nf, nb);
    const int64_t tiles = (E + 15) / 16;
    const int grid = (int)std::min<int64_t>(tiles, (int64_t)cus * grid_per_cu);
    if (form == MASS) {
        if (cell == TRI) hipLaunchKernelGGL((k_preeval_coef<MASS, TRI>), dim3(grid), dim3(64), lds, s, a);
        else if (cell == TET) hipLaunchKernelGGL((k_preeval_coef<MASS, TET>), dim3(grid), dim3(64), lds, s, a);
        else hipLaunchKernelGGL((k_preeval_coef<MASS, PRISM>), dim3(grid), dim3(64), lds, s, a);
    } else {
        if (cell == TRI) hipLaunchKernelGGL((k_preeval_coef<HELMHOLTZ, TRI>), dim3(grid), dim3(64), lds, s, a);
        else if (cell == TET) hipLaunchKernelGGL((k_preeval_coef<HELMHOLTZ, TET>), dim3(grid), dim3(64), lds, s, a);
        else hipLaunchKernelGGL((k_preeval_coef<HELMHOLTZ, PRISM>), dim3(grid), dim3(64), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace fe
