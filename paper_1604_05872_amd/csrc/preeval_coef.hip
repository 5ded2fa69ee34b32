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
    const double* coeff;   // element records of cstride doubles, the functions' [nf][nb] from coff
    double* out;           // [E][nn], or [E][vec_d nb][vec_d nb]
    int* status;
    const double* R;       // [nt][nn]
    const int* combos;     // [iota][nf], sorted multisets
    int64_t E;
    int nb, nn, nf, iota, nt, ntp;   // ntp: nt rounded up to a multiple of 8
    int r_lo, r_hi;        // geometry-tensor entries (monomials) evaluated here
    int accumulate;        // add to out instead of overwriting it
    int cstride, coff;     // coefficient record stride and the functions' offset
    int vec_d;             // 0: scalar output; d: each entry times `scale`
    double scale;          // into the d diagonal blocks of a vector matrix
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
        for (int i = lane; i < 16 * ncf; i += 64) {
            const int e = i / ncf;
            sCf[i] = e < ne ? a.coeff[(e0 + e) * a.cstride + a.coff + (i - e * ncf)] : 0.0;
        }
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
                    double v = acc0[r] + acc1[r];
                    if (a.vec_d) {
                        // the trace term: entry (j, k) of each diagonal block
                        v *= a.scale;
                        const int n = a.vec_d * nb, j = col / nb, k = col - (col / nb) * nb;
                        for (int c = 0; c < a.vec_d; ++c) {
                            double* o = a.out + (e0 + row) * (int64_t)n * n + (int64_t)(c * nb + j) * n + c * nb + k;
                            if (a.accumulate) *o += v;
                            else store_out(o, v, 0);
                        }
                    } else {
                        double* o = a.out + (e0 + row) * nn + col;
                        if (a.accumulate) *o += v;
                        else store_out(o, v, 0);
                    }
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
                               int iota, int grid_per_cu, int cus, hipStream_t s, int r_lo, int r_hi, int accumulate,
                               const CoefOut& o)
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
    a.cstride = o.cstride > 0 ? o.cstride : nf * nb;
    a.coff = o.coff;
    a.vec_d = o.vec_d;
    a.scale = o.scale;
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

// ---------------------------------------------------------------------------
// Elasticity with nf pre-multiplying functions, pre-evaluated.  The P1 Lame
// fields and the functions' product are both expanded out of the reduction:
//     lambda(X) prod_i f_i(X) = sum_{l,S} lambda_l C_S psi_l(X) prod_{s in S} phi_s(X)
// (likewise mu), so with the tables
//     T_{(l,S),a,b}[j][k] = sum_q W_q psi_l prod_{s in S} phi_s dphi_{j,a} dphi_{k,b}
// (iota = n_c C(n_s + nf - 1, nf) per term, Sec. 4.2) block (c, e) of the
// element matrix is
//     A[(c,j),(e,k)] = sum_{l,S,a,b} C_S |det J| (lambda_l K_ac K_be + mu_l K_ae K_bc
//                                  + delta_ce mu_l (K K^T)_ab) T_{(l,S),a,b}[j][k]:
// per block, one dense product of the tile's (16 elements) x (tables)
// coefficient rows with the table matrix on the FP64 matrix cores.
// ---------------------------------------------------------------------------

__global__ void k_elast_coef_tables(int nq, int nb, int d, int nc, int nf, int iota, const double* __restrict__ W,
                                    const double* __restrict__ phi, const double* __restrict__ psi,
                                    const double* __restrict__ dphi, const int* __restrict__ combos,
                                    double* __restrict__ T)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nn = nb * nb;
    if (tid >= (int64_t)nc * iota * nn) return;
    const int ls = (int)(tid / nn), jk = (int)(tid % nn), j = jk / nb, k = jk % nb;
    const int l = ls / iota, c = ls - l * iota;
    double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < nq; ++q) {
        double w = W[q] * psi[q * nc + l];
        for (int i = 0; i < nf; ++i) w *= phi[q * nb + combos[c * nf + i]];
        for (int aa = 0; aa < d; ++aa) {
            const double wa = w * dphi[(q * nb + j) * d + aa];
            for (int b = 0; b < d; ++b) acc[aa][b] = fma(wa, dphi[(q * nb + k) * d + b], acc[aa][b]);
        }
    }
    for (int aa = 0; aa < d; ++aa)
        for (int b = 0; b < d; ++b) T[((size_t)(ls * d + aa) * d + b) * nn + jk] = acc[aa][b];
}

struct ElastCoefArgs {
    const double* coords;
    const double* coeff;   // records [2 nc (Lame)][nf nb (functions)]
    double* out;           // [E][n][n], n = d nb
    int* status;
    const double* T;       // [nt][nb nb]
    const int* combos;     // [iota][nf]
    int64_t E;
    int nb, nf, iota, nt, ntp;
};

template <int CELL>
__global__ __launch_bounds__(64) void k_preeval_elast_coef(ElastCoefArgs a)
{
    constexpr int D = cell_dim(CELL), NC = cell_nv(CELL), NVD = NC * D;
    extern __shared__ double lds[];
    const int ntp = a.ntp, nb = a.nb, nn = nb * nb, nf = a.nf, iota = a.iota, n = D * nb;
    const int ncf = nf * nb, cst = 2 * NC + ncf;
    double* sA = lds;                      // [16][ntp] one block's coefficient rows
    double* sG = sA + 16 * ntp;            // [16][12]  K, |det J|, flag
    double* sL = sG + 16 * 12;             // [16][2 NC] Lame nodal values
    double* sCf = sL + 16 * 2 * NC;        // [16][nf][nb]
    double* sCS = sCf + 16 * ncf;          // [16][iota] symmetrised coefficient products
    const int lane = threadIdx.x, i16 = lane & 15, kq = lane >> 4;
    const int64_t ntiles = (a.E + 15) / 16;
    const int ncb = (nn + 15) / 16;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t e0 = t * 16;
        const int ne = a.E - e0 < 16 ? (int)(a.E - e0) : 16;
        if (lane < 16) {
            double K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, adet = 0.0;
            int bad = 0;
            if (lane < ne) {
                double v[NVD];
#pragma unroll
                for (int i = 0; i < NVD; ++i) v[i] = a.coords[(e0 + lane) * NVD + i];
                bad = affine_map<CELL>(v, K, adet);
                if (bad && a.status) atomicAdd(a.status, 1);
            }
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < 3; ++q) sG[lane * 12 + r * 3 + q] = K[r][q];
            sG[lane * 12 + 9] = adet;
            sG[lane * 12 + 10] = bad ? 1.0 : 0.0;
        }
        for (int i = lane; i < 16 * 2 * NC; i += 64) {
            const int e = i / (2 * NC);
            sL[i] = e < ne ? a.coeff[(e0 + e) * cst + (i - e * 2 * NC)] : 0.0;
        }
        for (int i = lane; i < 16 * ncf; i += 64) {
            const int e = i / ncf;
            sCf[i] = e < ne ? a.coeff[(e0 + e) * cst + 2 * NC + (i - e * ncf)] : 0.0;
        }
        __syncthreads();
        for (int i = lane; i < 16 * iota; i += 64) {
            const int e = i / iota, c = i - e * iota;
            sCS[i] = coef_product(sCf + e * ncf, nb, nf, a.combos + c * nf);
        }
        __syncthreads();
        for (int blk = 0; blk < D * D; ++blk) {
            const int c = blk / D, e2 = blk - c * D;
            // coefficient rows of block (c, e2), zero-padded to ntp
            for (int i = lane; i < 16 * ntp; i += 64) {
                const int e = i / ntp, tt = i - e * ntp;
                double x = 0.0;
                if (tt < a.nt) {
                    const int ls = tt / (D * D), aa = (tt / D) % D, b = tt % D;
                    const int l = ls / iota, s = ls - l * iota;
                    const double* K = sG + e * 12;
                    const double lam = sL[e * 2 * NC + l], mu = sL[e * 2 * NC + NC + l];
                    x = lam * (K[aa * 3 + c] * K[b * 3 + e2]) + mu * (K[aa * 3 + e2] * K[b * 3 + c]);
                    if (c == e2) {
                        double g = 0.0;
#pragma unroll
                        for (int m = 0; m < D; ++m) g = fma(K[aa * 3 + m], K[b * 3 + m], g);
                        x = fma(mu, g, x);
                    }
                    x *= K[9] * sCS[e * iota + s];
                }
                sA[i] = x;
            }
            __syncthreads();
            for (int cb = 0; cb < ncb; ++cb) {
                const int col = 16 * cb + i16;
                const bool cvalid = col < nn;
                v4d_c acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
                for (int kb = 0; kb < ntp / 4; kb += 2) {
                    const int k0 = 4 * kb + kq, k1 = k0 + 4;
                    const double b0 = (cvalid && k0 < a.nt) ? a.T[(size_t)k0 * nn + col] : 0.0;
                    const double b1 = (cvalid && k1 < a.nt) ? a.T[(size_t)k1 * nn + col] : 0.0;
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[i16 * ntp + k0], b0, acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[i16 * ntp + k1], b1, acc1, 0, 0, 0);
                }
                if (cvalid) {
                    const int j = col / nb, k = col - (col / nb) * nb;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = kq + 4 * r;
                        if (row < ne) {
                            const bool bad = sG[row * 12 + 10] != 0.0;
                            double* o = a.out + (e0 + row) * (int64_t)n * n + (int64_t)(c * nb + j) * n + e2 * nb + k;
                            store_out(o, bad ? __builtin_nan("") : acc0[r] + acc1[r], 0);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

size_t preeval_elast_coef_lds_bytes(int cell, int nt, int nf, int nb)
{
    const int nc = cell_nv(cell), d = cell_dim(cell);
    const size_t ntp = ((size_t)nt + 7) / 8 * 8, iota = (size_t)nt / ((size_t)nc * d * d);
    return sizeof(double) * 16 * (ntp + 12 + 2 * (size_t)nc + (size_t)nf * nb + iota);
}

hipError_t launch_elast_coef_tables(int nq, int nb, int d, int nc, int nf, int iota, const double* W,
                                    const double* phi, const double* psi, const double* dphi, const int* combos,
                                    double* T, hipStream_t s)
{
    const int64_t n = (int64_t)nc * iota * nb * nb;
    hipLaunchKernelGGL(k_elast_coef_tables, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, nq, nb, d, nc, nf,
                       iota, W, phi, psi, dphi, combos, T);
    return hipGetLastError();
}

hipError_t launch_preeval_elast_coef(int cell, const double* coords, const double* coeff, double* out, int* status,
                                     const double* T, const int* combos, int64_t E, int nb, int nf, int iota,
                                     int grid_per_cu, int cus, hipStream_t s)
{
    ElastCoefArgs a;
    a.coords = coords;
    a.coeff = coeff;
    a.out = out;
    a.status = status;
    a.T = T;
    a.combos = combos;
    a.E = E;
    a.nb = nb;
    a.nf = nf;
    a.iota = iota;
    a.nt = cell_nv(cell) * iota * cell_dim(cell) * cell_dim(cell);
    a.ntp = (a.nt + 7) / 8 * 8;
    const size_t lds = preeval_elast_coef_lds_bytes(cell, a.nt, nf, nb);
    const int64_t tiles = (E + 15) / 16;
    const int grid = (int)std::min<int64_t>(tiles, (int64_t)cus * grid_per_cu);
    if (cell == TRI) hipLaunchKernelGGL((k_preeval_elast_coef<TRI>), dim3(grid), dim3(64), lds, s, a);
    else if (cell == TET) hipLaunchKernelGGL((k_preeval_elast_coef<TET>), dim3(grid), dim3(64), lds, s, a);
    else hipLaunchKernelGGL((k_preeval_elast_coef<PRISM>), dim3(grid), dim3(64), lds, s, a);
    return hipGetLastError();
}

}  // namespace fe
