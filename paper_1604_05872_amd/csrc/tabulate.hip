// Reference tabulation (the local basis Phi_i at the quadrature points,
// Sec. 2.2), pre-evaluation of the reference tensors of the scalar forms
// (Sec. 2.3 Eqs. (8)-(9); Sec. 3.3 Algorithm 2, with the reduction over the
// quadrature loop executed numerically once per (cell, degree, rule)), and a
// standalone geometry kernel.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "fe_common.hpp"
#include "internal.hpp"

namespace fe {

namespace {

// Barycentric multi-index (|alpha| = p) of lattice node `idx` of a simplex of
// dimension d, in the order k, j, i with i fastest.
__device__ void simplex_node(int d, int p, int idx, int alpha[4])
{
    int count = 0;
    const int kmax = (d == 3) ? p : 0;
    for (int k = 0; k <= kmax; ++k)
        for (int j = 0; j <= p - k; ++j) {
            const int row = p - j - k + 1;
            if (idx < count + row) {
                const int i = idx - count;
                alpha[0] = p - i - j - k;
                alpha[1] = i;
                alpha[2] = j;
                alpha[3] = k;
                return;
            }
            count += row;
        }
}

// Factor f_a(t) = prod_{m<a} (p t - m) / (m + 1) and its derivative.
__device__ void lattice_factor(int p, int a, double t, double& f, double& df)
{
    f = 1.0;
    df = 0.0;
    for (int m = 0; m < a; ++m) {
        const double c = 1.0 / (m + 1);
        const double g = (p * t - m) * c;
        df = df * g + f * (p * c);
        f *= g;
    }
}

// Lagrange basis function of a simplex (Silvester's product of lattice
// factors of the barycentric coordinates) and its reference gradient.
__device__ void simplex_basis(int d, int p, int idx, const double* X, double& val, double* grad)
{
    int alpha[4];
    simplex_node(d, p, idx, alpha);
    double lam[4], f[4], df[4];
    lam[0] = 1.0;
    for (int c = 0; c < d; ++c) {
        lam[c + 1] = X[c];
        lam[0] -= X[c];
    }
    for (int v = 0; v <= d; ++v) lattice_factor(p, alpha[v], lam[v], f[v], df[v]);
    // d phi / d lam_v = df_v * prod_{w != v} f_w
    double dl[4];
    for (int v = 0; v <= d; ++v) {
        double pr = df[v];
        for (int w = 0; w <= d; ++w)
            if (w != v) pr *= f[w];
        dl[v] = pr;
    }
    val = f[0];
    for (int v = 1; v <= d; ++v) val *= f[v];
    for (int c = 0; c < d; ++c) grad[c] = dl[c + 1] - dl[0];
}

__global__ void k_tabulate(int cell, int p, int nq, const double* __restrict__ X, double* __restrict__ phi,
                           double* __restrict__ dphi)
{
    const int nb = n_scalar(cell, p);
    const int d = cell_dim(cell);
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nq * nb) return;
    const int q = tid / nb, j = tid % nb;
    const double* x = X + q * d;
    double val, g[3];
    if (cell == PRISM) {
        const int nt = (p + 1) * (p + 2) / 2;
        const int t = j % nt, l = j / nt;
        double vt, gt[2];
        simplex_basis(2, p, t, x, vt, gt);
        // 1-D lattice basis on [0,1]: barycentrics (1 - Z, Z), multi-index (p - l, l)
        double f0, df0, f1, df1;
        lattice_factor(p, p - l, 1.0 - x[2], f0, df0);
        lattice_factor(p, l, x[2], f1, df1);
        const double ez = f0 * f1, dez = f0 * df1 - df0 * f1;
        val = vt * ez;
        g[0] = gt[0] * ez;
        g[1] = gt[1] * ez;
        g[2] = vt * dez;
    } else {
        simplex_basis(d, p, j, x, val, g);
    }
    phi[q * nb + j] = val;
    for (int c = 0; c < d; ++c) dphi[(q * nb + j) * d + c] = g[c];
}

// R[r][j][k] (layout described with n_tables) from the tabulated basis.
__global__ void k_preeval_tables(int nq, int nb, int d, const double* __restrict__ W,
                                 const double* __restrict__ phi, const double* __restrict__ dphi,
                                 double* __restrict__ R)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nb * nb) return;
    const int j = tid / nb, k = tid % nb;
    double m = 0.0, K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < nq; ++q) {
        const double w = W[q];
        m += w * phi[q * nb + j] * phi[q * nb + k];
        for (int a = 0; a < d; ++a) {
            const double wa = w * dphi[(q * nb + j) * d + a];
            for (int b = 0; b < d; ++b) K[a][b] += wa * dphi[(q * nb + k) * d + b];
        }
    }
    const size_t nn = (size_t)nb * nb;
    R[tid] = m;
    for (int a = 0; a < d; ++a) R[(1 + a) * nn + tid] = K[a][a];
    int r = 1 + d;
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) R[(r++) * nn + tid] = K[a][b] + K[b][a];
}

template <int CELL>
__global__ void k_geometry(int64_t E, const double* __restrict__ coords, double* __restrict__ det_out,
                           double* __restrict__ kinv_out)
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        double v[NV * D];
#pragma unroll
        for (int k = 0; k < NV * D; ++k) v[k] = coords[e * NV * D + k];
        double K[3][3], adet, det;
        affine_map<CELL>(v, K, adet, &det);
        det_out[e] = det;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) kinv_out[(e * D + a) * D + b] = K[a][b];
    }
}

}  // namespace

hipError_t launch_tabulate(int cell, int p, int nq, const double* X, double* phi, double* dphi, hipStream_t s)
{
    const int n = nq * n_scalar(cell, p);
    hipLaunchKernelGGL(k_tabulate, dim3((n + 127) / 128), dim3(128), 0, s, cell, p, nq, X, phi, dphi);
    return hipGetLastError();
}

hipError_t launch_preeval_tables(int nq, int nb, int d, const double* W, const double* phi, const double* dphi,
                                 double* R, hipStream_t s)
{
    const int n = nb * nb;
    hipLaunchKernelGGL(k_preeval_tables, dim3((n + 127) / 128), dim3(128), 0, s, nq, nb, d, W, phi, dphi, R);
    return hipGetLastError();
}

hipError_t launch_geometry(int cell, int64_t E, const double* coords, double* det, double* kinv, hipStream_t s)
{
    const int64_t blocks64 = (E + 255) / 256;
    const int blocks = (int)(blocks64 < 65536 ? blocks64 : 65536);
    if (cell == TRI) hipLaunchKernelGGL(k_geometry<TRI>, dim3(blocks), dim3(256), 0, s, E, coords, det, kinv);
    else if (cell == TET) hipLaunchKernelGGL(k_geometry<TET>, dim3(blocks), dim3(256), 0, s, E, coords, det, kinv);
    else hipLaunchKernelGGL(k_geometry<PRISM>, dim3(blocks), dim3(256), 0, s, E, coords, det, kinv);
    return hipGetLastError();
}

}  // namespace fe
