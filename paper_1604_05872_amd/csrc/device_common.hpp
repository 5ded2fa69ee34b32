// Device helpers shared by the assembly kernels: affine geometry of an element
// and small fixed-size linear algebra.  All of it is float64.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "fe_common.hpp"

namespace fe {

// Geometry of the affine map F_K (Sec. 2.2): J has the edge vectors
// v_{a+1} - v_0 as columns (prism: v1-v0, v2-v0, v3-v0).  Produces
// K = J^{-1} (K[a][b] = dX_a/dx_b, the factors of Eq. (7)) and |det J|, and
// optionally det J and J itself (row-major 3x3, zero-padded).
// Returns nonzero when the map is unusable: |det J| not above
// 1e-13 * (max |J entry|)^d (degenerate, or NaN input), or a prism whose top
// face is not the bottom face translated (relative tolerance 1e-12).
template <int CELL>
__device__ __forceinline__ int affine_map(const double* __restrict__ v, double (&K)[3][3], double& adet,
                                          double* det_out = nullptr, double* J_out = nullptr)
{
    // every product rounded on its own: the same geometry bit for bit in
    // every kernel that inlines this
#pragma clang fp contract(off)
    constexpr int D = cell_dim(CELL);
    double J[3][3];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int r = 0; r < D; ++r) J[r][a] = v[(a + 1) * D + r] - v[r];
    double det, jmax = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int a = 0; a < D; ++a) jmax = fmax(jmax, fabs(J[r][a]));
    if (D == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double id = 1.0 / det;
        K[0][0] = J[1][1] * id;
        K[0][1] = -J[0][1] * id;
        K[1][0] = -J[1][0] * id;
        K[1][1] = J[0][0] * id;
    } else {
        const double a00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double a10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double a20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * a00 + J[0][1] * a10 + J[0][2] * a20;
        const double id = 1.0 / det;
        K[0][0] = a00 * id;
        K[1][0] = a10 * id;
        K[2][0] = a20 * id;
        K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
        K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
        K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    }
    if (det_out) *det_out = det;
    if (J_out)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int a = 0; a < 3; ++a) J_out[r * 3 + a] = (r < D && a < D) ? J[r][a] : 0.0;
    adet = fabs(det);
    double scale = jmax;
#pragma unroll
    for (int k = 1; k < D; ++k) scale *= jmax;
    int bad = !(adet > 1e-13 * scale);
    if (CELL == PRISM) {
        double vmax = 0.0;
#pragma unroll
        for (int k = 0; k < 18; ++k) vmax = fmax(vmax, fabs(v[k]));
        const double tol = 1e-12 * (vmax > 0.0 ? vmax : 1.0);
#pragma unroll
        for (int t = 1; t < 3; ++t)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double dev = (v[(t + 3) * 3 + r] - v[t * 3 + r]) - (v[9 + r] - v[r]);
                bad |= !(fabs(dev) <= tol);
            }
    }
    return bad;
}

// Jacobian of the vertex map x(X) = sum_v psi_v(X) v at one point:
// J[r][a] = sum_v v_r dpsi_v/dX_a, with dpsi [NV][D] the vertex basis
// gradients at that point.
template <int NV, int D>
__device__ __forceinline__ void vertex_map_jacobian(const double* __restrict__ v, const double* __restrict__ dpsi,
                                                    double (&J)[3][3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) J[r][c] = 0.0;
#pragma unroll
    for (int l = 0; l < NV; ++l)
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) J[r][c] = fma(v[l * D + r], dpsi[l * D + c], J[r][c]);
}

// 3x3 (or 2x2) inverse and determinant, row-major in a 3x3 array.
template <int D>
__device__ __forceinline__ double inverse_small(const double (&F)[3][3], double (&Fi)[3][3])
{
    if (D == 2) {
        const double det = F[0][0] * F[1][1] - F[0][1] * F[1][0];
        const double id = 1.0 / det;
        Fi[0][0] = F[1][1] * id;
        Fi[0][1] = -F[0][1] * id;
        Fi[1][0] = -F[1][0] * id;
        Fi[1][1] = F[0][0] * id;
        return det;
    }
    const double c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
    const double c10 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
    const double c20 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
    const double det = F[0][0] * c00 + F[0][1] * c10 + F[0][2] * c20;
    const double id = 1.0 / det;
    Fi[0][0] = c00 * id;
    Fi[1][0] = c10 * id;
    Fi[2][0] = c20 * id;
    Fi[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
    Fi[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
    Fi[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
    Fi[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
    Fi[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
    Fi[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
    return det;
}

// LDS ordering between the lanes of one wavefront (for an LDS area that
// only this wavefront uses)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Output store.  nt = 1 marks the store non-temporal (streaming); nt = 0 is an
// ordinary store, which lets L2 merge the partial lines that scattered row
// segments produce before they reach HBM.
__device__ __forceinline__ void store_out(double* p, double v, int nt)
{
    if (nt) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Coalesced copy of `n` consecutive doubles from global memory into LDS by
// the whole block.
__device__ __forceinline__ void load_to_lds(double* __restrict__ dst, const double* __restrict__ src, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

}  // namespace fe
