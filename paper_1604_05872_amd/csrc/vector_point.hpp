// Float64 per-point data of the vector forms, shared by the matrix-core
// kernels (a3 of the path): the point weights of the three weighted products
// and the matrix M that maps reference gradients to the operand columns.
//
// With K = J^{-1} and w = W_q |det J| (Eq. (7)):
//   elasticity (P1 Lame fields, Sec. 2.2's coefficient factor):
//       w0 = w lam(X_q), w1 = w mu(X_q), w2 = 0, M = K, so column (c, j) of the
//       operand at q is g_{q,j,c} = sum_a K[a][c] dphi_j/dX_a;
//   hyperelastic (compressible neo-Hookean tangent):
//       F = I + H K with H = sum_k u_k (x) grad_X phi_k, J_F = det F,
//       w0 = w lam, w1 = w (mu - lam ln J_F), w2 = w mu, M = K F^{-1}, so the
//       column is s = F^{-T} g; the element is flagged when J_F <= 0.
// With `collapse` (P1 on a simplex, every gradient constant in the point
// loop) the point loop is hoisted (generalised code motion, Sec. 3.2): the
// single point carries the integrated weights.
#pragma once
#include "device_common.hpp"

namespace fe {

struct PointTables {
    const double* W;      // [nq] reference weights
    const double* psi;    // [nq][nv] P1 (prism P1 x P1) basis at the points
    const double* dphi;   // [nq][ns][d] reference gradients
    int nq;               // points of the rule
    int collapse;
    double wsum;          // sum of W (collapse)
    double mu, lam;       // hyperelastic constants
};

// coef: the element's coefficients (Lame nodal values [2][nv], or
// displacement DOFs [d][ns]).  Returns nonzero when the element must be
// flagged.
template <int FORM, int CELL, int NS>
__device__ __forceinline__ int vector_point_data(const double* __restrict__ coef, const double (&K)[3][3], double adet,
                                                 int q, const PointTables& t, double& w0, double& w1, double& w2,
                                                 double (&M)[3][3])
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL);
    const double w = (t.collapse ? t.wsum : t.W[q]) * adet;
    if (FORM != HYPERELASTIC) {
        const double* ce = coef;
        double lam = 0.0, mu = 0.0;
        if (t.collapse) {
            for (int qq = 0; qq < t.nq; ++qq) {
                double l1 = 0.0, m1 = 0.0;
#pragma unroll
                for (int l = 0; l < NV; ++l) {
                    l1 = fma(ce[l], t.psi[qq * NV + l], l1);
                    m1 = fma(ce[NV + l], t.psi[qq * NV + l], m1);
                }
                lam = fma(t.W[qq], l1, lam);
                mu = fma(t.W[qq], m1, mu);
            }
            w0 = adet * lam;
            w1 = adet * mu;
        } else {
#pragma unroll
            for (int l = 0; l < NV; ++l) {
                lam = fma(ce[l], t.psi[q * NV + l], lam);
                mu = fma(ce[NV + l], t.psi[q * NV + l], mu);
            }
            w0 = w * lam;
            w1 = w * mu;
        }
        w2 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) M[r][c] = (r < D && c < D) ? K[r][c] : 0.0;
        return 0;
    }
    // H = sum_k u_k (x) grad_X phi_k ; F = I + H K
    const double* ue = coef;
    double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double* dg = t.dphi + (q * NS + k) * D;
#pragma unroll
        for (int r = 0; r < D; ++r) {
            const double ur = ue[r * NS + k];
#pragma unroll
            for (int c = 0; c < D; ++c) H[r][c] = fma(ur, dg[c], H[r][c]);
        }
    }
    double F[3][3], Fi[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double s = (r == b) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) s = fma(H[r][c], K[c][b], s);
            F[r][b] = s;
        }
    const double jf = inverse_small<D>(F, Fi);
    const int bad = !(jf > 0.0);
    const double lnj = log(jf);
    w0 = w * t.lam;
    w1 = w * (t.mu - t.lam * lnj);
    w2 = w * t.mu;
    // M = K F^{-1}: s_c = sum_a M[a][c] dphi/dX_a
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < D; ++b) s = fma(K[r][b], Fi[b][c], s);
            M[r][c] = (r < D && c < D) ? s : 0.0;
        }
    return bad;
}

// Hyperelastic point data from the gradient of the deformed map,
// A = dx/dX + du/dX = J + H.  Since F = A K, J_F = det A / det J and
// M = K F^{-1} = A^{-1}: the same quantities as vector_point_data without
// forming F, F^{-1} or K F^{-1}.  ue: displacement DOFs [d][ns]; Jm is J
// (row-major, zero-padded), det its determinant.
template <int CELL, int NS>
__device__ __forceinline__ int hyper_point_from_gradient(const double* __restrict__ ue, const double (&Jm)[9],
                                                         double det, double adet, int q, const PointTables& t,
                                                         double& w0, double& w1, double (&M)[3][3])
{
    constexpr int D = cell_dim(CELL);
    const double w = (t.collapse ? t.wsum : t.W[q]) * adet;
    double A[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) A[r][c] = Jm[r * 3 + c];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double* dg = t.dphi + (q * NS + k) * D;
#pragma unroll
        for (int r = 0; r < D; ++r) {
            const double ur = ue[r * NS + k];
#pragma unroll
            for (int c = 0; c < D; ++c) A[r][c] = fma(ur, dg[c], A[r][c]);
        }
    }
    const double da = inverse_small<D>(A, M);
    const double jf = da / det;
    const int bad = !(jf > 0.0);
    const double lnj = log(jf);
    w0 = w * t.lam;
    w1 = w * (t.mu - t.lam * lnj);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (r >= D || c >= D) M[r][c] = 0.0;
    return bad;
}

// Signed square root: the weighted product sum_q w_q x_q x_q^T is the Gram
// matrix Z^T diag(sign w) Z of z_q = sqrt|w_q| x_q; the root carries the
// sign of w.
__device__ __forceinline__ double signed_root(double w) { return copysign(sqrt(fabs(w)), w); }

}  // namespace fe
