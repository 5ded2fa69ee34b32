// Sharing-eliminated quadrature (Sec. 3.2, Algorithm 1, applied by hand to
// each form), float64 on the vector ALUs.  For every quadrature point the
// loop-invariant factors are hoisted out of the (j,k) nest (generalised code
// motion) and the test/trial symbols are factorised (Strategy 2), so the
// innermost body per scalar pair (j,k) and point q is:
//   mass          A[j][k]      += (w phi_j) phi_k
//   Helmholtz     A[j][k]      += (w g_j).g_k + (w phi_j) phi_k
//                 (a mixed plan of Algorithm 3 drops one of the two terms
//                 here and adds its pre-evaluated form at the end:
//                 |det J| Mhat[j][k], or sum_r G'_r Khat_r[j][k])
//   elasticity    A[cj][ek]    += (lam' g_jc) g_ke + (mu' g_je) g_kc
//                 A[cj][ck]    += (mu' g_j).g_k          (diagonal blocks)
//   hyperelastic  A[cj][ek]    += (lam' s_jc) s_ke + (alpha' s_je) s_kc
//                 A[cj][ck]    += (mu' g_j).g_k
// with w = W_q |det J|, lam' = w lambda(X_q), mu' = w mu(X_q) (P1 fields),
// g = K^T grad_X phi, and for the neo-Hookean tangent s = F^{-T} g,
// alpha' = w (mu - lambda ln det F).  (The factorised tangent equals
// sum_{b,d} g_jb dP_cb/dF_ed g_kd with P = mu (F - F^{-T}) + lambda ln J F^{-T}.)
//
// Work split: a workgroup takes `eb` elements; one unit of work is
// (element, j, block of KB consecutive k) and owns d*d*KB accumulators.
// Per-point data (g, s, scaled weights) for a chunk of `qc` points of all eb
// elements is staged in LDS, then every unit sweeps the chunk.  Units beyond
// the block size run in further passes.  Only A is written to global memory.
#pragma once
#include "device_common.hpp"

namespace fe {

struct QuadArgs {
    const double* coords;
    const double* coeff;
    double* out;
    int* status;
    const double* W;      // [nq]
    const double* phi;    // [nq][ns]
    const double* dphi;   // [nq][ns][d]
    const double* psi;    // [nq][nv]  P1 (prism: P1 x P1) basis for the Lame fields
    const double* mass_table;  // Helmholtz with its mass monomial pre-evaluated
                               // (a mixed plan of Algorithm 3): Mhat [ns][ns], else NULL
    const double* stiff_tables;  // Helmholtz with its gradient monomial pre-evaluated:
                                 // the pre-evaluated tensors [1 + d(d+1)/2][ns][ns]
                                 // (entries r >= 1 are used), else NULL
    int64_t E;
    int nq, ns;
    int collapse;         // gradients invariant in q (P1 on a simplex): the
                          // point loop is hoisted, one pass with summed weights
    int eb;               // elements per tile
    int qc;               // points per LDS chunk
    int nt;               // non-temporal output stores
    double mu, lam;       // hyperelastic constants
    int nf;               // pre-multiplying coefficient functions (Sec. 7.1): an
                          // element's coeff record is the form's own DOFs
                          // (own_coeff) followed by the functions' [nf][ns]
    int skip;             // Helmholtz: bit 0 leaves out the mass term, bit 1 the
                          // gradient term; hyperelastic: bit 1 leaves out the
                          // trace term (each added by another kernel afterwards)
    int pointgeo = 0;     // J, det J, J^{-1} at every point: 1 the vertex map of a
                          // prism, 2 the P2 coordinate field of a curved simplex
                          // (coords then [E][n_s(2)][d])
    const double* dpsi_grad = nullptr;   // [nq][nodes][d] gradients of the map's basis (pointgeo)
};

template <int FORM, int CELL>
struct QuadLayout {
    static constexpr int D = cell_dim(CELL);
    static constexpr int VEC = is_vector_form(FORM) ? 1 : 0;
    // per (element, point): g [ns][D], s [ns][D] (hyperelastic), F^{-1}
    // (hyperelastic, 9), 3 scaled weights, then with per-point geometry the
    // point's K (9) and |det J| (1)
    __host__ __device__ static int per_point(int ns, int pg = 0)
    {
        return ns * D + (FORM == HYPERELASTIC ? ns * D + 9 : 0) + 3 + (pg ? 10 : 0);
    }
    // per element: K (9), |det J|, flag, det J at the first point (per-point geometry)
    static constexpr int PER_ELEM = 12;
    __host__ __device__ static size_t lds_doubles(int ns, int eb, int qc, int pg = 0)
    {
        return (size_t)eb * PER_ELEM + (size_t)qc * ns + (size_t)eb * qc * per_point(ns, pg);
    }
};

template <int FORM, int CELL, int KB>
__device__ void quad_tile(const QuadArgs& a, int64_t e_begin, double* lds)
{
    using L = QuadLayout<FORM, CELL>;
    constexpr int D = L::D, NV = cell_nv(CELL);
    constexpr int NA = is_vector_form(FORM) ? D * D : 1;   // accumulators per (j,k)
    const int tid = threadIdx.x, B = blockDim.x;
    const int ns = a.ns, nq = a.nq, qc_max = a.qc;
    const int64_t rem = a.E - e_begin;
    const int eb = rem < a.eb ? (int)rem : a.eb;
    // per-point geometry: the vertex map of a prism, or the P2 coordinate
    // field of a curved triangle or tetrahedron (NM nodes per element)
    const int pg = a.pointgeo;
    constexpr int NM = CELL == PRISM ? NV : n_scalar(CELL, 2);
    const int ppt = L::per_point(ns, pg);
    // an element's coefficient record: the form's own DOFs, then nf functions
    const int own = FORM == ELASTICITY ? 2 * NV : FORM == HYPERELASTIC ? D * ns : 0;
    const int cst = own + a.nf * ns;

    double* sEl = lds;                                  // [eb][12]
    double* sPhi = lds + (size_t)a.eb * L::PER_ELEM;    // [qc][ns]
    double* sPt = sPhi + (size_t)qc_max * ns;           // [eb][qc][ppt]

    // element geometry (per-point geometry: only the sign of det J at the
    // first point, which every point must share)
    for (int i = tid; i < eb; i += B) {
        const int64_t e = e_begin + i;
        double* s = sEl + i * L::PER_ELEM;
        if (pg) {
            double v[NM * D];
#pragma unroll
            for (int k = 0; k < NM * D; ++k) v[k] = a.coords[e * (NM * D) + k];
            double J[3][3], Kq[3][3];
            vertex_map_jacobian<NM, D>(v, a.dpsi_grad, J);
            const double det = inverse_small<D>(J, Kq);
#pragma unroll
            for (int r = 0; r < 10; ++r) s[r] = 0.0;
            s[10] = (det != 0.0 && isfinite(det)) ? 0.0 : 1.0;
            s[11] = det;
            continue;
        }
        double v[NV * D];
#pragma unroll
        for (int k = 0; k < NV * D; ++k) v[k] = a.coords[e * (NV * D) + k];
        double K[3][3], adet;
        const int bad = affine_map<CELL>(v, K, adet);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) s[r * 3 + c] = (r < D && c < D) ? K[r][c] : 0.0;
        s[9] = adet;
        s[10] = bad ? 1.0 : 0.0;
    }
    __syncthreads();

    const int nkb = (ns + KB - 1) / KB;
    const int units_per_el = ns * nkb;
    const int units = eb * units_per_el;
    const int npass = (units + B - 1) / B;

    for (int pass = 0; pass < npass; ++pass) {
        const int u = pass * B + tid;
        const bool active = u < units;
        const int ui = active ? u / units_per_el : 0;
        const int ur = active ? u - ui * units_per_el : 0;
        const int uj = ur / nkb;
        const int k0 = (ur - uj * nkb) * KB;
        const int kn = active ? min(KB, ns - k0) : 0;
        double acc[KB][NA];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
#pragma unroll
            for (int x = 0; x < NA; ++x) acc[kk][x] = 0.0;

        const int nq_loop = a.collapse ? 1 : nq;
        for (int q0 = 0; q0 < nq_loop; q0 += qc_max) {
            const int qc = min(qc_max, nq_loop - q0);
            // --- stage per-point data -------------------------------------
            for (int idx = tid; idx < qc * ns; idx += B) sPhi[idx] = a.phi[q0 * ns + idx];
            if (pg) {
                // J(X_q) = sum_m x_m (x) grad psi_m(X_q), its inverse and |det J|
                for (int idx = tid; idx < eb * qc; idx += B) {
                    const int i = idx / qc, qq = idx - i * qc;
                    const int64_t e = e_begin + i;
                    double v[NM * D];
#pragma unroll
                    for (int k = 0; k < NM * D; ++k) v[k] = a.coords[e * (NM * D) + k];
                    double J[3][3], Kq[3][3];
                    vertex_map_jacobian<NM, D>(v, a.dpsi_grad + (size_t)(q0 + qq) * NM * D, J);
                    const double det = inverse_small<D>(J, Kq);
                    double* gq = sPt + ((size_t)i * qc_max + qq) * ppt + ppt - 10;
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c) gq[r * 3 + c] = Kq[r][c];
                    gq[9] = fabs(det);
                    const double det0 = sEl[i * L::PER_ELEM + 11];
                    if (!(det != 0.0 && isfinite(det)) || ((det > 0.0) != (det0 > 0.0)))
                        sEl[i * L::PER_ELEM + 10] = 1.0;
                }
                __syncthreads();
            }
            for (int idx = tid; idx < eb * qc * ns; idx += B) {
                const int i = idx / (qc * ns);
                const int r = idx - i * qc * ns;
                const int qq = r / ns, j = r - qq * ns;
                const double* K = pg ? sPt + ((size_t)i * qc_max + qq) * ppt + ppt - 10
                                                        : sEl + i * L::PER_ELEM;
                const double* gh = a.dphi + ((size_t)(q0 + qq) * ns + j) * D;
                double* g = sPt + ((size_t)i * qc_max + qq) * ppt + j * D;
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    double s = 0.0;
#pragma unroll
                    for (int c = 0; c < D; ++c) s = fma(K[c * 3 + b], gh[c], s);
                    g[b] = s;
                }
            }
            __syncthreads();
            for (int idx = tid; idx < eb * qc; idx += B) {
                const int i = idx / qc, qq = idx - i * qc;
                const int64_t e = e_begin + i;
                double wsum = a.W[q0 + qq];
                if (a.collapse) {
                    wsum = 0.0;
                    for (int q = 0; q < nq; ++q) wsum += a.W[q];
                }
                double* pt = sPt + ((size_t)i * qc_max + qq) * ppt;
                const double w = wsum * (pg ? pt[ppt - 1] : sEl[i * L::PER_ELEM + 9]);
                double* sw = pt + ns * D + (FORM == HYPERELASTIC ? ns * D + 9 : 0);
                // w times prod_i f_i(X_q), f_i = sum_l f_il phi_l (collapse
                // only without functions)
                double wf = w;
                for (int f = 0; f < a.nf; ++f) {
                    const double* cf = a.coeff + e * cst + own + f * ns;
                    double fv = 0.0;
                    for (int l = 0; l < ns; ++l) fv = fma(cf[l], sPhi[qq * ns + l], fv);
                    wf *= fv;
                }
                if (FORM == MASS || FORM == HELMHOLTZ) {
                    sw[0] = wf;
                } else if (FORM == ELASTICITY) {
                    const double* ce = a.coeff + e * cst;
                    if (a.collapse) {
                        // sum_q W_q lambda(X_q), sum_q W_q mu(X_q)
                        double lam = 0.0, mu = 0.0;
                        for (int q = 0; q < nq; ++q) {
                            const double* ps = a.psi + q * NV;
                            double l1 = 0.0, m1 = 0.0;
#pragma unroll
                            for (int l = 0; l < NV; ++l) {
                                l1 = fma(ce[l], ps[l], l1);
                                m1 = fma(ce[NV + l], ps[l], m1);
                            }
                            lam = fma(a.W[q], l1, lam);
                            mu = fma(a.W[q], m1, mu);
                        }
                        const double adet = sEl[i * L::PER_ELEM + 9];
                        sw[0] = adet * lam;
                        sw[1] = adet * mu;
                    } else {
                        const double* ps = a.psi + (q0 + qq) * NV;
                        double lam = 0.0, mu = 0.0;
#pragma unroll
                        for (int l = 0; l < NV; ++l) {
                            lam = fma(ce[l], ps[l], lam);
                            mu = fma(ce[NV + l], ps[l], mu);
                        }
                        sw[0] = wf * lam;
                        sw[1] = wf * mu;
                    }
                } else {
                    // F = I + sum_k u_k (x) g_k at this point
                    const double* ue = a.coeff + e * cst;
                    double F[3][3], Fi[3][3];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c) F[r][c] = (r == c) ? 1.0 : 0.0;
                    for (int k = 0; k < ns; ++k) {
                        const double* gk = pt + k * D;
#pragma unroll
                        for (int r = 0; r < D; ++r) {
                            const double ur_ = ue[r * ns + k];
#pragma unroll
                            for (int c = 0; c < D; ++c) F[r][c] = fma(ur_, gk[c], F[r][c]);
                        }
                    }
                    const double jf = inverse_small<D>(F, Fi);
                    double* fi = pt + 2 * ns * D;
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c) fi[r * 3 + c] = (r < D && c < D) ? Fi[r][c] : 0.0;
                    if (!(jf > 0.0)) sEl[i * L::PER_ELEM + 10] = 1.0;
                    const double lnj = log(jf);
                    sw[0] = wf * a.lam;                   // lambda'
                    sw[1] = wf * (a.mu - a.lam * lnj);    // alpha'
                    sw[2] = (a.skip & 2) ? 0.0 : wf * a.mu;   // mu' (the trace term)
                }
            }
            __syncthreads();
            if (FORM == HYPERELASTIC) {
                for (int idx = tid; idx < eb * qc * ns; idx += B) {
                    const int i = idx / (qc * ns);
                    const int r = idx - i * qc * ns;
                    const int qq = r / ns, j = r - qq * ns;
                    double* pt = sPt + ((size_t)i * qc_max + qq) * ppt;
                    const double* g = pt + j * D;
                    const double* fi = pt + 2 * ns * D;
                    double* s = pt + ns * D + j * D;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        double t = 0.0;
#pragma unroll
                        for (int b = 0; b < D; ++b) t = fma(fi[b * 3 + c], g[b], t);
                        s[c] = t;
                    }
                }
                __syncthreads();
            }
            // --- accumulate --------------------------------------------------
            if (active) {
                for (int qq = 0; qq < qc; ++qq) {
                    const double* pt = sPt + ((size_t)ui * qc_max + qq) * ppt;
                    const double* sw = pt + ns * D + (FORM == HYPERELASTIC ? ns * D + 9 : 0);
                    const double* gj = pt + uj * D;
                    if (FORM == MASS) {
                        const double tj = sw[0] * sPhi[qq * ns + uj];
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk)
                            if (kk < kn) acc[kk][0] = fma(tj, sPhi[qq * ns + k0 + kk], acc[kk][0]);
                    } else if (FORM == HELMHOLTZ) {
                        const double w = sw[0];
                        const double tj = (a.mass_table || (a.skip & 1)) ? 0.0 : w * sPhi[qq * ns + uj];
                        const double wgs = (a.stiff_tables || (a.skip & 2)) ? 0.0 : w;
                        double wg[D];
#pragma unroll
                        for (int b = 0; b < D; ++b) wg[b] = wgs * gj[b];
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk)
                            if (kk < kn) {
                                const double* gk = pt + (k0 + kk) * D;
                                double s = fma(tj, sPhi[qq * ns + k0 + kk], acc[kk][0]);
#pragma unroll
                                for (int b = 0; b < D; ++b) s = fma(wg[b], gk[b], s);
                                acc[kk][0] = s;
                            }
                    } else {
                        const double* xj = (FORM == HYPERELASTIC) ? pt + ns * D + uj * D : gj;
                        const double l1 = sw[0];
                        const double l2 = sw[1];
                        const double mu = (FORM == HYPERELASTIC) ? sw[2] : sw[1];
                        double a1[D], a2[D], mg[D];
#pragma unroll
                        for (int b = 0; b < D; ++b) {
                            a1[b] = l1 * xj[b];
                            a2[b] = l2 * xj[b];
                            mg[b] = mu * gj[b];
                        }
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk)
                            if (kk < kn) {
                                const double* gk = pt + (k0 + kk) * D;
                                const double* xk = (FORM == HYPERELASTIC) ? pt + ns * D + (k0 + kk) * D : gk;
                                double dot = mg[0] * gk[0];
#pragma unroll
                                for (int b = 1; b < D; ++b) dot = fma(mg[b], gk[b], dot);
#pragma unroll
                                for (int c = 0; c < D; ++c)
#pragma unroll
                                    for (int e2 = 0; e2 < D; ++e2) {
                                        double t = fma(a1[c], xk[e2], acc[kk][c * D + e2]);
                                        t = fma(a2[e2], xk[c], t);
                                        if (c == e2) t += dot;
                                        acc[kk][c * D + e2] = t;
                                    }
                            }
                    }
                }
            }
            __syncthreads();
        }
        // --- store -------------------------------------------------------------
        if (active) {
            const int64_t e = e_begin + ui;
            const bool bad = sEl[ui * L::PER_ELEM + 10] != 0.0;
            const int n = is_vector_form(FORM) ? D * ns : ns;
            double* o = a.out + e * (int64_t)n * n;
            const double nanv = __builtin_nan("");
            if (is_vector_form(FORM)) {
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2) {
                        double* row = o + (size_t)(c * ns + uj) * n + e2 * ns + k0;
#pragma unroll
                        for (int kk = 0; kk < KB; ++kk)
                            if (kk < kn) store_out(row + kk, bad ? nanv : acc[kk][c * D + e2], a.nt);
                    }
            } else {
                double* row = o + (size_t)uj * n + k0;
                const double* ke = sEl + ui * L::PER_ELEM;
                const double adet = ke[9];
                // geometry tensor G'_ab = |det J| sum_b K[a][b] K[a'][b] for the
                // pre-evaluated gradient tables (same order as the tables)
                double gt[6] = {0, 0, 0, 0, 0, 0};
                if (FORM == HELMHOLTZ && a.stiff_tables) {
                    int r = 0;
#pragma unroll
                    for (int x = 0; x < D; ++x) {
                        double s2 = 0.0;
#pragma unroll
                        for (int b = 0; b < D; ++b) s2 = fma(ke[x * 3 + b], ke[x * 3 + b], s2);
                        gt[r++] = adet * s2;
                    }
#pragma unroll
                    for (int x = 0; x < D; ++x)
#pragma unroll
                        for (int y = x + 1; y < D; ++y) {
                            double s2 = 0.0;
#pragma unroll
                            for (int b = 0; b < D; ++b) s2 = fma(ke[x * 3 + b], ke[y * 3 + b], s2);
                            gt[r++] = adet * s2;
                        }
                }
                const size_t nn = (size_t)ns * ns;
#pragma unroll
                for (int kk = 0; kk < KB; ++kk)
                    if (kk < kn) {
                        double v = acc[kk][0];
                        const size_t jk = (size_t)uj * ns + k0 + kk;
                        if (FORM == HELMHOLTZ && a.mass_table) v = fma(adet, a.mass_table[jk], v);
                        if (FORM == HELMHOLTZ && a.stiff_tables) {
#pragma unroll
                            for (int r = 0; r < D * (D + 1) / 2; ++r) v = fma(gt[r], a.stiff_tables[(1 + r) * nn + jk], v);
                        }
                        store_out(row + kk, bad ? nanv : v, a.nt);
                    }
            }
        }
    }
    if (a.status) {
        __syncthreads();
        for (int i = tid; i < eb; i += B)
            if (sEl[i * L::PER_ELEM + 10] != 0.0) atomicAdd(a.status, 1);
    }
    __syncthreads();
}

}  // namespace fe
