/*
 * fe_oracle.c -- reference implementation of finite-element local assembly.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * CPU oracle that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * What it computes (Luporini, Ham, Kelly, "An algorithm for the optimization
 * of finite element integration loops"):
 *   the quadrature-mode element tensor of Sec. 2.2, Eq. (7): for every element
 *   K with affine map F_K from the reference cell, and every test/trial pair,
 *       A_K[i][j] = sum_q W_q |det F_K'| * integrand(Phi_i, Phi_j, coeffs)(X_q)
 *   evaluated as the naive nest of Fig. 1 (element loop, quadrature reduction
 *   loop, then the test and trial loops), with the integrand written out in
 *   full (no factorisation, no hoisting beyond the reference tabulation
 *   Phi_i(X_q) that Eq. (7) itself names);
 *   and the global assembly of Sec. 2, which sums the element matrices into
 *   the compressed-row global matrix in element order (orc_csr_insert).
 *
 * Precision: IEEE double throughout; long double only while solving for
 * quadrature nodes.
 *
 * Conventions (independent of the library's own implementation):
 *   cells  0 triangle, 1 tetrahedron, 2 prism (triangle x [0,1])
 *   forms  0 mass, 1 Helmholtz, 2 linear elasticity (P1 Lame fields),
 *          3 neo-Hookean hyperelastic tangent
 *   basis  Lagrange P_p on the equispaced lattice, node order k,j,i with i
 *          fastest; prism node (t,l) -> l*n_tri + t; vector spaces are
 *          component-blocked (row c*n_s + j).
 *   coords [E][nv][gdim]; elasticity coeff [E][2][nc] (lambda, then mu);
 *   hyperelastic coeff [E][gdim*n_s]; mass / Helmholtz with nf
 *   pre-multiplying coefficient functions coeff [E][nf][n_s];
 *   out [E][n][n] row = test, col = trial.
 *
 * Pins: every function here is checked by the CPU test suite against exact
 * rational integration, closed forms, invariants and finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORC_MUTANT
#define ORC_MUTANT 0   /* tests/test_oracle_mutants.py builds planted-mistake variants */
#endif

#define ORC_MAXQ1 16          /* max points per collapsed direction  */
#define ORC_MAXNB 80          /* max scalar basis functions (prism P4 = 75) */
#define ORC_MAXQ  (ORC_MAXQ1 * ORC_MAXQ1 * ORC_MAXQ1)

static int tdim_of(int cell) { return cell == 0 ? 2 : 3; }
static int nvert_of(int cell) { return cell == 0 ? 3 : (cell == 1 ? 4 : 6); }

int orc_nbasis(int cell, int p)
{
    if (p < 1) return -1;
    if (cell == 0) return (p + 1) * (p + 2) / 2;
    if (cell == 1) return (p + 1) * (p + 2) * (p + 3) / 6;
    if (cell == 2) return (p + 1) * (p + 2) / 2 * (p + 1);
    return -1;
}

/* ------------------------------------------------------------------------ *
 * Quadrature (Sec. 7.1: exact Gauss-Legendre-Jacobi scheme).
 * Collapsed (conical product) rules: Gauss-Legendre in the first collapsed
 * coordinate, Gauss-Jacobi with weights (1-t)^1 and (1-u)^2 in the others,
 * m points each, exact for total degree 2m-1.  Nodes are the zeros of the
 * Jacobi polynomial P_m^(a,0), found by Newton iteration with deflation.
 * ------------------------------------------------------------------------ */

/* P_n^(a,0)(x) and its derivative by the three-term recurrence. */
static void jacobi_eval(int n, long double a, long double x, long double *pn, long double *dpn)
{
    long double p0 = 1.0L, p1 = 0.5L * ((a + 2.0L) * x + a);   /* b = 0 */
    if (n == 0) { *pn = 1.0L; *dpn = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        long double c = 2.0L * k + a;              /* 2k + a + b */
        long double a1 = 2.0L * k * (k + a) * (c - 2.0L);
        long double a2 = (c - 1.0L) * (a * a);     /* (c-1)(a^2 - b^2) */
        long double a3 = (c - 1.0L) * c * (c - 2.0L);
        long double a4 = 2.0L * (k + a - 1.0L) * (k - 1.0L) * c;
        long double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1; p1 = p2;
    }
    *pn = p1;
    /* (2n+a)(1-x^2) P_n' = n[a - (2n+a)x] P_n + 2(n+a) n P_{n-1}  (b = 0) */
    long double c = 2.0L * n + a;
    *dpn = (n * (a - c * x) * p1 + 2.0L * (n + a) * n * p0) / (c * (1.0L - x * x));
}

/* m-point Gauss-Jacobi rule for weight (1-t)^a on [0,1]. */
static void gauss_jacobi01(int m, int a, double *t, double *w)
{
    long double xs[ORC_MAXQ1];
    for (int i = 0; i < m; ++i) {
        long double x = -cosl((2.0L * i + 1.0L) * 3.14159265358979323846264338327950288L / (2.0L * m));
        if (i > 0 && x <= xs[i - 1]) x = xs[i - 1] + 1e-3L;
        for (int it = 0; it < 200; ++it) {
            long double pn, dpn;
            jacobi_eval(m, (long double)a, x, &pn, &dpn);
            long double s = 0.0L;
            for (int j = 0; j < i; ++j) s += 1.0L / (x - xs[j]);
            long double dx = pn / (dpn - s * pn);
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        xs[i] = x;
    }
    for (int i = 0; i < m; ++i) {
        long double pn, dpn;
        jacobi_eval(m, (long double)a, xs[i], &pn, &dpn);
        long double wx = powl(2.0L, a + 1) / ((1.0L - xs[i] * xs[i]) * dpn * dpn);
        t[i] = (double)(0.5L * (xs[i] + 1.0L));
        w[i] = (double)(wx / powl(2.0L, a + 1 + (ORC_MUTANT == 5 ? 1 : 0)));
    }
}

static int npts_dir(int qdeg) { int m = (qdeg + 2) / 2; return m < 1 ? 1 : m; }  /* ceil((D+1)/2) */

int orc_rule_size(int cell, int qdeg)
{
    if (qdeg < 0) return -1;
    int m = npts_dir(qdeg);
    if (m > ORC_MAXQ1) return -1;
    if (cell == 0) return qdeg <= 2 ? 3 : m * m;
    if (cell == 1) return m * m * m;
    if (cell == 2) return (qdeg <= 2 ? 3 : m * m) * m;
    return -1;
}

static int tri_rule(int qdeg, double *X, double *W)
{
    if (qdeg <= 2) {   /* interior three-point rule, exact for degree 2 */
        const double a = 1.0 / 6.0, b = 2.0 / 3.0;
        X[0] = a; X[1] = a; X[2] = b; X[3] = a; X[4] = a; X[5] = b;
        W[0] = W[1] = W[2] = 1.0 / 6.0;
        return 3;
    }
    int m = npts_dir(qdeg);
    double s[ORC_MAXQ1], ws[ORC_MAXQ1], t[ORC_MAXQ1], wt[ORC_MAXQ1];
    gauss_jacobi01(m, 0, s, ws);
    gauss_jacobi01(m, 1, t, wt);
    int n = 0;
    for (int it = 0; it < m; ++it)
        for (int is = 0; is < m; ++is) {
            X[2 * n] = s[is] * (1.0 - t[it]);
            X[2 * n + 1] = t[it];
            W[n] = ws[is] * wt[it];
            ++n;
        }
    return n;
}

int orc_rule(int cell, int qdeg, double *X, double *W)
{
    int nq = orc_rule_size(cell, qdeg);
    if (nq < 0) return -1;
    int m = npts_dir(qdeg);
    if (cell == 0) return tri_rule(qdeg, X, W);
    if (cell == 1) {
        double s[ORC_MAXQ1], ws[ORC_MAXQ1], t[ORC_MAXQ1], wt[ORC_MAXQ1], u[ORC_MAXQ1], wu[ORC_MAXQ1];
        gauss_jacobi01(m, 0, s, ws);
        gauss_jacobi01(m, 1, t, wt);
        gauss_jacobi01(m, 2, u, wu);
        int n = 0;
        for (int iu = 0; iu < m; ++iu)
            for (int it = 0; it < m; ++it)
                for (int is = 0; is < m; ++is) {
                    X[3 * n] = s[is] * (1.0 - t[it]) * (1.0 - u[iu]);
                    X[3 * n + 1] = t[it] * (1.0 - u[iu]);
                    X[3 * n + 2] = u[iu];
                    W[n] = ws[is] * wt[it] * wu[iu];
                    ++n;
                }
        return n;
    }
    /* prism: triangle rule x Gauss-Legendre in z */
    double XT[2 * ORC_MAXQ1 * ORC_MAXQ1], WT[ORC_MAXQ1 * ORC_MAXQ1], z[ORC_MAXQ1], wz[ORC_MAXQ1];
    int nt = tri_rule(qdeg, XT, WT);
    gauss_jacobi01(m, 0, z, wz);
    int n = 0;
    for (int iz = 0; iz < m; ++iz)
        for (int k = 0; k < nt; ++k) {
            X[3 * n] = XT[2 * k];
            X[3 * n + 1] = XT[2 * k + 1];
            X[3 * n + 2] = z[iz];
            W[n] = WT[k] * wz[iz];
            ++n;
        }
    return n;
}

/* ------------------------------------------------------------------------ *
 * Lagrange basis on the reference cell (Sec. 2.2: local basis Phi_i on K_0).
 * Silvester's closed form: for barycentric coordinates lam and node
 * multi-index alpha with |alpha| = p,
 *     Phi_alpha = prod_v prod_{m < alpha_v} (p*lam_v - m) / (m + 1),
 * derivatives by the product rule.
 * ------------------------------------------------------------------------ */

/* L_a(t) = prod_{m<a} (p t - m)/(m+1) and dL_a/dt */
static void silvester_1d(int p, int a, double t, double *L, double *dL)
{
    double v = 1.0, d = 0.0;
    for (int m = 0; m < a; ++m) {
        double f = (p * t - m) / (m + 1.0 + (ORC_MUTANT == 6 ? 1.0 : 0.0));
        double df = p / (m + 1.0 + (ORC_MUTANT == 6 ? 1.0 : 0.0));
        d = d * f + v * df;
        v = v * f;
    }
    *L = v; *dL = d;
}

/* Simplex basis: tdim = 2 or 3.  phi[nb], dphi[nb][tdim]. */
static void simplex_basis(int tdim, int p, const double *X, double *phi, double *dphi)
{
    double lam[4];
    lam[0] = 1.0;
    for (int c = 0; c < tdim; ++c) { lam[c + 1] = X[c]; lam[0] -= X[c]; }
    int idx = 0;
    int kmax = tdim == 3 ? p : 0;
    for (int k = 0; k <= kmax; ++k)
        for (int j = 0; j <= p - k; ++j)
            for (int i = 0; i <= p - j - k; ++i) {
                int alpha[4] = {p - i - j - k, i, j, k};
                double L[4], dL[4];
                for (int v = 0; v <= tdim; ++v) silvester_1d(p, alpha[v], lam[v], &L[v], &dL[v]);
                double val = 1.0;
                for (int v = 0; v <= tdim; ++v) val *= L[v];
                phi[idx] = val;
                for (int c = 0; c < tdim; ++c) {
                    /* d lam_0 / dX_c = -1, d lam_{c+1} / dX_c = +1 */
                    double g = 0.0;
                    for (int v = 0; v <= tdim; ++v) {
                        double dlv = (v == 0) ? -1.0 : (v == c + 1 ? 1.0 : 0.0);
                        if (dlv == 0.0) continue;
                        double prod = dL[v] * dlv;
                        for (int w = 0; w <= tdim; ++w) if (w != v) prod *= L[w];
                        g += prod;
                    }
                    dphi[idx * tdim + c] = g;
                }
                ++idx;
            }
}

int orc_basis(int cell, int p, const double *X, double *phi, double *dphi)
{
    int nb = orc_nbasis(cell, p);
    if (nb < 0 || nb > ORC_MAXNB) return -1;
    if (cell == 0 || cell == 1) { simplex_basis(tdim_of(cell), p, X, phi, dphi); return nb; }
    /* prism: Phi_(t,l)(X,Y,Z) = Phi_t(X,Y) * ell_l(Z), ell_l 1-D Lagrange on l/p */
    int nt = (p + 1) * (p + 2) / 2;
    double pt[ORC_MAXNB], dpt[2 * ORC_MAXNB];
    simplex_basis(2, p, X, pt, dpt);
    for (int l = 0; l <= p; ++l) {
        double La, dLa, Lb, dLb;
        silvester_1d(p, p - l, 1.0 - X[2], &La, &dLa);
        silvester_1d(p, l, X[2], &Lb, &dLb);
        double e = La * Lb, de = -dLa * Lb + La * dLb;
        for (int t = 0; t < nt; ++t) {
            int id = l * nt + t;
            phi[id] = pt[t] * e;
            dphi[3 * id] = dpt[2 * t] * e;
            dphi[3 * id + 1] = dpt[2 * t + 1] * e;
            dphi[3 * id + 2] = pt[t] * de;
        }
    }
    return nb;
}

/* P1 (prism: P1 x P1) basis used for the Lame coefficient fields and, with
 * its gradients, for the vertex map of a non-affine prism. */
static int p1_basis(int cell, const double *X, double *psi)
{
    double dpsi[3 * 6];
    return orc_basis(cell, 1, X, psi, dpsi);
}

static int p1_basis_grad(int cell, const double *X, double *psi, double *dpsi)
{
    return orc_basis(cell, 1, X, psi, dpsi);
}

/* det and inverse K = J^{-1} of a d x d Jacobian (row-major J[r][a] = dx_r/dX_a). */
static double jac_inverse(int d, const double *J, double *K)
{
    double det;
    if (d == 2) {
        det = J[0] * J[3] - J[1] * J[2];
        K[0] = J[3] / det; K[1] = -J[1] / det; K[2] = -J[2] / det; K[3] = J[0] / det;
        return det;
    }
    double c00 = J[4] * J[8] - J[5] * J[7];
    double c01 = J[5] * J[6] - J[3] * J[8];
    double c02 = J[3] * J[7] - J[4] * J[6];
    det = J[0] * c00 + J[1] * c01 + J[2] * c02;
    K[0] = c00 / det;
    K[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    K[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    K[3] = c01 / det;
    K[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    K[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    K[6] = c02 / det;
    K[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    K[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

/* ------------------------------------------------------------------------ *
 * Geometry of the affine map F_K (Sec. 2.2): x = v0 + J X with the columns of
 * J the edge vectors v_{a+1} - v0 (prism: v1-v0, v2-v0, v3-v0).  Returns
 * det J and K = J^{-1} (K[a][b] = dX_a/dx_b).
 * ------------------------------------------------------------------------ */
int orc_geometry(int cell, const double *v, double *J, double *detJ, double *K)
{
    int d = tdim_of(cell);
    for (int a = 0; a < d; ++a)
        for (int r = 0; r < d; ++r) J[r * d + a] = v[(a + 1) * d + r] - v[r];
    double det;
    if (d == 2) {
        det = J[0] * J[3] - J[1] * J[2];
        K[0] = J[3] / det; K[1] = -J[1] / det; K[2] = -J[2] / det; K[3] = J[0] / det;
    } else {
        /* cofactor expansion */
        double c00 = J[4] * J[8] - J[5] * J[7];
        double c01 = J[5] * J[6] - J[3] * J[8];
        double c02 = J[3] * J[7] - J[4] * J[6];
        det = J[0] * c00 + J[1] * c01 + J[2] * c02;
        K[0] = c00 / det;
        K[1] = (J[2] * J[7] - J[1] * J[8]) / det;
        K[2] = (J[1] * J[5] - J[2] * J[4]) / det;
        K[3] = c01 / det;
        K[4] = (J[0] * J[8] - J[2] * J[6]) / det;
        K[5] = (J[2] * J[3] - J[0] * J[5]) / det;
        K[6] = c02 / det;
        K[7] = (J[1] * J[6] - J[0] * J[7]) / det;
        K[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    }
    *detJ = det;
    if (cell == 2) {   /* affine prism: top face is the bottom face translated */
        double scale = 0.0;
        for (int k = 0; k < 18; ++k) scale = fmax(scale, fabs(v[k]));
        for (int t = 0; t < 3; ++t)
            for (int r = 0; r < 3; ++r) {
                double e = (v[(t + 3) * 3 + r] - v[t * 3 + r]) - (v[9 + r] - v[r]);
                if (fabs(e) > 1e-12 * (scale > 0 ? scale : 1.0)) return 1;
            }
    }
    return 0;
}

/* 3x3 / 2x2 determinant and inverse of a small matrix (row-major). */
static double small_inv(int d, const double *F, double *Fi)
{
    if (d == 2) {
        double det = F[0] * F[3] - F[1] * F[2];
        Fi[0] = F[3] / det; Fi[1] = -F[1] / det; Fi[2] = -F[2] / det; Fi[3] = F[0] / det;
        return det;
    }
    double c00 = F[4] * F[8] - F[5] * F[7];
    double c01 = F[5] * F[6] - F[3] * F[8];
    double c02 = F[3] * F[7] - F[4] * F[6];
    double det = F[0] * c00 + F[1] * c01 + F[2] * c02;
    Fi[0] = c00 / det; Fi[1] = (F[2] * F[7] - F[1] * F[8]) / det; Fi[2] = (F[1] * F[5] - F[2] * F[4]) / det;
    Fi[3] = c01 / det; Fi[4] = (F[0] * F[8] - F[2] * F[6]) / det; Fi[5] = (F[2] * F[3] - F[0] * F[5]) / det;
    Fi[6] = c02 / det; Fi[7] = (F[1] * F[6] - F[0] * F[7]) / det; Fi[8] = (F[0] * F[4] - F[1] * F[3]) / det;
    return det;
}

/* ------------------------------------------------------------------------ *
 * Integrands (one (test, trial) pair at one quadrature point), written from
 * the weak forms, not from any factorised expression.
 * ------------------------------------------------------------------------ */

/* Linear elasticity 2 mu eps(v):eps(u) + lambda div v div u with
 * v = phi_j e_c (test), u = phi_k e_e (trial); gj, gk physical gradients. */
static double elasticity_pair(int d, int c, int e, const double *gj, const double *gk, double lam, double mu)
{
    double Ev[9], Eu[9];
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            /* grad v = e_c (x) g_j  ->  (grad v)[a][b] = delta_ac g_j[b] */
            double gva = (a == c ? gj[b] : 0.0), gvb = (b == c ? gj[a] : 0.0);
            double gua = (a == e ? gk[b] : 0.0), gub = (b == e ? gk[a] : 0.0);
            Ev[a * d + b] = 0.5 * (gva + gvb);
            Eu[a * d + b] = 0.5 * (gua + gub);
        }
    double dd = 0.0, trv = 0.0, tru = 0.0;
    for (int a = 0; a < d; ++a) {
        trv += Ev[a * d + a];
        tru += Eu[a * d + a];
        for (int b = 0; b < d; ++b) dd += Ev[a * d + b] * Eu[a * d + b];
    }
    return 2.0 * mu * dd + (ORC_MUTANT == 1 ? 0.0 : lam) * trv * tru;
}

/* Neo-Hookean first Piola stress P = mu (F - F^{-T}) + lam ln J F^{-T} and
 * its derivative AA[c][b][e][g] = dP_cb / dF_eg. */
static void neo_hookean(int d, const double *F, double mu, double lam, double *P, double *AA, double *Jout)
{
    double Fi[9];
    double J = small_inv(d, F, Fi);
    *Jout = J;
    double lnJ = log(J);
    for (int c = 0; c < d; ++c)
        for (int b = 0; b < d; ++b)
            P[c * d + b] = mu * (F[c * d + b] - Fi[b * d + c]) + lam * lnJ * Fi[b * d + c];
    if (!AA) return;
    for (int c = 0; c < d; ++c)
        for (int b = 0; b < d; ++b)
            for (int e = 0; e < d; ++e)
                for (int g = 0; g < d; ++g) {
                    /* d F_cb / d F_eg = delta_ce delta_bg
                     * d (F^{-T})_cb / d F_eg = -Fi[b][e] Fi[g][c]
                     * d lnJ / d F_eg = Fi[g][e]                            */
                    double v = mu * ((c == e && b == g) ? 1.0 : 0.0)
                             + (ORC_MUTANT == 2 ? -mu : mu) * Fi[b * d + e] * Fi[g * d + c]
                             + lam * Fi[g * d + e] * Fi[b * d + c]
                             - (ORC_MUTANT == 7 ? 0.0 : lam) * lnJ * Fi[b * d + e] * Fi[g * d + c];
                    AA[((c * d + b) * d + e) * d + g] = v;
                }
}

/* ------------------------------------------------------------------------ *
 * Local assembly: the naive nest of Fig. 1 for Eq. (7).
 * Returns the number of elements flagged (degenerate map, non-affine prism,
 * or J_F <= 0 for the hyperelastic form); their blocks are filled with NaN.
 * ------------------------------------------------------------------------ */
static int64_t assemble_nest(int form, int cell, int p, int qdeg, int nf, int pointgeo, int64_t E,
                             const double *coords, const double *coeff,
                             double mu_c, double lam_c, double *out, int nthreads);

int64_t orc_assemble(int form, int cell, int p, int qdeg, int64_t E,
                     const double *coords, const double *coeff,
                     double mu_c, double lam_c, double *out, int nthreads)
{
    return assemble_nest(form, cell, p, qdeg, 0, 0, E, coords, coeff, mu_c, lam_c, out, nthreads);
}

/* Prisms without the affine assumption of Sec. 2.2: F_K is the vertex map
 * x(X) = sum_v psi_v(X) v with the P1 x P1 basis psi, so J, det J and
 * J^{-1} are evaluated at every quadrature point (J(X_q) = sum_v v (x)
 * grad psi_v(X_q)) instead of once per element.  An element is flagged when
 * det J is zero, not finite, or changes sign between points. */
int64_t orc_assemble_pointgeo(int form, int p, int qdeg, int64_t E, const double *coords,
                              const double *coeff, double mu_c, double lam_c, double *out, int nthreads)
{
    return assemble_nest(form, 2, p, qdeg, 0, 1, E, coords, coeff, mu_c, lam_c, out, nthreads);
}

/* A form pre-multiplied by nf coefficient functions (the experiment matrix
 * of Sec. 7.1, which pre-multiplies each of its forms): the integrand is
 * multiplied by prod_{i<nf} f_i(X_q), each f_i in the same Lagrange space as
 * the test and trial functions.  Per element the coefficient record is the
 * form's own coefficients (elasticity: the Lame DOFs [2][nv]; hyperelastic:
 * the displacement DOFs [d][n_s]; none for mass and Helmholtz) followed by
 * the DOFs of the functions [nf][n_s]. */
int64_t orc_assemble_coef(int form, int cell, int p, int qdeg, int nf, int64_t E,
                          const double *coords, const double *coeff, double mu_c, double lam_c,
                          double *out, int nthreads)
{
    if (form < 0 || form > 3 || nf < 0 || nf > 3 || (nf > 0 && !coeff)) return -1;
    return assemble_nest(form, cell, p, qdeg, nf, 0, E, coords, coeff, mu_c, lam_c, out, nthreads);
}

/* Curved triangles and tetrahedra: F_K is the isoparametric P2 map
 * x(X) = sum_m psi2_m(X) x_m over the element's six (triangle) or ten
 * (tetrahedron) P2 nodes, coords[E][n_2][d] in the lattice node order, so J,
 * det J and J^{-1} vary over the element and are evaluated at every
 * quadrature point (J(X_q) = sum_m x_m (x) grad psi2_m(X_q)).  The Lame
 * fields stay P1 in the reference coordinates.  Flagged as the non-affine
 * prisms above. */
int64_t orc_assemble_curved(int form, int cell, int p, int qdeg, int64_t E, const double *coords,
                            const double *coeff, double mu_c, double lam_c, double *out, int nthreads)
{
    if (cell != 0 && cell != 1) return -1;
    return assemble_nest(form, cell, p, qdeg, 0, 2, E, coords, coeff, mu_c, lam_c, out, nthreads);
}

static int64_t assemble_nest(int form, int cell, int p, int qdeg, int nf, int pointgeo, int64_t E,
                             const double *coords, const double *coeff,
                             double mu_c, double lam_c, double *out, int nthreads)
{
    int d = tdim_of(cell), nv = nvert_of(cell);
    /* nodes of the element map: the vertices, or the P2 nodes of a curved simplex */
    const int nmap = pointgeo == 2 ? orc_nbasis(cell, 2) : nv;
    int ns = orc_nbasis(cell, p);
    if (ns < 0 || form < 0 || form > 3) return -1;
    int vec = (form >= 2);
    int n = vec ? d * ns : ns;
    int nq = orc_rule_size(cell, qdeg);
    if (nq < 0) return -1;
    /* per-element coefficient record: the form's own DOFs, then nf functions */
    const int own = form == 2 ? 2 * nv : (form == 3 ? d * ns : 0);
    const int cstride = own + nf * ns;
    double *X = (double *)malloc(sizeof(double) * nq * 3);
    double *W = (double *)malloc(sizeof(double) * nq);
    double *PHI = (double *)malloc(sizeof(double) * nq * ns);
    double *DPHI = (double *)malloc(sizeof(double) * nq * ns * 3);
    double *PSI = (double *)malloc(sizeof(double) * nq * 6);
    double *DPSI = (double *)malloc(sizeof(double) * (nq + 1) * 30);
    orc_rule(cell, qdeg, X, W);
    /* reference tabulation Phi_i(X_q), dPhi_i/dX_a(X_q): the tables of Eq. (7) */
    for (int q = 0; q < nq; ++q) {
        orc_basis(cell, p, X + q * d, PHI + q * ns, DPHI + q * ns * d);
        p1_basis(cell, X + q * d, PSI + q * 6);
        if (pointgeo == 1) {
            double ps[6];
#if ORC_MUTANT == 12
            /* planted mistake: the vertex map's gradient at the centroid for every point */
            const double Xc[3] = {1.0 / 3.0, 1.0 / 3.0, 0.5};
            p1_basis_grad(cell, Xc, ps, DPSI + q * 30);
#else
            p1_basis_grad(cell, X + q * d, ps, DPSI + q * 30);
#endif
        } else if (pointgeo == 2) {
            double ps[10];
#if ORC_MUTANT == 14
            /* planted mistake: the curved map's gradient taken at the first point for every point */
            orc_basis(cell, 2, X, ps, DPSI + q * 30);
#else
            orc_basis(cell, 2, X + q * d, ps, DPSI + q * 30);
#endif
        }
    }
    int64_t flagged = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : flagged)
#endif
    for (int64_t e = 0; e < E; ++e) {
        double *A = out + (size_t)e * n * n;
        const double *v = coords + (size_t)e * nmap * d;
        double J[9], K[9], detJ, det0 = 0.0;
        int bad = 0;
        if (!pointgeo) {
            bad = orc_geometry(cell, v, J, &detJ, K);
            if (!(detJ != 0.0) || !isfinite(detJ)) bad = 1;
        }
        for (int k = 0; k < n * n; ++k) A[k] = 0.0;
        double g[ORC_MAXNB * 3];
        for (int q = 0; q < nq && !bad; ++q) {
            const double *phi = PHI + q * ns, *dphi = DPHI + q * ns * d;
            if (pointgeo) {
                /* J(X_q)[r][a] = sum_v v_r dpsi_v/dX_a(X_q) */
                for (int r = 0; r < d; ++r)
                    for (int a = 0; a < d; ++a) {
                        double s = 0.0;
                        for (int l = 0; l < nmap; ++l) s += v[l * d + r] * DPSI[q * 30 + l * d + a];
                        J[r * d + a] = s;
                    }
                detJ = jac_inverse(d, J, K);
                if (q == 0) det0 = detJ;
                if (!(detJ != 0.0) || !isfinite(detJ) || (detJ > 0.0) != (det0 > 0.0)) { bad = 1; break; }
            }
            double dx = W[q] * fabs(detJ);
            /* pre-multiplying coefficient functions f_i(X_q) = sum_l f_il Phi_l(X_q) */
            for (int f = 0; f < nf; ++f) {
                const double *cf = coeff + (size_t)e * cstride + own + (size_t)f * ns;
                double fv = 0.0;
                for (int l = 0; l < ns; ++l) fv += cf[l] * phi[ORC_MUTANT == 8 ? (l + 1) % ns : l];
                if (!(ORC_MUTANT == 9 && f > 0)) dx *= fv;
            }
            /* physical gradients g_i[b] = sum_a dX_a/dx_b dPhi_i/dX_a */
            for (int i = 0; i < ns; ++i)
                for (int b = 0; b < d; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += (ORC_MUTANT == 3 ? K[b * d + a] : K[a * d + b]) * dphi[i * d + a];
                    g[i * d + b] = s;
                }
            if (form == 0) {
                for (int i = 0; i < ns; ++i)
                    for (int j = 0; j < ns; ++j) A[i * n + j] += dx * phi[i] * phi[ORC_MUTANT == 4 ? i : j];
            } else if (form == 1) {
                for (int i = 0; i < ns; ++i)
                    for (int j = 0; j < ns; ++j) {
                        double gg = 0.0;
                        for (int b = 0; b < d; ++b) gg += g[i * d + b] * g[j * d + b];
                        A[i * n + j] += dx * (gg + phi[i] * phi[j]);
                    }
            } else if (form == 2) {
                const double *ce = coeff + (size_t)e * cstride;
                double lam = 0.0, mu = 0.0;
                for (int l = 0; l < nv; ++l) {
                    lam += ce[l] * PSI[q * 6 + l];
                    mu += ce[nv + l] * PSI[q * 6 + l];
                }
                for (int c = 0; c < d; ++c)
                    for (int i = 0; i < ns; ++i)
                        for (int f = 0; f < d; ++f)
                            for (int j = 0; j < ns; ++j)
                                A[(c * ns + i) * n + f * ns + j] +=
                                    dx * elasticity_pair(d, c, f, g + i * d, g + j * d, lam, mu);
            } else {
                const double *u = coeff + (size_t)e * cstride;
                double F[9], P[9], AA[81], JF;
                for (int a = 0; a < d; ++a)
                    for (int b = 0; b < d; ++b) {
                        double s = (a == b) ? 1.0 : 0.0;
                        for (int k = 0; k < ns; ++k) s += u[a * ns + k] * g[k * d + b];
                        F[a * d + b] = s;
                    }
                neo_hookean(d, F, mu_c, lam_c, P, AA, &JF);
                if (!(JF > 0.0)) { bad = 1; break; }
                for (int c = 0; c < d; ++c)
                    for (int i = 0; i < ns; ++i)
                        for (int f = 0; f < d; ++f)
                            for (int j = 0; j < ns; ++j) {
                                double s = 0.0;
                                for (int b = 0; b < d; ++b)
                                    for (int h = 0; h < d; ++h)
                                        s += g[i * d + b] * AA[((c * d + b) * d + f) * d + h] * g[j * d + h];
                                A[(c * ns + i) * n + f * ns + j] += dx * s;
                            }
            }
        }
        if (bad) {
            for (int k = 0; k < n * n; ++k) A[k] = NAN;
            flagged += 1;
        }
    }
    free(X); free(W); free(PHI); free(DPHI); free(PSI); free(DPSI);
    return flagged;
}

/* Hyperelastic residual R_(c,i) = sum_q W_q |det J| w(X_q) sum_b P_cb g_i[b]
 * (the form whose derivative the tangent above is); also the strain energy
 * Psi = sum_q W_q |det J| w(X_q) psi(F), psi = mu/2 (tr F^T F - d) - mu ln J
 * + lam/2 ln^2 J.  w = prod_{i<nf} f_i, the pre-multiplying functions laid
 * out after the displacement DOFs as in orc_assemble_coef (w = 1 for nf = 0). */
int64_t orc_hyper_residual_coef(int cell, int p, int qdeg, int nf, int64_t E, const double *coords,
                                const double *coeff, double mu_c, double lam_c,
                                double *R, double *energy);

int64_t orc_hyper_residual(int cell, int p, int qdeg, int64_t E, const double *coords,
                           const double *coeff, double mu_c, double lam_c,
                           double *R, double *energy)
{
    return orc_hyper_residual_coef(cell, p, qdeg, 0, E, coords, coeff, mu_c, lam_c, R, energy);
}

int64_t orc_hyper_residual_coef(int cell, int p, int qdeg, int nf, int64_t E, const double *coords,
                                const double *coeff, double mu_c, double lam_c,
                                double *R, double *energy)
{
    int d = tdim_of(cell), nv = nvert_of(cell);
    int ns = orc_nbasis(cell, p);
    int nq = orc_rule_size(cell, qdeg);
    if (ns < 0 || nq < 0) return -1;
    double *X = (double *)malloc(sizeof(double) * nq * 3);
    double *W = (double *)malloc(sizeof(double) * nq);
    double *PHI = (double *)malloc(sizeof(double) * nq * ns);
    double *DPHI = (double *)malloc(sizeof(double) * nq * ns * 3);
    orc_rule(cell, qdeg, X, W);
    for (int q = 0; q < nq; ++q) orc_basis(cell, p, X + q * d, PHI + q * ns, DPHI + q * ns * d);
    int64_t flagged = 0;
    for (int64_t e = 0; e < E; ++e) {
        double *r = R + (size_t)e * d * ns;
        double J[9], K[9], detJ, psi_sum = 0.0;
        for (int k = 0; k < d * ns; ++k) r[k] = 0.0;
        if (orc_geometry(cell, coords + (size_t)e * nv * d, J, &detJ, K)) { flagged++; continue; }
        const double *u = coeff + (size_t)e * (d + nf) * ns;
        for (int q = 0; q < nq; ++q) {
            double g[ORC_MAXNB * 3], F[9], P[9], JF;
            const double *dphi = DPHI + q * ns * d;
            double wf = 1.0;
            for (int f = 0; f < nf; ++f) {
                double fv = 0.0;
                for (int l = 0; l < ns; ++l) fv += u[(d + f) * ns + l] * PHI[q * ns + l];
                wf *= fv;
            }
            for (int i = 0; i < ns; ++i)
                for (int b = 0; b < d; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += K[a * d + b] * dphi[i * d + a];
                    g[i * d + b] = s;
                }
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double s = (a == b) ? 1.0 : 0.0;
                    for (int k = 0; k < ns; ++k) s += u[a * ns + k] * g[k * d + b];
                    F[a * d + b] = s;
                }
            neo_hookean(d, F, mu_c, lam_c, P, NULL, &JF);
            double dx = W[q] * fabs(detJ) * wf;
            for (int c = 0; c < d; ++c)
                for (int i = 0; i < ns; ++i) {
                    double s = 0.0;
                    for (int b = 0; b < d; ++b) s += P[c * d + b] * g[i * d + b];
                    r[c * ns + i] += dx * s;
                }
            double trc = 0.0;
            for (int k = 0; k < d * d; ++k) trc += F[k] * F[k];
            double lnJ = log(JF);
            psi_sum += dx * (0.5 * mu_c * (trc - d) - mu_c * lnJ + 0.5 * lam_c * lnJ * lnJ);
        }
        if (energy) energy[e] = psi_sum;
    }
    free(X); free(W); free(PHI); free(DPHI);
    return flagged;
}

/* Minimum of J_F = det(I + grad u) over the quadrature points, per element
 * (used by the tests to confirm that a seeded displacement is admissible). */
int64_t orc_hyper_min_jf(int cell, int p, int qdeg, int64_t E, const double *coords,
                         const double *coeff, double *minjf, int nthreads)
{
    int d = tdim_of(cell), nv = nvert_of(cell);
    int ns = orc_nbasis(cell, p);
    int nq = orc_rule_size(cell, qdeg);
    if (ns < 0 || nq < 0) return -1;
    double *X = (double *)malloc(sizeof(double) * nq * 3);
    double *W = (double *)malloc(sizeof(double) * nq);
    double *PHI = (double *)malloc(sizeof(double) * nq * ns);
    double *DPHI = (double *)malloc(sizeof(double) * nq * ns * 3);
    orc_rule(cell, qdeg, X, W);
    for (int q = 0; q < nq; ++q) orc_basis(cell, p, X + q * d, PHI + q * ns, DPHI + q * ns * d);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t e = 0; e < E; ++e) {
        double J[9], K[9], detJ, m = INFINITY;
        orc_geometry(cell, coords + (size_t)e * nv * d, J, &detJ, K);
        const double *u = coeff + (size_t)e * d * ns;
        for (int q = 0; q < nq; ++q) {
            double g[ORC_MAXNB * 3], F[9], Fi[9];
            const double *dphi = DPHI + q * ns * d;
            for (int i = 0; i < ns; ++i)
                for (int b = 0; b < d; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += K[a * d + b] * dphi[i * d + a];
                    g[i * d + b] = s;
                }
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double s = (a == b) ? 1.0 : 0.0;
                    for (int k = 0; k < ns; ++k) s += u[a * ns + k] * g[k * d + b];
                    F[a * d + b] = s;
                }
            double jf = small_inv(d, F, Fi);
            if (jf < m) m = jf;
        }
        minjf[e] = m;
    }
    free(X); free(W); free(PHI); free(DPHI);
    return 0;
}

/* ------------------------------------------------------------------------
 * Generic scalar bilinear forms: the integrand is a sum of terms
 *     scale_t * c_t(x) * s_test_t(phi_j) * s_trial_t(phi_k),
 * each symbol s being phi itself (0) or a physical derivative d/dx_b (1 + b),
 * and c_t = 1 (field < 0) or a P1 field interpolated from its vertex values
 * fields[e][field][v] -- the multilinear operands sharing elimination
 * (Sec. 3.2, Algorithm 1) works on.  Evaluated as the naive nest of Fig. 1
 * for Eq. (7): element, point, then every (j, k) pair with every term.
 * ------------------------------------------------------------------------ */
int64_t orc_assemble_spec(int n_terms, const int *test, const int *trial, const int *field, const double *scale,
                          int n_fields, int cell, int p, int qdeg, int64_t E, const double *coords,
                          const double *fields, double *out, int nthreads)
{
    int d = tdim_of(cell), nv = nvert_of(cell);
    int ns = orc_nbasis(cell, p);
    int nq = orc_rule_size(cell, qdeg);
    if (ns < 0 || nq < 0 || n_terms < 0 || n_terms > 32) return -1;
    for (int t = 0; t < n_terms; ++t)
        if (test[t] < 0 || test[t] > d || trial[t] < 0 || trial[t] > d || field[t] >= n_fields ||
            (field[t] >= 0 && !fields))
            return -1;
    double *X = (double *)malloc(sizeof(double) * nq * 3);
    double *W = (double *)malloc(sizeof(double) * nq);
    double *PHI = (double *)malloc(sizeof(double) * nq * ns);
    double *DPHI = (double *)malloc(sizeof(double) * nq * ns * 3);
    double *PSI = (double *)malloc(sizeof(double) * nq * 6);
    orc_rule(cell, qdeg, X, W);
    for (int q = 0; q < nq; ++q) {
        orc_basis(cell, p, X + q * d, PHI + q * ns, DPHI + q * ns * d);
        p1_basis(cell, X + q * d, PSI + q * 6);
    }
    int64_t flagged = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : flagged)
#endif
    for (int64_t e = 0; e < E; ++e) {
        double *A = out + (size_t)e * ns * ns;
        const double *v = coords + (size_t)e * nv * d;
        double J[9], K[9], detJ;
        int bad = orc_geometry(cell, v, J, &detJ, K);
        if (!(detJ != 0.0) || !isfinite(detJ)) bad = 1;
        for (int k = 0; k < ns * ns; ++k) A[k] = bad ? NAN : 0.0;
        if (bad) { flagged += 1; continue; }
        double sym[ORC_MAXNB * 4];
        for (int q = 0; q < nq; ++q) {
            const double *phi = PHI + q * ns, *dphi = DPHI + q * ns * d;
            double dx = W[q] * fabs(detJ);
            for (int i = 0; i < ns; ++i) {
                sym[i * 4] = phi[i];
                for (int b = 0; b < d; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += K[a * d + b] * dphi[i * d + a];
                    sym[i * 4 + 1 + b] = s;
                }
            }
            double c[32];
            for (int t = 0; t < n_terms; ++t) {
                double ct = scale[t];
                if (field[t] >= 0) {
                    double f = 0.0;
                    for (int l = 0; l < nv; ++l) f += fields[((size_t)e * n_fields + field[t]) * nv + l] * PSI[q * 6 + l];
                    ct *= f;
                }
                c[t] = ct;
            }
            for (int j = 0; j < ns; ++j)
                for (int k = 0; k < ns; ++k) {
                    double s = 0.0;
                    for (int t = 0; t < n_terms; ++t)
#if ORC_MUTANT == 13
                        s += c[t] * sym[k * 4 + test[t]] * sym[j * 4 + trial[t]];
#else
                        s += c[t] * sym[j * 4 + test[t]] * sym[k * 4 + trial[t]];
#endif
                    A[j * ns + k] += dx * s;
                }
        }
    }
    free(X); free(W); free(PHI); free(DPHI); free(PSI);
    return flagged;
}

/* ------------------------------------------------------------------------
 * Generic bilinear forms on a vector-valued Lagrange space of n_comp
 * components: basis functions phi_j e_c, numbered component-blocked
 * (c * n_s + j).  A term couples component test_comp of the test function
 * with component trial_comp of the trial function,
 *     scale_t * c_t(x) * s_test_t(phi_j) * s_trial_t(phi_k)
 * added at (test_comp * n_s + j, trial_comp * n_s + k); symbols and fields as
 * for the scalar forms above.  The same naive nest of Fig. 1 for Eq. (7),
 * over every (row, column) pair of the n_comp * n_s square matrix and every
 * term (zero unless the term's components are the row's and the column's).
 * ------------------------------------------------------------------------ */
int64_t orc_assemble_vspec(int n_terms, const int *test, const int *trial, const int *test_comp,
                           const int *trial_comp, const int *field, const double *scale, int n_fields, int n_comp,
                           int cell, int p, int qdeg, int64_t E, const double *coords, const double *fields,
                           double *out, int nthreads)
{
    int d = tdim_of(cell), nv = nvert_of(cell);
    int ns = orc_nbasis(cell, p);
    int nq = orc_rule_size(cell, qdeg);
    if (ns < 0 || nq < 0 || n_terms < 0 || n_terms > 64 || n_comp < 1 || n_comp > 3) return -1;
    for (int t = 0; t < n_terms; ++t)
        if (test[t] < 0 || test[t] > d || trial[t] < 0 || trial[t] > d || field[t] >= n_fields ||
            (field[t] >= 0 && !fields) || test_comp[t] < 0 || test_comp[t] >= n_comp || trial_comp[t] < 0 ||
            trial_comp[t] >= n_comp)
            return -1;
    int n = n_comp * ns;
    double *X = (double *)malloc(sizeof(double) * nq * 3);
    double *W = (double *)malloc(sizeof(double) * nq);
    double *PHI = (double *)malloc(sizeof(double) * nq * ns);
    double *DPHI = (double *)malloc(sizeof(double) * nq * ns * 3);
    double *PSI = (double *)malloc(sizeof(double) * nq * 6);
    orc_rule(cell, qdeg, X, W);
    for (int q = 0; q < nq; ++q) {
        orc_basis(cell, p, X + q * d, PHI + q * ns, DPHI + q * ns * d);
        p1_basis(cell, X + q * d, PSI + q * 6);
    }
    int64_t flagged = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : flagged)
#endif
    for (int64_t e = 0; e < E; ++e) {
        double *A = out + (size_t)e * n * n;
        const double *v = coords + (size_t)e * nv * d;
        double J[9], K[9], detJ;
        int bad = orc_geometry(cell, v, J, &detJ, K);
        if (!(detJ != 0.0) || !isfinite(detJ)) bad = 1;
        for (int k = 0; k < n * n; ++k) A[k] = bad ? NAN : 0.0;
        if (bad) { flagged += 1; continue; }
        double sym[ORC_MAXNB * 4];
        double c[64];
        for (int q = 0; q < nq; ++q) {
            const double *phi = PHI + q * ns, *dphi = DPHI + q * ns * d;
            double dx = W[q] * fabs(detJ);
            for (int i = 0; i < ns; ++i) {
                sym[i * 4] = phi[i];
                for (int b = 0; b < d; ++b) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) s += K[a * d + b] * dphi[i * d + a];
                    sym[i * 4 + 1 + b] = s;
                }
            }
            for (int t = 0; t < n_terms; ++t) {
                double ct = scale[t];
                if (field[t] >= 0) {
                    double f = 0.0;
                    for (int l = 0; l < nv; ++l) f += fields[((size_t)e * n_fields + field[t]) * nv + l] * PSI[q * 6 + l];
                    ct *= f;
                }
                c[t] = ct;
            }
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    int cr = r / ns, j = r % ns, cs = s / ns, k = s % ns;
                    double acc = 0.0;
                    for (int t = 0; t < n_terms; ++t) {
#if ORC_MUTANT == 15
                        if (trial_comp[t] != cr || test_comp[t] != cs) continue;
#else
                        if (test_comp[t] != cr || trial_comp[t] != cs) continue;
#endif
                        acc += c[t] * sym[j * 4 + test[t]] * sym[k * 4 + trial[t]];
                    }
                    A[r * n + s] += dx * acc;
                }
        }
    }
    free(X); free(W); free(PHI); free(DPHI); free(PSI);
    return flagged;
}

/* ------------------------------------------------------------------------
 * Global assembly (Sec. 2): the global matrix A_ij = a(phi_i, phi_j) of the
 * continuous space is the sum over elements of the element matrices, entry
 * (j, k) of element e added at (dofs[e][j], dofs[e][k]).  The compressed-row
 * pattern (row_ptr, cols, columns sorted within a row) is given; each stored
 * entry is found by bisection and the element contributions are added one
 * by one in increasing element order (then j, then k), starting from zero.
 * Returns 0, or -1 if some (row, column) pair is missing from the pattern.
 * ------------------------------------------------------------------------ */
int orc_csr_insert(int64_t E, int n, const int32_t *dofs, int64_t N, const int64_t *row_ptr,
                   const int32_t *cols, const double *A, double *values)
{
    for (int64_t i = 0; i < row_ptr[N]; i++) values[i] = 0.0;
    for (int64_t e = 0; e < E; e++)
        for (int j = 0; j < n; j++) {
            int64_t r = dofs[e * n + j];
            for (int k = 0; k < n; k++) {
#if ORC_MUTANT == 11
                if (k == n - 1) continue;
#endif
                int32_t c = dofs[e * n + k];
                int64_t lo = row_ptr[r], hi = row_ptr[r + 1];
                while (lo < hi) {
                    int64_t mid = lo + (hi - lo) / 2;
                    if (cols[mid] < c) lo = mid + 1; else hi = mid;
                }
                if (lo == row_ptr[r + 1] || cols[lo] != c) return -1;
#if ORC_MUTANT == 10
                values[lo] += A[(e * n + k) * n + j];
#else
                values[lo] += A[(e * n + j) * n + k];
#endif
            }
        }
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
