// Quadrature rules of the reference cells (exact Gauss-Legendre-Jacobi
// scheme named in Sec. 7.1 of the paper), built on the host once per
// (cell, degree).
//
// One-dimensional rules come from the Golub-Welsch construction: the nodes of
// the m-point Gauss rule for the Jacobi weight (1-x)^a on [-1,1] are the
// eigenvalues of the symmetric tridiagonal Jacobi matrix of that weight, and
// the weights are mu_0 times the squared first components of the normalised
// eigenvectors.  The eigenproblem is solved by the implicit QL method with
// Wilkinson shifts, in long double.  Simplices use the collapsed (Duffy /
// conical product) map, so a rule of m points per direction is exact for
// total degree 2m-1.
#include <cmath>
#include <vector>

#include "fe_common.hpp"

namespace fe {

namespace {

using ld = long double;

// Symmetric tridiagonal eigensolver (implicit QL).  d: diagonal (in), eigen-
// values (out); e: sub-diagonal e[0..n-2]; z: n x n row-major, starts as the
// identity and ends holding the eigenvectors in its columns.
void ql_implicit(int n, std::vector<ld>& d, std::vector<ld>& e, std::vector<ld>& z)
{
    e.resize(n);
    e[n - 1] = 0;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                ld dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-30L * dd || std::fabs(e[m]) < 1e-4000L) break;
            }
            if (m == l) break;
            ld g = (d[l + 1] - d[l]) / (2 * e[l]);
            ld r = std::hypot(g, (ld)1);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            ld s = 1, c = 1, p = 0;
            int i = m - 1;
            bool underflow = false;
            for (; i >= l; --i) {
                ld f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0) {
                    d[i + 1] -= p;
                    e[m] = 0;
                    underflow = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int k = 0; k < n; ++k) {
                    ld t = z[k * n + i + 1];
                    z[k * n + i + 1] = s * z[k * n + i] + c * t;
                    z[k * n + i] = c * z[k * n + i] - s * t;
                }
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0;
        }
    }
}

// m-point Gauss rule for the weight (1-t)^a on [0,1], nodes ascending.
void gauss_jacobi_01(int m, int a, std::vector<double>& t, std::vector<double>& w)
{
    std::vector<ld> d(m), e(m > 1 ? m - 1 : 1), z(m * m, 0);
    const ld al = a;   // weight (1-x)^al (1+x)^0 on [-1,1]
    for (int n = 0; n < m; ++n) {
        ld s = 2 * n + al;
        d[n] = (n == 0) ? -al / (al + 2) : -(al * al) / (s * (s + 2));
        if (n >= 1) {
            ld num = 4 * (ld)n * (n + al) * n * (n + al);
            ld den = s * s * (s + 1) * (s - 1);
            e[n - 1] = std::sqrt(num / den);
        }
    }
    for (int i = 0; i < m; ++i) z[i * m + i] = 1;
    ql_implicit(m, d, e, z);
    const ld mu0 = std::pow((ld)2, al + 1) / (al + 1);
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j)
            if (d[order[j]] < d[order[i]]) std::swap(order[i], order[j]);
    t.resize(m);
    w.resize(m);
    const ld scale = std::pow((ld)2, -(al + 1));   // map to [0,1] with weight (1-t)^a
    for (int i = 0; i < m; ++i) {
        int k = order[i];
        ld v0 = z[0 * m + k];
        t[i] = (double)((d[k] + 1) / 2);
        w[i] = (double)(mu0 * v0 * v0 * scale);
    }
}

void triangle_rule(int qdeg, std::vector<double>& X, std::vector<double>& W)
{
    X.clear();
    W.clear();
    if (qdeg <= 2) {
        const double a = 1.0 / 6.0, b = 2.0 / 3.0;
        X = {a, a, b, a, a, b};
        W = {1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
        return;
    }
    int m = rule_m(qdeg);
    std::vector<double> s, ws, t, wt;
    gauss_jacobi_01(m, 0, s, ws);
    gauss_jacobi_01(m, 1, t, wt);
    for (int is = 0; is < m; ++is)
        for (int it = 0; it < m; ++it) {
            X.push_back(s[is] * (1.0 - t[it]));
            X.push_back(t[it]);
            W.push_back(ws[is] * wt[it]);
        }
}

}  // namespace

// Fills X [nq][tdim] and W [nq]; returns nq, or -1 for an invalid request.
int build_rule(int cell, int qdeg, std::vector<double>& X, std::vector<double>& W)
{
    if (qdeg < 0 || qdeg > MAX_QDEG || cell < 0 || cell > 2) return -1;
    if (cell == TRI) {
        triangle_rule(qdeg, X, W);
        return (int)W.size();
    }
    int m = rule_m(qdeg);
    X.clear();
    W.clear();
    if (cell == TET) {
        std::vector<double> s, ws, t, wt, u, wu;
        gauss_jacobi_01(m, 0, s, ws);
        gauss_jacobi_01(m, 1, t, wt);
        gauss_jacobi_01(m, 2, u, wu);
        for (int is = 0; is < m; ++is)
            for (int it = 0; it < m; ++it)
                for (int iu = 0; iu < m; ++iu) {
                    X.push_back(s[is] * (1.0 - t[it]) * (1.0 - u[iu]));
                    X.push_back(t[it] * (1.0 - u[iu]));
                    X.push_back(u[iu]);
                    W.push_back(ws[is] * wt[it] * wu[iu]);
                }
        return (int)W.size();
    }
    std::vector<double> XT, WT, z, wz;
    triangle_rule(qdeg, XT, WT);
    gauss_jacobi_01(m, 0, z, wz);
    for (size_t k = 0; k < WT.size(); ++k)
        for (int iz = 0; iz < m; ++iz) {
            X.push_back(XT[2 * k]);
            X.push_back(XT[2 * k + 1]);
            X.push_back(z[iz]);
            W.push_back(WT[k] * wz[iz]);
        }
    return (int)W.size();
}

}  // namespace fe
