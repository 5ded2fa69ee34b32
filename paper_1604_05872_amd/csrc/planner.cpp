// Transformation algorithm (Sec. 4.1, Algorithm 3) with the cost function of
// Sec. 4.2, for the forms of the library.  Host-only.
//
// Operation counts are those of the innermost (j,k) loops per element
// (local optimality, Def. 10), counting each multiplication and each addition
// once, with the sharing-eliminated bodies the kernels execute:
//   theta_se(m)  = nq * (scalar pairs) * (ops per pair and point of m)
//   theta_pre(m) = 2 * rho * iota * (entries): rho pre-evaluable terms per
//                  entry, each expanded iota times (one multiply-add per term)
//   iota = C(n + k - 1, k): k coefficient functions in the monomial, n the
//          basis functions of the coefficient space (Sec. 4.2, Fig. 6); the
//          nf pre-multiplying functions of mass and Helmholtz live in the
//          test/trial space (n = n_s), the Lame fields of elasticity in P1.
// theta(m) = theta_pre(m) - theta_se(m); pre-evaluation is profitable iff
// theta < 0 (the sign convention of Sec. 4.1, which the algorithm's step 1
// uses).  Step 3 discards a bipartition whose pre-evaluated tables exceed T_H
// (Constraint 2, Sec. 3.4); identical tables are counted once (step 5 note).
// Argmin ties go to a plan with all monomials in one mode (one kernel),
// then to fewer pre-evaluated monomials (less memory).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>

#include "felocal.h"
#include "internal.hpp"

namespace fe {

static long binom(long n, long k)
{
    long r = 1;
    for (long i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

}  // namespace fe

using namespace fe;

extern "C" int fe_plan(fe_form_t form, fe_cell_t cell, int degree, int nf, int qdeg, size_t th_bytes,
                       fe_plan_t* plan)
{
    if (!plan || (int)form < 0 || (int)form > 3 || (int)cell < 0 || (int)cell > 2 || degree < 1 ||
        degree > MAX_DEGREE || qdeg > MAX_QDEG || nf < 0 || nf > 3)
        return FE_EINVAL;
    std::memset(plan, 0, sizeof(*plan));
    if (qdeg < 0) qdeg = default_qdeg(form, cell, degree, nf);
    if (qdeg > MAX_QDEG) return FE_EINVAL;
    if (th_bytes == 0) {
        // FE_TH_BYTES in the environment (a positive byte count) overrides the
        // device's L2 capacity
        const char* env = std::getenv("FE_TH_BYTES");
        const unsigned long long v = env ? std::strtoull(env, nullptr, 10) : 0ull;
        int ndev = 0;
        th_bytes = v > 0 ? (size_t)v
                         : (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) ? device_l2_bytes() : (size_t)4 << 20;
    }
    const double inf = std::numeric_limits<double>::infinity();
    const int d = cell_dim(cell), ns = n_scalar(cell, degree), nq = rule_size(cell, qdeg), nc = cell_nv(cell);
    const double pairs = (double)ns * ns;
    const size_t tbl = (size_t)ns * ns * sizeof(double);
    // nf pre-multiplying coefficient functions in the test/trial space: the
    // expansion of Sec. 4.2 has iota = C(n_s + nf - 1, nf) distinct tables
    const int iota_f = (int)binom(ns + nf - 1, nf);
    // table-set ids for the dedup of identical tables
    int table_set[4] = {0, 0, 0, 0};
    int nm = 0;
    bool legal[4] = {false, false, false, false};
    switch (form) {
    case FE_MASS:
        nm = 1;
        plan->theta_se[0] = nq * pairs * 2;
        plan->iota[0] = iota_f;
        plan->rho[0] = 1;
        plan->table_bytes[0] = (size_t)iota_f * tbl;
        table_set[0] = 1;
        legal[0] = true;
        break;
    case FE_HELMHOLTZ:
        nm = 2;   // grad v . grad u, then v u
        plan->theta_se[0] = nq * pairs * 2 * d;
        plan->iota[0] = iota_f;
        plan->rho[0] = d * (d + 1) / 2;
        plan->table_bytes[0] = (size_t)plan->rho[0] * iota_f * tbl;
        table_set[0] = 2;
        plan->theta_se[1] = nq * pairs * 2;
        plan->iota[1] = iota_f;
        plan->rho[1] = 1;
        plan->table_bytes[1] = (size_t)iota_f * tbl;
        table_set[1] = 1;
        legal[0] = legal[1] = true;
        break;
    case FE_ELASTICITY:
        nm = 2;   // lambda div v div u, then 2 mu eps(v):eps(u); one P1 coefficient each
        plan->theta_se[0] = nq * pairs * 2.0 * d * d;
        plan->theta_se[1] = nq * pairs * (2.0 * d * d + 3.0 * d);
        for (int m = 0; m < 2; ++m) {
            // the P1 Lame field (n_c functions) times the nf pre-multiplying
            // functions: iota = n_c C(n_s + nf - 1, nf) distinct tables per term
            plan->iota[m] = (int)binom(nc + 1 - 1, 1) * iota_f;
            // int psi_l prod_S phi dphi_j/dX_a dphi_k/dX_b
            plan->table_bytes[m] = (size_t)nc * iota_f * d * d * tbl;
            table_set[m] = 3;                                   // the same tables serve both
        }
        plan->rho[0] = d * d;
        plan->rho[1] = 2 * d * d;
        // the pre-evaluated kernel takes both monomials together (one set of
        // tables): a plan that splits them has no kernel (see below)
        legal[0] = legal[1] = true;
        break;
    default:
        // hyperelastic tangent: the terms in F (lambda' s_j,c s_k,e and
        // alpha' s_j,e s_k,c, 2 d^2 entries of two operations each per pair
        // and point) have a non-polynomial coefficient, so pre-evaluation is
        // not legal for them; the trace term mu |det J| g_j . g_k has a
        // constant coefficient (g_j . g_k: d products, d - 1 sums, then d
        // diagonal-block additions)
        nm = 2;
        plan->theta_se[0] = nq * pairs * 4.0 * d * d;
        plan->iota[0] = 0;
        plan->rho[0] = 0;
        plan->table_bytes[0] = 0;
        legal[0] = false;
        plan->theta_se[1] = nq * pairs * 3.0 * d;
        plan->iota[1] = iota_f;            // 1 without pre-multiplying functions
        plan->rho[1] = d * (d + 1) / 2;   // tables S_ab, a <= b
        plan->table_bytes[1] = (size_t)plan->rho[1] * iota_f * tbl;
        table_set[1] = 2;
        legal[1] = true;
        break;
    }
    // with coefficient functions the pre-evaluated kernel keeps a 16-element
    // tile of the expanded geometry tensor in LDS: a monomial whose tile
    // would not fit has no kernel (not legal)
    if (nf > 0) {
        int ndev = 0;
        const size_t lds_block =
            (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) ? device_lds_per_block() : (size_t)64 << 10;
        if (form == FE_ELASTICITY) {
            // one block's coefficient rows (the n_c iota_f d^2 tables) per tile
            if (preeval_elast_coef_lds_bytes(cell, nc * iota_f * d * d, nf, ns) > lds_block)
                legal[0] = legal[1] = false;
        } else if (form == FE_HYPERELASTIC) {
            // the trace term: the Helmholtz gradient tables with the functions
            const size_t nr = (size_t)n_tables(FE_HELMHOLTZ, cell), rho = (size_t)d * (d + 1) / 2;
            const size_t tile = 16 * sizeof(double) * ((rho * iota_f + 7) / 8 * 8 + nr + (size_t)nf * ns);
            if (tile > lds_block) legal[1] = false;
        } else {
            const size_t nr = (size_t)n_tables(form, cell);
            const size_t tile = 16 * sizeof(double) * ((nr * iota_f + 7) / 8 * 8 + nr + (size_t)nf * ns);
            if (tile > lds_block)
                for (int m = 0; m < nm; ++m) legal[m] = false;
        }
    }
    const double entries = is_vector_form(form) ? pairs * d * d : pairs;
    for (int m = 0; m < nm; ++m)
        plan->theta_pre[m] = plan->iota[m] > 0 ? 2.0 * plan->rho[m] * plan->iota[m] * entries : inf;
    if (form == FE_HYPERELASTIC) {
        plan->theta_pre[0] = inf;
        // the trace matrix is n_s x n_s, then added to the d diagonal blocks
        plan->theta_pre[1] = (2.0 * plan->rho[1] * plan->iota[1] + d) * pairs;
    }
    plan->n_monomials = nm;
    plan->th_bytes = th_bytes;

    // step 1: S = {theta > 0} (or pre-evaluation unavailable), P = M \ S
    int inP[4] = {0, 0, 0, 0};
    for (int m = 0; m < nm; ++m) inP[m] = legal[m] && (plan->theta_pre[m] - plan->theta_se[m] <= 0.0);
    // steps 2-4: enumerate bipartitions of P, discard those over T_H, argmin
    double best = inf;
    int best_mask = 0, best_count = 99;
    for (int mask = 0; mask < (1 << nm); ++mask) {
        bool ok = true;
        for (int m = 0; m < nm; ++m)
            if ((mask >> m & 1) && !inP[m]) ok = false;
        if (!ok) continue;
        // elasticity: both monomials in one mode
        if (form == FE_ELASTICITY && mask != 0 && mask != (1 << nm) - 1) continue;
        size_t mem = 0;
        int seen = 0;
        for (int m = 0; m < nm; ++m)
            if (mask >> m & 1) {
                if (!(seen & (1 << table_set[m]))) mem += plan->table_bytes[m];
                seen |= 1 << table_set[m];
            }
        if (mem > th_bytes) continue;
        double D = 0.0;
        int cnt = 0;
        for (int m = 0; m < nm; ++m) {
            if (mask >> m & 1) {
                D += plan->theta_pre[m];
                ++cnt;
            } else {
                D += plan->theta_se[m];
            }
        }
        // ties: a plan that keeps every monomial in one mode (one kernel),
        // then the fewest pre-evaluated monomials (least memory)
        const bool uniform = (cnt == 0 || cnt == nm);
        const bool best_uniform = (best_count == 0 || best_count == nm);
        if (D < best || (D == best && ((uniform && !best_uniform) ||
                                       (uniform == best_uniform && cnt < best_count)))) {
            best = D;
            best_mask = mask;
            best_count = cnt;
        }
    }
    plan->cost = best;
    bool all = nm > 0;
    for (int m = 0; m < nm; ++m) {
        plan->preevaluated[m] = (best_mask >> m) & 1;
        all = all && plan->preevaluated[m];
    }
    plan->mode = all ? FE_MODE_PREEVAL : FE_MODE_QUADRATURE;
    return FE_OK;
}
