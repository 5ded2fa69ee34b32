// Automatic sharing elimination (Sec. 3.2, Algorithm 1) for generic
// bilinear forms, scalar or on a vector-valued space, and a quadrature kernel
// generated from its result.
//
// A form is a sum of terms scale * c(x) * s_test(phi_j) * s_trial(phi_k),
// s being the basis function or one of its physical derivatives (the
// multilinear symbols) and c a constant or a P1 field (a coefficient, hoisted
// out of the (j, k) loops by generalised code motion, Strategy 1).  On a
// vector-valued space (basis functions phi_j e_c, component-blocked) a term
// couples one test and one trial component, so each component block of the
// element matrix is a (j, k) loop nest of its own, with its own products;
// the steps below run per block, and the symbols of phi_j are the same in
// every block.
//   * Terms with the same pair of symbols are merged into one product whose
//     coefficient is their sum (the partition of step 1).
//   * The sharing graph (step 3) has one vertex per distinct symbol of each
//     side and one edge per product.
//   * The ILP of step 5 -- minimise the number of factorised symbols such
//     that every product is grouped under exactly one factorised endpoint --
//     asks for a minimum vertex cover with an orientation of the edges; a
//     block's graph has at most 8 vertices, so it is solved exactly by
//     enumerating the vertex subsets (ties: the lower operation count, then
//     the first subset in enumeration order).
//   * Step 6 emits the loop nest: per point, each factorised test symbol u
//     gets a hoisted temporary h_u(k) = sum over its products of c s_trial(k)
//     (Strategy 2), each factorised trial symbol v a temporary h_v(j); the
//     innermost (j, k) body has one multiply-add per factorised symbol,
//     accumulated in per-lane register tiles of the element matrix.
// The kernel is written out as HIP source for the form, the cell and the
// degree, compiled at run time with hipRTC for the current device, and
// cached.  fe_options_t.shape.kernel = 5 selects the expanded loop nest
// instead (every product in the innermost body), for comparison.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "felocal.h"
#include "internal.hpp"

namespace fe {
namespace {

constexpr int MAXV = FE_MAX_VERTICES;
constexpr int MAXBV = 8;   // vertices of one block: 4 symbols per side

struct Graph {
    int nc = 1;   // components of the space (1: scalar form)
    int nv = 0, ne = 0;
    int blk[MAXV], side[MAXV], sym[MAXV];
    int et[FE_MAX_TERMS], er[FE_MAX_TERMS];      // vertex indices of each product
    std::vector<int> terms_of[FE_MAX_TERMS];      // terms merged into product e
    int nblocks() const { return nc * nc; }
};

int term_block(const fe_form_spec_t* s, int nc, int t) { return s->terms[t].test_comp * nc + s->terms[t].trial_comp; }

int vertex_of(Graph& g, int blk, int side, int sym)
{
    for (int i = 0; i < g.nv; ++i)
        if (g.blk[i] == blk && g.side[i] == side && g.sym[i] == sym) return i;
    g.blk[g.nv] = blk;
    g.side[g.nv] = side;
    g.sym[g.nv] = sym;
    return g.nv++;
}

int spec_components(const fe_form_spec_t* s) { return s->n_comp > 1 ? s->n_comp : 1; }

int validate_spec(const fe_form_spec_t* s, int d)
{
    if (!s || s->n_terms < 1 || s->n_terms > FE_MAX_TERMS || s->n_fields < 0 || s->n_fields > FE_MAX_FIELDS)
        return FE_EINVAL;
    if (s->n_comp < 0 || (s->n_comp > 1 && s->n_comp != d)) return FE_EINVAL;
    const int nc = spec_components(s);
    for (int t = 0; t < s->n_terms; ++t) {
        const fe_term_t& x = s->terms[t];
        if (x.test < 0 || x.test > d || x.trial < 0 || x.trial > d) return FE_EINVAL;
        if (x.field < -1 || x.field >= s->n_fields || !std::isfinite(x.scale)) return FE_EINVAL;
        if (x.test_comp < 0 || x.test_comp >= nc || x.trial_comp < 0 || x.trial_comp >= nc) return FE_EINVAL;
    }
    return FE_OK;
}

void build_graph(const fe_form_spec_t* s, Graph& g)
{
    g.nc = spec_components(s);
    // block by block; within a block test vertices first, then trial
    // vertices (symbol order within a side)
    for (int b = 0; b < g.nblocks(); ++b)
        for (int side = 0; side < 2; ++side)
            for (int sym = 0; sym < 4; ++sym)
                for (int t = 0; t < s->n_terms; ++t)
                    if (term_block(s, g.nc, t) == b && (side == 0 ? s->terms[t].test : s->terms[t].trial) == sym) {
                        vertex_of(g, b, side, sym);
                        break;
                    }
    for (int t = 0; t < s->n_terms; ++t) {
        const int b = term_block(s, g.nc, t);
        const int u = vertex_of(g, b, 0, s->terms[t].test), v = vertex_of(g, b, 1, s->terms[t].trial);
        int e = 0;
        while (e < g.ne && !(g.et[e] == u && g.er[e] == v)) ++e;
        if (e == g.ne) {
            g.et[e] = u;
            g.er[e] = v;
            g.terms_of[e].clear();
            ++g.ne;
        }
        g.terms_of[e].push_back(t);
    }
}

// Operation counts per element and block (multiply and add each count one;
// n is the block's width, the number of scalar basis functions).
//   expanded: per point w c_e s_test(j) for every product and j, then one
//             multiply-add per product and (j, k);
//   factorised: per point the temporaries (a multiply-add per grouped
//             product and index), w s(j) per factorised symbol and j, then one
//             multiply-add per factorised symbol and (j, k).
double theta_expanded(int ne, double n, double nq) { return nq * (2.0 * ne * n * n + 2.0 * ne * n); }

double theta_factorised(const Graph& g, const std::vector<int>& vs, const int* x, const int* owner, double n,
                        double nq)
{
    double inner = 0.0, hoist = 0.0;
    for (int i : vs)
        if (x[i]) {
            int deg = 0;
            for (int e = 0; e < g.ne; ++e) deg += owner[e] == i;
            inner += 2.0 * n * n;
            hoist += 2.0 * deg * n + n;
        }
    return nq * (inner + hoist);
}

// Exact solution of the ILP of Algorithm 1, step 5, for one block (its
// vertices vs and products es); writes x and owner for them.
void solve_ilp(const Graph& g, const std::vector<int>& vs, const std::vector<int>& es, double n, double nq, int* x,
               int* owner, double* best_theta)
{
    const int m = (int)vs.size();
    int best_count = MAXBV + 1;
    *best_theta = 0.0;
    int tx[MAXV], town[FE_MAX_TERMS];
    for (int e = 0; e < g.ne; ++e) town[e] = -2;   // other blocks' products stay unowned here
    for (unsigned sel = 1; sel < (1u << m); ++sel) {
        int count = 0;
        for (int a = 0; a < m; ++a) count += tx[vs[a]] = (sel >> a) & 1;
        bool cover = true;
        for (int e : es) {
            // y: a product goes to its factorised test symbol when both ends are
            // factorised (either choice gives the same count)
            if (tx[g.et[e]]) town[e] = g.et[e];
            else if (tx[g.er[e]]) town[e] = g.er[e];
            else {
                cover = false;
                break;
            }
        }
        if (!cover || count > best_count) continue;
        const double th = theta_factorised(g, vs, tx, town, n, nq);
        if (count < best_count || th < *best_theta) {
            best_count = count;
            *best_theta = th;
            for (int i : vs) x[i] = tx[i];
            for (int e : es) owner[e] = town[e];
        }
    }
}

int default_form_qdeg(const fe_form_spec_t* s, int p)
{
    bool field = false;
    for (int t = 0; t < s->n_terms; ++t) field |= s->terms[t].field >= 0;
    return 2 * p + (field ? 1 : 0);
}

const char* SYMNAME[4] = {"s0", "s1", "s2", "s3"};

// Layout of the generated nest.  A wavefront holds EPW elements, LPE =
// 64 / EPW lanes each, and each lane owns a TR x TC block of its element's
// matrix, so one K step costs TR + TC LDS reads and TR * TC multiply-adds per
// lane.  The layout minimises, per element, the larger of the two per K
// step: the VALU time (4 cycles per wavefront float64 multiply-add) and the
// LDS time (a wavefront read of one double returns 512 bytes, at 128 bytes
// per clock shared by the four SIMDs of a CU: 16 cycles), both shared by the
// EPW elements of the wavefront.
bool pick_layout(int ns, int* epw, int* tr, int* tc, int max_area = 64)
{
    *epw = 1;
    *tr = *tc = 8;
    double best = 1e30;
    for (int lim : {40, 64}) {
        bool found = false;
        for (int w = 1; w <= 8; w *= 2) {
            const int lpe = 64 / w;
            if (ns > lpe) continue;
            for (int a = 1; a <= 8; ++a)
                for (int b = 1; b <= 8; ++b) {
                    const int rt = (ns + a - 1) / a, ct = (ns + b - 1) / b;
                    if (a * b > lim || a * b > max_area || rt * ct > lpe || rt * a > lpe || ct * b > lpe) continue;
                    const double cost = std::max(4.0 * a * b, 16.0 * (a + b)) / w;
                    if (cost < best || (cost == best && a * b < *tr * *tc)) {
                        best = cost;
                        *epw = w;
                        *tr = a;
                        *tc = b;
                        found = true;
                    }
                }
        }
        if (found) return true;
    }
    return false;
}

// HIP source of the quadrature kernel of one form: EPW elements per
// wavefront.  Per element, the component blocks with products are taken one
// after the other (a scalar form has one block), or, for a vector form whose
// blocks' tiles fit together (allow_fused), all in one point loop (the fused
// nest below); an empty block is stored as zeros.  Per block and point, lane
// i of an element computes the symbols of
// basis function i and from them the row factor X_f(i) and the column factor
// Y_f(i) of every K step f of the block; the block is the sum over points and
// K steps of X_f Y_f^T, accumulated in register tiles.  Sharing-eliminated:
// one K step per factorised symbol (test symbol u: X = w s_u, Y = h_u, the
// hoisted sum of c_e s_trial over its products; trial symbol v: X = w h_v,
// Y = s_v).  Expanded: one K step per product (X = w c_e s_test, Y =
// s_trial).
std::string generate(const fe_form_spec_t* s, const Graph& g, const int* x, const int* owner, int cell, int p,
                     bool expanded, bool allow_fused = true)
{
    const int d = cell_dim(cell), nv = cell_nv(cell), ns = n_scalar(cell, p), nc = g.nc;
    struct Block {
        int a = 0, b = 0;
        std::vector<int> edges;
        std::vector<std::string> xs, ys;
    };
    std::vector<Block> blocks(g.nblocks());
    auto coef_sum = [&](int i, bool test_side) {
        std::string t = "(0.0";
        for (int e = 0; e < g.ne; ++e)
            if (owner[e] == i) t += std::string(" + c") + std::to_string(e) + " * " + SYMNAME[g.sym[test_side ? g.et[e] : g.er[e]]];
        return t + ")";
    };
    int nkmax = 1;
    for (int bi = 0; bi < g.nblocks(); ++bi) {
        Block& B = blocks[bi];
        B.a = bi / nc;
        B.b = bi % nc;
        bool any = false;
        for (int e = 0; e < g.ne; ++e)
            if (g.blk[g.et[e]] == bi) B.edges.push_back(e);
        for (int i = 0; i < g.nv; ++i) any |= g.blk[i] == bi && x[i] != 0;
        if (expanded || !any) {
            for (int e : B.edges) {
                B.xs.push_back(std::string("wq * c") + std::to_string(e) + " * " + SYMNAME[g.sym[g.et[e]]]);
                B.ys.push_back(SYMNAME[g.sym[g.er[e]]]);
            }
        } else {
            for (int i = 0; i < g.nv; ++i) {
                if (g.blk[i] != bi || !x[i]) continue;
                if (g.side[i] == 0) {
                    B.xs.push_back(std::string("wq * ") + SYMNAME[g.sym[i]]);
                    B.ys.push_back(coef_sum(i, false));
                } else {
                    B.xs.push_back("wq * " + coef_sum(i, true));
                    B.ys.push_back(SYMNAME[g.sym[i]]);
                }
            }
        }
        nkmax = std::max(nkmax, (int)B.xs.size());
    }
    // vector forms: the layout whose tiles of all non-empty blocks fit in 64
    // doubles per lane, for the fused nest below, if there is one and its K
    // step costs at most 1.5 times the unconstrained layout's (the fused nest
    // saves the per-block repetition of the point work, not K-step work;
    // measured on MI355X: elasticity tet P2 fused 2x2 tiles 9% faster, tet P3
    // fused 1x7 tiles 41% slower than the per-block nest)
    auto kcost = [](int w, int a, int b) { return std::max(4.0 * a * b, 16.0 * (a + b)) / w; };
    int nbne = 0;
    for (const Block& B : blocks) nbne += B.xs.empty() ? 0 : 1;
    int epw = 1, tr = 1, tc = 1;
    pick_layout(ns, &epw, &tr, &tc);
    bool fusable = false;
    if (allow_fused && nc > 1 && nbne > 1) {
        int fw = 1, fa = 1, fb = 1;
        if (pick_layout(ns, &fw, &fa, &fb, 64 / nbne) && kcost(fw, fa, fb) <= 1.5 * kcost(epw, tr, tc)) {
            fusable = true;
            epw = fw;
            tr = fa;
            tc = fb;
        }
    }
    const int rt = (ns + tr - 1) / tr, ct = (ns + tc - 1) / tc;
    // two buffers of factors per wavefront (one wave_sync per point) when
    // they fit in 48 KiB per block
    const int nbuf = 2 * 4 * epw * nkmax * (rt * tr + ct * tc) * 8 <= 48 * 1024 ? 2 : 1;
    std::ostringstream o;
    o.precision(17);
    o << "// generated: " << (nc > 1 ? "vector-valued" : "scalar") << " bilinear form, cell " << cell << ", degree "
      << p << (expanded ? ", expanded products\n" : ", sharing-eliminated\n");
    o << "#define NS " << ns << "\n#define NN " << nc * ns << "\n#define D " << d << "\n#define NV " << nv
      << "\n#define NF " << s->n_fields << "\n#define NK " << nkmax << "\n#define TR " << tr << "\n#define TC " << tc
      << "\n#define RT " << rt << "\n#define CT " << ct << "\n#define NXP " << rt * tr << "\n#define NYP " << ct * tc
      << "\n#define NBUF " << nbuf << "\n#define EPW " << epw << "\n#define LPE " << 64 / epw << "\n";
    o << R"(
__device__ static inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

extern "C" __global__ __launch_bounds__(256) void fe_form_kernel(
    const double* __restrict__ coords, const double* __restrict__ fields, double* __restrict__ out,
    int* __restrict__ status, const double* __restrict__ W, const double* __restrict__ phi,
    const double* __restrict__ dphi, const double* __restrict__ psi, long long E, int nq)
{
    // row and column factors of the current point, per wavefront
    __shared__ double sX[4][NBUF][EPW][NK][NXP];
    __shared__ double sY[4][NBUF][EPW][NK][NYP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sub = lane / LPE, li = lane - sub * LPE;     // element of the wavefront, lane within it
    const int rt = li / CT, ct = li - (li / CT) * CT;
    const bool act = li < RT * CT;
    for (long long e0 = ((long long)blockIdx.x * 4 + wv) * EPW; e0 < E; e0 += (long long)gridDim.x * 4 * EPW) {
        // lanes of an element past the end work on the last one and store nothing
        const bool valid = e0 + sub < E;
        const long long e = valid ? e0 + sub : E - 1;
        double v[NV * D];
        for (int i = 0; i < NV * D; ++i) v[i] = coords[e * NV * D + i];
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, K[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int a = 0; a < D; ++a)
            for (int r = 0; r < D; ++r) J[r][a] = v[(a + 1) * D + r] - v[r];
        double det;
        if (D == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            K[0][0] = J[1][1] / det; K[0][1] = -J[0][1] / det; K[1][0] = -J[1][0] / det; K[1][1] = J[0][0] / det;
        } else {
            const double c0 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c1 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c2 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            det = J[0][0] * c0 + J[0][1] * c1 + J[0][2] * c2;
            K[0][0] = c0 / det; K[1][0] = c1 / det; K[2][0] = c2 / det;
            K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
            K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
            K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
            K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        }
        const double adet = __builtin_fabs(det);
        double jmax = 0.0, vmax = 0.0;
        for (int r = 0; r < D; ++r)
            for (int a = 0; a < D; ++a) jmax = __builtin_fmax(jmax, __builtin_fabs(J[r][a]));
        double scale = jmax;
        for (int k = 1; k < D; ++k) scale *= jmax;
        int bad = !(adet > 1e-13 * scale);
        if (NV == 6) {   // prisms must be affine: top face = bottom face translated
            for (int i = 0; i < 18; ++i) vmax = __builtin_fmax(vmax, __builtin_fabs(v[i]));
            for (int t = 0; t < 3; ++t)
                for (int r = 0; r < 3; ++r)
                    if (__builtin_fabs((v[(t + 3) * 3 + r] - v[t * 3 + r]) - (v[9 + r] - v[r])) > 1e-12 * (vmax > 0 ? vmax : 1.0))
                        bad = 1;
        }
        // the element's coefficient-field values at its vertices, read once
        double fv[NF > 0 ? NF * NV : 1];
        for (int i = 0; i < NF * NV; ++i) fv[i] = fields[e * NF * NV + i];
        (void)fv;
)";
    // Vector forms whose non-empty blocks' register tiles fit together (at most
    // 64 doubles per lane): one point loop per element; the symbols and the
    // coefficient fields of a point are formed once and every non-empty block
    // accumulates from them (its factors through the same LDS buffer, two
    // wave_syncs per block and point).  Otherwise, for scalar forms, and when
    // the caller asks for it (the fused kernel would hold less than two
    // wavefronts per SIMD), the blocks take the point loop one after the other.
    const bool fused = fusable;
    if (fused) {
        o << "        // fused blocks: " << nbne << " non-empty of " << blocks.size() << "\n";
        o << "        double acc[" << nbne << "][TR][TC];\n";
        o << R"(#pragma unroll
        for (int bb = 0; bb < )" << nbne << R"(; ++bb)
#pragma unroll
            for (int r = 0; r < TR; ++r)
#pragma unroll
                for (int c = 0; c < TC; ++c) acc[bb][r][c] = 0.0;
        double np = 0.0, ng0 = 0.0, ng1 = 0.0, ng2 = 0.0;
        if (li < NS) {
            np = phi[li];
            ng0 = dphi[li * D];
            ng1 = dphi[li * D + 1];
            if (D == 3) ng2 = dphi[li * D + D - 1];
        }
        for (int q = 0; q < nq; ++q) {
            const double h0 = ng0, h1 = ng1, h2 = ng2;
            const double s0 = np;
            if (li < NS && q + 1 < nq) {
                np = phi[(q + 1) * NS + li];
                ng0 = dphi[((q + 1) * NS + li) * D];
                ng1 = dphi[((q + 1) * NS + li) * D + 1];
                if (D == 3) ng2 = dphi[((q + 1) * NS + li) * D + D - 1];
            }
            const double s1 = K[0][0] * h0 + K[1][0] * h1 + (D == 3 ? K[2][0] * h2 : 0.0);
            const double s2 = K[0][1] * h0 + K[1][1] * h1 + (D == 3 ? K[2][1] * h2 : 0.0);
            const double s3 = D == 3 ? K[0][2] * h0 + K[1][2] * h1 + K[2][2] * h2 : 0.0;
            (void)s0; (void)s1; (void)s2; (void)s3;
            double f[NF > 0 ? NF : 1];
            for (int i = 0; i < NF; ++i) {
                double t = 0.0;
                for (int l = 0; l < NV; ++l) t += fv[i * NV + l] * psi[q * NV + l];
                f[i] = t;
            }
            (void)f;
            const double wq = W[q] * adet;
)";
        int bb = 0;
        for (const Block& B : blocks) {
            const int nk = (int)B.xs.size();
            if (nk == 0) continue;
            o << "            {   // block (" << B.a << ", " << B.b << "): " << B.edges.size() << " products, " << nk
              << " K steps\n";
            for (int e : B.edges) {
                o << "            const double c" << e << " = 0.0";
                for (int t : g.terms_of[e]) {
                    o << " + " << s->terms[t].scale;
                    if (s->terms[t].field >= 0) o << " * f[" << s->terms[t].field << "]";
                }
                o << ";\n";
            }
            for (int k = 0; k < nk; ++k) {
                o << "            if (li < NXP) sX[wv][0][sub][" << k << "][li] = " << B.xs[k] << ";\n";
                o << "            if (li < NYP) sY[wv][0][sub][" << k << "][li] = " << B.ys[k] << ";\n";
            }
            o << "            wave_sync();\n            if (act) {\n#pragma unroll\n                for (int f = 0; f < "
              << nk << "; ++f) {\n";
            o << R"(                    double xr[TR], yc[TC];
#pragma unroll
                    for (int r = 0; r < TR; ++r) xr[r] = sX[wv][0][sub][f][rt * TR + r];
#pragma unroll
                    for (int c = 0; c < TC; ++c) yc[c] = sY[wv][0][sub][f][ct * TC + c];
#pragma unroll
                    for (int r = 0; r < TR; ++r)
#pragma unroll
                        for (int c = 0; c < TC; ++c) acc[)" << bb << R"(][r][c] = __builtin_fma(xr[r], yc[c], acc[)" << bb << R"(][r][c]);
                }
            }
            wave_sync();
            }
)";
            ++bb;
        }
        o << "        }\n";
        // stores: non-empty blocks from their tiles, empty blocks as zeros
        bb = 0;
        for (const Block& B : blocks) {
            const bool empty = B.xs.empty();
            o << "        {   // store block (" << B.a << ", " << B.b << ")\n";
            o << "        const int ro = " << B.a * ns << ", co = " << B.b * ns << ";\n";
            o << R"(        if (act && valid) {
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                const int j = rt * TR + r;
                if (j < NS) {
                    double* row = out + (e * NN + ro + j) * NN + co;
#pragma unroll
                    for (int c = 0; c < TC; ++c) {
                        const int k = ct * TC + c;
                        if (k < NS) row[k] = bad ? __builtin_nan("") : )"
              << (empty ? std::string("0.0") : "acc[" + std::to_string(bb) + "][r][c]") << R"(;
                    }
                }
            }
        }
        }
)";
            if (!empty) ++bb;
        }
    } else {
    for (const Block& B : blocks) {
        const int nk = (int)B.xs.size();
        o << "        // block (" << B.a << ", " << B.b << "): " << B.edges.size() << " products, " << nk
          << " K steps\n        {\n";
        if (nk == 0) {
            o << "        const int ro = " << B.a * ns << ", co = " << B.b * ns << ";\n";
            o << R"(        if (act && valid) {
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                const int j = rt * TR + r;
                if (j < NS) {
                    double* row = out + (e * NN + ro + j) * NN + co;
#pragma unroll
                    for (int c = 0; c < TC; ++c) {
                        const int k = ct * TC + c;
                        if (k < NS) row[k] = bad ? __builtin_nan("") : 0.0;
                    }
                }
            }
        }
        }
)";
            continue;
        }
        o << "        const int ro = " << B.a * ns << ", co = " << B.b * ns << ";\n";
        o << R"(        double acc[TR][TC];
#pragma unroll
        for (int r = 0; r < TR; ++r)
#pragma unroll
            for (int c = 0; c < TC; ++c) acc[r][c] = 0.0;
        // reference value and gradient of basis function `li`, one point
        // ahead (zero for lanes past the basis, whose factors are then zero)
        double np = 0.0, ng0 = 0.0, ng1 = 0.0, ng2 = 0.0;
        if (li < NS) {
            np = phi[li];
            ng0 = dphi[li * D];
            ng1 = dphi[li * D + 1];
            if (D == 3) ng2 = dphi[li * D + D - 1];
        }
        for (int q = 0; q < nq; ++q) {
            const double h0 = ng0, h1 = ng1, h2 = ng2;
            const double s0 = np;
            if (li < NS && q + 1 < nq) {
                np = phi[(q + 1) * NS + li];
                ng0 = dphi[((q + 1) * NS + li) * D];
                ng1 = dphi[((q + 1) * NS + li) * D + 1];
                if (D == 3) ng2 = dphi[((q + 1) * NS + li) * D + D - 1];
            }
            // symbols of basis function `li` at the point
            const double s1 = K[0][0] * h0 + K[1][0] * h1 + (D == 3 ? K[2][0] * h2 : 0.0);
            const double s2 = K[0][1] * h0 + K[1][1] * h1 + (D == 3 ? K[2][1] * h2 : 0.0);
            const double s3 = D == 3 ? K[0][2] * h0 + K[1][2] * h1 + K[2][2] * h2 : 0.0;
            (void)s0; (void)s1; (void)s2; (void)s3;
            // the coefficient of every product of the block at the point
            double f[NF > 0 ? NF : 1];
            for (int i = 0; i < NF; ++i) {
                double t = 0.0;
                for (int l = 0; l < NV; ++l) t += fv[i * NV + l] * psi[q * NV + l];
                f[i] = t;
            }
            (void)f;
)";
        for (int e : B.edges) {
            o << "            const double c" << e << " = 0.0";
            for (int t : g.terms_of[e]) {
                o << " + " << s->terms[t].scale;
                if (s->terms[t].field >= 0) o << " * f[" << s->terms[t].field << "]";
            }
            o << ";\n";
        }
        o << "            const double wq = W[q] * adet;\n";
        o << "            const int b = NBUF == 2 ? (q & 1) : 0;\n";
        for (int k = 0; k < nk; ++k) {
            o << "            if (li < NXP) sX[wv][b][sub][" << k << "][li] = " << B.xs[k] << ";\n";
            o << "            if (li < NYP) sY[wv][b][sub][" << k << "][li] = " << B.ys[k] << ";\n";
        }
        o << "            wave_sync();\n            if (act) {\n#pragma unroll\n                for (int f = 0; f < "
          << nk << "; ++f) {\n";
        o << R"(                    double xr[TR], yc[TC];
#pragma unroll
                    for (int r = 0; r < TR; ++r) xr[r] = sX[wv][b][sub][f][rt * TR + r];
#pragma unroll
                    for (int c = 0; c < TC; ++c) yc[c] = sY[wv][b][sub][f][ct * TC + c];
#pragma unroll
                    for (int r = 0; r < TR; ++r)
#pragma unroll
                        for (int c = 0; c < TC; ++c) acc[r][c] = __builtin_fma(xr[r], yc[c], acc[r][c]);
                }
            }
            if (NBUF == 1) wave_sync();
        }
        if (act && valid) {
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                const int j = rt * TR + r;
                if (j < NS) {
                    double* row = out + (e * NN + ro + j) * NN + co;
#pragma unroll
                    for (int c = 0; c < TC; ++c) {
                        const int k = ct * TC + c;
                        if (k < NS) row[k] = bad ? __builtin_nan("") : acc[r][c];
                    }
                }
            }
        }
        // the next block's first point may reuse this block's last buffer
        wave_sync();
        }
)";
    }
    }
    o << R"(        if (bad && valid && li == 0 && status) atomicAdd(status, 1);
    }
}
)";
    return o.str();
}

struct Compiled {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};
std::mutex g_gen_mu;
std::map<std::pair<int, std::string>, Compiled> g_gen;   // (device, source) -> kernel
std::map<std::string, hipFunction_t> g_chosen;           // call_key -> the kernel fe_assemble_form uses
std::string g_gen_log;

// The meaningful content of a call (the spec's used terms, not its padding).
std::string call_key(const fe_form_spec_t* s, int dev, int cell, int degree, int qdeg, int nest)
{
    std::ostringstream k;
    k.precision(17);
    k << dev << ' ' << cell << ' ' << degree << ' ' << qdeg << ' ' << nest << ' ' << s->n_fields << ' ' << s->n_comp
      << ' ' << s->n_terms;
    // (an out-of-range term count keys nothing that was ever planned)
    const int nt = s->n_terms < 0 ? 0 : s->n_terms > FE_MAX_TERMS ? FE_MAX_TERMS : s->n_terms;
    for (int t = 0; t < nt; ++t) {
        const fe_term_t& x = s->terms[t];
        k << ' ' << x.test << ' ' << x.trial << ' ' << x.field << ' ' << x.scale << ' ' << x.test_comp << ' '
          << x.trial_comp;
    }
    return k.str();
}

int compile(const std::string& src, hipFunction_t* fn)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_gen_mu);
    auto key = std::make_pair(dev, src);
    auto it = g_gen.find(key);
    if (it != g_gen.end()) {
        *fn = it->second.fn;
        return FE_OK;
    }
    hipDeviceProp_t prop;
    hipError_t he = hipGetDeviceProperties(&prop, dev);
    if (he != hipSuccess) return set_hip_error(he, "generated kernel: device properties");
    std::string arch = std::string("--offload-arch=") + prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "fe_form.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return set_hip_error(hipErrorInvalidValue, "generated kernel: hiprtcCreateProgram");
    // the same code-generation flags as the library's own kernels
    const char* opts[] = {arch.c_str(), "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, 6, opts);
    size_t logn = 0;
    hiprtcGetProgramLogSize(prog, &logn);
    g_gen_log.assign(logn, '\0');
    if (logn) hiprtcGetProgramLog(prog, &g_gen_log[0]);
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return set_hip_error(hipErrorInvalidValue, "generated kernel: compilation failed");
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    std::vector<char> code(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    Compiled c;
    he = hipModuleLoadData(&c.mod, code.data());
    if (he == hipSuccess) he = hipModuleGetFunction(&c.fn, c.mod, "fe_form_kernel");
    if (he != hipSuccess) return set_hip_error(he, "generated kernel: module load");
    g_gen[key] = c;
    *fn = c.fn;
    return FE_OK;
}

int plan_form(const fe_form_spec_t* spec, int cell, int degree, int qdeg, Graph& g, int* x, int* owner,
              fe_sharing_t* out)
{
    if ((int)cell < 0 || (int)cell > 2 || degree < 1 || degree > MAX_DEGREE) return FE_EINVAL;
    int rc = validate_spec(spec, cell_dim(cell));
    if (rc) return rc;
    if (qdeg < 0) qdeg = default_form_qdeg(spec, degree);
    if (qdeg > MAX_QDEG) return FE_EINVAL;
    build_graph(spec, g);
    const double n = n_scalar(cell, degree), nq = rule_size(cell, qdeg);
    double th = 0.0, th_exp = 0.0;
    for (int e = 0; e < g.ne; ++e) owner[e] = -1;
    for (int i = 0; i < g.nv; ++i) x[i] = 0;
    for (int b = 0; b < g.nblocks(); ++b) {
        std::vector<int> vs, es;
        for (int i = 0; i < g.nv; ++i)
            if (g.blk[i] == b) vs.push_back(i);
        for (int e = 0; e < g.ne; ++e)
            if (g.blk[g.et[e]] == b) es.push_back(e);
        if (es.empty()) continue;
        double thb = 0.0;
        solve_ilp(g, vs, es, n, nq, x, owner, &thb);
        // steps 2 and 4 keep only flop-decreasing factorisations: when grouping
        // does not pay for its temporaries (e.g. a perfect matching, as for the
        // Laplacian) the block's expanded nest (Strategy 1 alone) is kept
        const double thb_exp = theta_expanded((int)es.size(), n, nq);
        if (!(thb < thb_exp)) {
            for (int i : vs) x[i] = 0;
            for (int e : es) owner[e] = -1;
            thb = thb_exp;
        }
        th += thb;
        th_exp += thb_exp;
    }
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->n_vertices = g.nv;
        out->n_comp = g.nc;
        for (int i = 0; i < g.nv; ++i) {
            out->vertex_block[i] = g.blk[i];
            out->vertex_side[i] = g.side[i];
            out->vertex_symbol[i] = g.sym[i];
            out->factorized[i] = x[i];
        }
        out->n_edges = g.ne;
        for (int e = 0; e < g.ne; ++e) {
            out->edge_test[e] = g.et[e];
            out->edge_trial[e] = g.er[e];
            out->edge_owner[e] = owner[e];
        }
        out->theta_expanded = th_exp;
        out->theta_se = th;
    }
    return FE_OK;
}

}  // namespace

void release_generated()
{
    std::lock_guard<std::mutex> lk(g_gen_mu);
    g_chosen.clear();
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto& kv : g_gen) {
        if (!kv.second.mod) continue;
        // a module belongs to the device it was loaded on
        if (hipSetDevice(kv.first.first) == hipSuccess) (void)hipModuleUnload(kv.second.mod);
    }
    if (have_cur) (void)hipSetDevice(cur);
    g_gen.clear();
}

}  // namespace fe

using namespace fe;

extern "C" int fe_sharing_plan(const fe_form_spec_t* spec, fe_cell_t cell, int degree, int qdeg, fe_sharing_t* plan)
{
    if (!plan) return FE_EINVAL;
    Graph g;
    int x[MAXV] = {0}, owner[FE_MAX_TERMS] = {0};
    return plan_form(spec, cell, degree, qdeg, g, x, owner, plan);
}

extern "C" int fe_form_source(const fe_form_spec_t* spec, fe_cell_t cell, int degree, int expanded, char* buf,
                              size_t* len)
{
    if (!len) return FE_EINVAL;
    Graph g;
    int x[MAXV] = {0}, owner[FE_MAX_TERMS] = {0};
    int rc = plan_form(spec, cell, degree, -1, g, x, owner, nullptr);
    if (rc) return rc;
    const std::string src = generate(spec, g, x, owner, cell, degree, expanded != 0);
    if (buf && *len > 0) {
        const size_t m = std::min(*len - 1, src.size());
        std::memcpy(buf, src.data(), m);
        buf[m] = '\0';
    }
    *len = src.size() + 1;
    return FE_OK;
}

extern "C" int fe_assemble_form(const fe_form_spec_t* spec, fe_cell_t cell, int degree, int64_t n_elems,
                                const double* coords, const double* fields, double* out_A, const fe_options_t* opt)
{
    fe_options_t o;
    if (opt) o = *opt;
    else fe_options_init(&o);
    if (n_elems < 0) return FE_EINVAL;
    if (o.shape.kernel != 0 && o.shape.kernel != 5) return FE_EINVAL;
    if (o.coord_degree < 0 || o.coord_degree > 2) return FE_EINVAL;
    if (o.coord_degree == 2) return FE_ENOTSUP;   // affine cells only
    Graph g;
    int x[MAXV] = {0}, owner[FE_MAX_TERMS] = {0};
    const int qdeg = o.qdeg < 0 ? -1 : o.qdeg;
    if (!spec) return FE_EINVAL;
    // the kernel chosen for this (device, form, cell, degree, rule, nest) is
    // kept (only after the form was planned and validated), so a repeated
    // call skips the planning, the generation and the source lookup
    int dev = 0;
    (void)hipGetDevice(&dev);
    const std::string key = call_key(spec, dev, cell, degree, qdeg, o.shape.kernel);
    hipFunction_t fn = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_gen_mu);
        auto it = g_chosen.find(key);
        if (it != g_chosen.end()) fn = it->second;
    }
    int rc = FE_OK;
    if (!fn) {
        rc = plan_form(spec, cell, degree, qdeg, g, x, owner, nullptr);
        if (rc) return rc;
        if (n_scalar(cell, degree) > 64) return FE_ENOTSUP;
    }
    if (n_elems == 0) return FE_OK;
    if (!coords || !out_A || (spec->n_fields > 0 && !fields)) return FE_EINVAL;
    const RefTables* t = nullptr;
    rc = get_tables(cell, degree, qdeg < 0 ? default_form_qdeg(spec, degree) : qdeg, (hipStream_t)o.stream, &t);
    if (rc) return rc;
    if (!fn) {
        rc = compile(generate(spec, g, x, owner, cell, degree, o.shape.kernel == 5), &fn);
        if (rc) return rc;
        if (spec->n_comp > 1) {
            // the fused vector nest keeps every block's tile in registers; where
            // that leaves less than two wavefronts per SIMD (measured on MI355X:
            // slower than the per-block nest) the per-block nest is used
            int per_cu = 0;
            const hipError_t oe = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
            if (oe != hipSuccess) return set_hip_error(oe, "generated kernel occupancy");
            if (per_cu < 2) {
                rc = compile(generate(spec, g, x, owner, cell, degree, o.shape.kernel == 5, false), &fn);
                if (rc) return rc;
            }
        }
        std::lock_guard<std::mutex> lk(g_gen_mu);
        g_chosen[key] = fn;
    }
    const double* W = t->dW;
    const double* phi = t->dphi;
    const double* dphi = t->ddphi;
    const double* psi = t->dpsi;
    int* status = o.d_status;
    long long E = n_elems;
    int nq = t->nq;
    void* args[] = {(void*)&coords, (void*)&fields, (void*)&out_A, (void*)&status, (void*)&W, (void*)&phi,
                    (void*)&dphi,   (void*)&psi,    (void*)&E,     (void*)&nq};
    const int64_t blocks = (n_elems + 3) / 4;
    const int grid = (int)std::min<int64_t>(blocks, (int64_t)device_cus() * 8);
    hipError_t e = hipModuleLaunchKernel(fn, grid, 1, 1, 256, 1, 1, 0, (hipStream_t)o.stream, args, nullptr);
    return e == hipSuccess ? FE_OK : set_hip_error(e, "generated kernel launch");
}
