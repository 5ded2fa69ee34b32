// Automatic sharing elimination (Sec. 3.2, Algorithm 1) for generic scalar
// bilinear forms, and a quadrature kernel generated from its result.
//
// A form is a sum of terms scale * c(x) * s_test(phi_j) * s_trial(phi_k),
// s being the basis function or one of its physical derivatives (the
// multilinear symbols) and c a constant or a P1 field (a coefficient, hoisted
// out of the (j, k) loops by generalised code motion, Strategy 1).
//   * Terms with the same pair of symbols are merged into one product whose
//     coefficient is their sum (the partition of step 1).
//   * The sharing graph (step 3) has one vertex per distinct symbol of each
//     side and one edge per product.
//   * The ILP of step 5 -- minimise the number of factorised symbols such
//     that every product is grouped under exactly one factorised endpoint --
//     asks for a minimum vertex cover with an orientation of the edges; the
//     graphs have at most 8 vertices, so it is solved exactly by enumerating
//     the vertex subsets (ties: the lower operation count, then the first
//     subset in enumeration order).
//   * Step 6 emits the loop nest: per point, each factorised test symbol u
//     gets a hoisted temporary h_u(k) = sum over its products of c s_trial(k)
//     (Strategy 2), each factorised trial symbol v a temporary h_v(j); the
//     innermost (j, k) body has one multiply-add per factorised symbol.
// The kernel is written out as HIP source for the form, the cell and the
// degree, compiled at run time with hipRTC for the current device, and
// cached.  fe_options_t.shape.kernel = 5 selects the expanded loop nest
// instead (every product in the innermost body), for comparison.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

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

constexpr int MAXV = 8;

struct Graph {
    int nv = 0, ne = 0;
    int side[MAXV], sym[MAXV];
    int et[FE_MAX_TERMS], er[FE_MAX_TERMS];      // vertex indices of each product
    std::vector<int> terms_of[FE_MAX_TERMS];      // terms merged into product e
};

int vertex_of(Graph& g, int side, int sym)
{
    for (int i = 0; i < g.nv; ++i)
        if (g.side[i] == side && g.sym[i] == sym) return i;
    g.side[g.nv] = side;
    g.sym[g.nv] = sym;
    return g.nv++;
}

int validate_spec(const fe_form_spec_t* s, int d)
{
    if (!s || s->n_terms < 1 || s->n_terms > FE_MAX_TERMS || s->n_fields < 0 || s->n_fields > FE_MAX_FIELDS)
        return FE_EINVAL;
    for (int t = 0; t < s->n_terms; ++t) {
        const fe_term_t& x = s->terms[t];
        if (x.test < 0 || x.test > d || x.trial < 0 || x.trial > d) return FE_EINVAL;
        if (x.field < -1 || x.field >= s->n_fields || !std::isfinite(x.scale)) return FE_EINVAL;
    }
    return FE_OK;
}

void build_graph(const fe_form_spec_t* s, Graph& g)
{
    // test vertices first, then trial vertices (symbol order within a side)
    for (int side = 0; side < 2; ++side)
        for (int sym = 0; sym < 4; ++sym)
            for (int t = 0; t < s->n_terms; ++t)
                if ((side == 0 ? s->terms[t].test : s->terms[t].trial) == sym) {
                    vertex_of(g, side, sym);
                    break;
                }
    for (int t = 0; t < s->n_terms; ++t) {
        const int u = vertex_of(g, 0, s->terms[t].test), v = vertex_of(g, 1, s->terms[t].trial);
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

// Operation counts per element (multiply and add each count one).
//   expanded: per point w c_e s_test(j) for every product and j, then one
//             multiply-add per product and (j, k);
//   factorised: per point the temporaries (a multiply-add per grouped
//             product and index), w s(j) per factorised symbol and j, then one
//             multiply-add per factorised symbol and (j, k).
double theta_expanded(const Graph& g, double n, double nq) { return nq * (2.0 * g.ne * n * n + 2.0 * g.ne * n); }

double theta_factorised(const Graph& g, const int* x, const int* owner, double n, double nq)
{
    double inner = 0.0, hoist = 0.0;
    for (int i = 0; i < g.nv; ++i)
        if (x[i]) {
            int deg = 0;
            for (int e = 0; e < g.ne; ++e) deg += owner[e] == i;
            inner += 2.0 * n * n;
            hoist += 2.0 * deg * n + n;
        }
    return nq * (inner + hoist);
}

// Exact solution of the ILP of Algorithm 1, step 5.
void solve_ilp(const Graph& g, double n, double nq, int* best_x, int* best_owner, double* best_theta)
{
    int best_count = MAXV + 1;
    *best_theta = 0.0;
    for (unsigned m = 1; m < (1u << g.nv); ++m) {
        int x[MAXV], owner[FE_MAX_TERMS], count = 0;
        for (int i = 0; i < g.nv; ++i) count += x[i] = (m >> i) & 1;
        bool cover = true;
        for (int e = 0; e < g.ne && cover; ++e) {
            // y: a product goes to its factorised test symbol when both ends are
            // factorised (either choice gives the same count)
            if (x[g.et[e]]) owner[e] = g.et[e];
            else if (x[g.er[e]]) owner[e] = g.er[e];
            else cover = false;
        }
        if (!cover || count > best_count) continue;
        const double th = theta_factorised(g, x, owner, n, nq);
        if (count < best_count || th < *best_theta) {
            best_count = count;
            *best_theta = th;
            for (int i = 0; i < g.nv; ++i) best_x[i] = x[i];
            for (int e = 0; e < g.ne; ++e) best_owner[e] = owner[e];
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

// HIP source of the quadrature kernel of one form (one wavefront per
// element, lane j < NS owns row j of the element matrix).
std::string generate(const fe_form_spec_t* s, const Graph& g, const int* x, const int* owner, int cell, int p,
                     bool expanded)
{
    bool any = false;
    for (int i = 0; i < g.nv; ++i) any |= x[i] != 0;
    expanded = expanded || !any;
    const int d = cell_dim(cell), nv = cell_nv(cell), ns = n_scalar(cell, p);
    std::ostringstream o;
    o.precision(17);
    o << "// generated: scalar bilinear form, cell " << cell << ", degree " << p
      << (expanded ? ", expanded products\n" : ", sharing-eliminated\n");
    o << "#define NS " << ns << "\n#define D " << d << "\n#define NV " << nv << "\n#define NF " << s->n_fields
      << "\n";
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
    __shared__ double sS[4][4][NS];    // symbols of the current point, per wavefront
)";
    int nht = 0;   // factorised test symbols: temporaries over k in LDS
    for (int i = 0; i < g.nv; ++i) nht += (!expanded && x[i] && g.side[i] == 0);
    if (nht) o << "    __shared__ double sH[4][" << nht << "][NS];\n";
    o << R"(    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (long long e = (long long)blockIdx.x * 4 + wv; e < E; e += (long long)gridDim.x * 4) {
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
        double acc[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] = 0.0;
        for (int q = 0; q < nq; ++q) {
            // symbols of basis function `lane` at the point
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            if (lane < NS) {
                s0 = phi[q * NS + lane];
                const double* gh = dphi + (q * NS + lane) * D;
                s1 = K[0][0] * gh[0] + K[1][0] * gh[1] + (D == 3 ? K[2][0] * gh[D - 1] : 0.0);
                s2 = K[0][1] * gh[0] + K[1][1] * gh[1] + (D == 3 ? K[2][1] * gh[D - 1] : 0.0);
                s3 = D == 3 ? K[0][2] * gh[0] + K[1][2] * gh[1] + K[2][2] * gh[D - 1] : 0.0;
                sS[wv][0][lane] = s0;
                sS[wv][1][lane] = s1;
                sS[wv][2][lane] = s2;
                sS[wv][3][lane] = s3;
            }
            // the coefficient of every product at the point
            double f[NF > 0 ? NF : 1];
            for (int i = 0; i < NF; ++i) {
                double t = 0.0;
                for (int l = 0; l < NV; ++l) t += fields[(e * NF + i) * NV + l] * psi[q * NV + l];
                f[i] = t;
            }
            (void)f;
)";
    // coefficient of each product: sum of its terms
    for (int e = 0; e < g.ne; ++e) {
        o << "            const double c" << e << " = 0.0";
        for (int t : g.terms_of[e]) {
            o << " + " << s->terms[t].scale;
            if (s->terms[t].field >= 0) o << " * f[" << s->terms[t].field << "]";
        }
        o << ";\n";
    }
    o << "            const double wq = W[q] * adet;\n";
    if (expanded) {
        o << "            wave_sync();\n            if (lane < NS) {\n";
        for (int e = 0; e < g.ne; ++e)
            o << "                const double a" << e << " = wq * c" << e << " * " << SYMNAME[g.sym[g.et[e]]] << ";\n";
        o << "#pragma unroll\n                for (int k = 0; k < NS; ++k) {\n                    double t = acc[k];\n";
        for (int e = 0; e < g.ne; ++e) o << "                    t += a" << e << " * sS[wv][" << g.sym[g.er[e]] << "][k];\n";
        o << "                    acc[k] = t;\n                }\n            }\n";
    } else {
        // temporaries of factorised test symbols: h_u(k) over the products grouped under u
        int h = 0;
        for (int i = 0; i < g.nv; ++i) {
            if (!(x[i] && g.side[i] == 0)) continue;
            o << "            if (lane < NS) sH[wv][" << h << "][lane] = 0.0";
            for (int e = 0; e < g.ne; ++e)
                if (owner[e] == i) o << " + c" << e << " * " << SYMNAME[g.sym[g.er[e]]];
            o << ";\n";
            ++h;
        }
        o << "            wave_sync();\n            if (lane < NS) {\n";
        // per-row factors: w s_u(j) for factorised test symbols, w h_v(j) for trial ones
        h = 0;
        for (int i = 0; i < g.nv; ++i) {
            if (!x[i]) continue;
            if (g.side[i] == 0) {
                o << "                const double a" << i << " = wq * " << SYMNAME[g.sym[i]] << ";\n";
            } else {
                o << "                const double a" << i << " = wq * (0.0";
                for (int e = 0; e < g.ne; ++e)
                    if (owner[e] == i) o << " + c" << e << " * " << SYMNAME[g.sym[g.et[e]]];
                o << ");\n";
            }
        }
        o << "#pragma unroll\n                for (int k = 0; k < NS; ++k) {\n                    double t = acc[k];\n";
        h = 0;
        for (int i = 0; i < g.nv; ++i) {
            if (!x[i]) continue;
            if (g.side[i] == 0) o << "                    t += a" << i << " * sH[wv][" << h++ << "][k];\n";
            else o << "                    t += a" << i << " * sS[wv][" << g.sym[i] << "][k];\n";
        }
        o << "                    acc[k] = t;\n                }\n            }\n";
    }
    o << R"(            wave_sync();
        }
        if (lane < NS) {
            double* row = out + (e * NS + lane) * NS;
#pragma unroll
            for (int k = 0; k < NS; ++k) row[k] = bad ? __builtin_nan("") : acc[k];
        }
        if (bad && lane == 0 && status) atomicAdd(status, 1);
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
std::string g_gen_log;

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
    double th = 0.0;
    solve_ilp(g, n, nq, x, owner, &th);
    // steps 2 and 4 keep only flop-decreasing factorisations: when grouping
    // does not pay for its temporaries (e.g. a perfect matching, as for the
    // Laplacian) the expanded nest (Strategy 1 alone) is kept
    const double th_exp = theta_expanded(g, n, nq);
    if (!(th < th_exp)) {
        for (int i = 0; i < g.nv; ++i) x[i] = 0;
        for (int e = 0; e < g.ne; ++e) owner[e] = -1;
        th = th_exp;
    }
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->n_vertices = g.nv;
        for (int i = 0; i < g.nv; ++i) {
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
    Graph g;
    int x[MAXV] = {0}, owner[FE_MAX_TERMS] = {0};
    const int qdeg = o.qdeg < 0 ? -1 : o.qdeg;
    int rc = plan_form(spec, cell, degree, qdeg, g, x, owner, nullptr);
    if (rc) return rc;
    if (n_scalar(cell, degree) > 64) return FE_ENOTSUP;
    if (n_elems == 0) return FE_OK;
    if (!coords || !out_A || (spec->n_fields > 0 && !fields)) return FE_EINVAL;
    const RefTables* t = nullptr;
    rc = get_tables(cell, degree, qdeg < 0 ? default_form_qdeg(spec, degree) : qdeg, (hipStream_t)o.stream, &t);
    if (rc) return rc;
    hipFunction_t fn = nullptr;
    rc = compile(generate(spec, g, x, owner, cell, degree, o.shape.kernel == 5), &fn);
    if (rc) return rc;
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
