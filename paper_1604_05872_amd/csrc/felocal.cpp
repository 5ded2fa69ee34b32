// C ABI of the local-assembly library (include/felocal.h): argument
// validation, reference-table cache, variant selection and launches.
#include "felocal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gram64.hpp"
#include "internal.hpp"
#include "preeval.hpp"
#include "quad.hpp"
#include "split.hpp"

namespace fe {

namespace {

std::mutex g_mu;
thread_local std::string g_hip_msg = "no HIP error recorded";
std::map<std::tuple<int, int, int, int>, RefTables*> g_tables;   // (device, cell, p, qdeg)
std::map<std::tuple<int, int, int, int, int, int>, CoefTables*> g_coef;   // (device, form, cell, p, qdeg, nf)

int current_device()
{
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

}  // namespace

int set_hip_error(hipError_t e, const char* where)
{
    g_hip_msg = std::string(where) + ": " + hipGetErrorString(e);
    return FE_EHIP;
}

int device_cus()
{
    static int cus[64] = {0};
    int d = current_device();
    if (d < 0 || d >= 64) return 256;
    if (cus[d] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || v <= 0) v = 256;
        cus[d] = v;
    }
    return cus[d];
}

// LDS capacity of one compute unit: the default memory threshold T_H
// (160 KiB on gfx950 when the runtime does not report it).
size_t device_lds_per_cu()
{
    static size_t lds[64] = {0};
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return 160 * 1024;
    if (lds[d] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, d) != hipSuccess || v <= 0)
            v = 160 * 1024;
        lds[d] = (size_t)v;
    }
    return lds[d];
}

// L2 capacity of the current device (one XCD's L2 on MI355X: 4 MiB when the
// runtime does not report it).
size_t device_l2_bytes()
{
    static size_t l2[64] = {0};
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return 4u << 20;
    if (l2[d] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeL2CacheSize, d) != hipSuccess || v <= 0) v = 4 << 20;
        l2[d] = (size_t)v;
    }
    return l2[d];
}

// Builds (once) the rule, the tabulated basis, the P1 coefficient basis and
// the pre-evaluated tensors of (cell, p, qdeg) on the current device.
int get_tables(int cell, int p, int qdeg, hipStream_t s, const RefTables** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(current_device(), cell, p, qdeg);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) {
        *out = it->second;
        return FE_OK;
    }
    RefTables* t = new RefTables();
    t->cell = cell;
    t->p = p;
    t->qdeg = qdeg;
    t->d = cell_dim(cell);
    t->nv = cell_nv(cell);
    t->nb = n_scalar(cell, p);
    t->nq = build_rule(cell, qdeg, t->X, t->W);
    if (t->nq <= 0) {
        delete t;
        return FE_EINVAL;
    }
    const int nq = t->nq, nb = t->nb, d = t->d;
    const int nt = n_tables(HELMHOLTZ, cell);
    hipError_t e = hipSuccess;
    auto M = [&](double** p_, size_t n) {
        if (e == hipSuccess) e = hipMalloc((void**)p_, n * sizeof(double));
    };
    M(&t->dX, (size_t)nq * d);
    M(&t->dW, nq);
    M(&t->dphi, (size_t)nq * nb);
    M(&t->ddphi, (size_t)nq * nb * d);
    M(&t->dpsi, (size_t)nq * t->nv);
    M(&t->dR, (size_t)nt * nb * nb);
    M(&t->ddpsi, (size_t)nq * t->nv * d);
    if (e == hipSuccess) e = hipMemcpyAsync(t->dX, t->X.data(), sizeof(double) * nq * d, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(t->dW, t->W.data(), sizeof(double) * nq, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_tabulate(cell, p, nq, t->dX, t->dphi, t->ddphi, s);
    if (e == hipSuccess) e = launch_tabulate(cell, 1, nq, t->dX, t->dpsi, t->ddpsi, s);
    if (e == hipSuccess) e = launch_preeval_tables(nq, nb, d, t->dW, t->dphi, t->ddphi, t->dR, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        for (double* p_ : {t->dX, t->dW, t->dphi, t->ddphi, t->dpsi, t->ddpsi, t->dR})
            if (p_) (void)hipFree(p_);
        delete t;
        return set_hip_error(e, "building reference tables");
    }
    g_tables[key] = t;
    *out = t;
    return FE_OK;
}

// The cached reference tables of (cell, p, qdeg) on the current device,
// without building them: FE_EINVAL when no earlier call built them.
int find_tables(int cell, int p, int qdeg, const RefTables** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tables.find(std::make_tuple(current_device(), cell, p, qdeg));
    if (it == g_tables.end()) return FE_EINVAL;
    *out = it->second;
    return FE_OK;
}

// Builds (once) the multisets and the coefficient-expanded reference tensors
// of (form, cell, p, qdeg, nf) on the current device.
int get_coef_tables(int form, int cell, int p, int qdeg, int nf, hipStream_t s, const CoefTables** out)
{
    const RefTables* rt = nullptr;
    int rc = get_tables(cell, p, qdeg, s, &rt);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(current_device(), form, cell, p, qdeg, nf);
    auto it = g_coef.find(key);
    if (it != g_coef.end()) {
        *out = it->second;
        return FE_OK;
    }
    const int nb = rt->nb;
    if (form == ELASTICITY && nf == 0) {
        // T[(l, a, b)][j][k] = sum_q W_q psi_l dphi_{j,a} dphi_{k,b}
        CoefTables* t = new CoefTables();
        t->iota = rt->nv;
        t->nt = rt->nv * rt->d * rt->d;
        hipError_t e = hipMalloc((void**)&t->dR, elast_table_doubles(cell, nb) * sizeof(double));
        if (e == hipSuccess) e = launch_elast_tables(rt->nq, nb, rt->d, rt->nv, rt->dW, rt->dpsi, rt->ddphi, t->dR, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            if (t->dR) (void)hipFree(t->dR);
            delete t;
            return set_hip_error(e, "building elasticity tables");
        }
        g_coef[key] = t;
        *out = t;
        return FE_OK;
    }
    // sorted multisets l_1 <= ... <= l_nf, lexicographic
    std::vector<int> combos;
    std::vector<int> cur(nf, 0);
    for (;;) {
        combos.insert(combos.end(), cur.begin(), cur.end());
        int i = nf - 1;
        while (i >= 0 && cur[i] == nb - 1) --i;
        if (i < 0) break;
        ++cur[i];
        for (int k = i + 1; k < nf; ++k) cur[k] = cur[i];
    }
    CoefTables* t = new CoefTables();
    t->iota = (int)(combos.size() / nf);
    // elasticity: T[((l * iota + S) * d + a) * d + b] for the P1 Lame basis
    // psi_l and the multisets S; the scalar forms: R[(r, S)]
    const int nr = form == ELASTICITY ? rt->nv * rt->d * rt->d : n_tables(form, cell);
    t->nt = nr * t->iota;
    hipError_t e = hipMalloc((void**)&t->dCombos, combos.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&t->dR, (size_t)t->nt * nb * nb * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpyAsync(t->dCombos, combos.data(), combos.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && form == ELASTICITY)
        e = launch_elast_coef_tables(rt->nq, nb, rt->d, rt->nv, nf, t->iota, rt->dW, rt->dphi, rt->dpsi, rt->ddphi,
                                     t->dCombos, t->dR, s);
    else if (e == hipSuccess)
        e = launch_coef_tables(rt->nq, nb, rt->d, nf, t->iota, nr, rt->dW, rt->dphi, rt->ddphi, t->dCombos, t->dR, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        if (t->dCombos) (void)hipFree(t->dCombos);
        if (t->dR) (void)hipFree(t->dR);
        delete t;
        return set_hip_error(e, "building coefficient tables");
    }
    g_coef[key] = t;
    *out = t;
    return FE_OK;
}

Config default_preeval_tiled_config(int nn, int mm)
{
    // choose (block, epi) with the least idle slots, one pass when possible
    Config best;
    double best_waste = 1e9;
    for (int block : {256, 320, 384, 448, 512}) {
        for (int epi = 1; epi <= 64; ++epi) {
            const int slots = epi * nn;
            const int m = (slots + block - 1) / block;
            if (m > mm && epi > 1) break;
            const int passes = (m + mm - 1) / mm;
            const double waste = (double)(passes * mm * block - slots) / (passes * mm * block) * 0.25 +
                                 (double)(m * block - slots) / (m * block) + (epi * nn < 512 ? 0.5 : 0.0) +
                                 0.01 * passes;
            if (waste < best_waste - 1e-9) {
                best_waste = waste;
                best.block = block;
                best.epi = epi;
            }
        }
    }
    best.chunk = best.epi * std::max(1, 256 / best.epi);
    return best;
}

Config default_preeval_config(int form, int nn)
{
    // Streaming kernel when a step fits in registers: the fewest idle slots
    // at 4 (else 8, mass 16) slots per thread, at least 1024 stores a step.
    Config best;
    double best_score = 1e9;
    for (int block : {256, 320, 384, 448, 512}) {
        for (int mm : {4, 8, 16}) {
            if (mm == 16 && form != MASS) continue;
            const int epi = std::min(block, mm * block / nn);
            if (epi < 1) continue;
            const int slots = epi * nn;
            if (preeval_stream_mm(form, slots, block) != mm) continue;
            const double score = 1.0 - (double)slots / (mm * block) + (slots < 1024 ? 0.3 : 0.0) +
                                 (mm > 4 ? 0.05 * (mm / 8) : 0.0);
            if (score < best_score - 1e-9) {
                best_score = score;
                best.block = block;
                best.epi = epi;
                best.chunk = 0;
                best.variant = 1;
            }
        }
    }
    if (best_score < 1e9) return best;
    return default_preeval_tiled_config(nn, preeval_mm(form));
}

Config default_quad_config(int form, int cell, int p, int nq, int pointgeo)
{
    Config c;
    c.block = QUAD_BLOCK;
    const int ns = n_scalar(cell, p);
    const int kb = quad_kb(cell, p);
    const int units = ns * ((ns + kb - 1) / kb);
    c.eb = std::max(1, QUAD_BLOCK / units);
    const int D = cell_dim(cell);
    const int ppt = ns * D + (form == HYPERELASTIC ? ns * D + 9 : 0) + 3 + (pointgeo ? 10 : 0);
    const size_t fixed = (size_t)c.eb * 12 * 8;
    const size_t per_q = ((size_t)ns + (size_t)c.eb * ppt) * 8;
    int qc = (int)((QUAD_LDS_BUDGET - fixed) / per_q);
    c.qc = std::max(1, std::min(nq, qc));
    return c;
}

size_t quad_lds_bytes(int form, int cell, int ns, int eb, int qc, int pointgeo)
{
    const int D = cell_dim(cell);
    const int ppt = ns * D + (form == HYPERELASTIC ? ns * D + 9 : 0) + 3 + (pointgeo ? 10 : 0);
    return ((size_t)eb * 12 + (size_t)qc * ns + (size_t)eb * qc * ppt) * 8;
}

}  // namespace fe

using namespace fe;

extern "C" {

void fe_options_init(fe_options_t* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->qdeg = -1;
    opt->precision = FE_FP64;
    opt->mode = FE_MODE_AUTO;
    opt->stream = nullptr;
    opt->mu = 1.0;
    opt->lambda = 10.0;
    opt->d_status = nullptr;
    opt->th_bytes = 0;
    opt->validate = 0;
}

const char* fe_version(void) { return "felocal 0.1 (gfx950)"; }

const char* fe_strerror(int code)
{
    switch (code) {
    case FE_OK: return "success";
    case FE_EINVAL: return "invalid argument";
    case FE_ENOTSUP: return "unsupported combination of form, cell, degree, precision or size";
    case FE_EHIP: return g_hip_msg.c_str();
    case FE_ENONAFFINE: return "a prism element is not affine";
    case FE_ENOMEM: return "out of memory or size limit exceeded";
    default: return "unknown error code";
    }
}

int fe_local_dims(fe_form_t form, fe_cell_t cell, int degree, int* n_rows_out, int* n_coeff)
{
    if ((int)form < 0 || (int)form > 3 || (int)cell < 0 || (int)cell > 2 || degree < 1 || degree > MAX_DEGREE)
        return FE_EINVAL;
    if (n_rows_out) *n_rows_out = n_rows(form, cell, degree);
    if (n_coeff) {
        const int nv = cell_nv(cell);
        *n_coeff = form == ELASTICITY ? 2 * nv : form == HYPERELASTIC ? cell_dim(cell) * n_scalar(cell, degree) : 0;
    }
    return FE_OK;
}

int fe_tabulate(fe_cell_t cell, int degree, int qdeg, double* points, double* weights, double* phi, double* dphi,
                int* info)
{
    if (!info || (int)cell < 0 || (int)cell > 2 || degree < 1 || degree > MAX_DEGREE || qdeg < 0 || qdeg > MAX_QDEG)
        return FE_EINVAL;
    std::vector<double> X, W;
    const int nq = build_rule(cell, qdeg, X, W);
    if (nq <= 0) return FE_EINVAL;
    const int nb = n_scalar(cell, degree), d = cell_dim(cell);
    info[0] = nq;
    info[1] = nb;
    info[2] = d;
    if (!points) return FE_OK;
    if (!weights) return FE_EINVAL;
    std::memcpy(points, X.data(), sizeof(double) * nq * d);
    std::memcpy(weights, W.data(), sizeof(double) * nq);
    if (!phi && !dphi) return FE_OK;   // rule only: host-side, no device needed
    if (!phi || !dphi) return FE_EINVAL;
    const RefTables* t = nullptr;
    int rc = get_tables(cell, degree, qdeg, nullptr, &t);
    if (rc) return rc;
    hipError_t e = hipMemcpy(phi, t->dphi, sizeof(double) * nq * nb, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(dphi, t->ddphi, sizeof(double) * nq * nb * d, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_hip_error(e, "fe_tabulate copy");
    return FE_OK;
}

int fe_geometry(fe_cell_t cell, int64_t n_elems, const double* coords, double* out_detJ, double* out_Kinv,
                void* stream)
{
    if ((int)cell < 0 || (int)cell > 2 || n_elems < 0) return FE_EINVAL;
    if (n_elems == 0) return FE_OK;
    if (!coords || !out_detJ || !out_Kinv) return FE_EINVAL;
    hipError_t e = launch_geometry(cell, n_elems, coords, out_detJ, out_Kinv, (hipStream_t)stream);
    if (e != hipSuccess) return set_hip_error(e, "fe_geometry launch");
    return FE_OK;
}

}  // extern "C"

// host-side affinity check of prisms (opt->validate)
static int validate_prisms(int64_t E, const double* d_coords, hipStream_t s)
{
    std::vector<double> h((size_t)E * 18);
    hipError_t e = hipMemcpyAsync(h.data(), d_coords, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_hip_error(e, "validate copy");
    for (int64_t i = 0; i < E; ++i) {
        const double* v = &h[(size_t)i * 18];
        double vmax = 0.0;
        for (int k = 0; k < 18; ++k) vmax = std::fmax(vmax, std::fabs(v[k]));
        const double tol = 1e-12 * (vmax > 0 ? vmax : 1.0);
        for (int t = 1; t < 3; ++t)
            for (int r = 0; r < 3; ++r)
                if (!(std::fabs((v[(t + 3) * 3 + r] - v[t * 3 + r]) - (v[9 + r] - v[r])) <= tol))
                    return FE_ENONAFFINE;
    }
    return FE_OK;
}

extern "C" {

// Resolves the variant of one call: mode (Algorithm 3) and kernel family.
// *mass_pre is set for a Helmholtz plan that pre-evaluates only the mass
// monomial (the quadrature kernel then adds |det J| Mhat).
int fe_resolve_variant(int form, int cell, int degree, int qdeg, const fe_options_t* o, int* mode_out,
                       int* mass_pre)
{
    *mass_pre = 0;   // bit 0: mass monomial pre-evaluated; bit 1: gradient monomial pre-evaluated
    if (o->precision != FE_FP64) {
        if (!is_vector_form(form)) return FE_ENOTSUP;
        if (o->mode == FE_MODE_PREEVAL) return FE_ENOTSUP;
        const int n = n_rows(form, cell, degree);
        if (n > 32 || rule_size(cell, qdeg) > 32) return FE_ENOTSUP;
        *mode_out = FE_MODE_QUADRATURE;
        return FE_OK;
    }
    if (o->mode == FE_MODE_PREEVAL) {
        if (form == HYPERELASTIC) return FE_ENOTSUP;   // a non-polynomial coefficient
        *mode_out = FE_MODE_PREEVAL;
        return FE_OK;
    }
    if (o->mode == FE_MODE_QUADRATURE) {
        *mode_out = FE_MODE_QUADRATURE;
        return FE_OK;
    }
    fe_plan_t plan;
    int rc = fe_plan((fe_form_t)form, (fe_cell_t)cell, degree, o->nf, qdeg, o->th_bytes, &plan);
    if (rc) return rc;
    *mode_out = plan.mode;
    // fe_autotune measured the other mode faster for this variant: run it
    // (the whole form in one mode)
    int tm = 0;
    if (tuned_mode(form, cell, degree, qdeg, FE_FP64, o->nf, &tm) && tm != plan.mode) {
        *mode_out = tm;
        return FE_OK;
    }
    // a mixed Helmholtz plan: with nf = 0 the quadrature kernel adds the
    // pre-evaluated monomial's tables; with coefficient functions the
    // coefficient pre-evaluation kernel adds that monomial afterwards
    if (form == HELMHOLTZ && plan.mode == FE_MODE_QUADRATURE)
        *mass_pre = (plan.preevaluated[1] ? 1 : 0) | (plan.preevaluated[0] ? 2 : 0);
    // the hyperelastic trace monomial mu |det J| w g_j . g_k with nf > 0
    // pre-multiplying functions w: pre-evaluated by the coefficient kernel,
    // added to the diagonal blocks after the quadrature kernel (with nf = 0
    // the matrix-core kernels pre-evaluate it themselves)
    if (form == HYPERELASTIC && o->nf > 0 && plan.preevaluated[1]) *mass_pre = 2;
    return FE_OK;
}

}  // extern "C"

namespace fe {

// FE_LOG=1 in the environment (read at every call): one line on stderr per
// dispatched call (the plan's mode, the precision and the launch
// configuration).
bool log_enabled()
{
    const char* v = std::getenv("FE_LOG");
    return v && v[0] == '1';
}

void log_call(const Call& c, const Config& cfg)
{
    static const char* forms[] = {"mass", "helmholtz", "elasticity", "hyperelastic"};
    static const char* cells[] = {"triangle", "tetrahedron", "prism"};
    static const char* precs[] = {"fp64", "fp32", "bf16x3"};
    std::fprintf(stderr,
                 "felocal: %s %s P%d E=%lld qdeg=%d nf=%d mode=%s precision=%s pointgeo=%d variant=%d block=%d "
                 "epi=%d chunk=%d eb=%d qc=%d grid_per_cu=%d\n",
                 forms[c.form & 3], cells[c.cell % 3], c.degree, (long long)c.E, c.qdeg, c.nf,
                 c.mode == FE_MODE_PREEVAL ? "preevaluated" : "quadrature", precs[c.prec % 3], c.pointgeo,
                 cfg.variant, cfg.block, cfg.epi, cfg.chunk, cfg.eb, cfg.qc, cfg.grid_per_cu);
}

// Output store mode: ordinary stores unless FE_NT_STORES=1 in the environment.
int store_mode()
{
    static int mode = -1;
    if (mode < 0) {
        const char* v = std::getenv("FE_NT_STORES");
        mode = (v && v[0] == '1') ? 1 : 0;
    }
    return mode;
}

// Generalised code motion (Sec. 3.2): with P1 on a simplex every gradient,
// hence F, is invariant in the quadrature loop, so the vector forms hoist
// the point loop and integrate the remaining scalar weights only.
bool q_invariant(const Call& c)
{
    // (pre-multiplying functions and a curved map vary over the element)
    return is_vector_form(c.form) && c.degree == 1 && c.cell != PRISM && c.nf == 0 && !c.pointgeo;
}

// the hoisted degree-1 kernel: float64 quadrature mode, vector forms on
// simplices
bool vec_p1_eligible(const Call& c)
{
    return c.prec == FE_FP64 && c.mode == FE_MODE_QUADRATURE && q_invariant(c) && !c.pointgeo;
}

bool gram64_eligible(const Call& c)
{
    if (!is_vector_form(c.form)) {
        // scalar Gram kernel: element matrices up to 48 x 48, any rule, per-point
        // prism geometry and coefficient functions; a mixed plan without
        // coefficient functions adds its pre-evaluated tables in the VALU kernel
        if (c.prec != FE_FP64 || c.mode != FE_MODE_QUADRATURE) return false;
        if (n_scalar(c.cell, c.degree) > 48) return false;
        return !(c.nf == 0 && c.mass_pre != 0);
    }
    if (c.pointgeo) return false;   // the vector matrix-core kernels take one map per element
    if (c.nf > 0) return false;      // and no pre-multiplying functions
    if (n_rows(c.form, c.cell, c.degree) > 32) return false;
    if (n_scalar(c.cell, c.degree) > 16) return false;
    const int nq = q_invariant(c) ? 1 : c.tables->nq;
    return nq <= 32;
}

int split_nqp(int nq) { return nq <= 8 ? 8 : nq <= 16 ? 16 : 32; }
int gram64_nqp(int nq) { return nq <= 4 ? 4 : nq <= 8 ? 8 : nq <= 16 ? 16 : nq <= 28 ? 28 : 32; }

// Launches one resolved call with an explicit configuration.
int launch_call(const Call& c, const Config& cfg)
{
    const RefTables* t = c.tables;
    const int cus = device_cus();
    hipError_t e;
    if (c.prec == FE_FP64 && c.mode == FE_MODE_QUADRATURE && cfg.variant == 2) {
        // degree 1 on a simplex: the hoisted streaming kernel
        if (!vec_p1_eligible(c)) return FE_EINVAL;
        VecP1Args v;
        v.coords = c.coords;
        v.coeff = c.coeff;
        v.out = c.out;
        v.status = c.status;
        v.W = t->dW;
        v.psi = t->dpsi;
        v.dphi = t->ddphi;
        v.E = c.E;
        v.nq = t->nq;
        v.nt = store_mode();
        v.mu = c.mu;
        v.lam = c.lam;
        const int64_t tiles = (c.E + vec_p1_elems_per_block() - 1) / vec_p1_elems_per_block();
        const int grid = (int)std::min<int64_t>(tiles, (int64_t)cus * cfg.grid_per_cu);
        e = launch_vec_p1(c.form, c.cell, v, grid, c.stream);
        if (e != hipSuccess) return set_hip_error(e, "degree-1 vector launch");
        return FE_OK;
    }
    if (c.prec != FE_FP64 || (c.mode == FE_MODE_QUADRATURE && cfg.variant == 1 && is_vector_form(c.form))) {
        SplitArgs a;
        a.coords = c.coords;
        a.coeff = c.coeff;
        a.out = c.out;
        a.status = c.status;
        a.W = t->dW;
        a.dphi = t->ddphi;
        a.psi = t->dpsi;
        a.E = c.E;
        a.nq = t->nq;
        a.ns = t->nb;
        a.collapse = q_invariant(c) ? 1 : 0;
        a.nt = store_mode();
        a.mu = c.mu;
        a.lam = c.lam;
        const int nq_eff = a.collapse ? 1 : t->nq;
        if (c.prec == FE_FP64) {
            if (!gram64_eligible(c)) return FE_EINVAL;
            const int nqp = gram64_nqp(nq_eff);
            const int per_block = G64_WAVES * g64_eb(c.form);
            const int64_t steps = (c.E + per_block - 1) / per_block;
            const int grid = (int)std::min<int64_t>(steps, (int64_t)cus * cfg.grid_per_cu);
            const size_t lds = gram64_lds_bytes(c.form, c.cell, nqp, t->nq, t->nb);
            e = c.form == ELASTICITY ? launch_gram64_elasticity(c.cell, c.degree, nqp, a, grid, lds, c.stream)
                                     : launch_gram64_hyperelastic(c.cell, c.degree, nqp, a, grid, lds, c.stream);
            if (e != hipSuccess) return set_hip_error(e, "float64 matrix-core launch");
            return FE_OK;
        }
        const int nqp = split_nqp(nq_eff);
        const int per_block = SPLIT_WAVES * split_eb(c.form);
        const int64_t steps = (c.E + per_block - 1) / per_block;
        const int grid = (int)std::min<int64_t>(steps, (int64_t)cus * cfg.grid_per_cu);
        const size_t lds = split_lds_bytes(c.form, c.cell, t->nq, t->nb);
        e = launch_split(c.form, c.cell, c.degree, c.prec == FE_SPLIT_FP32 ? SPLIT_FP32 : SPLIT_BF16X3, nqp, a, grid,
                         lds, c.stream);
        if (e != hipSuccess) return set_hip_error(e, "split-precision launch");
        return FE_OK;
    }
    if (c.mode == FE_MODE_PREEVAL && c.form == ELASTICITY && c.nf > 0) {
        // the P1 Lame fields and the nf functions expanded (iota = n_c C(n_s + nf - 1, nf))
        const CoefTables* ct = nullptr;
        int rc = get_coef_tables(c.form, c.cell, c.degree, c.qdeg, c.nf, c.stream, &ct);
        if (rc) return rc;
        e = launch_preeval_elast_coef(c.cell, c.coords, c.coeff, c.out, c.status, ct->dR, ct->dCombos, c.E, t->nb,
                                      c.nf, ct->iota, cfg.grid_per_cu, cus, c.stream);
        if (e != hipSuccess) return set_hip_error(e, "pre-evaluated elasticity launch");
        return FE_OK;
    }
    if (c.mode == FE_MODE_PREEVAL && c.form == ELASTICITY) {
        // the P1 Lame fields expanded out of the reduction (iota = n_c)
        const CoefTables* ct = nullptr;
        int rc = get_coef_tables(c.form, c.cell, c.degree, c.qdeg, 0, c.stream, &ct);
        if (rc) return rc;
        e = launch_preeval_elast(c.cell, c.coords, c.coeff, c.out, c.status, ct->dR, c.E, t->nb, cfg.grid_per_cu, cus,
                                 c.stream);
        if (e != hipSuccess) return set_hip_error(e, "pre-evaluated elasticity launch");
        return FE_OK;
    }
    if (c.mode == FE_MODE_PREEVAL && c.nf > 0) {
        const CoefTables* ct = nullptr;
        int rc = get_coef_tables(c.form, c.cell, c.degree, c.qdeg, c.nf, c.stream, &ct);
        if (rc) return rc;
        e = launch_preeval_coef(c.form, c.cell, c.coords, c.coeff, c.out, c.status, ct->dR, ct->dCombos, c.E, t->nb,
                                c.nf, ct->iota, cfg.grid_per_cu, cus, c.stream);
        if (e != hipSuccess) return set_hip_error(e, "coefficient pre-evaluated launch");
        return FE_OK;
    }
    if (c.mode == FE_MODE_PREEVAL) {
        PreevalArgs a;
        a.coords = c.coords;
        a.tables = t->dR;
        a.out = c.out;
        a.status = c.status;
        a.E = c.E;
        a.nn = t->nb * t->nb;
        a.epi = cfg.epi;
        a.chunk = cfg.chunk;
        a.nt = store_mode();
        if (cfg.variant) {
            if (cfg.epi < 1 || cfg.epi > cfg.block || cfg.chunk < 0 || cfg.chunk % cfg.epi ||
                preeval_stream_mm(c.form, cfg.epi * a.nn, cfg.block) == 0)
                return FE_EINVAL;   // a streaming step must fit in registers
            e = launch_preeval_stream(c.form, c.cell, a, cfg.block, cfg.grid_per_cu, cus, c.stream);
            if (e != hipSuccess) return set_hip_error(e, "pre-evaluated launch");
            return FE_OK;
        }
        const int64_t tiles = (c.E + a.chunk - 1) / a.chunk;
        const int grid = (int)std::min<int64_t>(tiles, (int64_t)cus * cfg.grid_per_cu);
        e = launch_preeval(c.form, c.cell, a, cfg.block, grid, c.stream);
        if (e != hipSuccess) return set_hip_error(e, "pre-evaluated launch");
        return FE_OK;
    }
    if (cfg.variant == 1) {
        // mass and Helmholtz on the float64 matrix cores
        if (!gram64_eligible(c)) return FE_EINVAL;
        GramScalarArgs g;
        g.coords = c.coords;
        g.coeff = c.coeff;
        g.out = c.out;
        g.status = c.status;
        g.W = t->dW;
        g.phi = t->dphi;
        g.dphi = t->ddphi;
        g.dpsi_grad = t->ddpsi;
        g.E = c.E;
        g.nq = t->nq;
        g.nf = c.nf;
        g.skip = c.nf > 0 ? c.mass_pre : 0;
        g.pointgeo = c.pointgeo;
        if (c.pointgeo == 2) g.dpsi_grad = c.map_tables->ddphi;
        g.nt = store_mode();
        const int64_t blocks =
            (c.E + gram64_scalar_elems_per_block(c.cell) - 1) / gram64_scalar_elems_per_block(c.cell);
        const int grid = (int)std::min<int64_t>(blocks, (int64_t)cus * cfg.grid_per_cu);
        e = launch_gram64_scalar(c.form, c.cell, c.degree, g, grid, c.stream);
        if (e != hipSuccess) return set_hip_error(e, "float64 matrix-core launch");
        return add_coef_monomial(c, cfg);
    }
    QuadArgs a;
    a.coords = c.coords;
    a.coeff = c.coeff;
    a.out = c.out;
    a.status = c.status;
    a.W = t->dW;
    a.phi = t->dphi;
    a.dphi = t->ddphi;
    a.psi = t->dpsi;
    a.mass_table = (c.nf == 0 && (c.mass_pre & 1)) ? t->dR : nullptr;
    a.stiff_tables = (c.nf == 0 && (c.mass_pre & 2)) ? t->dR : nullptr;
    a.skip = c.nf > 0 ? c.mass_pre : 0;
    a.E = c.E;
    a.nq = t->nq;
    a.ns = t->nb;
    a.collapse = q_invariant(c) ? 1 : 0;
    a.nt = store_mode();
    a.eb = cfg.eb;
    a.qc = cfg.qc;
    a.mu = c.mu;
    a.lam = c.lam;
    a.nf = c.nf;
    a.pointgeo = c.pointgeo;
    a.dpsi_grad = c.pointgeo == 2 ? c.map_tables->ddphi : t->ddpsi;
    const int64_t tiles = (c.E + a.eb - 1) / a.eb;
    const int grid = (int)std::min<int64_t>(tiles, (int64_t)cus * cfg.grid_per_cu);
    const size_t lds = quad_lds_bytes(c.form, c.cell, t->nb, a.eb, a.qc, c.pointgeo);
    e = launch_quad(c.form, c.cell, quad_kb(c.cell, c.degree), a, grid, lds, c.stream);
    if (e != hipSuccess) return set_hip_error(e, "quadrature launch");
    return add_coef_monomial(c, cfg);
}

// A mixed plan with coefficient functions: the pre-evaluated monomial is
// added to the quadrature part by the coefficient pre-evaluation kernel.
int add_coef_monomial(const Call& c, const Config& cfg)
{
    (void)cfg;
    if (!(c.nf > 0 && c.mass_pre)) return FE_OK;
    const RefTables* t = c.tables;
    const CoefTables* ct = nullptr;
    // the hyperelastic trace monomial is the Helmholtz gradient monomial with
    // the constant mu, on each of the d diagonal blocks: Helmholtz's tables
    const int tform = c.form == HYPERELASTIC ? HELMHOLTZ : c.form;
    int rc = get_coef_tables(tform, c.cell, c.degree, c.qdeg, c.nf, c.stream, &ct);
    if (rc) return rc;
    const int r_lo = (c.mass_pre & 1) ? 0 : 1, r_hi = (c.mass_pre & 2) ? n_tables(tform, c.cell) : 1;
    CoefOut o;
    if (c.form == HYPERELASTIC) {
        o.vec_d = cell_dim(c.cell);
        o.scale = c.mu;
        o.cstride = own_coeff(c.form, c.cell, c.degree) + c.nf * t->nb;
        o.coff = own_coeff(c.form, c.cell, c.degree);
    }
    hipError_t e = launch_preeval_coef(tform, c.cell, c.coords, c.coeff, c.out, nullptr, ct->dR, ct->dCombos, c.E,
                                       t->nb, c.nf, ct->iota, 8, device_cus(), c.stream, r_lo, r_hi, 1, o);
    if (e != hipSuccess) return set_hip_error(e, "coefficient pre-evaluated launch");
    return FE_OK;
}

size_t device_lds_per_block()
{
    static size_t lds[64] = {0};
    int d = current_device();
    if (d < 0 || d >= 64) return 64 * 1024;
    if (lds[d] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d) != hipSuccess || v <= 0)
            v = 64 * 1024;
        lds[d] = (size_t)v;
    }
    return lds[d];
}

int check_config(const Call& c, const Config& cfg)
{
    if (cfg.grid_per_cu < 1 || cfg.grid_per_cu > 64) return FE_EINVAL;
    if (c.prec != FE_FP64) return FE_OK;
    const RefTables* t = c.tables;
    const size_t max_lds = device_lds_per_block();
    if (c.mode == FE_MODE_PREEVAL && c.form == ELASTICITY && c.nf > 0) {
        // one wavefront per 16-element tile; one block's coefficient rows in LDS
        long iota = 1;
        for (int i = 1; i <= c.nf; ++i) iota = iota * (t->nb + i - 1) / i;
        const long nt = (long)cell_nv(c.cell) * iota * cell_dim(c.cell) * cell_dim(c.cell);
        return preeval_elast_coef_lds_bytes(c.cell, (int)std::min<long>(nt, 1L << 30), c.nf, t->nb) <= max_lds
                   ? FE_OK
                   : FE_EINVAL;
    }
    if (c.mode == FE_MODE_PREEVAL && c.form == ELASTICITY) return FE_OK;   // static LDS, grid only
    if (c.mode == FE_MODE_PREEVAL && c.nf > 0) {
        // one wavefront per block; the element rows of a 16-element tile
        // (n_tables * iota of them) sit in LDS
        long iota = 1;
        for (int i = 1; i <= c.nf; ++i) iota = iota * (t->nb + i - 1) / i;
        const long ntp = (n_tables(c.form, c.cell) * iota + 7) / 8 * 8;
        return preeval_coef_lds_bytes(c.form, c.cell, (int)std::min<long>(ntp, 1L << 30), c.nf, t->nb) <= max_lds
                   ? FE_OK
                   : FE_EINVAL;
    }
    if (c.mode == FE_MODE_PREEVAL) {
        const int nn = t->nb * t->nb;
        if (cfg.block < 64 || cfg.block > 512 || cfg.block % 64 || cfg.epi < 1 || cfg.epi > cfg.block)
            return FE_EINVAL;
        if (cfg.chunk < 0 || cfg.chunk % cfg.epi) return FE_EINVAL;
        if (cfg.variant) {
            if (preeval_stream_mm(c.form, cfg.epi * nn, cfg.block) == 0) return FE_EINVAL;
            return preeval_stream_lds_bytes(c.form, c.cell, cfg.block, cfg.epi) <= max_lds ? FE_OK : FE_EINVAL;
        }
        if (cfg.chunk == 0) return FE_EINVAL;
        return preeval_lds_bytes(c.form, c.cell, cfg.chunk) <= max_lds ? FE_OK : FE_EINVAL;
    }
    if (cfg.variant == 2)
        return vec_p1_eligible(c) && vec_p1_lds_bytes(c.cell) <= max_lds ? FE_OK : FE_EINVAL;
    if (cfg.variant) {
        if (!gram64_eligible(c)) return FE_EINVAL;
        if (cfg.grid_per_cu < 1) return FE_EINVAL;
        if (!is_vector_form(c.form)) return gram64_scalar_lds_bytes(c.cell, c.degree) <= max_lds ? FE_OK : FE_EINVAL;
        const int nq = q_invariant(c) ? 1 : t->nq;
        return gram64_lds_bytes(c.form, c.cell, gram64_nqp(nq), t->nq, t->nb) <= max_lds ? FE_OK : FE_EINVAL;
    }
    if (cfg.eb < 1 || cfg.qc < 1 || cfg.qc > t->nq) return FE_EINVAL;
    return quad_lds_bytes(c.form, c.cell, t->nb, cfg.eb, cfg.qc, c.pointgeo) <= max_lds ? FE_OK : FE_EINVAL;
}

int final_config(const Call& c, Config* cfg)
{
    lookup_config(c, cfg);
    const int* s = c.shape;   // kernel, block, epi, chunk, eb, qc, grid_per_cu
    const Config autocfg = *cfg;
    if (s[0]) {
        // 1, 2: tiled or streaming pre-evaluated kernel; 3, 4: VALU or matrix-core
        // quadrature; 5: the hoisted degree-1 vector kernel
        const bool pre = c.mode == FE_MODE_PREEVAL && c.prec == FE_FP64;
        if (pre != (s[0] <= 2) || (c.prec != FE_FP64 && s[0] != 4)) return FE_EINVAL;
        if (c.prec == FE_FP64) {
            const int v = s[0] == 5 ? 2 : (s[0] == 2 || s[0] == 4) ? 1 : 0;
            if (!pre && v != autocfg.variant) {
                *cfg = v ? Config() : default_quad_config(c.form, c.cell, c.degree, c.tables->nq, c.pointgeo);
                cfg->variant = v;
            }
            cfg->variant = v;
        }
    }
    if (s[1]) cfg->block = s[1];
    if (s[2]) cfg->epi = s[2];
    if (s[3]) cfg->chunk = s[3];
    else if (c.mode == FE_MODE_PREEVAL && (cfg->variant != autocfg.variant || cfg->epi != autocfg.epi))
        cfg->chunk = cfg->variant ? 0 : cfg->epi * std::max(1, 256 / cfg->epi);
    if (s[4]) cfg->eb = s[4];
    if (s[5]) cfg->qc = s[5];
    if (s[6]) cfg->grid_per_cu = s[6];
    return check_config(c, *cfg);
}

// Validates the arguments of fe_assemble_local and resolves them into a Call.
int resolve_call(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                 const double* coeff_dofs, double* out_A, const fe_options_t* opt, Call* c, int lookup_only)
{
    fe_options_t o;
    if (opt) o = *opt;
    else fe_options_init(&o);
    if ((int)form < 0 || (int)form > 3 || (int)cell < 0 || (int)cell > 2 || degree < 1 || degree > MAX_DEGREE ||
        n_elems < 0)
        return FE_EINVAL;
    if ((int)o.precision < 0 || (int)o.precision > 2 || (int)o.mode < 0 || (int)o.mode > 2) return FE_EINVAL;
    if (o.nf < 0 || o.nf > 3) return FE_EINVAL;
    if (o.nf > 0 && o.precision != FE_FP64) return FE_ENOTSUP;
    if (o.coord_degree < 0 || o.coord_degree > 2) return FE_EINVAL;
    if (o.coord_degree == 2 && cell == PRISM) return FE_ENOTSUP;
    // the vertex map of a simplex is affine: the vertex map at every point
    // only changes prisms; a P2 coordinate field curves a simplex
    const int pg = o.coord_degree == 2 ? 2 : (o.pointgeo && cell == PRISM) ? 1 : 0;
    if (pg && (o.nf > 0 || o.precision != FE_FP64 || o.mode == FE_MODE_PREEVAL)) return FE_ENOTSUP;
    // a per-point map adds the degree of det J: 1 (prism heights), d (P2 map)
    const int qdeg = o.qdeg < 0 ? default_qdeg(form, cell, degree, o.nf) + (pg == 2 ? cell_dim(cell) : pg) : o.qdeg;
    if (qdeg > MAX_QDEG) return FE_EINVAL;
    c->nf = o.nf;
    c->pointgeo = pg;
    c->form = form;
    c->cell = cell;
    c->degree = degree;
    c->qdeg = qdeg;
    c->E = n_elems;
    c->prec = o.precision;
    c->coords = coords;
    c->coeff = coeff_dofs;
    c->out = out_A;
    c->status = o.d_status;
    c->mu = o.mu;
    c->lam = o.lambda;
    c->stream = (hipStream_t)o.stream;
    const int sh[7] = {o.shape.kernel, o.shape.block, o.shape.epi, o.shape.chunk,
                       o.shape.eb,     o.shape.qc,    o.shape.grid_per_cu};
    for (int i = 0; i < 7; ++i) {
        if (sh[i] < 0 || (i == 0 && sh[i] > 5)) return FE_EINVAL;
        c->shape[i] = sh[i];
    }
    if (n_elems == 0) return FE_OK;
    if (!coords || !out_A) return FE_EINVAL;
    if ((is_vector_form(form) || o.nf > 0) && !coeff_dofs) return FE_EINVAL;
    if (form == HYPERELASTIC && !(std::isfinite(o.mu) && std::isfinite(o.lambda))) return FE_EINVAL;
    int rc = FE_OK;
    if (pg) {
        // pre-evaluation needs a geometry tensor that is constant over the
        // element (Sec. 3.3); with per-point maps every monomial is evaluated
        // by quadrature
        c->mode = FE_MODE_QUADRATURE;
        c->mass_pre = 0;
    } else {
        rc = fe_resolve_variant(form, cell, degree, qdeg, &o, &c->mode, &c->mass_pre);
        if (rc) return rc;
    }
    if (o.validate && cell == PRISM && !pg) {
        rc = validate_prisms(n_elems, coords, c->stream);
        if (rc) return rc;
    }
    if (lookup_only) return find_tables(cell, degree, qdeg, &c->tables);
    if (pg == 2) {
        // the P2 basis gradients at the same rule: the map's tables
        rc = get_tables(cell, 2, qdeg, c->stream, &c->map_tables);
        if (rc) return rc;
    }
    return get_tables(cell, degree, qdeg, c->stream, &c->tables);
}

}  // namespace fe

extern "C" {

int fe_assemble_local(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                      const double* coeff_dofs, double* out_A, const fe_options_t* opt)
{
    Call c;
    int rc = resolve_call(form, cell, degree, n_elems, coords, coeff_dofs, out_A, opt, &c, 0);
    if (rc || n_elems == 0) return rc;
    // at degree 1 on a simplex the point loop is hoisted and the contraction is
    // one record per element: the split precisions take the float64 hoisted
    // kernel there (faster than the matrix-core split kernel, and exact)
    if (c.prec != FE_FP64 && q_invariant(c) && c.shape[0] == 0) c.prec = FE_FP64;
    Config cfg;
    rc = final_config(c, &cfg);
    if (rc) return rc;
    if (log_enabled()) log_call(c, cfg);
    return launch_call(c, cfg);
}

void fe_autotune_clear(void);

void fe_release_caches(void)
{
    fe_autotune_clear();
    release_generated();
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_tables) {
        RefTables* t = kv.second;
        for (double* p_ : {t->dX, t->dW, t->dphi, t->ddphi, t->dpsi, t->ddpsi, t->dR})
            if (p_) (void)hipFree(p_);
        delete t;
    }
    g_tables.clear();
    for (auto& kv : g_coef) {
        CoefTables* t = kv.second;
        if (t->dCombos) (void)hipFree(t->dCombos);
        if (t->dR) (void)hipFree(t->dR);
        delete t;
    }
    g_coef.clear();
}

}  // extern "C"
