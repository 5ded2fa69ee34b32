// Mixed batches: sub-batches of different (form, cell, degree) run in ONE
// persistent kernel.  The host turns every sub-batch into element tiles with
// the tile shape of its variant (from the autotune cache or the defaults) and
// lays the tiles out as one global index range; each workgroup repeatedly
// takes the next tile index from a device counter and runs the matching
// device routine (the same tile routines the standalone kernels use).  The
// counter reset (a one-thread kernel, not a memset node) and the persistent
// launch are captured once into a HIP graph; fe_batch_run replays it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "felocal.h"
#include "internal.hpp"
#include "preeval.hpp"
#include "quad.hpp"

namespace fe {

// Variants the persistent kernel can run (FP64): kind 0 = pre-evaluated,
// kind 1 = quadrature; the switch below enumerates every (kind, form, cell,
// kb) instance.
struct SubDesc {
    int variant;          // index into the dispatch switch
    int pad_;
    int64_t tile_begin;   // first global tile of this sub-batch
    int64_t n_tiles;
    PreevalArgs pa;
    QuadArgs qa;
};

__host__ __device__ constexpr int variant_id(int kind, int form, int cell, int kb_small)
{
    // kind 0: 2 forms x 3 cells; kind 1: 3 forms x 3 cells x 2 k-block widths
    return kind == 0 ? form * 3 + cell : 6 + (form * 3 + cell) * 2 + kb_small;
}

template <int FORM, int CELL, int KB>
__device__ __forceinline__ void run_quad(const SubDesc& d, int64_t local, double* lds)
{
    quad_tile<FORM, CELL, KB>(d.qa, local * d.qa.eb, lds);
}

__global__ __launch_bounds__(256) void k_batch(const SubDesc* __restrict__ subs, int n_subs, int64_t total,
                                               unsigned long long* counter)
{
    extern __shared__ double lds[];
    __shared__ long long s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (long long)atomicAdd(counter, 1ULL);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= total) break;
        int lo = 0, hi = n_subs - 1;
        while (lo < hi) {   // last sub-batch with tile_begin <= tile
            const int mid = (lo + hi + 1) >> 1;
            if (subs[mid].tile_begin <= tile) lo = mid;
            else hi = mid - 1;
        }
        const SubDesc& d = subs[lo];
        const int64_t local = tile - d.tile_begin;
        switch (d.variant) {
        case variant_id(0, MASS, TRI, 0): preeval_tile<MASS, TRI, preeval_mm(MASS)>(d.pa, local * d.pa.chunk, lds); break;
        case variant_id(0, MASS, TET, 0): preeval_tile<MASS, TET, preeval_mm(MASS)>(d.pa, local * d.pa.chunk, lds); break;
        case variant_id(0, MASS, PRISM, 0): preeval_tile<MASS, PRISM, preeval_mm(MASS)>(d.pa, local * d.pa.chunk, lds); break;
        case variant_id(0, HELMHOLTZ, TRI, 0): preeval_tile<HELMHOLTZ, TRI, preeval_mm(HELMHOLTZ)>(d.pa, local * d.pa.chunk, lds); break;
        case variant_id(0, HELMHOLTZ, TET, 0): preeval_tile<HELMHOLTZ, TET, preeval_mm(HELMHOLTZ)>(d.pa, local * d.pa.chunk, lds); break;
        case variant_id(0, HELMHOLTZ, PRISM, 0): preeval_tile<HELMHOLTZ, PRISM, preeval_mm(HELMHOLTZ)>(d.pa, local * d.pa.chunk, lds); break;
        case variant_id(1, MASS, TRI, 1): run_quad<MASS, TRI, 3>(d, local, lds); break;
        case variant_id(1, MASS, TRI, 0): run_quad<MASS, TRI, 5>(d, local, lds); break;
        case variant_id(1, MASS, TET, 1): run_quad<MASS, TET, 4>(d, local, lds); break;
        case variant_id(1, MASS, TET, 0): run_quad<MASS, TET, 5>(d, local, lds); break;
        case variant_id(1, MASS, PRISM, 1): run_quad<MASS, PRISM, 3>(d, local, lds); break;
        case variant_id(1, MASS, PRISM, 0): run_quad<MASS, PRISM, 5>(d, local, lds); break;
        case variant_id(1, HELMHOLTZ, TRI, 1): run_quad<HELMHOLTZ, TRI, 3>(d, local, lds); break;
        case variant_id(1, HELMHOLTZ, TRI, 0): run_quad<HELMHOLTZ, TRI, 5>(d, local, lds); break;
        case variant_id(1, HELMHOLTZ, TET, 1): run_quad<HELMHOLTZ, TET, 4>(d, local, lds); break;
        case variant_id(1, HELMHOLTZ, TET, 0): run_quad<HELMHOLTZ, TET, 5>(d, local, lds); break;
        case variant_id(1, HELMHOLTZ, PRISM, 1): run_quad<HELMHOLTZ, PRISM, 3>(d, local, lds); break;
        case variant_id(1, HELMHOLTZ, PRISM, 0): run_quad<HELMHOLTZ, PRISM, 5>(d, local, lds); break;
        case variant_id(1, ELASTICITY, TRI, 1): run_quad<ELASTICITY, TRI, 3>(d, local, lds); break;
        case variant_id(1, ELASTICITY, TRI, 0): run_quad<ELASTICITY, TRI, 5>(d, local, lds); break;
        case variant_id(1, ELASTICITY, TET, 1): run_quad<ELASTICITY, TET, 4>(d, local, lds); break;
        case variant_id(1, ELASTICITY, TET, 0): run_quad<ELASTICITY, TET, 5>(d, local, lds); break;
        case variant_id(1, ELASTICITY, PRISM, 1): run_quad<ELASTICITY, PRISM, 3>(d, local, lds); break;
        case variant_id(1, ELASTICITY, PRISM, 0): run_quad<ELASTICITY, PRISM, 5>(d, local, lds); break;
        default: break;
        }
    }
}

__global__ void k_reset_counter(unsigned long long* counter) { *counter = 0ULL; }

}  // namespace fe

using namespace fe;

struct fe_batch {
    SubDesc* d_subs = nullptr;
    unsigned long long* d_counter = nullptr;
    int n_subs = 0;
    int64_t total = 0;
    int grid = 0;
    size_t lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void destroy(fe_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_subs) (void)hipFree(b->d_subs);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

// pre-evaluated tile shape with the persistent kernel's block of 256
Config batch_preeval_config(const Config& tuned, int nn, int mm)
{
    if (tuned.block == 256 && !tuned.variant) return tuned;
    Config best;
    best.block = 256;
    double best_w = 1e9;
    for (int epi = 1; epi <= 64; ++epi) {
        const int slots = epi * nn, m = (slots + 255) / 256;
        if (m > mm && epi > 1) break;
        const double w = (double)(m * 256 - slots) / (m * 256) + (slots < 512 ? 0.5 : 0.0);
        if (w < best_w - 1e-9) {
            best_w = w;
            best.epi = epi;
        }
    }
    best.chunk = best.epi * std::max(1, 256 / best.epi);
    best.grid_per_cu = tuned.grid_per_cu;
    return best;
}

}  // namespace

extern "C" {

int fe_resolve_variant(int form, int cell, int degree, int qdeg, const fe_options_t* o, int* mode_out, int* mass_pre);

int fe_batch_create(const fe_subbatch_t* subs, int n_subs, const fe_options_t* opt, fe_batch_t** out)
{
    if (!out || !subs || n_subs < 1 || n_subs > 4096) return FE_EINVAL;
    *out = nullptr;
    fe_options_t o;
    if (opt) o = *opt;
    else fe_options_init(&o);
    if (o.precision != FE_FP64) return FE_ENOTSUP;
    hipStream_t s = (hipStream_t)o.stream;
    std::vector<SubDesc> h(n_subs);
    int64_t total = 0;
    size_t lds = 0;
    for (int i = 0; i < n_subs; ++i) {
        const fe_subbatch_t& sb = subs[i];
        if ((int)sb.form < 0 || (int)sb.form > 2 || (int)sb.cell < 0 || (int)sb.cell > 2 || sb.degree < 1 ||
            sb.degree > MAX_DEGREE || sb.n_elems < 0)
            return sb.form == FE_HYPERELASTIC ? FE_ENOTSUP : FE_EINVAL;
        if (sb.n_elems > 0 && (!sb.coords || !sb.out_A || (sb.form == FE_ELASTICITY && !sb.coeff_dofs)))
            return FE_EINVAL;
        const int qdeg = sb.qdeg < 0 ? default_qdeg(sb.form, sb.cell, sb.degree) : sb.qdeg;
        if (qdeg > MAX_QDEG) return FE_EINVAL;
        fe_options_t so = o;
        so.qdeg = qdeg;
        Call c;
        c.form = sb.form;
        c.cell = sb.cell;
        c.degree = sb.degree;
        c.qdeg = qdeg;
        c.prec = FE_FP64;
        c.E = sb.n_elems;
        int rc = fe_resolve_variant(sb.form, sb.cell, sb.degree, qdeg, &so, &c.mode, &c.mass_pre);
        if (rc) return rc;
        rc = get_tables(sb.cell, sb.degree, qdeg, s, &c.tables);
        if (rc) return rc;
        const RefTables* t = c.tables;
        Config cfg;
        lookup_config(c, &cfg);
        SubDesc& d = h[i];
        std::memset(&d, 0, sizeof(d));
        d.tile_begin = total;
        if (c.mode == FE_MODE_PREEVAL) {
            cfg = batch_preeval_config(cfg, t->nb * t->nb, preeval_mm(sb.form));
            d.variant = variant_id(0, sb.form, sb.cell, 0);
            d.pa.coords = sb.coords;
            d.pa.tables = t->dR;
            d.pa.out = sb.out_A;
            d.pa.status = o.d_status;
            d.pa.E = sb.n_elems;
            d.pa.nn = t->nb * t->nb;
            d.pa.epi = cfg.epi;
            d.pa.chunk = cfg.chunk;
            d.n_tiles = (sb.n_elems + cfg.chunk - 1) / cfg.chunk;
            lds = std::max(lds, preeval_lds_bytes(sb.form, sb.cell, cfg.chunk));
            d.pa.nt = store_mode();
        } else {
            // the persistent kernel runs the VALU quadrature tile
            if (cfg.variant) cfg = default_quad_config(sb.form, sb.cell, sb.degree, t->nq);
            const int kb = quad_kb(sb.cell, sb.degree);
            d.variant = variant_id(1, sb.form, sb.cell, (kb == 5) ? 0 : 1);
            d.qa.coords = sb.coords;
            d.qa.coeff = sb.coeff_dofs;
            d.qa.out = sb.out_A;
            d.qa.status = o.d_status;
            d.qa.W = t->dW;
            d.qa.phi = t->dphi;
            d.qa.dphi = t->ddphi;
            d.qa.psi = t->dpsi;
            d.qa.mass_table = (c.mass_pre & 1) ? t->dR : nullptr;
            d.qa.stiff_tables = (c.mass_pre & 2) ? t->dR : nullptr;
            d.qa.E = sb.n_elems;
            d.qa.nq = t->nq;
            d.qa.ns = t->nb;
            d.qa.collapse = (sb.form == FE_ELASTICITY && sb.degree == 1 && sb.cell != FE_PRISM) ? 1 : 0;
            d.qa.eb = cfg.eb;
            d.qa.qc = cfg.qc;
            d.qa.nt = store_mode();
            d.n_tiles = (sb.n_elems + cfg.eb - 1) / cfg.eb;
            lds = std::max(lds, quad_lds_bytes(sb.form, sb.cell, t->nb, cfg.eb, cfg.qc));
        }
        total += d.n_tiles;
    }
    fe_batch* b = new fe_batch();
    b->n_subs = n_subs;
    b->total = total;
    b->lds = lds;
    hipError_t e = hipMalloc((void**)&b->d_subs, sizeof(SubDesc) * n_subs);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_counter, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemcpy(b->d_subs, h.data(), sizeof(SubDesc) * n_subs, hipMemcpyHostToDevice);
    int per_cu = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, 256, lds);
    if (e != hipSuccess) {
        destroy(b);
        return set_hip_error(e, "fe_batch_create setup");
    }
    per_cu = std::max(1, per_cu);
    b->grid = (int)std::max<int64_t>(1, std::min<int64_t>(total, (int64_t)device_cus() * per_cu));
    // capture: counter reset + persistent launch
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, cs, b->d_counter);
        hipLaunchKernelGGL(k_batch, dim3(b->grid), dim3(256), lds, cs, b->d_subs, n_subs, total, b->d_counter);
        hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
        e = (e2 != hipSuccess) ? e2 : hipGetLastError();
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        destroy(b);
        return set_hip_error(e, "fe_batch_create capture");
    }
    *out = b;
    return FE_OK;
}

int fe_batch_run(fe_batch_t* batch, void* stream)
{
    if (!batch || !batch->exec) return FE_EINVAL;
    hipError_t e = hipGraphLaunch(batch->exec, (hipStream_t)stream);
    if (e != hipSuccess) return set_hip_error(e, "fe_batch_run");
    return FE_OK;
}

int fe_batch_destroy(fe_batch_t* batch)
{
    if (!batch) return FE_EINVAL;
    destroy(batch);
    return FE_OK;
}

int fe_batch_info(const fe_batch_t* batch, int64_t* n_tiles, int* grid)
{
    if (!batch) return FE_EINVAL;
    if (n_tiles) *n_tiles = batch->total;
    if (grid) *grid = batch->grid;
    return FE_OK;
}

}  // extern "C"
