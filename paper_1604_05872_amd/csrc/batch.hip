// Mixed batches: sub-batches of different (form, cell, degree) in one
// HIP graph of persistent work-queue kernels.  The host turns every
// sub-batch into element tiles with the tile shape of its variant (from the
// autotune cache or the defaults) and groups the sub-batches by kernel
// variant (kind, form, cell, k-block width).  Each group gets one persistent
// kernel, specialised for its variant so that it runs at that variant's
// register budget and occupancy (one kernel for every variant would run all
// of them at the worst one), whose workgroups repeatedly take the next tile
// of the group from a device counter.  A one-block kernel clears the
// counters (no memset node), the group kernels are captured on parallel
// branches of one graph, pre-evaluated elasticity sub-batches follow the
// join one after another, and fe_batch_run replays it with one graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "felocal.h"
#include "internal.hpp"
#include "preeval.hpp"
#include "quad.hpp"

namespace fe {

// kind 0 = pre-evaluated (2 forms x 3 cells), kind 1 = quadrature (3 forms x
// 3 cells x 2 k-block widths): 24 variants
constexpr int N_VARIANTS = 24;

struct SubDesc {
    int64_t tile_begin;   // first tile of this sub-batch within its group
    int64_t n_tiles;
    PreevalArgs pa;
    QuadArgs qa;
};

__host__ __device__ constexpr int variant_id(int kind, int form, int cell, int kb_small)
{
    return kind == 0 ? form * 3 + cell : 6 + (form * 3 + cell) * 2 + kb_small;
}

template <int VID>
__device__ __forceinline__ void run_tile(const SubDesc& d, int64_t local, double* lds)
{
    if constexpr (VID < 6) {
        constexpr int FORM = VID / 3, CELL = VID % 3;
        preeval_tile<FORM, CELL, preeval_mm(FORM)>(d.pa, local * d.pa.chunk, lds);
    } else {
        constexpr int v = VID - 6, FORM = (v / 2) / 3, CELL = (v / 2) % 3;
        constexpr int KB = (v % 2) ? (CELL == TET ? 4 : 3) : 5;
        quad_tile<FORM, CELL, KB>(d.qa, local * d.qa.eb, lds);
    }
}

template <int VID>
__global__ __launch_bounds__(256) void k_batch_group(const SubDesc* __restrict__ subs, int n_subs, int64_t total,
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
        run_tile<VID>(subs[lo], tile - subs[lo].tile_begin, lds);
    }
}

__global__ void k_reset_counters(unsigned long long* counters, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0ULL;
}

// runtime variant id -> the group kernel's launch and occupancy
template <int V = 0>
hipError_t launch_group(int vid, int grid, size_t lds, hipStream_t s, const SubDesc* subs, int n, int64_t total,
                        unsigned long long* ctr)
{
    if (vid == V) {
        hipLaunchKernelGGL((k_batch_group<V>), dim3(grid), dim3(256), lds, s, subs, n, total, ctr);
        return hipGetLastError();
    }
    if constexpr (V + 1 < N_VARIANTS) return launch_group<V + 1>(vid, grid, lds, s, subs, n, total, ctr);
    return hipErrorInvalidValue;
}

template <int V = 0>
hipError_t group_occupancy(int vid, size_t lds, int* per_cu)
{
    if (vid == V) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_group<V>, 256, lds);
    if constexpr (V + 1 < N_VARIANTS) return group_occupancy<V + 1>(vid, lds, per_cu);
    return hipErrorInvalidValue;
}

}  // namespace fe

using namespace fe;

struct fe_batch {
    struct Group {
        int vid = 0;
        int n_subs = 0;
        int64_t total = 0;
        int grid = 0;
        size_t lds = 0;
        SubDesc* d_subs = nullptr;
    };
    std::vector<Group> groups;
    // elasticity sub-batches that Algorithm 3 pre-evaluates: the pre-evaluated
    // elasticity kernel, one launch each, in sequence after the groups
    struct ElastSub {
        int cell = 0, ns = 0;
        const double* coords = nullptr;
        const double* coeff = nullptr;
        double* out = nullptr;
        const double* T = nullptr;
        int64_t E = 0;
        int grid_per_cu = 1;   // the single call's (autotuned or default) launch width
    };
    std::vector<ElastSub> elast;
    // sub-batches whose single-call kernel is not a group tile (the streaming
    // pre-evaluated kernel, the float64 matrix-core and hoisted degree-1
    // quadrature kernels): launched as single calls, with the same shape
    struct Direct {
        Call c;
        Config cfg;
    };
    std::vector<Direct> direct;
    unsigned long long* d_counters = nullptr;
    int64_t total = 0;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void destroy(fe_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& g : b->groups)
        if (g.d_subs) (void)hipFree(g.d_subs);
    if (b->d_counters) (void)hipFree(b->d_counters);
    delete b;
}

// pre-evaluated tile shape with the group kernel's block of 256: the fewest
// idle slots, and tiles of about 256 KiB of output
Config batch_preeval_config(const Config& tuned, int nn, int mm)
{
    Config best;
    best.block = 256;
    if (tuned.block == 256 && !tuned.variant) {
        best = tuned;
    } else {
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
    }
    const int steps = std::max(1, (int)((256 * 1024) / ((int64_t)best.epi * nn * 8)));
    best.chunk = best.epi * std::min(steps, std::max(1, 256 / best.epi));
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
    if (o.precision != FE_FP64 || o.nf != 0 || o.pointgeo != 0 || o.coord_degree > 1) return FE_ENOTSUP;
    hipStream_t s = (hipStream_t)o.stream;
    std::vector<std::vector<SubDesc>> by_vid(N_VARIANTS);
    std::vector<size_t> lds_vid(N_VARIANTS, 0);
    std::vector<fe_batch::ElastSub> elast;
    std::vector<fe_batch::Direct> direct;
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
        if (sb.n_elems == 0) continue;
        rc = get_tables(sb.cell, sb.degree, qdeg, s, &c.tables);
        if (rc) return rc;
        const RefTables* t = c.tables;
        if (sb.form == FE_ELASTICITY && c.mode == FE_MODE_PREEVAL) {
            const CoefTables* ct = nullptr;
            rc = get_coef_tables(ELASTICITY, sb.cell, sb.degree, qdeg, 0, s, &ct);
            if (rc) return rc;
            fe_batch::ElastSub es;
            es.cell = sb.cell;
            es.ns = t->nb;
            es.coords = sb.coords;
            es.coeff = sb.coeff_dofs;
            es.out = sb.out_A;
            es.T = ct->dR;
            es.E = sb.n_elems;
            Config ecfg;
            lookup_config(c, &ecfg);
            es.grid_per_cu = ecfg.grid_per_cu > 0 ? ecfg.grid_per_cu : preeval_elast_grid_per_cu(sb.cell, t->nb);
            elast.push_back(es);
            continue;
        }
        Config cfg;
        lookup_config(c, &cfg);
        // the sub-batch's single-call kernel and shape (the autotuner's when it
        // has tuned the variant): launched as is where no group tile serves it
        if ((c.mode == FE_MODE_PREEVAL && cfg.variant == 1) || (c.mode == FE_MODE_QUADRATURE && cfg.variant != 0)) {
            c.coords = sb.coords;
            c.coeff = sb.coeff_dofs;
            c.out = sb.out_A;
            c.status = o.d_status;
            c.mu = o.mu;
            c.lam = o.lambda;
            if (check_config(c, cfg) != FE_OK) return FE_EINVAL;
            direct.push_back({c, cfg});
            continue;
        }
        SubDesc d;
        std::memset(&d, 0, sizeof(d));
        int vid;
        size_t lds;
        if (c.mode == FE_MODE_PREEVAL) {
            cfg = batch_preeval_config(cfg, t->nb * t->nb, preeval_mm(sb.form));
            vid = variant_id(0, sb.form, sb.cell, 0);
            d.pa.coords = sb.coords;
            d.pa.tables = t->dR;
            d.pa.out = sb.out_A;
            d.pa.status = o.d_status;
            d.pa.E = sb.n_elems;
            d.pa.nn = t->nb * t->nb;
            d.pa.epi = cfg.epi;
            d.pa.chunk = cfg.chunk;
            d.pa.nt = store_mode();
            d.n_tiles = (sb.n_elems + cfg.chunk - 1) / cfg.chunk;
            lds = preeval_lds_bytes(sb.form, sb.cell, cfg.chunk);
        } else {
            // the group kernels run the VALU quadrature tile
            const int kb = quad_kb(sb.cell, sb.degree);
            vid = variant_id(1, sb.form, sb.cell, (kb == 5) ? 0 : 1);
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
            lds = quad_lds_bytes(sb.form, sb.cell, t->nb, cfg.eb, cfg.qc);
        }
        auto& grp = by_vid[vid];
        d.tile_begin = grp.empty() ? 0 : grp.back().tile_begin + grp.back().n_tiles;
        grp.push_back(d);
        lds_vid[vid] = std::max(lds_vid[vid], lds);
    }
    fe_batch* b = new fe_batch();
    b->elast = elast;
    b->direct = direct;
    hipError_t e = hipSuccess;
    const int cus = device_cus();
    for (int v = 0; v < N_VARIANTS && e == hipSuccess; ++v) {
        if (by_vid[v].empty()) continue;
        fe_batch::Group g;
        g.vid = v;
        g.n_subs = (int)by_vid[v].size();
        g.total = by_vid[v].back().tile_begin + by_vid[v].back().n_tiles;
        g.lds = lds_vid[v];
        int per_cu = 0;
        e = group_occupancy(v, g.lds, &per_cu);
        if (e != hipSuccess) break;
        g.grid = (int)std::max<int64_t>(1, std::min<int64_t>(g.total, (int64_t)cus * std::max(1, per_cu)));
        e = hipMalloc((void**)&g.d_subs, sizeof(SubDesc) * g.n_subs);
        if (e == hipSuccess)
            e = hipMemcpy(g.d_subs, by_vid[v].data(), sizeof(SubDesc) * g.n_subs, hipMemcpyHostToDevice);
        b->total += g.total;
        b->grid += g.grid;
        b->groups.push_back(g);
    }
    const int ng = (int)b->groups.size();
    // parallel branches of the graph: one per group; the single-call
    // sub-batches follow the join one after another (each fills the GPU; on
    // parallel branches they contend for the L2 and ran slower on MI355X)
    const int nd = (int)b->direct.size();
    const int nbr = ng;
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_counters, sizeof(unsigned long long) * std::max(1, ng));
    if (e != hipSuccess) {
        destroy(b);
        return set_hip_error(e, "fe_batch_create setup");
    }
    // capture: counter reset, then the group kernels on parallel branches
    std::vector<hipStream_t> br(nbr, nullptr);
    std::vector<hipEvent_t> done(nbr, nullptr);
    hipStream_t cs = nullptr;
    hipEvent_t start = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    for (int i = 0; i < nbr && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
    }
    bool capturing = false;
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        capturing = e == hipSuccess;
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, cs, b->d_counters, ng);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(start, cs);
    for (int i = 0; i < ng && e == hipSuccess; ++i) {
        const fe_batch::Group& g = b->groups[i];
        e = hipStreamWaitEvent(br[i], start, 0);
        if (e == hipSuccess)
            e = launch_group(g.vid, g.grid, g.lds, br[i], g.d_subs, g.n_subs, g.total, b->d_counters + i);
        if (e == hipSuccess) e = hipEventRecord(done[i], br[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, done[i], 0);
    }
    for (int i = 0; i < nd && e == hipSuccess; ++i) {
        fe_batch::Direct& dsub = b->direct[i];
        dsub.c.stream = cs;
        if (launch_call(dsub.c, dsub.cfg) != FE_OK) e = hipErrorLaunchFailure;
    }
    // pre-evaluated elasticity after the join, one sub-batch at a time: each
    // fills the GPU, and two running at once write partial lines over twice
    // the span, which the L2 merges less well (measured on MI355X: 4.2 ms
    // for the mixed batch against 5.4 ms with a branch per sub-batch)
    for (size_t i = 0; i < b->elast.size() && e == hipSuccess; ++i) {
        const fe_batch::ElastSub& es = b->elast[i];
        e = launch_preeval_elast(es.cell, es.coords, es.coeff, es.out, o.d_status, es.T, es.E, es.ns,
                                 es.grid_per_cu, cus, cs);
    }
    if (capturing) {
        const hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    for (int i = 0; i < nbr; ++i) {
        if (done[i]) (void)hipEventDestroy(done[i]);
        if (br[i]) (void)hipStreamDestroy(br[i]);
    }
    if (start) (void)hipEventDestroy(start);
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
