// Tile-shape autotuner and configuration cache.
//
// A variant is (form, cell, degree, rule, mode, precision).  Its tunable
// shape is, for the pre-evaluated kernel, the block size, the elements per
// step and per tile; for the quadrature kernel, the elements per tile and the
// points per LDS chunk; for every kernel, the resident blocks per CU of the
// persistent grid.  fe_autotune times each candidate with HIP events on the
// caller's inputs and keeps the fastest in memory (and, when the environment
// variable FE_AUTOTUNE_CACHE names a file, appends it there as one JSON object
// per line; the file is read back on first use, so tuning persists).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "felocal.h"
#include "internal.hpp"

namespace fe {

namespace {

using Key = std::tuple<int, int, int, int, int, int, int>;
using ModeKey = std::tuple<int, int, int, int, int, int>;   // form, cell, degree, qdeg, precision, nf
std::mutex g_tmu;
std::map<Key, Config> g_tuned;
std::map<ModeKey, int> g_mode;   // the measured faster mode of an AUTO request
bool g_loaded = false;

Key key_of(const Call& c) { return Key(c.form, c.cell, c.degree, c.qdeg, c.mode, c.prec, c.nf); }

void load_file_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char* path = std::getenv("FE_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        int v[7];
        Config c;
        if (std::sscanf(line,
                        "{\"form\": %d, \"cell\": %d, \"degree\": %d, \"qdeg\": %d, \"mode\": %d, \"precision\": %d, "
                        "\"block\": %d, \"epi\": %d, \"chunk\": %d, \"eb\": %d, \"qc\": %d, \"grid_per_cu\": %d, "
                        "\"variant\": %d, \"nf\": %d",
                        &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &c.block, &c.epi, &c.chunk, &c.eb, &c.qc,
                        &c.grid_per_cu, &c.variant, &v[6]) == 14)
            g_tuned[Key(v[0], v[1], v[2], v[3], v[4], v[5], v[6])] = c;
        else if (std::sscanf(line,
                             "{\"form\": %d, \"cell\": %d, \"degree\": %d, \"qdeg\": %d, \"precision\": %d, "
                             "\"nf\": %d, \"tuned_mode\": %d",
                             &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6]) == 7)
            g_mode[ModeKey(v[0], v[1], v[2], v[3], v[4], v[5])] = v[6];
    }
    std::fclose(f);
}

Config default_for(const Call& c)
{
    if (c.prec != FE_FP64) return Config();
    if (c.mode == FE_MODE_PREEVAL && c.form == ELASTICITY) {
        // resident workgroups per CU by matrix width: the fewer tiles write
        // partial lines at once, the more of them the L2 merges (measured on
        // MI355X; the autotuner may find a better count for a given shape)
        Config x;
        x.grid_per_cu = preeval_elast_grid_per_cu(c.cell, c.tables->nb);
        return x;
    }
    if (c.mode == FE_MODE_PREEVAL && c.nf > 0) return Config();
    if (c.mode == FE_MODE_PREEVAL) return default_preeval_config(c.form, c.tables->nb * c.tables->nb);
    // float64 matrix-core Gram kernel where the point loop is not hoisted
    // (with one point per element the VALU kernel is faster).  For the scalar
    // forms it wins where its tiles are well filled (measured on MI355X over
    // every cell, degree and nf = 0..2): mass from n = 10, Helmholtz (four
    // rows per point) with three tiles or one nearly full tile.
    if (vec_p1_eligible(c)) {
        // degree 1 on a simplex: the hoisted streaming kernel; two resident
        // blocks per CU measured fastest on MI355X (the grid's store window
        // stays small)
        Config x;
        x.variant = 2;
        x.grid_per_cu = 2;
        return x;
    }
    bool gram = gram64_eligible(c) && !q_invariant(c);
    if (gram && !is_vector_form(c.form)) {
        const int ns = c.tables->nb;
        gram = c.form == MASS ? ns >= 10 : (ns > 32 || (ns >= 13 && ns <= 16));
    }
    if (gram) {
        Config x;
        x.variant = 1;
        return x;
    }
    return default_quad_config(c.form, c.cell, c.degree, c.tables->nq, c.pointgeo);
}

std::vector<Config> candidates(const Call& c)
{
    std::vector<Config> out;
    const Config base = default_for(c);
    if (c.prec != FE_FP64) {
        for (int g : {4, 8, 16}) {
            Config x = base;
            x.grid_per_cu = g;
            out.push_back(x);
        }
        return out;
    }
    if (c.mode == FE_MODE_PREEVAL && (c.nf > 0 || c.form == ELASTICITY)) {
        for (int g : {1, 2, 4, 8, 16}) {
            Config x;
            x.grid_per_cu = g;
            out.push_back(x);
        }
        return out;
    }
    if (c.mode == FE_MODE_PREEVAL) {
        const int nn = c.tables->nb * c.tables->nb, mm = preeval_mm(c.form);
        // streaming shapes: largest step that fits 4, 8 (mass 16) slots per thread
        for (int block : {256, 320, 384, 448, 512}) {
            for (int smm : {4, 8, 16}) {
                if (smm == 16 && c.form != MASS) continue;
                const int epi = std::min(block, smm * block / nn);
                if (epi < 1 || preeval_stream_mm(c.form, epi * nn, block) != smm) continue;
                if ((double)(epi * nn) / (smm * block) < 0.75) continue;
                Config x;
                x.block = block;
                x.epi = epi;
                x.variant = 1;
                x.grid_per_cu = 8;   // capped by occupancy at launch
                for (int t : {0, 4, 8, 16, 24, 32}) {
                    x.chunk = t * epi;
                    out.push_back(x);
                }
            }
        }
        for (int block : {256, 320, 384, 512}) {
            for (int epi : {1, 2, 4, 8, 16, 32, 64}) {
                const int m = (epi * nn + block - 1) / block;
                if (m > 2 * mm || (epi > 1 && epi * nn > 8 * block * mm)) continue;
                const double waste = 1.0 - (double)(epi * nn) / (m * block);
                if (waste > 0.2) continue;
                for (int per : {16, 256}) {
                    Config x;
                    x.block = block;
                    x.epi = epi;
                    x.chunk = epi * std::max(1, per / epi);
                    x.grid_per_cu = 8;
                    out.push_back(x);
                }
            }
        }
        if (out.empty()) out.push_back(base);
        return out;
    }
    if (vec_p1_eligible(c))
        for (int g : {2, 4, 8}) {
            Config x;
            x.variant = 2;
            x.grid_per_cu = g;
            out.push_back(x);
        }
    if (gram64_eligible(c))
        for (int g : {2, 4, 8}) {
            Config x;
            x.variant = 1;
            x.grid_per_cu = g;
            out.push_back(x);
        }
    const Config vb = default_quad_config(c.form, c.cell, c.degree, c.tables->nq, c.pointgeo);
    for (int div : {1, 2, 4}) {
        for (int g : {4, 8}) {
            Config x = vb;
            x.eb = std::max(1, vb.eb / div);
            const int D = cell_dim(c.cell), ns = c.tables->nb;
            const int ppt = ns * D + (c.form == HYPERELASTIC ? ns * D + 9 : 0) + 3;
            const size_t per_q = ((size_t)ns + (size_t)x.eb * ppt) * 8;
            x.qc = std::max(1, std::min(c.tables->nq, (int)((QUAD_LDS_BUDGET - x.eb * 96) / per_q)));
            x.grid_per_cu = g;
            out.push_back(x);
        }
    }
    return out;
}

}  // namespace

void lookup_config(const Call& c, Config* cfg)
{
    if (!c.pointgeo) {
        std::lock_guard<std::mutex> lk(g_tmu);
        load_file_locked();
        auto it = g_tuned.find(key_of(c));
        if (it != g_tuned.end() && check_config(c, it->second) == FE_OK) {
            *cfg = it->second;
            return;
        }
    }
    *cfg = default_for(c);
}

bool tuned_mode(int form, int cell, int degree, int qdeg, int prec, int nf, int* mode)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    load_file_locked();
    auto it = g_mode.find(ModeKey(form, cell, degree, qdeg, prec, nf));
    if (it == g_mode.end()) return false;
    *mode = it->second;
    return true;
}

int resolve_call(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                 const double* coeff_dofs, double* out_A, const fe_options_t* opt, Call* c, int lookup_only);

namespace {

// Times every valid candidate shape of the call\"s kernel (a warm-up launch,
// then three timed ones) and stores the fastest in the cache.
int tune_call(const Call& c, double* best_out, Config* best_cfg_out)
{
    std::vector<Config> cands;
    for (const Config& x : candidates(c))
        if (check_config(c, x) == FE_OK) cands.push_back(x);
    if (cands.empty()) return FE_EINVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_hip_error(hipErrorUnknown, "autotune events");
    double best = 1e30;
    Config best_cfg = cands[0];
    int rc = FE_OK;
    for (const Config& x : cands) {
        rc = launch_call(c, x);   // warm-up
        if (rc) break;
        hipError_t e = hipEventRecord(e0, c.stream);
        for (int r = 0; r < 3 && e == hipSuccess && rc == FE_OK; ++r) rc = launch_call(c, x);
        if (e == hipSuccess) e = hipEventRecord(e1, c.stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = set_hip_error(e, "autotune timing");
            break;
        }
        if (rc) break;
        if (ms / 3.0 < best) {
            best = ms / 3.0;
            best_cfg = x;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tmu);
    load_file_locked();
    g_tuned[key_of(c)] = best_cfg;
    const char* path = std::getenv("FE_AUTOTUNE_CACHE");
    if (path) {
        FILE* f = std::fopen(path, "a");
        if (f) {
            std::fprintf(f,
                         "{\"form\": %d, \"cell\": %d, \"degree\": %d, \"qdeg\": %d, \"mode\": %d, "
                         "\"precision\": %d, \"block\": %d, \"epi\": %d, \"chunk\": %d, \"eb\": %d, \"qc\": %d, "
                         "\"grid_per_cu\": %d, \"variant\": %d, \"nf\": %d, \"ms\": %.6f}\n",
                         c.form, c.cell, c.degree, c.qdeg, c.mode, c.prec, best_cfg.block, best_cfg.epi,
                         best_cfg.chunk, best_cfg.eb, best_cfg.qc, best_cfg.grid_per_cu, best_cfg.variant, c.nf, best);
            std::fclose(f);
        }
    }
    *best_out = best;
    *best_cfg_out = best_cfg;
    return FE_OK;
}

void record_mode(const Call& c, int mode)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_mode[ModeKey(c.form, c.cell, c.degree, c.qdeg, c.prec, c.nf)] = mode;
    const char* path = std::getenv("FE_AUTOTUNE_CACHE");
    if (path) {
        FILE* f = std::fopen(path, "a");
        if (f) {
            std::fprintf(f,
                         "{\"form\": %d, \"cell\": %d, \"degree\": %d, \"qdeg\": %d, \"precision\": %d, "
                         "\"nf\": %d, \"tuned_mode\": %d}\n",
                         c.form, c.cell, c.degree, c.qdeg, c.prec, c.nf, mode);
            std::fclose(f);
        }
    }
}

}  // namespace

}  // namespace fe

using namespace fe;

extern "C" int fe_autotune(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                           const double* coeff_dofs, double* out_A, const fe_options_t* opt, double* best_ms,
                           fe_shape_t* best_shape)
{
    if (n_elems < 1) return FE_EINVAL;
    Call c;
    int rc = resolve_call(form, cell, degree, n_elems, coords, coeff_dofs, out_A, opt, &c, 0);
    if (rc) return rc;
    if (c.pointgeo) return FE_ENOTSUP;   // per-point maps use the built-in shape
    // the kernel fe_assemble_local runs: split precisions at degree 1 on a
    // simplex take the float64 hoisted kernel
    if (c.prec != FE_FP64 && q_invariant(c)) c.prec = FE_FP64;
    double best = 0.0;
    Config best_cfg;
    rc = tune_call(c, &best, &best_cfg);
    if (rc) return rc;
    // an AUTO request of a form with two legal modes: time the other mode as
    // well (with its own best shape), and let later AUTO calls of the variant
    // run the faster one -- operation counts and run times need not agree
    // (Sec. 7.2); fe_plan keeps reporting Algorithm 3's choice
    fe_options_t o;
    if (opt) o = *opt;
    else fe_options_init(&o);
    if (o.mode == FE_MODE_AUTO && c.prec == FE_FP64 && c.form != HYPERELASTIC) {
        Call c2 = c;
        c2.mode = c.mode == FE_MODE_PREEVAL ? FE_MODE_QUADRATURE : FE_MODE_PREEVAL;
        c2.mass_pre = 0;
        double best2 = 0.0;
        Config cfg2;
        if (tune_call(c2, &best2, &cfg2) == FE_OK) {
            const bool other = best2 < best;
            record_mode(c, other ? c2.mode : c.mode);
            if (other) {
                c = c2;
                best = best2;
                best_cfg = cfg2;
            }
        }
        (void)hipGetLastError();
    }
    if (best_ms) *best_ms = best;
    if (best_shape) {
        best_shape->kernel = c.prec != FE_FP64                  ? 4
                             : c.mode == FE_MODE_PREEVAL && (c.nf || c.form == ELASTICITY) ? 0   // a single kernel
                             : c.mode == FE_MODE_PREEVAL         ? (best_cfg.variant ? 2 : 1)
                                                                 : (best_cfg.variant == 2 ? 5 : best_cfg.variant ? 4 : 3);
        best_shape->block = best_cfg.block;
        best_shape->epi = best_cfg.epi;
        best_shape->chunk = best_cfg.chunk;
        best_shape->eb = best_cfg.eb;
        best_shape->qc = best_cfg.qc;
        best_shape->grid_per_cu = best_cfg.grid_per_cu;
    }
    return FE_OK;
}

extern "C" void fe_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_tuned.clear();
    g_mode.clear();
}
