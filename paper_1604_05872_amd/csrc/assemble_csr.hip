// Local and global assembly in one pass for the pre-evaluated forms.
//
// Global assembly (Sec. 2) adds every element matrix into the matrix of the
// continuous space; for mass and Helmholtz the element matrix is the
// pre-evaluated contraction A_e[j][k] = sum_r c_r(e) R_r[j][k] (Sec. 3.3,
// Algorithm 2), a few flops per entry.  Writing A_e to memory and reading it
// back for the insertion would cost more than forming it again, so this pass
// forms each entry where it is added: the insertion kernel's row-by-row
// schedule (one lane group per row, the row's elements in increasing order,
// values accumulated in LDS and stored contiguously), with the entry
// computed from the element's geometry tensor (precomputed, 64 B per
// element) and the reference tables (staged in LDS once per workgroup).  The
// arithmetic of an entry is that of the pre-evaluated local kernels, term by
// term, so the result equals fe_csr_insert of fe_assemble_local's output bit
// for bit.
#include <hip/hip_runtime.h>

#include <mutex>

#include "csr.hpp"
#include "felocal.h"
#include "internal.hpp"
#include "preeval.hpp"

namespace fe {

int resolve_call(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                 const double* coeff_dofs, double* out_A, const fe_options_t* opt, Call* c, int lookup_only);

namespace {

constexpr int GEO_STRIDE = 8;              // doubles per element of the geometry workspace
constexpr size_t CSR_TABLE_LDS_MAX = 96 * 1024;
constexpr int FUSED_MAX_WAVES = 16;        // wavefronts per workgroup

// Geometry tensor of every element (the pre-evaluated kernels' c(e)); a
// flagged element gets NaN and is counted once.
template <int FORM, int CELL>
__global__ void k_csr_geometry(int64_t E, const double* __restrict__ coords, double* __restrict__ geo,
                               int* __restrict__ status)
{
    constexpr int NT = n_tables(FORM, CELL);
    constexpr int NVD = cell_nv(CELL) * cell_dim(CELL);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double c[NT];
    if (preeval_coeffs<FORM, CELL>(coords + e * NVD, c)) {
#pragma unroll
        for (int r = 0; r < NT; ++r) c[r] = __builtin_nan("");
        if (status) atomicAdd(status, 1);
    }
#pragma unroll
    for (int r = 0; r < GEO_STRIDE; ++r) geo[e * GEO_STRIDE + r] = r < NT ? c[r] : 0.0;
}


// Workgroups of `waves` independent wavefronts that share the tables in LDS.
// Wavefront w of workgroup b takes visits of VISIT_ROWS rows, W lanes per
// row (64 / W rows side by side), KPL entries per lane, B elements per row
// per batch of loads.
template <int FORM, int CELL, int W, int KPL, int B>
__global__ __launch_bounds__(1024) void k_csr_preeval(int64_t N, int n, const int64_t* __restrict__ row_ptr,
                                                      const int64_t* __restrict__ pair_ptr,
                                                      const uint32_t* __restrict__ list,
                                                      const uint16_t* __restrict__ pos,
                                                      const double* __restrict__ geo,
                                                      const double* __restrict__ tables,
                                                      double* __restrict__ vals, int round_cap, int visit_pairs)
{
    // an entry is rounded before it is added, as when it is stored first
#pragma clang fp contract(off)
    constexpr int NT = n_tables(FORM, CELL);
    constexpr int RR = CSR_WAVE / W;
    extern __shared__ double smem[];
    const int nn = n * n;
    const int waves = blockDim.x / CSR_WAVE;
    const int wid = threadIdx.x / CSR_WAVE;
    const int t = threadIdx.x % CSR_WAVE;
    const int g = t / W;
    const int kl = t % W;
    double* sR = smem;   // [NT][n][n]
    const size_t per_wave = ((size_t)round_cap * 8 + (size_t)visit_pairs * 4 + 7) / 8;   // doubles
    double* acc = smem + (size_t)NT * nn + wid * per_wave;
    uint32_t* seg = reinterpret_cast<uint32_t*>(acc + round_cap);
    for (int i = threadIdx.x; i < NT * nn; i += blockDim.x) sR[i] = tables[i];
    __syncthreads();
    // from here on the wavefronts are independent
    const int G = gridDim.x;
    const int b = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const int64_t gw = (int64_t)b * waves + wid;
    const int64_t GW = (int64_t)G * waves;
    for (int64_t v0 = gw * VISIT_ROWS; v0 < N; v0 += GW * VISIT_ROWS) {
        const int nv = (int)(N - v0 < VISIT_ROWS ? N - v0 : VISIT_ROWS);
        int64_t my_rp = 0, my_pp = 0;
        if (t <= nv) {
            my_rp = row_ptr[v0 + t];
            my_pp = pair_ptr[v0 + t];
        }
        const int64_t P0 = __shfl(my_pp, 0);
        const int np = (int)(__shfl(my_pp, nv) - P0);
        wave_sync();   // the previous visit's reads of seg are done
        for (int i = t; i < np; i += CSR_WAVE) seg[i] = list[P0 + i];
        wave_sync();
        for (int r0 = 0; r0 < nv; r0 += RR) {
            const int nr = nv - r0 < RR ? nv - r0 : RR;
            const int64_t vb = __shfl(my_rp, r0);
            const int V = (int)(__shfl(my_rp, r0 + nr) - vb);
            for (int i = t; i < V; i += CSR_WAVE) acc[i] = 0.0;
            const int li = r0 + g;   // < VISIT_ROWS
            const int64_t rp = __shfl(my_rp, li);
            const int64_t pp = __shfl(my_pp, li);
            const int64_t pe = __shfl(my_pp, li + 1);
            const bool okr = g < nr;
            const int off = okr ? (int)(rp - vb) : 0;
            const int cnt = okr ? (int)(pe - pp) : 0;
            const int lp = (int)(pp - P0);
            int cmax = cnt;
            for (int o = CSR_WAVE / 2; o > 0; o >>= 1) {
                const int x = __shfl_xor(cmax, o);
                cmax = x > cmax ? x : cmax;
            }
            wave_sync();
            for (int s0 = 0; s0 < cmax; s0 += B) {
                // unconditional loads (see k_csr_insert): a slot past the row's
                // last element re-reads that element, a lane past n entry n - 1
                int q[B][KPL];
                double gm[B][NT];
                int jn[B];
#pragma unroll
                for (int u = 0; u < B; u++) {
                    const int sl = s0 + u < cnt ? lp + s0 + u : cnt > 0 ? lp + cnt - 1 : 0;
                    const uint32_t ej = np > 0 ? seg[sl] : 0u;
                    const uint32_t e = ej / (uint32_t)n;
                    jn[u] = (int)(ej - e * (uint32_t)n) * n;
                    const uint64_t pbase = (uint64_t)(np > 0 ? P0 + sl : 0) * (uint32_t)n;
#pragma unroll
                    for (int kk = 0; kk < KPL; kk++) {
                        const int k = kl + W * kk < n ? kl + W * kk : n - 1;
                        q[u][kk] = pos[pbase + k];
                    }
                    const double* gp = geo + (uint64_t)e * GEO_STRIDE;
#pragma unroll
                    for (int r = 0; r < NT; r++) gm[u][r] = gp[r];
                }
#pragma unroll
                for (int u = 0; u < B; u++) {
                    if (s0 + u < cnt) {
#pragma unroll
                        for (int kk = 0; kk < KPL; kk++) {
                            const int k = kl + W * kk;
                            if (k < n) {
                                const double* R = sR + jn[u] + k;
                                double x = gm[u][0] * R[0];
#pragma unroll
                                for (int r = 1; r < NT; ++r) x = fma(gm[u][r], R[r * nn], x);
                                acc[off + q[u][kk]] += x;
                            }
                        }
                    }
                    // the next element of a row may add to the same entries from other lanes
                    wave_sync();
                }
            }
            for (int i = t; i < V; i += CSR_WAVE) vals[vb + i] = acc[i];
            wave_sync();
        }
    }
}

template <int FORM, int CELL, int W, int KPL, int B>
hipError_t launch_fused(const fe_csr* c, const double* geo, const double* tables, double* vals, int round_cap,
                        hipStream_t s)
{
    constexpr int NT = n_tables(FORM, CELL);
    const size_t tab = sizeof(double) * (size_t)NT * c->n * c->n;
    const int vp = c->visit_pairs > 0 ? c->visit_pairs : 1;
    const size_t per_wave = 8 * (((size_t)round_cap * 8 + (size_t)vp * 4 + 7) / 8);
    const size_t limit = device_lds_per_block();
    int waves = FUSED_MAX_WAVES;
    while (waves > 1 && tab + waves * per_wave > limit) waves--;
    if (tab + waves * per_wave > limit) return hipErrorInvalidConfiguration;
    const size_t lds = tab + waves * per_wave;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_csr_preeval<FORM, CELL, W, KPL, B>, waves * CSR_WAVE,
                                                     lds) != hipSuccess ||
        occ <= 0)
        occ = 1;
    const int64_t visits = (c->N + VISIT_ROWS - 1) / VISIT_ROWS;
    int64_t grid = (int64_t)device_cus() * occ;
    if (grid * waves > visits) grid = (visits + waves - 1) / waves;
    if (grid < 1) grid = 1;
    k_csr_preeval<FORM, CELL, W, KPL, B><<<(unsigned)grid, waves * CSR_WAVE, lds, s>>>(
        c->N, c->n, c->row_ptr, c->pair_ptr, c->list, c->pos, geo, tables, vals, round_cap, vp);
    return hipGetLastError();
}

// Lanes per row: narrow groups with several entries per lane put several
// rows side by side in a wavefront, so that more rows have their loads in
// flight at once (each row's chain of dependent loads is what bounds the pass).
template <int FORM, int CELL>
hipError_t fused_shape(const fe_csr* c, const double* geo, const double* tables, double* vals, hipStream_t s);

// The measured shape first; where its rounds do not fit in LDS beside the
// tables (rows shared by very many elements), one row per round (the
// smallest round).  hipErrorInvalidConfiguration when even that does not fit.
template <int FORM, int CELL>
hipError_t fused_for_n(const fe_csr* c, const double* geo, const double* tables, double* vals, hipStream_t s)
{
    const hipError_t e = fused_shape<FORM, CELL>(c, geo, tables, vals, s);
    if (e != hipErrorInvalidConfiguration) return e;
    const int cap0 = c->round_len[0] > 0 ? c->round_len[0] : 1;
    if (c->n <= 64) return launch_fused<FORM, CELL, 64, 1, 2>(c, geo, tables, vals, cap0, s);
    return launch_fused<FORM, CELL, 64, 2, 2>(c, geo, tables, vals, cap0, s);
}

template <int FORM, int CELL>
hipError_t fused_shape(const fe_csr* c, const double* geo, const double* tables, double* vals, hipStream_t s)
{
    const int n = c->n;
    // lanes per row: 8 up to n = 32 (eight rows side by side; measured on
    // MI355X, Helmholtz tet P2 0.59 -> 0.38 ms and P3 1.75 -> 1.10 ms against
    // 16 lanes), then 16, 32, 64
    const int W = n <= 4 ? 4 : n <= 32 ? 8 : n <= 64 ? 16 : n <= 96 ? 32 : 64;
    int level = 0;
    while ((1 << level) < CSR_WAVE / W) level++;
    const int cap = c->round_len[level] > 0 ? c->round_len[level] : 1;
    // the geometry tensors of B elements sit in registers: fewer per batch
    // for the seven-term Helmholtz tensors
    constexpr int BS = n_tables(FORM, CELL) > 1 ? 4 : 8;
    constexpr int B8 = BS / 2;
    if (n <= 4) return launch_fused<FORM, CELL, 4, 1, BS>(c, geo, tables, vals, cap, s);
    if (n <= 8) return launch_fused<FORM, CELL, 8, 1, BS>(c, geo, tables, vals, cap, s);
    if (n <= 16) return launch_fused<FORM, CELL, 8, 2, B8>(c, geo, tables, vals, cap, s);
    if (n <= 24) return launch_fused<FORM, CELL, 8, 3, B8>(c, geo, tables, vals, cap, s);
    if (n <= 32) return launch_fused<FORM, CELL, 8, 4, B8>(c, geo, tables, vals, cap, s);
    if (n <= 48) return launch_fused<FORM, CELL, 16, 3, BS == 4 ? 3 : 4>(c, geo, tables, vals, cap, s);
    if (n <= 64) return launch_fused<FORM, CELL, 16, 4, BS == 4 ? 2 : 4>(c, geo, tables, vals, cap, s);
    if (n <= 96) return launch_fused<FORM, CELL, 32, 3, 2>(c, geo, tables, vals, cap, s);
    return launch_fused<FORM, CELL, 64, 2, 2>(c, geo, tables, vals, cap, s);
}

// geo: the geometry workspace, [E][GEO_STRIDE] doubles
template <int FORM, int CELL>
hipError_t run_fused(const fe_csr* c, double* geo, const double* coords, const double* tables, double* vals,
                     int* status, hipStream_t s)
{
    const unsigned blocks = (unsigned)((c->E + 255) / 256);
    k_csr_geometry<FORM, CELL><<<blocks, 256, 0, s>>>(c->E, coords, geo, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return fused_for_n<FORM, CELL>(c, geo, tables, vals, s);
}

hipError_t run_fused_form(int form, int cell, const fe_csr* c, double* geo, const double* coords,
                          const double* R, double* values, int* status, hipStream_t s)
{
    if (form == FE_MASS)
        return cell == FE_TRIANGLE      ? run_fused<MASS, TRI>(c, geo, coords, R, values, status, s)
               : cell == FE_TETRAHEDRON ? run_fused<MASS, TET>(c, geo, coords, R, values, status, s)
                                        : run_fused<MASS, PRISM>(c, geo, coords, R, values, status, s);
    return cell == FE_TRIANGLE      ? run_fused<HELMHOLTZ, TRI>(c, geo, coords, R, values, status, s)
           : cell == FE_TETRAHEDRON ? run_fused<HELMHOLTZ, TET>(c, geo, coords, R, values, status, s)
                                    : run_fused<HELMHOLTZ, PRISM>(c, geo, coords, R, values, status, s);
}

// The geometry workspace of fe_assemble_csr_noalloc: file-scope device
// memory (every GPU the library runs on holds its own copy until the process
// ends), so the entry point allocates nothing.  In host code the array's
// name is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr int64_t NOALLOC_MAX_ELEMS = (int64_t)1 << 20;   // 64 MiB of workspace
__device__ __align__(256) double scratch[GEO_STRIDE * NOALLOC_MAX_ELEMS];

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {nullptr};

// the current device's address of `scratch`, or nullptr (error set)
double* scratch_address()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "fe_assemble_csr_noalloc workspace address");
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace fe

extern "C" int fe_assemble_csr(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                               fe_csr_t* csr, double* values, const fe_options_t* opt)
{
    using namespace fe;
    if (!csr) return FE_EINVAL;
    Call c;
    // out_A is not written here: pass values so that argument checks see a buffer
    int rc = resolve_call(form, cell, degree, n_elems, coords, nullptr, values, opt, &c, 0);
    if (rc) return rc;
    if (csr->E != n_elems || csr->n != n_rows(form, cell, degree)) return FE_EINVAL;
    if ((form != FE_MASS && form != FE_HELMHOLTZ) || c.nf != 0 || c.prec != FE_FP64) return FE_ENOTSUP;
    if (n_elems == 0 || csr->nnz == 0) return FE_OK;
    if (c.mode != FE_MODE_PREEVAL) return FE_ENOTSUP;
    const size_t tab = sizeof(double) * (size_t)n_tables(form, cell) * csr->n * csr->n;
    if (tab > CSR_TABLE_LDS_MAX || tab > device_lds_per_block()) return FE_ENOTSUP;
    if (!csr->geo) {
        if (hipMalloc(&csr->geo, sizeof(double) * GEO_STRIDE * (size_t)n_elems) != hipSuccess) {
            (void)hipGetLastError();
            csr->geo = nullptr;
            return FE_ENOMEM;
        }
    }
    const hipError_t e = run_fused_form(form, cell, csr, csr->geo, coords, c.tables->dR, values, c.status, c.stream);
    if (e == hipErrorInvalidConfiguration) return FE_ENOTSUP;   // one row and the tables exceed the LDS
    return e == hipSuccess ? FE_OK : set_hip_error(e, "fe_assemble_csr");
}

extern "C" int fe_assemble_csr_noalloc(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems,
                                       const double* coords, fe_csr_t* csr, double* values, const fe_options_t* opt)
{
    using namespace fe;
    if (!csr) return FE_EINVAL;
    if (n_elems > NOALLOC_MAX_ELEMS) return FE_ENOMEM;
    Call c;
    // the reference tables must already be cached: look them up, never build
    int rc = resolve_call(form, cell, degree, n_elems, coords, nullptr, values, opt, &c, /*lookup_only=*/1);
    if (rc) return rc;
    if (csr->E != n_elems || csr->n != n_rows(form, cell, degree)) return FE_EINVAL;
    if ((form != FE_MASS && form != FE_HELMHOLTZ) || c.nf != 0 || c.prec != FE_FP64) return FE_ENOTSUP;
    if (n_elems == 0 || csr->nnz == 0) return FE_OK;
    if (c.mode != FE_MODE_PREEVAL) return FE_ENOTSUP;
    const size_t tab = sizeof(double) * (size_t)n_tables(form, cell) * csr->n * csr->n;
    if (tab > CSR_TABLE_LDS_MAX || tab > device_lds_per_block()) return FE_ENOTSUP;
    double* geo = scratch_address();
    if (!geo) return FE_EHIP;
    const hipError_t e = run_fused_form(form, cell, csr, geo, coords, c.tables->dR, values, c.status, c.stream);
    if (e == hipErrorInvalidConfiguration) return FE_ENOTSUP;
    return e == hipSuccess ? FE_OK : set_hip_error(e, "fe_assemble_csr_noalloc");
}
