// Internal host-side interfaces of the local-assembly library.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "fe_common.hpp"

namespace fe {

struct PreevalArgs;
struct QuadArgs;
struct SplitArgs;

// quadrature.cpp
int build_rule(int cell, int qdeg, std::vector<double>& X, std::vector<double>& W);

// tabulate.hip
hipError_t launch_tabulate(int cell, int p, int nq, const double* X, double* phi, double* dphi, hipStream_t s);
hipError_t launch_preeval_tables(int nq, int nb, int d, const double* W, const double* phi, const double* dphi,
                                 double* R, hipStream_t s);
hipError_t launch_geometry(int cell, int64_t E, const double* coords, double* det, double* kinv, hipStream_t s);

// assemble_*.hip
hipError_t launch_preeval(int form, int cell, const PreevalArgs& a, int block, int grid, hipStream_t s);
// streaming pre-evaluated kernel: persistent grid of at most max_per_cu
// resident blocks per CU
hipError_t launch_preeval_stream(int form, int cell, const PreevalArgs& a, int block, int max_per_cu, int cus,
                                 hipStream_t s);
// preeval_coef.hip: pre-evaluation with nf pre-multiplying coefficient functions
hipError_t launch_coef_tables(int nq, int nb, int d, int nf, int iota, int nr, const double* W, const double* phi,
                              const double* dphi, const int* combos, double* R, hipStream_t s);
// Output and coefficient layout of the coefficient pre-evaluation: scalar
// forms write [E][nb][nb] with the functions' DOFs [E][nf][nb]; for the
// hyperelastic trace monomial each entry, times `scale` (mu), goes to the
// vec_d diagonal blocks of [E][vec_d nb][vec_d nb], and an element's record
// is `cstride` doubles with the functions' DOFs from `coff`.
struct CoefOut {
    int vec_d = 0;
    double scale = 1.0;
    int cstride = 0;   // 0: nf * nb
    int coff = 0;
};
// geometry-tensor entries [r_lo, r_hi) only (r_hi < 0: all), adding to out
// when accumulate is set (the pre-evaluated half of a mixed plan)
hipError_t launch_preeval_coef(int form, int cell, const double* coords, const double* coeff, double* out,
                               int* status, const double* R, const int* combos, int64_t E, int nb, int nf,
                               int iota, int grid_per_cu, int cus, hipStream_t s, int r_lo = 0, int r_hi = -1,
                               int accumulate = 0, const CoefOut& o = CoefOut());
size_t preeval_coef_lds_bytes(int form, int cell, int ntp, int nf, int nb);
// elasticity pre-evaluated with its P1 Lame fields and nf functions expanded:
// tables T[((l * iota + S) * d + a) * d + b][j][k] and the kernel
hipError_t launch_elast_coef_tables(int nq, int nb, int d, int nc, int nf, int iota, const double* W,
                                    const double* phi, const double* psi, const double* dphi, const int* combos,
                                    double* T, hipStream_t s);
hipError_t launch_preeval_elast_coef(int cell, const double* coords, const double* coeff, double* out, int* status,
                                     const double* T, const int* combos, int64_t E, int nb, int nf, int iota,
                                     int grid_per_cu, int cus, hipStream_t s);
size_t preeval_elast_coef_lds_bytes(int cell, int nt, int nf, int nb);
// preeval_elast.hip: pre-evaluated linear elasticity with P1 Lame fields
hipError_t launch_elast_tables(int nq, int ns, int d, int nc, const double* W, const double* psi, const double* dphi,
                               double* T, hipStream_t s);
// doubles in the blocked elasticity tables of a cell with n_s basis functions
size_t elast_table_doubles(int cell, int ns);
hipError_t launch_preeval_elast(int cell, const double* coords, const double* coeff, double* out, int* status,
                                const double* T, int64_t E, int ns, int grid_per_cu, int cus, hipStream_t s);
// default resident workgroups (four wavefronts each) per CU of k_preeval_elast
int preeval_elast_grid_per_cu(int cell, int ns);
hipError_t launch_quad_mass(int cell, int kb, const QuadArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t launch_quad_helmholtz(int cell, int kb, const QuadArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t launch_quad_elasticity(int cell, int kb, const QuadArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t launch_quad_hyperelastic(int cell, int kb, const QuadArgs& a, int grid, size_t lds, hipStream_t s);
inline hipError_t launch_quad(int form, int cell, int kb, const QuadArgs& a, int grid, size_t lds, hipStream_t s)
{
    switch (form) {
    case MASS: return launch_quad_mass(cell, kb, a, grid, lds, s);
    case HELMHOLTZ: return launch_quad_helmholtz(cell, kb, a, grid, lds, s);
    case ELASTICITY: return launch_quad_elasticity(cell, kb, a, grid, lds, s);
    default: return launch_quad_hyperelastic(cell, kb, a, grid, lds, s);
    }
}
hipError_t launch_split_elasticity_fp32(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds,
                                       hipStream_t s);
hipError_t launch_split_elasticity_bf16x3(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds,
                                         hipStream_t s);
hipError_t launch_split_hyperelastic_fp32(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds,
                                         hipStream_t s);
hipError_t launch_split_hyperelastic_bf16x3(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds,
                                           hipStream_t s);
hipError_t launch_gram64_elasticity(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds,
                                    hipStream_t s);
hipError_t launch_gram64_hyperelastic(int cell, int p, int nqp, const SplitArgs& a, int grid, size_t lds,
                                      hipStream_t s);
// assemble_gram64_scalar.hip: float64 matrix-core quadrature of mass and Helmholtz
struct GramScalarArgs {
    const double* coords;
    const double* coeff;        // nf coefficient functions [E][nf][ns]
    double* out;
    int* status;
    const double* W;            // [nq]
    const double* phi;          // [nq][ns]
    const double* dphi;         // [nq][ns][d]
    const double* dpsi_grad;    // [nq][nv][d] (per-point prism geometry)
    int64_t E;
    int nq, nf;
    int skip;                   // bit 0: no value rows, bit 1: no gradient rows
    int pointgeo;
    int nt;
};
hipError_t launch_gram64_scalar(int form, int cell, int p, const GramScalarArgs& a, int grid, hipStream_t s);
size_t gram64_scalar_lds_bytes(int cell, int p);
int gram64_scalar_elems_per_block(int cell);
// assemble_vec_p1.hip: the vector forms at degree 1 on simplices (every
// gradient constant, the point loop hoisted), float64
struct VecP1Args {
    const double* coords;
    const double* coeff;
    double* out;
    int* status;
    const double* W;            // [nq]
    const double* psi;          // [nq][nv] P1 basis at the points
    const double* dphi;         // [nq][ns][d] (the first point's gradients are used)
    int64_t E;
    int nq;
    int nt;
    double mu, lam;
};
hipError_t launch_vec_p1(int form, int cell, const VecP1Args& a, int grid, hipStream_t s);
size_t vec_p1_lds_bytes(int cell);
int vec_p1_elems_per_block();
// prec: 1 = fp32 operands, 2 = bf16 hi/lo split
inline hipError_t launch_split(int form, int cell, int p, int prec, int nqp, const SplitArgs& a, int grid,
                               size_t lds, hipStream_t s)
{
    if (form == ELASTICITY)
        return prec == 1 ? launch_split_elasticity_fp32(cell, p, nqp, a, grid, lds, s)
                         : launch_split_elasticity_bf16x3(cell, p, nqp, a, grid, lds, s);
    return prec == 1 ? launch_split_hyperelastic_fp32(cell, p, nqp, a, grid, lds, s)
                     : launch_split_hyperelastic_bf16x3(cell, p, nqp, a, grid, lds, s);
}

// slot tile of the pre-evaluated kernel (registers per pass) per form
constexpr int preeval_mm(int form) { return form == MASS ? 16 : 8; }
// Slots per thread of the streaming kernel for `slots` = epi * n^2 entries
// per step: 4, 8 (or 16 for the one-table mass form); 0 when a step does
// not fit in registers (the tiled kernel is used then).
constexpr int preeval_stream_mm(int form, int slots, int block)
{
    return slots <= 4 * block ? 4 : slots <= 8 * block ? 8 : (form == MASS && slots <= 16 * block) ? 16 : 0;
}
// (upper bound: a geometry group is at most block / epi steps)
inline size_t preeval_stream_lds_bytes(int form, int cell, int block, int epi)
{
    return (size_t)2 * (block / epi) * epi * n_tables(form, cell) * sizeof(double);
}
// k-block width of the quadrature kernel
constexpr int quad_kb(int cell, int p)
{
    return cell == TET ? (p == 1 ? 4 : 5) : (p <= 2 ? 3 : 5);
}
constexpr int QUAD_BLOCK = 256;
constexpr int SPLIT_BLOCK = 256;
constexpr size_t QUAD_LDS_BUDGET = 48 * 1024;

// Reference tables of one (cell, degree, rule), device resident.
struct RefTables {
    int cell = 0, p = 0, qdeg = 0, nq = 0, nb = 0, d = 0, nv = 0;
    std::vector<double> X, W;          // host copy of the rule
    double* dX = nullptr;              // [nq][d]
    double* dW = nullptr;              // [nq]
    double* dphi = nullptr;            // [nq][nb]
    double* ddphi = nullptr;           // [nq][nb][d]
    double* dpsi = nullptr;            // [nq][nv] P1 (prism P1 x P1) basis
    double* ddpsi = nullptr;           // [nq][nv][d] its gradients (the vertex map's)
    double* dR = nullptr;              // [1 + d(d+1)/2][nb][nb] pre-evaluated tensors
};

// Tables of the pre-evaluation with nf coefficient functions: the sorted
// multisets S of nf basis indices and R[(r, S)][j][k], device resident.
// For elasticity (nf = 0, the P1 Lame fields): iota = n_c, no multisets,
// and R = T[(l, a, b)][j][k].
struct CoefTables {
    int iota = 0, nt = 0;
    int* dCombos = nullptr;   // [iota][nf]
    double* dR = nullptr;     // [nt][nb][nb]
};

// felocal.cpp
int get_tables(int cell, int p, int qdeg, hipStream_t s, const RefTables** out);
int find_tables(int cell, int p, int qdeg, const RefTables** out);
int get_coef_tables(int form, int cell, int p, int qdeg, int nf, hipStream_t s, const CoefTables** out);
int device_cus();
size_t device_lds_per_cu();
size_t device_l2_bytes();
int set_hip_error(hipError_t e, const char* where);

// Launch configuration of one variant.
struct Config {
    int block = 256;
    int epi = 1;      // pre-evaluated: elements per step
    int chunk = 256;  // pre-evaluated: elements per tile (streaming: per visit, 0 = automatic)
    int eb = 1;       // quadrature: elements per tile
    int qc = 1;       // quadrature: points per LDS chunk
    int grid_per_cu = 8;
    int variant = 0;  // pre-evaluated: 1 = streaming, 0 = tiled kernel;
                      // quadrature: 1 = float64 matrix-core Gram kernel, 0 = VALU kernel
};

// pre-evaluated kernel: streaming when a step fits in registers, else tiled
Config default_preeval_config(int form, int nn);
Config default_preeval_tiled_config(int nn, int mm);
// LDS of one pre-evaluated tile: geometry tensors plus the staged coordinates
inline size_t preeval_lds_bytes(int form, int cell, int chunk)
{
    return (size_t)chunk * (n_tables(form, cell) + cell_nv(cell) * cell_dim(cell)) * sizeof(double);
}
Config default_quad_config(int form, int cell, int p, int nq, int pointgeo = 0);
size_t quad_lds_bytes(int form, int cell, int ns, int eb, int qc, int pointgeo = 0);

// One resolved assembly call.
struct Call {
    int form = 0, cell = 0, degree = 1, qdeg = 2;
    int mode = 0;       // FE_MODE_PREEVAL or FE_MODE_QUADRATURE
    int nf = 0;         // pre-multiplying coefficient functions
    int pointgeo = 0;   // J at every point: 1 the vertex map of a (non-affine)
                        // prism, 2 the P2 coordinate field of a curved simplex
    const RefTables* map_tables = nullptr;   // pointgeo 2: the P2 tables at the rule
    int shape[7] = {0, 0, 0, 0, 0, 0, 0};   // caller's launch-shape override (fe_shape_t order)
    int mass_pre = 0;   // Helmholtz quadrature: bit 0 mass monomial pre-evaluated,
                        // bit 1 gradient monomial pre-evaluated; hyperelastic
                        // with nf > 0: bit 1 the trace monomial pre-evaluated
    int prec = 0;       // fe_precision_t
    int64_t E = 0;
    const double* coords = nullptr;
    const double* coeff = nullptr;
    double* out = nullptr;
    int* status = nullptr;
    double mu = 1.0, lam = 10.0;
    hipStream_t stream = nullptr;
    const RefTables* tables = nullptr;
};

int launch_call(const Call& c, const Config& cfg);
int add_coef_monomial(const Call& c, const Config& cfg);
int store_mode();
// configuration from the autotune cache, else the built-in default
void lookup_config(const Call& c, Config* cfg);
// the mode fe_autotune measured faster for an AUTO request of this variant
bool tuned_mode(int form, int cell, int degree, int qdeg, int prec, int nf, int* mode);
// the float64 matrix-core kernel serves this call (vector form, n <= 32,
// at most 32 contraction points)
bool gram64_eligible(const Call& c);
// the hoisted degree-1 vector kernel serves this call (float64 quadrature,
// vector form at degree 1 on a simplex)
bool vec_p1_eligible(const Call& c);
// P1 vector form on a simplex: every gradient is constant over the element,
// so the point loop is hoisted (generalised code motion, Sec. 3.2)
bool q_invariant(const Call& c);
// padded point count of the matrix-core kernels for nq contraction points
int split_nqp(int nq);
int gram64_nqp(int nq);
// 0 when the kernel selected by c can take cfg, else FE_EINVAL
int check_config(const Call& c, const Config& cfg);
// automatic shape with the caller's override applied and checked
int final_config(const Call& c, Config* cfg);
size_t device_lds_per_block();
// unloads every kernel module fe_assemble_form compiled and forgets the
// kernels chosen per call (no generated kernel may be in flight)
void release_generated();

}  // namespace fe
