// Float64 matrix-core quadrature for the scalar forms (mass, Helmholtz).
//
// The sharing-eliminated quadrature sum (Sec. 3.2, Algorithm 1) of a scalar
// form is a weighted Gram product over the points:
//     A[j][k] = sum_q w_q ( phi_j(q) phi_k(q) + sum_b g_jb(q) g_kb(q) ),
// w_q = W_q |det J| (times prod_i f_i(X_q) with coefficient functions, Sec.
// 7.1), g = K^T grad_X phi.  With the rows R = (q, c) of the point data
// (c: the value, then the D gradient components) and the signed square roots
// r_q of the weights,
//     A = Z^T diag(sign r) Z,   Z[(q, c)][j] = |r_q| x_c(q, j),
// a dense product whose reduction dimension is the (point, component) index.
// It runs on v_mfma_f64_16x16x4_f64: the n x n matrix is covered by T x T
// tiles of 16 (T = ceil(n / 16)), only the tiles on and above the diagonal
// are computed (A is symmetric), 4 rows R per instruction.  One wavefront
// per element; each lane forms the operand entries the instruction layout
// assigns to it (row R0 + lane / 16, column 16 t + lane % 16), the same
// entry serving as the A operand of tile row t and, with the sign of r_q, as
// the B operand of tile column t.  Per-point data (the roots and, for
// non-affine prisms, each point's K) is staged in LDS for chunks of points.
// The epilogue stores each tile row by row, the mirrored tiles through an LDS
// transpose.  In a mixed plan (Fig. 5) the rows of the pre-evaluated
// monomial are left out (skip) and another kernel adds that monomial.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace fe {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

// wavefronts (elements) per block: the point chunks' tables are staged once
// per block, so prisms (the largest tables) share them among 8; 4 elsewhere
// (measured on MI355X: non-affine Helmholtz prism P3 20.8 -> 13.3 ms with 8,
// tetrahedra with large rules a few per cent slower with 8)
__host__ __device__ constexpr int gs_waves(int cell) { return cell == PRISM ? 8 : 4; }
constexpr int GS_QC = 32;                       // points per staged chunk
constexpr int GS_PT = 12;                       // doubles per staged point: root, K (9), pad
constexpr int GS_TILE_LD = 17;
constexpr int GS_WAVE_DOUBLES = GS_QC * GS_PT + 16 * GS_TILE_LD;

__device__ __forceinline__ void gs_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Operand entries of one step of 4 rows R0 .. R0 + 3 for the lane's row
// R0 + rsub and columns 16 t + m16: z = |r_q| x_c(q, j) (A operand) and
// r_q x_c(q, j) (B operand), zero past the rows or columns.
template <int CELL, int NS, int T, int D>
__device__ __forceinline__ void gs_operands(int R0, int nrows, int NC, int c_first, int rsub, int m16, bool pg,
                                            const double* sQ, const double* sPhi, const double* sDphi, double k00,
                                            double k01, double k02, double k10, double k11, double k12, double k20,
                                            double k21, double k22, double (&za)[T], double (&zb)[T])
{
    const int R = R0 + rsub;
    const bool rv = R < nrows;
    const int qq = rv ? R / NC : 0;
    const int comp = rv ? R - qq * NC + c_first : 0;   // 0: value, 1 + b: gradient b
    const double root = rv ? sQ[qq * GS_PT] : 0.0;
    // column b of K (b = comp - 1), chosen by selects
    const int b = comp > 0 ? comp - 1 : 0;
    double kb0, kb1, kb2;
    if (pg) {
        kb0 = sQ[qq * GS_PT + 1 + b];
        kb1 = sQ[qq * GS_PT + 4 + b];
        kb2 = sQ[qq * GS_PT + 7 + b];
    } else {
        kb0 = b == 0 ? k00 : b == 1 ? k01 : k02;
        kb1 = b == 0 ? k10 : b == 1 ? k11 : k12;
        kb2 = b == 0 ? k20 : b == 1 ? k21 : k22;
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int j = 16 * t + m16;
        const int jj = j < NS ? j : NS - 1;
        double x;
        if (comp == 0) {
            x = sPhi[qq * NS + jj];
        } else {
            const double* gh = sDphi + (qq * NS + jj) * D;
            x = kb0 * gh[0];
            x = fma(kb1, gh[1], x);
            if (D == 3) x = fma(kb2, gh[2], x);
        }
        x = (rv && j < NS) ? x : 0.0;
        za[t] = fabs(root) * x;
        zb[t] = root * x;
    }
}

template <int FORM, int CELL, int P>
__global__ __launch_bounds__(gs_waves(CELL) * 64) void k_gram64_scalar(GramScalarArgs a)
{
    constexpr int GS_WAVES = gs_waves(CELL);
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL), NVD = NV * D;
    // nodes of a per-point map: the prism's vertices, or the P2 nodes of a
    // curved triangle or tetrahedron
    constexpr int NM = CELL == PRISM ? NV : n_scalar(CELL, 2), NMD = NM * D;
    constexpr int NS = n_scalar(CELL, P);
    constexpr int T = (NS + 15) / 16;
    constexpr int NPAIR = T * (T + 1) / 2;
    extern __shared__ double smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* sQ = smem + wave * GS_WAVE_DOUBLES;        // [GS_QC][GS_PT]
    double* sT = sQ + GS_QC * GS_PT;                   // [16][GS_TILE_LD]
    // the chunk's reference tables, shared by the block's wavefronts
    double* sPhi = smem + GS_WAVES * GS_WAVE_DOUBLES;  // [GS_QC][NS]
    double* sDphi = sPhi + GS_QC * NS;                 // [GS_QC][NS][D]
    const int nq = a.nq;
    // active components of the rows: value (unless the mass monomial is
    // pre-evaluated or skipped), then the gradient components
    const bool with_phi = FORM == MASS || !(a.skip & 1);
    const bool with_grad = FORM == HELMHOLTZ && !(a.skip & 2);
    const int NC = (with_phi ? 1 : 0) + (with_grad ? D : 0);
    const int c_first = with_phi ? 0 : 1;              // component id of row c = 0
    const int m16 = lane & 15, rsub = lane >> 4;
    const double nanv = __builtin_nan("");

    // every wavefront of the block runs the same iterations (the tables are
    // staged with block barriers); a wavefront past the last element idles
    for (int64_t base = (int64_t)blockIdx.x * GS_WAVES; base < a.E; base += (int64_t)gridDim.x * GS_WAVES) {
        const int64_t e = base + wave;
        const bool live = e < a.E;
        const int64_t ec = live ? e : a.E - 1;
        const int nvd = a.pointgeo ? NMD : NVD;
        double v[NMD > NVD ? NMD : NVD];
#pragma unroll
        for (int k = 0; k < (NMD > NVD ? NMD : NVD); ++k) v[k] = k < nvd ? a.coords[ec * nvd + k] : 0.0;
        double K[3][3], adet = 0.0, det0 = 0.0;
        int bad = 0;
        if (a.pointgeo) {
            double J[3][3];
            vertex_map_jacobian<NM, D>(v, a.dpsi_grad, J);
            det0 = inverse_small<D>(J, K);
            bad = !(det0 != 0.0 && isfinite(det0));
        } else {
            bad = affine_map<CELL>(v, K, adet);
        }
        v4d acc[NPAIR];
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};

        for (int q0 = 0; q0 < nq; q0 += GS_QC) {
            const int qc = nq - q0 < GS_QC ? nq - q0 : GS_QC;
            // --- the chunk's tables (one contiguous range of each) -------------
            __syncthreads();
            for (int i = threadIdx.x; i < qc * NS; i += GS_WAVES * 64) sPhi[i] = a.phi[(size_t)q0 * NS + i];
            for (int i = threadIdx.x; i < qc * NS * D; i += GS_WAVES * 64) sDphi[i] = a.dphi[(size_t)q0 * NS * D + i];
            __syncthreads();
            // --- per-point data: the signed root of the weight, the point's K
            if (lane < qc) {
                const int q = q0 + lane;
                double* s = sQ + lane * GS_PT;
                double w = a.W[q];
                if (a.pointgeo) {
                    double J[3][3], Kq[3][3];
                    vertex_map_jacobian<NM, D>(v, a.dpsi_grad + (size_t)q * NMD, J);
                    const double det = inverse_small<D>(J, Kq);
                    if (!(det != 0.0 && isfinite(det)) || ((det > 0.0) != (det0 > 0.0))) bad = 1;
                    w *= fabs(det);
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c) s[1 + r * 3 + c] = Kq[r][c];
                } else {
                    w *= adet;
                }
                for (int f = 0; f < a.nf; ++f) {
                    const double* cf = a.coeff + (ec * a.nf + f) * NS;
                    double fv = 0.0;
                    for (int l = 0; l < NS; ++l) fv = fma(cf[l], sPhi[lane * NS + l], fv);
                    w *= fv;
                }
                s[0] = copysign(sqrt(fabs(w)), w);
            }
            gs_wave_sync();
            // --- rows of the chunk, 4 per instruction --------------------------
            // The operands of step i + 1 are formed while the matrix cores run
            // step i (they depend only on LDS data, not on the accumulators).
            const int nrows = qc * NC;
            // the element's K as scalars (no array whose address escapes)
            const double k00 = K[0][0], k01 = K[0][1], k02 = K[0][2], k10 = K[1][0], k11 = K[1][1],
                         k12 = K[1][2], k20 = K[2][0], k21 = K[2][1], k22 = K[2][2];
            const bool pg = a.pointgeo != 0;
            double za[T], zb[T];
            gs_operands<CELL, NS, T, D>(0, nrows, NC, c_first, rsub, m16, pg, sQ, sPhi, sDphi, k00, k01, k02, k10,
                                        k11, k12, k20, k21, k22, za, zb);
#pragma unroll 1
            for (int R0 = 0; R0 < nrows; R0 += 4) {
                double zn[T], zbn[T];
                int p = 0;
#pragma unroll
                for (int jt = 0; jt < T; ++jt)
#pragma unroll
                    for (int kt = jt; kt < T; ++kt, ++p)
                        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[jt], zb[kt], acc[p], 0, 0, 0);
                gs_operands<CELL, NS, T, D>(R0 + 4, nrows, NC, c_first, rsub, m16, pg, sQ, sPhi, sDphi, k00, k01, k02,
                                            k10, k11, k12, k20, k21, k22, zn, zbn);
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    za[t] = zn[t];
                    zb[t] = zbn[t];
                }
            }
        }
        bad = __ballot(bad) != 0ull;

        // --- epilogue: each tile row by row, the mirrored tiles through LDS ------
        double* o = a.out + ec * (int64_t)NS * NS;
        int p = 0;
#pragma unroll
        for (int jt = 0; jt < T; ++jt)
#pragma unroll
            for (int kt = jt; kt < T; ++kt, ++p) {
                // lane holds D[m][n], m = lane / 16 + 4 r, n = lane % 16
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = rsub + 4 * r;
                    const int j = 16 * jt + m, k = 16 * kt + m16;
                    const double val = acc[p][r];
                    if (live && j < NS && k < NS) store_out(o + (size_t)j * NS + k, bad ? nanv : val, a.nt);
                    if (jt != kt) sT[m * GS_TILE_LD + m16] = val;
                }
                if (jt != kt) {
                    // mirrored tile: row 16 kt + m', column 16 jt + n' gets D[n'][m']
                    gs_wave_sync();
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m2 = rsub + 4 * r;
                        const int j = 16 * kt + m2, k = 16 * jt + m16;
                        const double val = sT[m16 * GS_TILE_LD + m2];
                        if (live && j < NS && k < NS) store_out(o + (size_t)j * NS + k, bad ? nanv : val, a.nt);
                    }
                    gs_wave_sync();
                }
            }
        if (live && bad && lane == 0 && a.status) atomicAdd(a.status, 1);
    }
}

// instantiated for element matrices of at most 48 x 48 (3 x 3 tiles): every
// triangle and tetrahedron degree, prisms up to P3
template <int FORM, int CELL>
hipError_t launch_p(int p, const GramScalarArgs& a, int grid, size_t lds, hipStream_t s)
{
    switch (p) {
    case 1: k_gram64_scalar<FORM, CELL, 1><<<grid, gs_waves(CELL) * 64, lds, s>>>(a); break;
    case 2: k_gram64_scalar<FORM, CELL, 2><<<grid, gs_waves(CELL) * 64, lds, s>>>(a); break;
    case 3: k_gram64_scalar<FORM, CELL, 3><<<grid, gs_waves(CELL) * 64, lds, s>>>(a); break;
    default:
        if constexpr (CELL != PRISM) {
            k_gram64_scalar<FORM, CELL, 4><<<grid, gs_waves(CELL) * 64, lds, s>>>(a);
            break;
        }
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

size_t gram64_scalar_lds_bytes(int cell, int p)
{
    const int ns = n_scalar(cell, p);
    return sizeof(double) * ((size_t)gs_waves(cell) * GS_WAVE_DOUBLES + (size_t)GS_QC * ns * (1 + cell_dim(cell)));
}
int gram64_scalar_elems_per_block(int cell) { return gs_waves(cell); }

hipError_t launch_gram64_scalar(int form, int cell, int p, const GramScalarArgs& a, int grid, hipStream_t s)
{
    const size_t lds = gram64_scalar_lds_bytes(cell, p);
    if (form == MASS) {
        return cell == TRI ? launch_p<MASS, TRI>(p, a, grid, lds, s)
             : cell == TET ? launch_p<MASS, TET>(p, a, grid, lds, s)
                           : launch_p<MASS, PRISM>(p, a, grid, lds, s);
    }
    return cell == TRI ? launch_p<HELMHOLTZ, TRI>(p, a, grid, lds, s)
         : cell == TET ? launch_p<HELMHOLTZ, TET>(p, a, grid, lds, s)
                       : launch_p<HELMHOLTZ, PRISM>(p, a, grid, lds, s);
}

}  // namespace fe
