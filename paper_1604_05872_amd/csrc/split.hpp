// Split-precision MFMA contraction for the vector forms.
//
// The sharing-eliminated quadrature sum of the elasticity and hyperelastic
// forms is, per element, a sum of weighted Gram products of one matrix of
// per-point basis data.  With X[q][(c,j)] = g_{q,j,c} (hyperelastic:
// s = F^{-T} g) and diagonal point weights,
//     P_lam = X^T diag(lam') X,   P_2 = X^T diag(mu' or alpha') X,
//     D[j][k] = sum_b Pg[(b,j),(b,k)],  Pg = G^T diag(mu') G,
//     A[(c,j),(e,k)] = P_lam[(c,j),(e,k)] + P_2[(e,j),(c,k)] + delta_ce D[j][k]
// (for elasticity G = X, so Pg = P_2).  Each product is evaluated as a Gram
// matrix Z^T diag(sign) Z of the square-root-scaled columns Z = sqrt|w| X,
// so only one operand per product is rounded.  The products run on the matrix cores:
// one wavefront per element, the element matrix (n = d*n_s <= 32) padded to a
// 32x32 tile, the quadrature point as the reduction dimension (zero-padded).
//
// Precision: geometry, the Lame fields, F, F^{-1}, ln det F and the point
// weights are float64.  The operand entries (3-term dot products of a 3x3
// matrix computed in float64 with a reference gradient) are formed in fp32
// and then
//   * fed to v_mfma_f32_32x32x2_f32 (FE_SPLIT_FP32), or
//   * split into bf16 hi + lo (hardware round-to-nearest-even conversion)
//     with three products hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16
//     (v_mfma_f32_32x32x8_bf16 when the rule has at most 8 points), dropping
//     lo*lo (FE_SPLIT_BF16X3),
// accumulated in fp32; the three-term combination is summed in fp32 and
// stored as float64.
//
// Each wavefront owns its LDS area and walks its own elements; no block-wide
// barrier is taken after the tables are staged, so wavefronts of a block
// overlap their VALU, matrix-core and store phases.  Per element:
//   A. (once per batch of SPLIT_EB elements) the batch's coordinates and
//      coefficients, loaded into registers during the previous batch, go to
//      LDS, and the loads of the next batch are issued, so one global round
//      trip is hidden behind a whole batch;
//   B. one lane per (element, quadrature point) of the batch computes the
//      float64 point data for the whole batch;
//   C. every lane builds exactly the operand entries the instruction layout
//      assigns to it (column (c,j) = lane % 32) and runs the MFMAs;
//   D. the block-transposed and trace terms are exchanged through LDS and the
//      element matrix is stored row by row.
#pragma once
#include "device_common.hpp"
#include "vector_point.hpp"

namespace fe {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

enum SplitPrec { SPLIT_FP32 = 1, SPLIT_BF16X3 = 2 };

struct SplitArgs {
    const double* coords;
    const double* coeff;
    double* out;
    int* status;
    const double* W;      // [nq]
    const double* dphi;   // [nq][ns][d]
    const double* psi;    // [nq][nv]
    int64_t E;
    int nq, ns;
    int collapse;         // P1 on a simplex: one point with summed weights
    int nt;               // non-temporal output stores
    double mu, lam;
};

constexpr int SPLIT_WAVES = 4;
constexpr int SPLIT_TILE_LD = 33;   // padded rows against bank conflicts
constexpr int SPLIT_MAX_IN = 48;    // nv*d + coefficients of one element (at most 42 when n <= 32)
constexpr int SPLIT_EB = 4;         // elements per wavefront batch (one global round trip)
constexpr int SPLIT_PRE = (SPLIT_EB * SPLIT_MAX_IN + 63) / 64;   // prefetch registers per lane

// per-wave LDS (bytes)
constexpr int SPW_IN = 0;                                          // inputs [EB][48] f64
constexpr int SPW_W = SPW_IN + SPLIT_EB * SPLIT_MAX_IN * 8;        // signed weight roots [EB][32][4] f32
constexpr int SPW_M = SPW_W + SPLIT_EB * 32 * 4 * 4;               // M^T [EB][32][3][3] f32
constexpr int SPW_K = SPW_M + SPLIT_EB * 32 * 9 * 4;               // K^T [EB][12] f32
constexpr int SPW_FLAG = SPW_K + SPLIT_EB * 12 * 4;                // flags [EB] (+pad)
constexpr int SPW_GEO = SPW_FLAG + 16;                             // K [EB][9] f64, |det J| [EB] f64
constexpr int SPW_T2 = SPW_GEO + SPLIT_EB * 10 * 8;        // P_2 tile [32][33] f32
constexpr int SPW_TG = SPW_T2 + 32 * SPLIT_TILE_LD * 4;    // P_g tile [32][33] f32
constexpr int SPLIT_WAVE_BYTES = SPW_TG + 32 * SPLIT_TILE_LD * 4;

// block LDS: 4 wave areas, then W [nq] f64, psi [nq][nv] f64, reference
// gradients [nq][ns][d] as f64 (for F) and as f32 zero-padded to 32 points
// (for the operands)
__host__ __device__ constexpr size_t split_lds_bytes(int cell, int nq, int ns)
{
    return (size_t)SPLIT_WAVES * SPLIT_WAVE_BYTES +
           ((size_t)nq + (size_t)nq * cell_nv(cell) + (size_t)nq * ns * cell_dim(cell)) * 8 +
           (size_t)32 * ns * cell_dim(cell) * 4;
}

template <int FORM, int CELL>
__host__ __device__ constexpr int split_coeffs_per_elem(int ns)
{
    return FORM == HYPERELASTIC ? cell_dim(CELL) * ns : 2 * cell_nv(CELL);
}

// LDS ordering between the lanes of one wavefront (its LDS area is private)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// P: polynomial degree (the scalar space size is then a compile-time
// constant); NQP: padded point count (8, 16 or 32).  Every thread of the
// block runs it.
template <int FORM, int CELL, int PREC, int P, int NQP>
__device__ void split_kernel_body(const SplitArgs& a, char* lds)
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL), NVD = NV * D;
    constexpr bool HYP = (FORM == HYPERELASTIC);
    constexpr int ns = n_scalar(CELL, P), n = D * ns;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nq_all = a.nq;
    const int nq = a.collapse ? 1 : nq_all;     // points of the contraction
    constexpr int ncf = split_coeffs_per_elem<FORM, CELL>(ns);
    constexpr int nin = NVD + ncf;               // inputs per element

    char* wl = lds + wave * SPLIT_WAVE_BYTES;
    double* sBuf = (double*)(wl + SPW_IN);
    float* sWall = (float*)(wl + SPW_W);
    float* sMall = (float*)(wl + SPW_M);
    float* sKall = (float*)(wl + SPW_K);
    int* sFlag = (int*)(wl + SPW_FLAG);
    float* tP2 = (float*)(wl + SPW_T2);
    float* tPg = (float*)(wl + SPW_TG);
    double* gW = (double*)(lds + SPLIT_WAVES * SPLIT_WAVE_BYTES);
    double* gPsi = gW + nq_all;
    double* gTab = gPsi + nq_all * NV;
    float* gTabF = (float*)(gTab + nq_all * ns * D);

    // tables, once per block
    for (int i = tid; i < nq_all; i += blockDim.x) gW[i] = a.W[i];
    for (int i = tid; i < nq_all * NV; i += blockDim.x) gPsi[i] = a.psi[i];
    for (int i = tid; i < nq_all * ns * D; i += blockDim.x) gTab[i] = a.dphi[i];
    for (int i = tid; i < 32 * ns * D; i += blockDim.x) gTabF[i] = i < nq * ns * D ? (float)a.dphi[i] : 0.f;
    // padding points q >= nq carry zero weights and zero matrices
    for (int i = lane; i < SPLIT_EB * 32 * 4; i += 64) {
        const int q = (i >> 2) & 31;
        if (q >= nq) ((float*)(wl + SPW_W))[i] = 0.f;
    }
    for (int i = lane; i < SPLIT_EB * 32 * 9; i += 64) {
        const int q = (i / 9) & 31;
        if (q >= nq) ((float*)(wl + SPW_M))[i] = 0.f;
    }
    // summed weights for the hoisted point loop of P1 simplices
    double wsum = 0.0;
    for (int q = 0; q < nq_all; ++q) wsum += a.W[q];
    const PointTables pt{gW, gPsi, gTab, nq_all, a.collapse, wsum, a.mu, a.lam};
    __syncthreads();

    const int64_t stride = (int64_t)gridDim.x * SPLIT_WAVES * SPLIT_EB;
    constexpr int nbatch_in = SPLIT_EB * nin;
    double pre[SPLIT_PRE];
    auto fetch = [&](int64_t first) {
#pragma unroll
        for (int k = 0; k < SPLIT_PRE; ++k) {
            const int t = lane + 64 * k;
            const int i = t / nin, x = t - (t / nin) * nin;
            const int64_t ee = first + i;
            pre[k] = 0.0;
            if (t < nbatch_in && ee < a.E)
                pre[k] = x < NVD ? a.coords[ee * NVD + x] : a.coeff[ee * ncf + (x - NVD)];
        }
    };
    int64_t b0 = ((int64_t)blockIdx.x * SPLIT_WAVES + wave) * SPLIT_EB;
    fetch(b0);

    const int col = lane & 31, half = lane >> 5;
    // columns >= n only feed rows/columns of the 32x32 tile that are never
    // stored, so their operand values just have to stay finite
    const bool cvalid = col < n;
    const int cc = cvalid ? col / ns : 0;
    const int cj = cvalid ? col - cc * ns : 0;
    (void)cvalid;
    static_assert(n <= 32 && nin <= SPLIT_MAX_IN, "element matrix must fit one 32x32 tile");

    for (; b0 < a.E; b0 += stride) {
        // --- A: this batch's inputs to LDS; loads of the next batch ----------
#pragma unroll
        for (int k = 0; k < SPLIT_PRE; ++k) {
            const int t = lane + 64 * k;
            if (t < nbatch_in) {
                const int i = t / nin;
                sBuf[i * SPLIT_MAX_IN + (t - i * nin)] = pre[k];
            }
        }
        if (lane < SPLIT_EB) sFlag[lane] = 0;
        fetch(b0 + stride);
        wave_sync();

        // --- B0: geometry, one lane per element of the batch ------------------
        double* sGeo = (double*)(wl + SPW_GEO);
        if (lane < SPLIT_EB && b0 + lane < a.E) {
            double K[3][3], adet;
            const int bad = affine_map<CELL>(sBuf + lane * SPLIT_MAX_IN, K, adet);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) sGeo[lane * 10 + r * 3 + c] = (r < D && c < D) ? K[r][c] : 0.0;
            sGeo[lane * 10 + 9] = adet;
            if (bad) sFlag[lane] = 1;
        }
        wave_sync();

        // --- B: float64 point data, one lane per (element, point) -----------
#pragma unroll 1
        for (int t = lane; t < SPLIT_EB * nq; t += 64) {
            const int ib = t / nq, q = t - ib * nq;
            if (b0 + ib >= a.E) continue;
            double K[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) K[r][c] = sGeo[ib * 10 + r * 3 + c];
            const double adet = sGeo[ib * 10 + 9];
            double w0, w1, w2, M[3][3];
            const int bad =
                vector_point_data<FORM, CELL, ns>(sBuf + ib * SPLIT_MAX_IN, K, adet, q, pt, w0, w1, w2, M);
            // signed square roots of the three product weights (the operands
            // are fp32, so the root is taken in fp32); bit t of the element's
            // flag word records a negative weight of product t
            float* sW = sWall + ib * 32 * 4;
            float* sMt = sMall + ib * 32 * 9;
            const float f0 = (float)w0, f1 = (float)w1, f2 = (float)w2;
            sW[q * 4 + 0] = copysignf(sqrtf(fabsf(f0)), f0);
            sW[q * 4 + 1] = copysignf(sqrtf(fabsf(f1)), f1);
            sW[q * 4 + 2] = copysignf(sqrtf(fabsf(f2)), f2);
            const int neg = (f0 < 0.f ? 2 : 0) | (f1 < 0.f ? 4 : 0) | (f2 < 0.f ? 8 : 0);
            if (neg) atomicOr(&sFlag[ib], neg);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) sMt[q * 9 + c * 3 + r] = (float)M[r][c];
            if (q == 0)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int r = 0; r < 3; ++r) sKall[ib * 12 + c * 3 + r] = (r < D && c < D) ? (float)K[r][c] : 0.f;
            if (bad) atomicOr(&sFlag[ib], 1);
        }
        wave_sync();

        // --- C, D: per element of the batch ------------------------------------
#pragma unroll 1
        for (int ib = 0; ib < SPLIT_EB; ++ib) {
            const int64_t e = b0 + ib;
            if (e >= a.E) break;
            const float* sW = sWall + ib * 32 * 4;
            const float* sMt = sMall + ib * 32 * 9;
            const int negw = __builtin_amdgcn_readfirstlane(sFlag[ib]);
            float kc[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) kc[b] = sKall[ib * 12 + cc * 3 + b];

            v16f accL, acc2, accG;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                accL[r] = 0.f;
                acc2[r] = 0.f;
                accG[r] = 0.f;
            }
            // Scaled columns at point q (zero at padding points): with the signed
            // roots r_t of the weights, z_t = |r_t| x enters as the A operand and
            // sign(r_t) z_t as the B operand (an exact sign-bit flip), for
            //   P_lam = Z_0^T S_0 Z_0, P_2 = Z_1^T S_1 Z_1, P_g = Z_2^T S_2 Z_2,
            // x = s (hyperelastic) or g, and g for P_g.
            auto colx = [&](int q) -> float {
                const float* gh = gTabF + (q * ns + cj) * D;
                const float* m = sMt + q * 9 + cc * 3;
                float x = m[0] * gh[0];
#pragma unroll
                for (int b = 1; b < D; ++b) x = fmaf(m[b], gh[b], x);
                return x;
            };
            auto colg = [&](int q) -> float {
                const float* gh = gTabF + (q * ns + cj) * D;
                float g = kc[0] * gh[0];
#pragma unroll
                for (int b = 1; b < D; ++b) g = fmaf(kc[b], gh[b], g);
                return g;
            };
            auto sgn = [&](int q, int t) -> unsigned { return __float_as_uint(sW[q * 4 + t]) & 0x80000000u; };
            if (PREC == SPLIT_BF16X3) {
                constexpr int KW = NQP == 8 ? 4 : 8;    // points per lane per instruction
                typedef __bf16 vbf __attribute__((ext_vector_type(KW)));
                typedef unsigned vu __attribute__((ext_vector_type(KW / 2)));
                auto mma = [&](const vbf& x, const vbf& y, v16f& acc) {
                    if constexpr (KW == 4)
                        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(v4s, x),
                                                                       __builtin_bit_cast(v4s, y), acc, 0, 0, 0);
                    else
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
                };
                // split |r_t| x into bf16 hi + lo; hi*hi + hi*lo + lo*hi with the
                // point signs on the B operand
                auto product = [&](const float* x, int q0, int t, v16f& acc) {
                    vbf h, l;
#pragma unroll
                    for (int i = 0; i < KW; ++i) {
                        const float z = fabsf(sW[(q0 + i) * 4 + t]) * x[i];
                        const __bf16 hi = (__bf16)z;
                        h[i] = hi;
                        l[i] = (__bf16)(z - (float)hi);
                    }
                    if (negw & (2 << t)) {   // uniform over the wavefront (one element)
                        vu sm;
#pragma unroll
                        for (int i = 0; i < KW / 2; ++i)
                            sm[i] = (sgn(q0 + 2 * i, t) >> 16) | sgn(q0 + 2 * i + 1, t);
                        const vbf hb = __builtin_bit_cast(vbf, __builtin_bit_cast(vu, h) ^ sm);
                        const vbf lb = __builtin_bit_cast(vbf, __builtin_bit_cast(vu, l) ^ sm);
                        mma(l, hb, acc);
                        mma(h, lb, acc);
                        mma(h, hb, acc);
                    } else {
                        mma(l, h, acc);
                        mma(h, l, acc);
                        mma(h, h, acc);
                    }
                };
#pragma unroll 1
                for (int kb = 0; kb < NQP / (2 * KW); ++kb) {
                    const int q0 = 2 * KW * kb + KW * half;
                    float x[KW], g[KW];
                    // x and g of the lane's column at its KW points, from one
                    // read of the reference gradients
#pragma unroll
                    for (int i = 0; i < KW; ++i) {
                        const int q = q0 + i;
                        const float* gh = gTabF + (q * ns + cj) * D;
                        float gv[3];
#pragma unroll
                        for (int b = 0; b < D; ++b) gv[b] = gh[b];
                        const float* m = sMt + q * 9 + cc * 3;
                        float xv = m[0] * gv[0], g0 = kc[0] * gv[0];
#pragma unroll
                        for (int b = 1; b < D; ++b) {
                            xv = fmaf(m[b], gv[b], xv);
                            g0 = fmaf(kc[b], gv[b], g0);
                        }
                        x[i] = xv;
                        g[i] = g0;
                    }
                    product(x, q0, 0, accL);
                    product(x, q0, 1, acc2);
                    if (HYP) product(g, q0, 2, accG);
                }
            } else {
#pragma unroll 2
                for (int ks = 0; ks < NQP / 2; ++ks) {
                    const int q = 2 * ks + half;
                    const float x = colx(q);
                    const float r0 = sW[q * 4 + 0], r1 = sW[q * 4 + 1];
                    accL = __builtin_amdgcn_mfma_f32_32x32x2f32(fabsf(r0) * x, r0 * x, accL, 0, 0, 0);
                    acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(fabsf(r1) * x, r1 * x, acc2, 0, 0, 0);
                    if (HYP) {
                        const float g = colg(q), r2 = sW[q * 4 + 2];
                        accG = __builtin_amdgcn_mfma_f32_32x32x2f32(fabsf(r2) * g, r2 * g, accG, 0, 0, 0);
                    }
                }
            }

            // --- D: epilogue ------------------------------------------------
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * half + (r & 3);
                tP2[row * SPLIT_TILE_LD + col] = acc2[r];
                if (HYP) tPg[row * SPLIT_TILE_LD + col] = accG[r];
            }
            wave_sync();
            const bool bad = (negw & 1) != 0;
            const float* tD = HYP ? tPg : tP2;
            double* o = a.out + e * (int64_t)n * n;
            const double nanv = __builtin_nan("");
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * half + (r & 3);
                if (row < n && col < n) {
                    const int c = row / ns, j = row - c * ns;
                    const int d2 = col / ns, k = col - d2 * ns;
                    float v = accL[r] + tP2[(d2 * ns + j) * SPLIT_TILE_LD + c * ns + k];
                    if (c == d2) {
#pragma unroll
                        for (int b = 0; b < D; ++b) v += tD[(b * ns + j) * SPLIT_TILE_LD + b * ns + k];
                    }
                    store_out(o + (size_t)row * n + col, bad ? nanv : (double)v, a.nt);
                }
            }
            if (bad && lane == 0 && a.status) atomicAdd(a.status, 1);
            wave_sync();
        }
    }
}

}  // namespace fe
