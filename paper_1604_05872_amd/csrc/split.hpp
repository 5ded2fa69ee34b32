// Split-precision MFMA contraction for the vector forms.
//
// The sharing-eliminated quadrature sum of the elasticity and hyperelastic
// forms is, per element, a sum of weighted Gram products of one matrix of
// per-point basis data.  With X[q][(c,j)] = g_{q,j,c} (hyperelastic:
// s = F^{-T} g) and diagonal point weights,
//     P_lam = X^T diag(lam') X,   P_2 = X^T diag(mu' or alpha') X,
//     D[j][k] = sum_b Pg[(b,j),(b,k)],  Pg = G^T diag(mu') G,
//     A[(c,j),(e,k)] = P_lam[(c,j),(e,k)] + P_2[(e,j),(c,k)] + delta_ce D[j][k]
// (for elasticity G = X, so Pg = P_2).  The products run on the matrix cores:
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
// accumulated in fp32; the final three-term combination is float64.
//
// Each wavefront owns its LDS area and walks its own elements; no block-wide
// barrier is taken after the tables are staged, so wavefronts of a block
// overlap their VALU, matrix-core and store phases.  Per element:
//   A. the element's coordinates and coefficients (prefetched into one
//      register per lane during the previous element) go to LDS;
//   B. one lane per quadrature point computes the float64 point data;
//   C. every lane builds exactly the operand entries the instruction layout
//      assigns to it (column (c,j) = lane % 32) and runs the MFMAs;
//   D. the block-transposed and trace terms are exchanged through LDS and the
//      element matrix is stored row by row.
#pragma once
#include "device_common.hpp"

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

// per-wave LDS (bytes)
constexpr int SPW_IN = 0;                                  // inputs [48] f64
constexpr int SPW_W = SPW_IN + SPLIT_MAX_IN * 8;           // weights [32][4] f32
constexpr int SPW_M = SPW_W + 32 * 4 * 4;                  // M^T per point [32][3][3] f32 (row c: M[0..2][c])
constexpr int SPW_K = SPW_M + 32 * 9 * 4;                  // K^T [3][3] f32
constexpr int SPW_FLAG = SPW_K + 12 * 4;
constexpr int SPW_T2 = SPW_FLAG + 16;                      // P_2 tile [32][33] f32
constexpr int SPW_TG = SPW_T2 + 32 * SPLIT_TILE_LD * 4;    // P_g tile [32][33] f32
constexpr int SPLIT_WAVE_BYTES = SPW_TG + 32 * SPLIT_TILE_LD * 4;

// block LDS: 4 wave areas, then W [nq] f64, psi [nq][nv] f64, reference
// gradients [nq][ns][d] as f64 (for F) and as f32 (for the operands)
__host__ __device__ constexpr size_t split_lds_bytes(int cell, int nq, int ns)
{
    return (size_t)SPLIT_WAVES * SPLIT_WAVE_BYTES +
           ((size_t)nq + (size_t)nq * cell_nv(cell) + (size_t)nq * ns * cell_dim(cell)) * 8 +
           (size_t)nq * ns * cell_dim(cell) * 4;
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

// NQP: padded point count (8, 16 or 32).  Every thread of the block runs it.
template <int FORM, int CELL, int PREC, int NQP>
__device__ void split_kernel_body(const SplitArgs& a, char* lds)
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL), NVD = NV * D;
    constexpr bool HYP = (FORM == HYPERELASTIC);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ns = a.ns, n = D * ns, nq_all = a.nq;
    const int nq = a.collapse ? 1 : nq_all;     // points of the contraction
    const int ncf = split_coeffs_per_elem<FORM, CELL>(ns);
    const int nin = NVD + ncf;                   // inputs per element

    char* wl = lds + wave * SPLIT_WAVE_BYTES;
    double* sIn = (double*)(wl + SPW_IN);
    float* sW = (float*)(wl + SPW_W);
    float* sMt = (float*)(wl + SPW_M);
    float* sKt = (float*)(wl + SPW_K);
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
    for (int i = tid; i < nq_all * ns * D; i += blockDim.x) {
        gTab[i] = a.dphi[i];
        gTabF[i] = (float)a.dphi[i];
    }
    // summed weights for the hoisted point loop of P1 simplices
    double wsum = 0.0;
    for (int q = 0; q < nq_all; ++q) wsum += a.W[q];
    __syncthreads();

    int64_t e = (int64_t)blockIdx.x * SPLIT_WAVES + wave;
    const int64_t stride = (int64_t)gridDim.x * SPLIT_WAVES;
    auto fetch = [&](int64_t ee) -> double {
        if (lane >= nin || ee >= a.E) return 0.0;
        return lane < NVD ? a.coords[ee * NVD + lane] : a.coeff[ee * ncf + (lane - NVD)];
    };
    double pre = fetch(e);

    const int col = lane & 31, half = lane >> 5;
    const bool cvalid = col < n;
    const int cc = cvalid ? col / ns : 0;
    const int cj = cvalid ? col - cc * ns : 0;

    for (; e < a.E; e += stride) {
        // --- A: inputs to LDS; prefetch the next element -------------------
        if (lane < nin) sIn[lane] = pre;
        pre = fetch(e + stride);
        wave_sync();

        // --- B: float64 point data, one lane per point ----------------------
        int bad = 0;
        if (lane < nq) {
            const int q = lane;
            double K[3][3], adet;
            bad = affine_map<CELL>(sIn, K, adet);
            const double w = (a.collapse ? wsum : gW[q]) * adet;
            double M[3][3];
            float w0, w1, w2 = 0.f;
            if (!HYP) {
                const double* ce = sIn + NVD;
                double lam = 0.0, mu = 0.0;
                if (a.collapse) {
                    for (int qq = 0; qq < nq_all; ++qq) {
                        double l1 = 0.0, m1 = 0.0;
#pragma unroll
                        for (int l = 0; l < NV; ++l) {
                            l1 = fma(ce[l], gPsi[qq * NV + l], l1);
                            m1 = fma(ce[NV + l], gPsi[qq * NV + l], m1);
                        }
                        lam = fma(gW[qq], l1, lam);
                        mu = fma(gW[qq], m1, mu);
                    }
                    w0 = (float)(adet * lam);
                    w1 = (float)(adet * mu);
                } else {
#pragma unroll
                    for (int l = 0; l < NV; ++l) {
                        lam = fma(ce[l], gPsi[q * NV + l], lam);
                        mu = fma(ce[NV + l], gPsi[q * NV + l], mu);
                    }
                    w0 = (float)(w * lam);
                    w1 = (float)(w * mu);
                }
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) M[r][c] = (r < D && c < D) ? K[r][c] : 0.0;
            } else {
                // H = sum_k u_k (x) grad_X phi_k ; F = I + H K
                const double* ue = sIn + NVD;
                double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int k = 0; k < ns; ++k) {
                    const double* dg = gTab + (q * ns + k) * D;
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        const double ur = ue[r * ns + k];
#pragma unroll
                        for (int c = 0; c < D; ++c) H[r][c] = fma(ur, dg[c], H[r][c]);
                    }
                }
                double F[3][3], Fi[3][3];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        double s = (r == b) ? 1.0 : 0.0;
#pragma unroll
                        for (int c = 0; c < D; ++c) s = fma(H[r][c], K[c][b], s);
                        F[r][b] = s;
                    }
                const double jf = inverse_small<D>(F, Fi);
                bad |= !(jf > 0.0);
                const double lnj = log(jf);
                w0 = (float)(w * a.lam);
                w1 = (float)(w * (a.mu - a.lam * lnj));
                w2 = (float)(w * a.mu);
                // M = K F^{-1}: s_c = sum_a M[a][c] dphi/dX_a
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double s = 0.0;
#pragma unroll
                        for (int b = 0; b < D; ++b) s = fma(K[r][b], Fi[b][c], s);
                        M[r][c] = (r < D && c < D) ? s : 0.0;
                    }
            }
            sW[q * 4 + 0] = w0;
            sW[q * 4 + 1] = w1;
            sW[q * 4 + 2] = w2;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) sMt[q * 9 + c * 3 + r] = (float)M[r][c];
            if (q == 0)
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int r = 0; r < 3; ++r) sKt[c * 3 + r] = (r < D && c < D) ? (float)K[r][c] : 0.f;
        }
        bad = __any(bad) ? 1 : 0;
        wave_sync();

        // --- C: operands and matrix-core products ---------------------------
        float kc[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) kc[b] = sKt[cc * 3 + b];

        v16f accL, acc2, accG;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            accL[r] = 0.f;
            acc2[r] = 0.f;
            accG[r] = 0.f;
        }
        // x (s for the hyperelastic form, else g) of the lane's column at
        // point q with the weights of P_lam and P_2; g with the weight of P_g
        auto colx = [&](int q, float& x, float& w1, float& w2) {
            x = w1 = w2 = 0.f;
            if (cvalid && q < nq) {
                const float* gh = gTabF + (q * ns + cj) * D;
                const float* m = sMt + q * 9 + cc * 3;
                float sx = m[0] * gh[0];
#pragma unroll
                for (int b = 1; b < D; ++b) sx = fmaf(m[b], gh[b], sx);
                x = sx;
                w1 = sW[q * 4 + 0];
                w2 = sW[q * 4 + 1];
            }
        };
        auto colg = [&](int q, float& g, float& w3) {
            g = w3 = 0.f;
            if (cvalid && q < nq) {
                const float* gh = gTabF + (q * ns + cj) * D;
                float sg = kc[0] * gh[0];
#pragma unroll
                for (int b = 1; b < D; ++b) sg = fmaf(kc[b], gh[b], sg);
                g = sg;
                w3 = sW[q * 4 + 2];
            }
        };
        if (PREC == SPLIT_BF16X3) {
            if (NQP == 8) {
                auto gram4 = [&](const float* xv, const float* wv, v16f& acc) {
                    v4bf xh, xl, yh, yl;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const __bf16 h = (__bf16)xv[i];
                        xh[i] = h;
                        xl[i] = (__bf16)(xv[i] - (float)h);
                        const float y = wv[i] * xv[i];
                        const __bf16 yh_ = (__bf16)y;
                        yh[i] = yh_;
                        yl[i] = (__bf16)(y - (float)yh_);
                    }
                    const v4s a_h = __builtin_bit_cast(v4s, xh), a_l = __builtin_bit_cast(v4s, xl);
                    const v4s b_h = __builtin_bit_cast(v4s, yh), b_l = __builtin_bit_cast(v4s, yl);
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a_l, b_h, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a_h, b_l, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a_h, b_h, acc, 0, 0, 0);
                };
                float xv[4], w1v[4], w2v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) colx(4 * half + i, xv[i], w1v[i], w2v[i]);
                gram4(xv, w1v, accL);
                gram4(xv, w2v, acc2);
                if (HYP) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) colg(4 * half + i, xv[i], w1v[i]);
                    gram4(xv, w1v, accG);
                }
            } else {
                auto gram8 = [&](const float* xv, const float* wv, v16f& acc) {
                    v8bf xh, xl, yh, yl;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const __bf16 h = (__bf16)xv[i];
                        xh[i] = h;
                        xl[i] = (__bf16)(xv[i] - (float)h);
                        const float y = wv[i] * xv[i];
                        const __bf16 yh_ = (__bf16)y;
                        yh[i] = yh_;
                        yl[i] = (__bf16)(y - (float)yh_);
                    }
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl, yh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, yl, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, yh, acc, 0, 0, 0);
                };
#pragma unroll 1
                for (int kb = 0; kb < NQP / 16; ++kb) {
                    float xv[8], w1v[8], w2v[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) colx(16 * kb + 8 * half + i, xv[i], w1v[i], w2v[i]);
                    gram8(xv, w1v, accL);
                    gram8(xv, w2v, acc2);
                    if (HYP) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) colg(16 * kb + 8 * half + i, xv[i], w1v[i]);
                        gram8(xv, w1v, accG);
                    }
                }
            }
        } else {
#pragma unroll 2
            for (int ks = 0; ks < NQP / 2; ++ks) {
                float x, w1, w2;
                colx(2 * ks + half, x, w1, w2);
                accL = __builtin_amdgcn_mfma_f32_32x32x2f32(x, w1 * x, accL, 0, 0, 0);
                acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, w2 * x, acc2, 0, 0, 0);
                if (HYP) {
                    float g, w3;
                    colg(2 * ks + half, g, w3);
                    accG = __builtin_amdgcn_mfma_f32_32x32x2f32(g, w3 * g, accG, 0, 0, 0);
                }
            }
        }

        // --- D: epilogue --------------------------------------------------
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * half + (r & 3);
            tP2[row * SPLIT_TILE_LD + col] = acc2[r];
            if (HYP) tPg[row * SPLIT_TILE_LD + col] = accG[r];
        }
        wave_sync();
        {
            const float* tD = HYP ? tPg : tP2;
            double* o = a.out + e * (int64_t)n * n;
            const double nanv = __builtin_nan("");
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * half + (r & 3);
                if (row < n && col < n) {
                    const int c = row / ns, j = row - c * ns;
                    const int d2 = col / ns, k = col - d2 * ns;
                    double v = (double)accL[r] + (double)tP2[(d2 * ns + j) * SPLIT_TILE_LD + c * ns + k];
                    if (c == d2) {
                        double t = 0.0;
#pragma unroll
                        for (int b = 0; b < D; ++b) t += (double)tD[(b * ns + j) * SPLIT_TILE_LD + b * ns + k];
                        v += t;
                    }
                    store_out(o + (size_t)row * n + col, bad ? nanv : v, a.nt);
                }
            }
            if (bad && lane == 0 && a.status) atomicAdd(a.status, 1);
        }
        wave_sync();
    }
}

}  // namespace fe
