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
// 32x32 tile, the point index as the reduction dimension (zero-padded to a
// multiple of 8).  Geometry, the Lame fields, F, F^{-1}, ln det F and the
// point weights are float64; operands are rounded to
//   * fp32 (v_mfma_f32_32x32x2_f32), or
//   * bf16 hi + lo with three products hi*hi + hi*lo + lo*hi
//     (v_mfma_f32_32x32x8_bf16), dropping lo*lo,
// accumulated in fp32, and the final three-term combination is float64.
//
// Each lane builds exactly the operand entries the instruction layout assigns
// to it (column (c,j) = lane % 32, a fixed set of points), so no operand is
// staged through LDS; LDS holds the per-point float64 data, the reference
// gradient table and the fp32 product tiles for the transposed-block epilogue.
#pragma once
#include "device_common.hpp"

namespace fe {

typedef short v4s __attribute__((ext_vector_type(4)));
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
    double mu, lam;
};

__device__ __forceinline__ unsigned short bf16_rne(float x)
{
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// LDS per wave (doubles): per-point weights (3) and matrix (9) for 32 points,
// plus two 32x33 fp32 tiles.
constexpr int SPLIT_PT_STRIDE = 12;
constexpr int SPLIT_TILE_LD = 33;   // padded row to avoid bank conflicts
constexpr int SPLIT_WAVE_DOUBLES = 32 * SPLIT_PT_STRIDE + 32 * SPLIT_TILE_LD;   // 2 tiles of floats = 1 tile of doubles
constexpr int SPLIT_WAVES = 4;

template <int FORM, int CELL>
__host__ __device__ constexpr size_t split_lds_bytes(int nq, int ns)
{
    return (size_t)SPLIT_WAVES * SPLIT_WAVE_DOUBLES * 8 + (size_t)nq * ns * cell_dim(CELL) * 8;
}

// One element per wavefront; the block (4 waves) processes 4 consecutive
// elements per step.  Every thread of the block must call it with the same
// e_base sequence.
template <int FORM, int CELL, int PREC, int NKB>
__device__ void split_step(const SplitArgs& a, int64_t e_base, double* lds, const double* sTab)
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL);
    constexpr bool HYP = (FORM == HYPERELASTIC);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ns = a.ns, n = D * ns, nq = a.nq;
    const int64_t e = e_base + wave;
    const bool valid = e < a.E;
    double* wl = lds + wave * SPLIT_WAVE_DOUBLES;
    double* sPt = wl;                                      // [32][12]
    float* tP2 = (float*)(wl + 32 * SPLIT_PT_STRIDE);       // [32][33]
    float* tPg = tP2 + 32 * SPLIT_TILE_LD;                  // [32][33] (hyperelastic)

    // geometry (float64, every lane; the loads are uniform across the wave)
    double K[3][3], adet = 0.0;
    int bad = 1;
    if (valid) {
        double v[NV * D];
#pragma unroll
        for (int k = 0; k < NV * D; ++k) v[k] = a.coords[e * (NV * D) + k];
        bad = affine_map<CELL>(v, K, adet);
    }
    // per-point float64 data: lane q handles point q
    if (valid && lane < 32) {
        const int q = lane;
        double* pt = sPt + q * SPLIT_PT_STRIDE;
        if (q < nq) {
            const double w = a.W[q] * adet;
            if (!HYP) {
                const double* ce = a.coeff + e * 2 * NV;
                const double* ps = a.psi + q * NV;
                double lam = 0.0, mu = 0.0;
#pragma unroll
                for (int l = 0; l < NV; ++l) {
                    lam = fma(ce[l], ps[l], lam);
                    mu = fma(ce[NV + l], ps[l], mu);
                }
                pt[0] = w * lam;
                pt[1] = w * mu;
                pt[2] = 0.0;
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) pt[3 + r * 3 + c] = (r < D && c < D) ? K[r][c] : 0.0;
            } else {
                // H = sum_k u_k (x) grad_X phi_k ; F = I + H K
                const double* ue = a.coeff + e * (D * ns);
                double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int k = 0; k < ns; ++k) {
                    const double* gh = sTab + (q * ns + k) * D;
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        const double ur = ue[r * ns + k];
#pragma unroll
                        for (int c = 0; c < D; ++c) H[r][c] = fma(ur, gh[c], H[r][c]);
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
                if (!(jf > 0.0)) bad = 1;
                const double lnj = log(jf);
                pt[0] = w * a.lam;
                pt[1] = w * (a.mu - a.lam * lnj);
                pt[2] = w * a.mu;
                // M = K F^{-1}: s_c = sum_a M[a][c] dphi/dX_a
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double s = 0.0;
#pragma unroll
                        for (int b = 0; b < D; ++b) s = fma(K[r][b], Fi[b][c], s);
                        pt[3 + r * 3 + c] = (r < D && c < D) ? s : 0.0;
                    }
            }
        } else {
#pragma unroll
            for (int k = 0; k < SPLIT_PT_STRIDE; ++k) pt[k] = 0.0;
        }
    }
    // any lane flagged the element (J_F <= 0 at its point, or the map)
    bad = __any(bad) ? 1 : 0;
    __syncthreads();

    // operands: column (c, j) of this lane
    const int col = lane & 31, half = lane >> 5;
    const bool cvalid = valid && col < n;
    const int cc = cvalid ? col / ns : 0;
    const int cj = cvalid ? col - cc * ns : 0;

    v16f accL, acc2, accG;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        accL[r] = 0.f;
        acc2[r] = 0.f;
        accG[r] = 0.f;
    }

    // x = value of the lane's column at point q: X (s or g) and G (g)
    auto column_values = [&](int q, double& x, double& g, double& wl_, double& w2, double& wg) {
        x = 0.0;
        g = 0.0;
        wl_ = 0.0;
        w2 = 0.0;
        wg = 0.0;
        if (cvalid && q < nq) {
            const double* pt = sPt + q * SPLIT_PT_STRIDE;
            const double* gh = sTab + (q * ns + cj) * D;
            double sx = 0.0, sg = 0.0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                sx = fma(pt[3 + b * 3 + cc], gh[b], sx);
                if (HYP) sg = fma(K[b][cc], gh[b], sg);
            }
            x = sx;
            g = HYP ? sg : sx;
            wl_ = pt[0];
            w2 = pt[1];
            wg = HYP ? pt[2] : 0.0;
        }
    };

    if (PREC == SPLIT_BF16X3) {
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            v4s xh, xl, lh, ll, th, tl, gh_, gl_, mh, ml;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = 8 * kb + 4 * half + i;
                double x, g, wl_, w2, wg;
                column_values(q, x, g, wl_, w2, wg);
                auto split = [](double v, short& h, short& l) {
                    const float f = (float)v;
                    const unsigned short hb = bf16_rne(f);
                    h = (short)hb;
                    l = (short)bf16_rne(f - bf16_to_f(hb));
                };
                short h, l;
                split(x, h, l);
                xh[i] = h;
                xl[i] = l;
                split(wl_ * x, h, l);
                lh[i] = h;
                ll[i] = l;
                split(w2 * x, h, l);
                th[i] = h;
                tl[i] = l;
                if (HYP) {
                    split(g, h, l);
                    gh_[i] = h;
                    gl_[i] = l;
                    split(wg * g, h, l);
                    mh[i] = h;
                    ml[i] = l;
                }
            }
            accL = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(xl, lh, accL, 0, 0, 0);
            accL = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(xh, ll, accL, 0, 0, 0);
            accL = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(xh, lh, accL, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(xl, th, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(xh, tl, acc2, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(xh, th, acc2, 0, 0, 0);
            if (HYP) {
                accG = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(gl_, mh, accG, 0, 0, 0);
                accG = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(gh_, ml, accG, 0, 0, 0);
                accG = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(gh_, mh, accG, 0, 0, 0);
            }
        }
    } else {
#pragma unroll
        for (int ks = 0; ks < 4 * NKB; ++ks) {
            const int q = 2 * ks + half;
            double x, g, wl_, w2, wg;
            column_values(q, x, g, wl_, w2, wg);
            const float xf = (float)x;
            accL = __builtin_amdgcn_mfma_f32_32x32x2f32(xf, (float)(wl_ * x), accL, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(xf, (float)(w2 * x), acc2, 0, 0, 0);
            if (HYP) accG = __builtin_amdgcn_mfma_f32_32x32x2f32((float)g, (float)(wg * g), accG, 0, 0, 0);
        }
    }

    // epilogue: the block-transposed term and the trace term come from LDS
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * half + (r & 3);
        tP2[row * SPLIT_TILE_LD + col] = acc2[r];
        if (HYP) tPg[row * SPLIT_TILE_LD + col] = accG[r];
    }
    __syncthreads();
    if (valid) {
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
                store_out(o + (size_t)row * n + col, bad ? nanv : v);
            }
        }
        if (bad && lane == 0 && a.status) atomicAdd(a.status, 1);
    }
    __syncthreads();
}

}  // namespace fe
