// Split-precision MFMA contraction for the vector forms.
//
// The sharing-eliminated quadrature sum of the elasticity and hyperelastic
// forms is, per element, a sum of weighted Gram products of one matrix of
// per-point basis data.  With X[q][(c,j)] = g_{q,j,c} (hyperelastic:
// s = F^{-T} g) and diagonal point weights,
//     P_lam = X^T diag(lam') X,   P_2 = X^T diag(mu' or alpha') X,
//     A[(c,j),(e,k)] = P_lam[(c,j),(e,k)] + P_2[(e,j),(c,k)] + delta_ce D[j][k],
// with the trace term D[j][k] = sum_q mu'_q g_{q,j} . g_{q,k}.  Each product is
// evaluated as a Gram matrix Z^T diag(sign) Z of the square-root-scaled
// columns Z = sqrt|w| X, so only one operand per product is rounded.  The
// products run on the matrix cores: one wavefront per element, the element
// matrix (n = d*n_s <= 32) padded to a 32x32 tile, the quadrature point as
// the reduction dimension (zero-padded).
//
// The trace term is split off the way Alg. 3 splits a form into monomials
// (Sec. 4).  For elasticity mu varies over the element and D is the block
// trace of P_2 (G = X).  For the hyperelastic form mu is a constant, so the
// monomial mu |det J| g_j . g_k is pre-evaluated (Sec. 3.3): with K = J^{-1},
//     D[j][k] = mu |det J| sum_{a<=b} (K K^T)_ab S_ab[j][k],
//     S_aa = T_aa, S_ab = T_ab + T_ba, T_ab[j][k] = sum_q W_q dphi_{q,j,a} dphi_{q,k,b},
// with the tables formed once per workgroup from the staged reference
// gradients; the matrix cores then carry two products instead of three.
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
// accumulated in fp32; the pre-evaluated trace term is an fp32 sum of
// fp32-rounded coefficients and tables; the combination is summed in fp32 and
// stored as float64.
//
// Each wavefront owns its LDS area and walks its own elements; no block-wide
// barrier is taken after the tables are staged, so wavefronts of a block
// overlap their VALU, matrix-core and store phases.  Per element:
//   A. (once per batch of EB elements) the batch's inputs are already in
//      LDS: they were loaded into registers two batches ahead and staged
//      right after the previous batch's point phase;
//   B. one lane per (element, quadrature point) of the batch maps its element
//      and computes the float64 point data for the whole batch; then the next
//      batch's inputs go to LDS and the loads of the one after are issued;
//   C. every lane builds exactly the operand entries the instruction layout
//      assigns to it (column (c,j) = lane % 32) and runs the MFMAs;
//   D. the block-transposed and trace terms are exchanged through LDS and the
//      element matrix is stored row by row.
#pragma once
#include <type_traits>
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

// elements per wavefront batch (one global round trip).  A hyperelastic
// point is expensive, so two elements (54 of 64 lanes for a 27-point rule)
// keep the LDS small enough for three workgroups per CU.
__host__ __device__ constexpr int split_eb(int form) { return form == HYPERELASTIC ? 2 : 4; }
// pre-evaluated trace tables (hyperelastic): one per pair a <= b
__host__ __device__ constexpr int split_trace_tables(int form, int cell)
{
    return form == HYPERELASTIC ? cell_dim(cell) * (cell_dim(cell) + 1) / 2 : 0;
}

// per-wave LDS (bytes), for a batch of eb elements
struct SplitLayout {
    int in;     // inputs: coordinates [eb][nv d], then coefficients [eb][ncf] (f64, at most eb x 48)
    int w;      // signed weight roots [eb][32][2] f32
    int m;      // M^T [eb][32][3][3] f32
    int flag;   // flags [eb] (+pad)
    int dco;    // trace coefficients [eb][8] f32
    int dtr;    // trace term of the current element [16][16] f32
    int t2;     // P_2 tile [32][33] f32
    int bytes;
};
__host__ __device__ constexpr SplitLayout split_layout(int eb)
{
    SplitLayout L{};
    L.in = 0;
    L.w = L.in + eb * SPLIT_MAX_IN * 8;
    L.m = L.w + eb * 32 * 2 * 4;
    L.flag = L.m + eb * 32 * 9 * 4;
    L.dco = L.flag + 16;
    L.dtr = L.dco + eb * 8 * 4;
    L.t2 = L.dtr + 16 * 16 * 4;
    L.bytes = L.t2 + 32 * SPLIT_TILE_LD * 4;
    return L;
}

// block LDS: 4 wave areas, then W [nq] f64, psi [nq][nv] f64, reference
// gradients [nq][ns][d] as f64 (for F) and as f32 zero-padded to 32 points
// (for the operands), then the trace tables [ntr][ns][ns] f32
__host__ __device__ constexpr size_t split_lds_bytes(int form, int cell, int nq, int ns)
{
    return (size_t)SPLIT_WAVES * split_layout(split_eb(form)).bytes +
           ((size_t)nq + (size_t)nq * cell_nv(cell) + (size_t)nq * ns * cell_dim(cell)) * 8 +
           (size_t)32 * ns * cell_dim(cell) * 4 + (size_t)split_trace_tables(form, cell) * ns * ns * 4;
}

template <int FORM, int CELL>
__host__ __device__ constexpr int split_coeffs_per_elem(int ns)
{
    return FORM == HYPERELASTIC ? cell_dim(CELL) * ns : 2 * cell_nv(CELL);
}

// P: polynomial degree (the scalar space size is then a compile-time
// constant); NQP: padded point count (8, 16 or 32).  Every thread of the
// block runs it.
template <int FORM, int CELL, int PREC, int P, int NQP>
__device__ void split_kernel_body(const SplitArgs& a, char* lds)
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL), NVD = NV * D;
    constexpr bool HYP = (FORM == HYPERELASTIC);
    constexpr int EB = split_eb(FORM);
    constexpr SplitLayout L = split_layout(EB);
    constexpr int NTR = split_trace_tables(FORM, CELL);
    constexpr int ns = n_scalar(CELL, P), n = D * ns;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nq_all = a.nq;
    const int nq = a.collapse ? 1 : nq_all;     // points of the contraction
    constexpr int ncf = split_coeffs_per_elem<FORM, CELL>(ns);
    constexpr int nin = NVD + ncf;               // inputs per element

    char* wl = lds + wave * L.bytes;
    double* sBuf = (double*)(wl + L.in);
    float* sWall = (float*)(wl + L.w);
    float* sMall = (float*)(wl + L.m);
    int* sFlag = (int*)(wl + L.flag);
    float* sDtr = (float*)(wl + L.dtr);
    float* sDco = (float*)(wl + L.dco);
    float* tP2 = (float*)(wl + L.t2);
    double* gW = (double*)(lds + SPLIT_WAVES * L.bytes);
    double* gPsi = gW + nq_all;
    double* gTab = gPsi + nq_all * NV;
    float* gTabF = (float*)(gTab + nq_all * ns * D);
    float* gTr = gTabF + 32 * ns * D;            // [NTR][ns][ns]

    // tables, once per block
    for (int i = tid; i < nq_all; i += blockDim.x) gW[i] = a.W[i];
    for (int i = tid; i < nq_all * NV; i += blockDim.x) gPsi[i] = a.psi[i];
    for (int i = tid; i < nq_all * ns * D; i += blockDim.x) gTab[i] = a.dphi[i];
    for (int i = tid; i < 32 * ns * D; i += blockDim.x) gTabF[i] = i < nq * ns * D ? (float)a.dphi[i] : 0.f;
    // padding points q >= nq carry zero weights and zero matrices
    for (int i = lane; i < EB * 32 * 2; i += 64) {
        const int q = (i >> 1) & 31;
        if (q >= nq) sWall[i] = 0.f;
    }
    for (int i = lane; i < EB * 32 * 9; i += 64) {
        const int q = (i / 9) & 31;
        if (q >= nq) sMall[i] = 0.f;
    }
    // summed weights for the hoisted point loop of P1 simplices
    double wsum = 0.0;
    for (int q = 0; q < nq_all; ++q) wsum += a.W[q];
    const PointTables pt{gW, gPsi, gTab, nq_all, a.collapse, wsum, a.mu, a.lam};
    __syncthreads();
    if (NTR > 0) {
        // trace tables S_ab over the whole rule (pairs a <= b in row order)
        for (int i = tid; i < NTR * ns * ns; i += blockDim.x) {
            const int r = i / (ns * ns), jk = i - r * ns * ns, j = jk / ns, k = jk - j * ns;
            const int ta = D == 3 ? (r < 3 ? 0 : r < 5 ? 1 : 2) : (r < 2 ? 0 : 1);
            const int tb = D == 3 ? (r < 3 ? r : r < 5 ? r - 2 : 2) : (r < 2 ? r : 1);
            double x = 0.0;
            for (int q = 0; q < nq_all; ++q) {
                const double* gq = gTab + q * ns * D;
                double t = gq[j * D + ta] * gq[k * D + tb];
                if (ta != tb) t += gq[j * D + tb] * gq[k * D + ta];
                x = fma(gW[q], t, x);
            }
            gTr[i] = (float)x;
        }
        __syncthreads();
    }

    constexpr int S2 = (ns * ns + 63) / 64;   // trace entries per lane: e = lane + 64 s

    const int64_t stride = (int64_t)gridDim.x * SPLIT_WAVES * EB;
    constexpr int nbatch_in = EB * nin;
    constexpr int NPRE = (nbatch_in + 63) / 64;   // prefetch registers per lane
    // a batch's inputs are two contiguous ranges: coordinates [EB][NVD], then
    // coefficients [EB][ncf]; sBuf keeps that layout
    double pre[NPRE];
    auto fetch = [&](int64_t first) {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int t = lane + 64 * k;
            pre[k] = 0.0;
            if (t < EB * NVD) {
                if (first * NVD + t < a.E * NVD) pre[k] = a.coords[first * NVD + t];
            } else if (t < nbatch_in) {
                if (first * ncf + (t - EB * NVD) < a.E * ncf) pre[k] = a.coeff[first * ncf + (t - EB * NVD)];
            }
        }
    };
    int64_t b0 = ((int64_t)blockIdx.x * SPLIT_WAVES + wave) * EB;
    // inputs of a batch go to LDS right after the previous batch's point
    // phase (the only reader of sBuf).  The compiler's wait for their loads
    // is a full one (it cannot count the element loop's stores), so it also
    // waits for the stores of the batch before; a variant whose stores were
    // counted exactly (the wait then left them in flight) ran no faster
    auto stage = [&]() {
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int t = lane + 64 * k;
            if (t < nbatch_in) sBuf[t] = pre[k];
        }
    };
    fetch(b0);
    stage();
    fetch(b0 + stride);

    const int col = lane & 31, half = lane >> 5;
    // columns >= n only feed rows/columns of the 32x32 tile that are never
    // stored, so their operand values just have to stay finite
    const bool cvalid = col < n;
    const int cc = cvalid ? col / ns : 0;
    const int cj = cvalid ? col - cc * ns : 0;
    static_assert(n <= 32 && nin <= SPLIT_MAX_IN, "element matrix must fit one 32x32 tile");

    for (; b0 < a.E; b0 += stride) {
        // --- A: flags of this batch (its inputs are in LDS) --------------------
        if (lane < EB) sFlag[lane] = 0;
        wave_sync();

        // --- B: float64 point data, one lane per (element, point); every lane
        // maps its own element (no serial geometry pass) ------------------------
#pragma unroll 1
        for (int t = lane; t < EB * nq; t += 64) {
            const int ib = t / nq, q = t - ib * nq;
            if (b0 + ib >= a.E) continue;
            const double* xe = sBuf + ib * NVD;                 // coordinates
            const double* ce = sBuf + EB * NVD + ib * ncf;      // coefficients
            double K[3][3], adet, det, Jm[9];
            const int bad_geo = affine_map<CELL>(xe, K, adet, &det, Jm);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (r >= D || c >= D) K[r][c] = 0.0;
            double w0, w1, M[3][3];
            int bad;
            if (HYP) {
                bad = hyper_point_from_gradient<CELL, ns>(ce, Jm, det, adet, q, pt, w0, w1, M);
            } else {
                double w2;
                bad = vector_point_data<FORM, CELL, ns>(ce, K, adet, q, pt, w0, w1, w2, M);
            }
            // signed square roots of the two product weights (the operands
            // are fp32, so the root is taken in fp32); bit t + 1 of the
            // element's flag word records a negative weight of product t
            float* sW = sWall + ib * 32 * 2;
            float* sMt = sMall + ib * 32 * 9;
            const float f0 = (float)w0, f1 = (float)w1;
            sW[q * 2 + 0] = copysignf(sqrtf(fabsf(f0)), f0);
            sW[q * 2 + 1] = copysignf(sqrtf(fabsf(f1)), f1);
            const int neg = (f0 < 0.f ? 2 : 0) | (f1 < 0.f ? 4 : 0) | (bad || bad_geo ? 1 : 0);
            if (neg) atomicOr(&sFlag[ib], neg);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) sMt[q * 9 + c * 3 + r] = (float)M[r][c];
            if (HYP && q == 0) {
                // coefficients mu |det J| (K K^T)_ab of the trace tables
                const double sc = a.mu * adet;
#pragma unroll
                for (int r = 0; r < NTR; ++r) {
                    const int ta = D == 3 ? (r < 3 ? 0 : r < 5 ? 1 : 2) : (r < 2 ? 0 : 1);
                    const int tb = D == 3 ? (r < 3 ? r : r < 5 ? r - 2 : 2) : (r < 2 ? r : 1);
                    double g = 0.0;
#pragma unroll
                    for (int c = 0; c < D; ++c) g = fma(K[ta][c], K[tb][c], g);
                    sDco[ib * 8 + r] = (float)(sc * g);
                }
            }
        }
        wave_sync();
        // the next batch's inputs (loaded during this batch's point phase)
        stage();
        fetch(b0 + 2 * stride);

        // --- C, D: per element of the batch ------------------------------------
#pragma unroll 1
        for (int ib = 0; ib < EB; ++ib) {
            const int64_t e = b0 + ib;
            if (e >= a.E) break;
            const float* sW = sWall + ib * 32 * 2;
            const float* sMt = sMall + ib * 32 * 9;
            const int negw = __builtin_amdgcn_readfirstlane(sFlag[ib]);

            v16f accL, acc2;
            // column (c, j) of the operand at point q: x = sum_a M[a][c] dphi_{q,j,a}
            auto colx = [&](int q) -> float {
                const float* gh = gTabF + (q * ns + cj) * D;
                const float* m = sMt + q * 9 + cc * 3;
                float x = m[0] * gh[0];
#pragma unroll
                for (int b = 1; b < D; ++b) x = fmaf(m[b], gh[b], x);
                return x;
            };
            auto sgn = [&](int q, int t) -> unsigned { return __float_as_uint(sW[q * 2 + t]) & 0x80000000u; };
            if (PREC == SPLIT_BF16X3) {
                constexpr int KW = NQP == 8 ? 4 : 8;    // points per lane per instruction
                typedef __bf16 vbf __attribute__((ext_vector_type(KW)));
                typedef unsigned vu __attribute__((ext_vector_type(KW / 2)));
                auto mma = [&](const vbf& x, const vbf& y, const v16f& acc) -> v16f {
                    if constexpr (KW == 4)
                        return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(__builtin_bit_cast(v4s, x),
                                                                        __builtin_bit_cast(v4s, y), acc, 0, 0, 0);
                    else
                        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
                };
                // Scaled columns at the lane's KW points: with the signed roots
                // r_t of the weights, z = |r_t| x enters as the A operand and
                // sign(r_t) z as the B operand (an exact sign-bit flip); z is
                // split into bf16 hi + lo and hi*hi + hi*lo + lo*hi accumulated
                // SG: the product's weights may be negative (a branch on the
                // element's flag word, taken once per element)
                auto product = [&](auto sg, const float* x, int q0, int t, v16f acc) -> v16f {
                    typedef float v2f __attribute__((ext_vector_type(2)));
                    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
                    vu hu, lu;
#pragma unroll
                    for (int i = 0; i < KW / 2; ++i) {
                        // one packed conversion gives both his; their fp32
                        // values are the upper halves of the packed word
                        const float z0 = fabsf(sW[(q0 + 2 * i) * 2 + t]) * x[2 * i];
                        const float z1 = fabsf(sW[(q0 + 2 * i + 1) * 2 + t]) * x[2 * i + 1];
                        const unsigned hb = __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){z0, z1}, v2bf));
                        const float h0 = __uint_as_float(hb << 16), h1 = __uint_as_float(hb & 0xffff0000u);
                        hu[i] = hb;
                        lu[i] = __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){z0 - h0, z1 - h1}, v2bf));
                    }
                    const vbf h = __builtin_bit_cast(vbf, hu), l = __builtin_bit_cast(vbf, lu);
                    if constexpr (decltype(sg)::value) {
                        vu sm;
#pragma unroll
                        for (int i = 0; i < KW / 2; ++i)
                            sm[i] = (sgn(q0 + 2 * i, t) >> 16) | sgn(q0 + 2 * i + 1, t);
                        const vbf hb = __builtin_bit_cast(vbf, hu ^ sm);
                        const vbf lb = __builtin_bit_cast(vbf, lu ^ sm);
                        acc = mma(l, hb, acc);
                        acc = mma(h, lb, acc);
                        return mma(h, hb, acc);
                    } else {
                        acc = mma(l, h, acc);
                        acc = mma(h, l, acc);
                        return mma(h, h, acc);
                    }
                };
                // both point blocks' columns first, then the products, with no
                // branch in between
                auto run = [&](auto s0, auto s1) {
                    constexpr int NKB = NQP / (2 * KW);
                    float x[NKB][KW];
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                        for (int i = 0; i < KW; ++i) x[kb][i] = colx(2 * KW * kb + KW * half + i);
                    const v16f zero = {};
                    accL = zero;
                    acc2 = zero;
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb) {
                        const int q0 = 2 * KW * kb + KW * half;
                        accL = product(s0, x[kb], q0, 0, accL);
                        acc2 = product(s1, x[kb], q0, 1, acc2);
                    }
                };
                typedef std::integral_constant<bool, true> Neg;
                typedef std::integral_constant<bool, false> Pos;
                if (negw & 6) run(Neg(), Neg());
                else run(Pos(), Pos());
            } else {
                const v16f zero = {};
                accL = zero;
                acc2 = zero;
#pragma unroll 2
                for (int ks = 0; ks < NQP / 2; ++ks) {
                    const int q = 2 * ks + half;
                    const float x = colx(q);
                    const float r0 = sW[q * 2 + 0], r1 = sW[q * 2 + 1];
                    accL = __builtin_amdgcn_mfma_f32_32x32x2f32(fabsf(r0) * x, r0 * x, accL, 0, 0, 0);
                    acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(fabsf(r1) * x, r1 * x, acc2, 0, 0, 0);
                }
            }

            // --- D: epilogue ------------------------------------------------
            // P_2 to LDS, then the trace term D of this element into a 16x16
            // LDS matrix (lane entries e = lane + 64 s)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * half + (r & 3);
                tP2[row * SPLIT_TILE_LD + col] = acc2[r];
            }
            if (HYP) {
                float dco[NTR > 0 ? NTR : 1];
#pragma unroll
                for (int t = 0; t < NTR; ++t) dco[t] = sDco[ib * 8 + t];
#pragma unroll
                for (int s2 = 0; s2 < S2; ++s2) {
                    const int ee = lane + 64 * s2;
                    if (ee < ns * ns) {
                        float dv = 0.f;
#pragma unroll
                        for (int t = 0; t < NTR; ++t) dv = fmaf(dco[t], gTr[t * ns * ns + ee], dv);
                        sDtr[(ee / ns) * 16 + ee % ns] = dv;
                    }
                }
                wave_sync();
            } else {
                wave_sync();
#pragma unroll
                for (int s2 = 0; s2 < S2; ++s2) {
                    const int ee = lane + 64 * s2;
                    if (ee < ns * ns) {
                        const int j = ee / ns, k = ee % ns;
                        float dv = 0.f;
#pragma unroll
                        for (int b = 0; b < D; ++b) dv += tP2[(b * ns + j) * SPLIT_TILE_LD + b * ns + k];
                        sDtr[j * 16 + k] = dv;
                    }
                }
                wave_sync();
            }
            // A[(c,j),(cc,cj)] = P_lam + P_2[(cc,j),(c,cj)] + delta_{c,cc} D[j][cj];
            // the lane's rows are 8 (r / 4) + r % 4 (+4 in the upper half)
            const bool bad = (negw & 1) != 0;
            const double nanv = __builtin_nan("");
            if (col < n) {
                // lane base: its column, and the upper half's four-row shift,
                // so every row offset below is a constant
                double* o = a.out + e * (int64_t)n * n + col + (half ? 4 * n : 0);
                const float* tb = tP2 + cc * ns * SPLIT_TILE_LD + cj;
                const float* db = sDtr + cj;
                if (bad) {   // uniform over the wavefront
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row0 = 8 * (r >> 2) + (r & 3);
                        if (half ? row0 + 4 < n : row0 < n) store_out(o + row0 * n, nanv, a.nt);
                    }
                } else {
                    // every LDS read first, unpredicated (rows past the matrix
                    // read row 0's entries), so that their latencies overlap;
                    // then the sums and the stores
                    float tv[16], dvv[16];
                    bool diag[16];
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row0 = 8 * (r >> 2) + (r & 3), row1 = row0 + 4;
                        const int c0 = row0 < n ? row0 / ns : 0, j0 = row0 < n ? row0 - c0 * ns : 0;
                        const int c1 = row1 < n ? row1 / ns : 0, j1 = row1 < n ? row1 - c1 * ns : 0;
                        const int c = half ? c1 : c0, j = half ? j1 : j0;
                        tv[r] = tb[j * SPLIT_TILE_LD + c * ns];
                        dvv[r] = db[j * 16];
                        diag[r] = c == cc;
                    }
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row0 = 8 * (r >> 2) + (r & 3), row1 = row0 + 4;
                        if (half ? row1 < n : row0 < n) {
                            const float v = accL[r] + tv[r] + (diag[r] ? dvv[r] : 0.f);
                            store_out(o + row0 * n, (double)v, a.nt);
                        }
                    }
                }
            }
            if (bad && lane == 0 && a.status) atomicAdd(a.status, 1);
            wave_sync();
        }
    }
}

}  // namespace fe
