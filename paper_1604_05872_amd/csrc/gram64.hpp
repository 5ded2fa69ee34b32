// Float64 matrix-core contraction for the vector forms (n = d * n_s <= 32).
//
// The sharing-eliminated quadrature sum of the elasticity and hyperelastic
// forms (Sec. 3.2, Algorithm 1) is, per element, a sum of weighted Gram
// products of one matrix of per-point basis data (see split.hpp for the
// derivation).  Here every step stays float64: with the signed roots r_t of
// the point weights (vector_point.hpp),
//     P_t = Z_t^T diag(sign r_t) Z_t,   Z_t[q][(c,j)] = |r_t(q)| x_q[(c,j)],
// x = g (elasticity) or s = F^{-T} g (hyperelastic).  P_lam (t = 0) and P_2
// (t = 1) are symmetric, so the 16x16 tiles 00, 01 and 11 of the padded
// 32x32 matrix cover them, one v_mfma_f64_16x16x4_f64 per tile and 4 points.
// The trace term D[j][k] = sum_q mu'_q g_{q,j} . g_{q,k}: for elasticity
// (mu varies over the element) it is the block trace of the P_2 tile; for
// the hyperelastic form mu is a constant, so D is pre-evaluated (Sec. 3.3) as
//     D[j][k] = mu |det J| sum_{a<=b} (K K^T)_ab S_ab[j][k]
// from tables S_ab formed once per workgroup (the same split of the form as
// in split.hpp), all in float64.  Then
//     A[(c,j),(e,k)] = P_lam[(c,j),(e,k)] + P_2[(e,j),(c,k)] + delta_ce D[j][k].
//
// Instruction layout (16x16x4, f64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; it holds D[l / 16 + 4 r][l % 16], r = 0..3.
//
// Schedule as in split.hpp: one wavefront per element, four wavefronts per
// block with private LDS areas, batches of EB elements whose inputs are
// prefetched one batch ahead, one lane per (element, point) for the point
// data, then per element the MFMA products and an epilogue that reads the
// transposed P_2 blocks (and D) from one LDS tile and stores from registers.
#pragma once
#include "device_common.hpp"
#include "split.hpp"
#include "vector_point.hpp"

namespace fe {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int G64_WAVES = 4;
// elements per wavefront batch: hyperelastic 2 (per-point matrices in LDS),
// elasticity 4
__host__ __device__ constexpr int g64_eb(int form) { return form == HYPERELASTIC ? 2 : 4; }
constexpr int G64_TLD = 33;                     // padded tile rows
__host__ __device__ constexpr int g64_pre(int form) { return (g64_eb(form) * SPLIT_MAX_IN + 63) / 64; }

// per-wave LDS layout (bytes) for a padded point count nqp
__host__ __device__ constexpr int g64_off_rw(int form) { return g64_eb(form) * SPLIT_MAX_IN * 8; }
__host__ __device__ constexpr int g64_off_m(int form, int nqp) { return g64_off_rw(form) + g64_eb(form) * nqp * 3 * 8; }
__host__ __device__ constexpr int g64_off_geo(int form, int nqp)
{
    return g64_off_m(form, nqp) + (form == HYPERELASTIC ? g64_eb(form) * nqp * 9 * 8 : 0);
}
// hyperelastic: trace coefficients mu |det J| (K K^T)_ab [eb][8] f64
__host__ __device__ constexpr int g64_off_dco(int form, int nqp) { return g64_off_geo(form, nqp) + g64_eb(form) * 10 * 8; }
__host__ __device__ constexpr int g64_off_flag(int form, int nqp)
{
    return g64_off_dco(form, nqp) + (form == HYPERELASTIC ? g64_eb(form) * 8 * 8 : 0);
}
__host__ __device__ constexpr int g64_off_t(int form, int nqp) { return g64_off_flag(form, nqp) + 16; }
__host__ __device__ constexpr int g64_off_d(int form, int nqp) { return g64_off_t(form, nqp) + 32 * G64_TLD * 8; }
__host__ __device__ constexpr int g64_wave_bytes(int form, int nqp)
{
    return g64_off_d(form, nqp) + (form == HYPERELASTIC ? 16 * 17 * 8 : 0);
}
// block LDS: the wave areas, then W [nq], psi [nq][nv] (elasticity), dphi
// [nq][ns][d] and (hyperelastic) the trace tables [ntr][ns][ns], all f64
__host__ __device__ constexpr size_t gram64_lds_bytes(int form, int cell, int nqp, int nq, int ns)
{
    return (size_t)G64_WAVES * g64_wave_bytes(form, nqp) +
           ((size_t)nq + (form == HYPERELASTIC ? 0 : (size_t)nq * cell_nv(cell)) + (size_t)nq * ns * cell_dim(cell) +
            (size_t)split_trace_tables(form, cell) * ns * ns) * 8;
}

template <int FORM, int CELL, int P, int NQP>
__device__ void gram64_kernel_body(const SplitArgs& a, char* lds)
{
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL), NVD = NV * D;
    constexpr bool HYP = (FORM == HYPERELASTIC);
    constexpr int ns = n_scalar(CELL, P), n = D * ns;
    constexpr int NTILE = n > 16 ? 2 : 1;
    constexpr int ncf = split_coeffs_per_elem<FORM, CELL>(ns);
    constexpr int nin = NVD + ncf;
    static_assert(n <= 32 && ns <= 16 && nin <= SPLIT_MAX_IN, "element matrix must fit one 32x32 tile");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nq_all = a.nq;
    const int nq = a.collapse ? 1 : nq_all;

    char* wl = lds + wave * g64_wave_bytes(FORM, NQP);
    double* sIn = (double*)wl;
    constexpr int EB = g64_eb(FORM), PRE = g64_pre(FORM);
    double* sRw = (double*)(wl + g64_off_rw(FORM));
    double* sM = (double*)(wl + g64_off_m(FORM, NQP));
    double* sGeo = (double*)(wl + g64_off_geo(FORM, NQP));
    double* sDco = (double*)(wl + g64_off_dco(FORM, NQP));
    constexpr int NTR = split_trace_tables(FORM, CELL);
    int* sFlag = (int*)(wl + g64_off_flag(FORM, NQP));
    double* sT = (double*)(wl + g64_off_t(FORM, NQP));
    double* sD = (double*)(wl + g64_off_d(FORM, NQP));
    double* gW = (double*)(lds + G64_WAVES * g64_wave_bytes(FORM, NQP));
    double* gPsi = gW + nq_all;
    double* gTab = gPsi + (HYP ? 0 : nq_all * NV);   // the hyperelastic form has no Lame field
    double* gTr = gTab + nq_all * ns * D;             // [NTR][ns][ns]

    for (int i = tid; i < nq_all; i += blockDim.x) gW[i] = a.W[i];
    if (!HYP)
        for (int i = tid; i < nq_all * NV; i += blockDim.x) gPsi[i] = a.psi[i];
    for (int i = tid; i < nq_all * ns * D; i += blockDim.x) gTab[i] = a.dphi[i];
    // padding points q >= nq carry zero weights and zero matrices
    for (int i = lane; i < EB * NQP * 3; i += 64)
        if ((i / 3) % NQP >= nq) sRw[i] = 0.0;
    if (HYP)
        for (int i = lane; i < EB * NQP * 9; i += 64)
            if ((i / 9) % NQP >= nq) sM[i] = 0.0;
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
            gTr[i] = x;
        }
        __syncthreads();
    }

    const int64_t stride = (int64_t)gridDim.x * G64_WAVES * EB;
    constexpr int nbatch_in = EB * nin;
    double pre[PRE];
    auto fetch = [&](int64_t first) {
#pragma unroll
        for (int k = 0; k < PRE; ++k) {
            const int t = lane + 64 * k;
            const int i = t / nin, x = t - (t / nin) * nin;
            const int64_t ee = first + i;
            pre[k] = 0.0;
            if (t < nbatch_in && ee < a.E)
                pre[k] = x < NVD ? a.coords[ee * NVD + x] : a.coeff[ee * ncf + (x - NVD)];
        }
    };
    int64_t b0 = ((int64_t)blockIdx.x * G64_WAVES + wave) * EB;
    fetch(b0);

    // this lane's operand columns (c, j) = col0, col1 and its point slot
    const int i16 = lane & 15, kq = lane >> 4;
    int ccol[2], jcol[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int col = 16 * h + i16;
        ccol[h] = col < n ? col / ns : 0;     // columns >= n feed entries that are never stored
        jcol[h] = col < n ? col - (col / ns) * ns : 0;
    }

    for (; b0 < a.E; b0 += stride) {
        // --- A: inputs of this batch to LDS; loads of the next batch ----------
#pragma unroll
        for (int k = 0; k < PRE; ++k) {
            const int t = lane + 64 * k;
            if (t < nbatch_in) {
                const int i = t / nin;
                sIn[i * SPLIT_MAX_IN + (t - i * nin)] = pre[k];
            }
        }
        if (lane < EB) sFlag[lane] = 0;
        fetch(b0 + stride);
        wave_sync();

        // --- B0: geometry, one lane per element ------------------------------
        if (lane < EB && b0 + lane < a.E) {
            double K[3][3], adet;
            const int bad = affine_map<CELL>(sIn + lane * SPLIT_MAX_IN, K, adet);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) sGeo[lane * 10 + r * 3 + c] = (r < D && c < D) ? K[r][c] : 0.0;
            sGeo[lane * 10 + 9] = adet;
            if (HYP) {
                const double sc = a.mu * adet;
#pragma unroll
                for (int r = 0; r < NTR; ++r) {
                    const int ta = D == 3 ? (r < 3 ? 0 : r < 5 ? 1 : 2) : (r < 2 ? 0 : 1);
                    const int tb = D == 3 ? (r < 3 ? r : r < 5 ? r - 2 : 2) : (r < 2 ? r : 1);
                    double g = 0.0;
#pragma unroll
                    for (int c = 0; c < D; ++c) g = fma(K[ta][c], K[tb][c], g);
                    sDco[lane * 8 + r] = sc * g;
                }
            }
            if (bad) sFlag[lane] = 1;
        }
        wave_sync();

        // --- B: float64 point data, one lane per (element, point) -----------
#pragma unroll 1
        for (int t = lane; t < EB * nq; t += 64) {
            const int ib = t / nq, q = t - ib * nq;
            if (b0 + ib >= a.E) continue;
            double K[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) K[r][c] = sGeo[ib * 10 + r * 3 + c];
            double w0, w1, w2, M[3][3];
            const int bad = vector_point_data<FORM, CELL, ns>(sIn + ib * SPLIT_MAX_IN + NVD, K, sGeo[ib * 10 + 9], q, pt,
                                                              w0, w1, w2, M);
            double* rw = sRw + (ib * NQP + q) * 3;
            rw[0] = signed_root(w0);
            rw[1] = signed_root(w1);
            (void)w2;
            if (HYP) {
                double* mt = sM + (ib * NQP + q) * 9;     // [c][a] = M[a][c]
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int r = 0; r < 3; ++r) mt[c * 3 + r] = M[r][c];
            }
            if (bad) sFlag[ib] = 1;
        }
        wave_sync();

        // --- C, D: per element of the batch ------------------------------------
#pragma unroll 1
        for (int ib = 0; ib < EB; ++ib) {
            const int64_t e = b0 + ib;
            if (e >= a.E) break;
            const double* rwe = sRw + ib * NQP * 3;
            const double* me = sM + ib * NQP * 9;
            const double* ge = sGeo + ib * 10;
            double kc[2][3];   // elasticity: K[a][c] of the lane's two columns
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int b = 0; b < 3; ++b) kc[h][b] = ge[b * 3 + ccol[h]];

            v4d aL[3], a2[3];
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    aL[t][r] = 0.0;
                    a2[t][r] = 0.0;
                }

            // column value x_q[(c,j)] of the operand
            auto colx = [&](int q, int h) -> double {
                const int qt = q < nq ? q : nq - 1;      // padding points: any finite table row
                const double* gh = gTab + (qt * ns + jcol[h]) * D;
                double x;
                if (HYP) {
                    const double* m = me + q * 9 + ccol[h] * 3;
                    x = m[0] * gh[0];
#pragma unroll
                    for (int b = 1; b < D; ++b) x = fma(m[b], gh[b], x);
                } else {
                    x = kc[h][0] * gh[0];
#pragma unroll
                    for (int b = 1; b < D; ++b) x = fma(kc[h][b], gh[b], x);
                }
                return x;
            };
#pragma unroll 1
            for (int kb = 0; kb < NQP / 4; ++kb) {
                const int q = 4 * kb + kq;
                const double r0 = rwe[q * 3 + 0], r1 = rwe[q * 3 + 1];
                const double x0 = colx(q, 0);
                const double x1 = NTILE == 2 ? colx(q, 1) : 0.0;
                const double l0 = fabs(r0) * x0, l1 = fabs(r0) * x1;
                aL[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(l0, r0 * x0, aL[0], 0, 0, 0);
                const double m0 = fabs(r1) * x0, m1 = fabs(r1) * x1;
                a2[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(m0, r1 * x0, a2[0], 0, 0, 0);
                if (NTILE == 2) {
                    aL[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(l0, r0 * x1, aL[1], 0, 0, 0);
                    aL[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(l1, r0 * x1, aL[2], 0, 0, 0);
                    a2[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(m0, r1 * x1, a2[1], 0, 0, 0);
                    a2[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(m1, r1 * x1, a2[2], 0, 0, 0);
                }
            }
            // --- epilogue -----------------------------------------------------
            // P_2 (both triangles) and D to LDS; each lane then combines the
            // entries its P_lam tiles hold, and the element matrix leaves
            // through LDS
#pragma unroll
            for (int t = 0; t < (NTILE == 2 ? 3 : 1); ++t) {
                const int I = t == 2 ? 1 : 0, J = t == 0 ? 0 : 1;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + kq + 4 * r, col = 16 * J + i16;
                    sT[row * G64_TLD + col] = a2[t][r];
                    if (I != J) sT[col * G64_TLD + row] = a2[t][r];
                }
            }
            if (HYP) {
                // pre-evaluated trace term, entries e = lane + 64 s
                const double* dco = sDco + ib * 8;
#pragma unroll
                for (int s2 = 0; s2 < (ns * ns + 63) / 64; ++s2) {
                    const int ee = lane + 64 * s2;
                    if (ee < ns * ns) {
                        double dv = 0.0;
#pragma unroll
                        for (int t = 0; t < NTR; ++t) dv = fma(dco[t], gTr[t * ns * ns + ee], dv);
                        sD[(ee / ns) * 17 + ee % ns] = dv;
                    }
                }
            }
            wave_sync();
            const bool bad = sFlag[ib] != 0;
            const double nanv = __builtin_nan("");
            // the combined entry (row, col) of the element matrix from a
            // P_lam value of the lane's tiles, P_2 (and D) in LDS
            auto value = [&](int row, int col, double pl) -> double {
                if (row >= n || col >= n) return 0.0;
                const int c = row / ns, j = row - c * ns;
                const int e2 = col / ns, k = col - e2 * ns;
                double v = pl + sT[(e2 * ns + j) * G64_TLD + c * ns + k];
                if (c == e2) {
                    if (HYP) v += sD[j * 17 + k];
                    else
#pragma unroll
                        for (int b = 0; b < D; ++b) v += sT[(b * ns + j) * G64_TLD + b * ns + k];
                }
                return v;
            };
            double* o = a.out + e * (int64_t)(n * n);
            if constexpr (!HYP) {
                // every entry the lane's P_lam tiles hold (the 01 tile also
                // gives the mirrored 10 entries), kept in registers until all
                // reads of sT are done; then the element matrix is packed into
                // sT and stored as contiguous 512-byte pieces (scattered 8-byte
                // stores of single entries leave partial lines to merge:
                // elasticity P2 on 1.97M tets 4.22 -> 3.38 ms).  The
                // hyperelastic kernel keeps the scattered stores: the 16
                // values would cost it a wavefront per SIMD
                constexpr int NVAL = NTILE == 2 ? 16 : 4;
                double vals[NVAL];
                {
                    int kv = 0;
#pragma unroll
                    for (int t = 0; t < (NTILE == 2 ? 3 : 1); ++t) {
                        const int I = t == 2 ? 1 : 0, J = t == 0 ? 0 : 1;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = 16 * I + kq + 4 * r, col = 16 * J + i16;
                            vals[kv++] = value(row, col, aL[t][r]);
                            if (I != J) vals[kv++] = value(col, row, aL[t][r]);
                        }
                    }
                }
                wave_sync();
                {
                    int kv = 0;
#pragma unroll
                    for (int t = 0; t < (NTILE == 2 ? 3 : 1); ++t) {
                        const int I = t == 2 ? 1 : 0, J = t == 0 ? 0 : 1;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = 16 * I + kq + 4 * r, col = 16 * J + i16;
                            if (row < n && col < n) sT[row * n + col] = vals[kv];
                            ++kv;
                            if (I != J) {
                                if (row < n && col < n) sT[col * n + row] = vals[kv];
                                ++kv;
                            }
                        }
                    }
                }
                wave_sync();
                if (bad) {   // uniform over the wavefront
                    for (int i = lane; i < n * n; i += 64) store_out(o + i, nanv, a.nt);
                } else {
                    for (int i = lane; i < n * n; i += 64) store_out(o + i, sT[i], a.nt);
                }
            } else {
                // each entry as it is formed (rows of 16 consecutive columns;
                // the mirrored 10 tile scatters, merged in L2)
#pragma unroll
                for (int t = 0; t < (NTILE == 2 ? 3 : 1); ++t) {
                    const int I = t == 2 ? 1 : 0, J = t == 0 ? 0 : 1;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * I + kq + 4 * r, col = 16 * J + i16;
                        if (row < n && col < n) store_out(o + row * n + col, bad ? nanv : value(row, col, aL[t][r]), a.nt);
                        if (I != J && row < n && col < n)
                            store_out(o + col * n + row, bad ? nanv : value(col, row, aL[t][r]), a.nt);
                    }
                }
            }
            if (bad && lane == 0 && a.status) atomicAdd(a.status, 1);
            wave_sync();
        }
    }
}

}  // namespace fe
