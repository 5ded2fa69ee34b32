// Streaming kernel for the vector forms at degree 1 on simplices, where
// every reference gradient is constant, so F and the operand columns are
// invariant in the point loop (generalised code motion, Sec. 3.2): the
// point loop collapses to integrated weights and an element is its
// geometry, three scalars and two small sets of vectors.
//
// With K = J^{-1}, g_j = K^T dphi_j (the physical gradients) and, for the
// hyperelastic form, A = J + H (H = sum_k u_k (x) dphi_k), M = A^{-1},
// s_j = M^T dphi_j = F^{-T} g_j, J_F = det A / det J:
//   A_e[(c,j),(e,k)] = w0 s_{j,c} s_{k,e} + w1 s_{j,e} s_{k,c} + delta_ce w2 g_j . g_k
// elasticity: s = g, w0 = |det J| int lambda, w1 = w2 = |det J| int mu
// (the P1 Lame fields integrated exactly over the reference cell);
// hyperelastic: w = |det J| sum_q W_q, w0 = w lambda,
// w1 = w (mu - lambda ln J_F), w2 = w mu.  All float64.
//
// Schedule: a persistent grid over tiles of VP1_TE consecutive elements.
// One lane per element maps it and writes its record (s, g, w) to LDS; then
// one lane per (element, row) forms the row from the records.  A tile's
// rows are contiguous in memory, so a wavefront's 64 rows are one stretch:
// the wavefront stages them in its own LDS area and stores the stretch in
// consecutive 16-byte pieces, lane after lane.
#include "device_common.hpp"
#include "internal.hpp"

namespace fe {

namespace {

constexpr int VP1_TE = 64;       // elements per tile
constexpr int VP1_BLOCK = 256;
constexpr int VP1_WAVES = VP1_BLOCK / 64;

template <int CELL>
struct VP1 {
    static constexpr int D = cell_dim(CELL), NS = D + 1, N = D * NS, NVD = NS * D;
    static constexpr int DP = D == 3 ? 4 : 2;             // padded vector
    // record: s [NS][DP], g [NS][DP], w0 w1 w2 flag
    static constexpr int REC = 2 * NS * DP + 4;
};

template <int FORM, int CELL>
__global__ __launch_bounds__(VP1_BLOCK) void k_vec_p1(VecP1Args a)
{
    using T = VP1<CELL>;
    constexpr int D = T::D, NS = T::NS, N = T::N, NVD = T::NVD, DP = T::DP, REC = T::REC;
    constexpr bool HYP = FORM == HYPERELASTIC;
    constexpr int NCF = HYP ? D * NS : 2 * NS;
    __shared__ double sG[NS][D];          // reference gradients (constant)
    __shared__ double sPsi[NS];           // integrals of the P1 basis over the reference cell
    __shared__ double sRec[VP1_TE * REC];
    __shared__ double sStage[VP1_WAVES][64 * N];   // a wavefront's rows
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < NS * D) sG[tid / D][tid % D] = a.dphi[tid];
    if (tid < NS) {
        double x = 0.0;
        for (int q = 0; q < a.nq; ++q) x = fma(a.W[q], a.psi[q * NS + tid], x);
        sPsi[tid] = x;
    }
    double wsum = 0.0;
    for (int q = 0; q < a.nq; ++q) wsum += a.W[q];
    __syncthreads();

    for (int64_t t0 = (int64_t)blockIdx.x * VP1_TE; t0 < a.E; t0 += (int64_t)gridDim.x * VP1_TE) {
        // --- one lane per element: geometry, point data, record --------------
        if (tid < VP1_TE && t0 + tid < a.E) {
            const int64_t e = t0 + tid;
            double v[NVD], cf[NCF];
#pragma unroll
            for (int i = 0; i < NVD; ++i) v[i] = a.coords[e * NVD + i];
#pragma unroll
            for (int i = 0; i < NCF; ++i) cf[i] = a.coeff[e * NCF + i];
            double K[3][3], adet, det, Jm[9];
            int bad = affine_map<CELL>(v, K, adet, &det, Jm);
            double* r = sRec + tid * REC;
            double w0, w1, w2, M[3][3];
            if (HYP) {
                double A[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int c = 0; c < 3; ++c) A[i][c] = Jm[i * 3 + c];
#pragma unroll
                for (int k = 0; k < NS; ++k)
#pragma unroll
                    for (int i = 0; i < D; ++i)
#pragma unroll
                        for (int c = 0; c < D; ++c) A[i][c] = fma(cf[i * NS + k], sG[k][c], A[i][c]);
                const double da = inverse_small<D>(A, M);
                const double jf = da / det;
                bad |= !(jf > 0.0);
                const double w = wsum * adet;
                w0 = w * a.lam;
                w1 = w * (a.mu - a.lam * log(jf));
                w2 = w * a.mu;
            } else {
                double lam = 0.0, mu = 0.0;
#pragma unroll
                for (int l = 0; l < NS; ++l) {
                    lam = fma(cf[l], sPsi[l], lam);
                    mu = fma(cf[NS + l], sPsi[l], mu);
                }
                w0 = adet * lam;
                w1 = adet * mu;
                w2 = w1;
            }
            // g_j = K^T dphi_j; s_j = M^T dphi_j (elasticity: s = g)
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int c = 0; c < DP; ++c) {
                    double g = 0.0, s = 0.0;
                    if (c < D)
#pragma unroll
                        for (int b = 0; b < D; ++b) {
                            g = fma(K[b][c], sG[j][b], g);
                            if (HYP) s = fma(M[b][c], sG[j][b], s);
                        }
                    r[NS * DP + j * DP + c] = g;
                    r[j * DP + c] = HYP ? s : g;
                }
            r[2 * NS * DP + 0] = w0;
            r[2 * NS * DP + 1] = w1;
            r[2 * NS * DP + 2] = w2;
            r[2 * NS * DP + 3] = bad ? 1.0 : 0.0;
            if (bad && a.status) atomicAdd(a.status, 1);
        }
        __syncthreads();

        // --- one lane per (element, row): the row from the records -----------
        const int nrows = (int)((a.E - t0 < VP1_TE ? a.E - t0 : VP1_TE) * N);
        typedef double d2 __attribute__((ext_vector_type(2)));
        double* st = sStage[wave];
        for (int u0 = wave * 64; u0 < nrows; u0 += VP1_BLOCK) {
            const int u = u0 + lane;
            if (u < nrows) {
                const int el = u / N, row = u - el * N;
                const int c = row / NS, j = row - c * NS;
                const double* r = sRec + el * REC;
                const double w0 = r[2 * NS * DP + 0], w1 = r[2 * NS * DP + 1], w2 = r[2 * NS * DP + 2];
                const bool bad = r[2 * NS * DP + 3] != 0.0;
                double sj[D], gj[D];
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    sj[b] = r[j * DP + b];
                    gj[b] = r[NS * DP + j * DP + b];
                }
                // the column coefficients of this row: w0 s_{j,c}, w1 s_{j,e}
                const double a0 = w0 * sj[c];
                double vals[N];
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    double sk[D], gk[D];
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        sk[b] = r[k * DP + b];
                        gk[b] = r[NS * DP + k * DP + b];
                    }
                    double gg = gj[0] * gk[0];
#pragma unroll
                    for (int b = 1; b < D; ++b) gg = fma(gj[b], gk[b], gg);
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2) {
                        double x = fma(a0, sk[e2], w1 * sj[e2] * sk[c]);
                        if (e2 == c) x = fma(w2, gg, x);
                        vals[e2 * NS + k] = bad ? __builtin_nan("") : x;
                    }
                }
#pragma unroll
                for (int i = 0; i < N; i += 2) *reinterpret_cast<d2*>(st + lane * N + i) = (d2){vals[i], vals[i + 1]};
            }
            wave_sync();
            // the stretch of rows u0 .. u0 + 63 in 16-byte pieces
            const int npieces = ((nrows - u0 < 64 ? nrows - u0 : 64) * N) / 2;
            d2* o = reinterpret_cast<d2*>(a.out + t0 * (int64_t)(N * N) + (int64_t)u0 * N);
            const d2* sp = reinterpret_cast<const d2*>(st);
            for (int pc = lane; pc < npieces; pc += 64) {
                if (a.nt) __builtin_nontemporal_store(sp[pc], o + pc);
                else o[pc] = sp[pc];
            }
            wave_sync();
        }
        __syncthreads();
    }
}

template <int FORM>
hipError_t go(int cell, const VecP1Args& a, int grid, hipStream_t s)
{
    if (cell == TRI) hipLaunchKernelGGL((k_vec_p1<FORM, TRI>), dim3(grid), dim3(VP1_BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_vec_p1<FORM, TET>), dim3(grid), dim3(VP1_BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace

size_t vec_p1_lds_bytes(int cell)
{
    return cell == TRI ? sizeof(double) * (VP1_TE * VP1<TRI>::REC + 3 * 2 + 3 + VP1_WAVES * 64 * VP1<TRI>::N)
                       : sizeof(double) * (VP1_TE * VP1<TET>::REC + 4 * 3 + 4 + VP1_WAVES * 64 * VP1<TET>::N);
}

int vec_p1_elems_per_block() { return VP1_TE; }

hipError_t launch_vec_p1(int form, int cell, const VecP1Args& a, int grid, hipStream_t s)
{
    if (cell != TRI && cell != TET) return hipErrorInvalidValue;
    return form == ELASTICITY ? go<ELASTICITY>(cell, a, grid, s) : go<HYPERELASTIC>(cell, a, grid, s);
}

}  // namespace fe
