// Pre-evaluated contraction for the scalar forms (mass, Helmholtz):
//     A_e[j][k] = sum_r c_r(e) R_r[j][k]
// with reference tensors R_r pre-evaluated once (Sec. 3.3, Algorithm 2; the
// tensor-contraction mode of Sec. 2.3, Eqs. (8)-(9)) and the geometry tensor
// c(e) = (|det J|, G'_00, G'_11, ..., G'_01, ...), G' = |det J| K K^T.
//
// The work is bound by the store of A (a few flops per 8-byte entry), so the
// kernel is organised around the output stream:
//   * a workgroup owns a tile of `chunk` consecutive elements, whose output
//     blocks are one contiguous span of chunk*n^2 doubles;
//   * the span is walked `epi` elements at a time; thread t owns the fixed
//     slots f = t + B*m of the epi*n^2 entries of one step, so every step
//     stores a contiguous range with consecutive lanes on consecutive words;
//   * because a slot always maps to the same table entry (j,k), the thread
//     keeps R_r[j][k] for its slots in registers (MM slots per pass, more
//     passes when n^2 is large), and only the per-element geometry tensor is
//     read from LDS.
// Nothing proportional to the element count is stored besides A itself
// (Constraint 1, Sec. 3.4).
#pragma once
#include "device_common.hpp"

namespace fe {

struct PreevalArgs {
    const double* coords;
    const double* tables;   // [NT][nn]
    double* out;            // [E][nn]
    int* status;
    int64_t E;
    int nn;                 // n^2
    int epi;                // elements per step
    int chunk;              // elements per tile (multiple of epi)
    int nt;                 // non-temporal output stores
};

template <int FORM, int CELL>
constexpr int preeval_nt() { return n_tables(FORM, CELL); }

// Geometry tensor of one element (vertices v); returns nonzero when the
// element is flagged.
template <int FORM, int CELL>
__device__ __forceinline__ int preeval_coeffs(const double* __restrict__ vsrc, double* c)
{
    // no contraction, so that every kernel computes the same tensor bit for bit
#pragma clang fp contract(off)
    constexpr int D = cell_dim(CELL), NV = cell_nv(CELL);
    double v[NV * D];
#pragma unroll
    for (int k = 0; k < NV * D; ++k) v[k] = vsrc[k];
    double K[3][3], adet;
    const int bad = affine_map<CELL>(v, K, adet);
    c[0] = adet;
    if (FORM == HELMHOLTZ) {
        int r = 1;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < D; ++b) s += K[a][b] * K[a][b];
            c[r++] = adet * s;
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int a2 = a + 1; a2 < D; ++a2) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < D; ++b) s += K[a][b] * K[a2][b];
                c[r++] = adet * s;
            }
    }
    return bad;
}

// One tile of elements [e_begin, min(e_begin + chunk, E)).  sG: LDS of
// chunk * (NT + nv * d) doubles (geometry tensors, then the staged
// coordinates).  Every thread of the block must call it.
template <int FORM, int CELL, int MM>
__device__ void preeval_tile(const PreevalArgs& a, int64_t e_begin, double* sG)
{
    constexpr int NT = preeval_nt<FORM, CELL>();
    constexpr int NVD = cell_nv(CELL) * cell_dim(CELL);
    const int tid = threadIdx.x, B = blockDim.x;
    const int64_t rem = a.E - e_begin;
    const int ne = rem < a.chunk ? (int)rem : a.chunk;
    double* sV = sG + (size_t)a.chunk * NT;

    // coordinates of the tile: one contiguous span, loaded coalesced
    load_to_lds(sV, a.coords + e_begin * NVD, ne * NVD);
    __syncthreads();
    for (int i = tid; i < ne; i += B) {
        double c[NT];
        const int bad = preeval_coeffs<FORM, CELL>(sV + i * NVD, c);
        if (bad) {
#pragma unroll
            for (int r = 0; r < NT; ++r) c[r] = __builtin_nan("");
            if (a.status) atomicAdd(a.status, 1);
        }
#pragma unroll
        for (int r = 0; r < NT; ++r) sG[i * NT + r] = c[r];
    }
    __syncthreads();

    const int nn = a.nn, epi = a.epi;
    const int slots = epi * nn;
    const int per_pass = B * MM;
    const int npass = (slots + per_pass - 1) / per_pass;
    const int steps = (ne + epi - 1) / epi;
    for (int pass = 0; pass < npass; ++pass) {
        double R[MM][NT];
        int el[MM], fs[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const int f = tid + B * (pass * MM + m);
            fs[m] = f;
            if (f < slots) {
                el[m] = f / nn;
                const int jk = f - el[m] * nn;
#pragma unroll
                for (int r = 0; r < NT; ++r) R[m][r] = a.tables[r * nn + jk];
            } else {
                el[m] = 1 << 30;
#pragma unroll
                for (int r = 0; r < NT; ++r) R[m][r] = 0.0;
            }
        }
        if (epi == 1) {
            // one element per step: its geometry tensor is shared by every slot
            for (int it = 0; it < steps; ++it) {
                double* o = a.out + (e_begin + (int64_t)it) * nn;
                double g[NT];
#pragma unroll
                for (int r = 0; r < NT; ++r) g[r] = sG[it * NT + r];
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    if (el[m] == 0) {
                        double v = g[0] * R[m][0];
#pragma unroll
                        for (int r = 1; r < NT; ++r) v = fma(g[r], R[m][r], v);
                        store_out(o + fs[m], v, a.nt);
                    }
                }
            }
        } else {
            for (int it = 0; it < steps; ++it) {
                const int lim = ne - it * epi;
                double* o = a.out + (e_begin + (int64_t)it * epi) * nn;
                const double* g0 = sG + it * epi * NT;
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    if (el[m] < lim) {
                        const double* g = g0 + el[m] * NT;
                        double v = g[0] * R[m][0];
#pragma unroll
                        for (int r = 1; r < NT; ++r) v = fma(g[r], R[m][r], v);
                        store_out(o + fs[m], v, a.nt);
                    }
                }
            }
        }
    }
    __syncthreads();
}

// Streaming variant, used when one step's slots fit in registers
// (epi * n^2 <= blockDim * MM): every block loads its table entries once and
// keeps them for the whole launch.  The grid is persistent and the steps of
// epi consecutive elements are grouped into visits of T = chunk / epi
// consecutive steps; block b (after the XCD-aware renumbering below) takes
// the visits b, b + G, b + 2G, ..., so the grid writes one window of G
// visits that sweeps through the output, each block one contiguous run at a
// time.  Geometry tensors are produced one element per thread for the next
// S = min(T, blockDim / epi) steps of the block at a time, double-buffered in
// LDS: the coordinate loads of the next group are issued before the stores of
// the current group.  sG: 2 * S * epi * NT doubles.
template <int FORM, int CELL, int MM>
__device__ void preeval_stream(const PreevalArgs& a, double* sG)
{
    constexpr int NT = preeval_nt<FORM, CELL>();
    constexpr int NVD = cell_nv(CELL) * cell_dim(CELL);
    const int tid = threadIdx.x, B = blockDim.x;
    const int nn = a.nn, epi = a.epi;
    const int G = gridDim.x;
    // Consecutive workgroups are dealt to the 8 XCDs in turn; renumber them
    // so that consecutive logical blocks (adjacent visits, hence adjacent
    // coordinates and output lines) share an XCD and its L2.
    const int b = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const int T = a.chunk / epi;                    // steps per visit
    const int64_t nsteps = (a.E + epi - 1) / epi;
    const int64_t nvisits = (nsteps + T - 1) / T;
    if (b >= nvisits) return;
    const int64_t K = ((nvisits - 1 - b) / G + 1) * T;   // local steps (the last visit may run past the end)
    // Steps per geometry group: at most one visit, so that a group's
    // coordinates are one contiguous range (one page) of the input.
    const int S = T < B / epi ? T : B / epi;
    const int GE = S * epi;                         // elements per group (<= B)

    // table entries of this thread's slots (one pass covers a step)
    double R[MM][NT];
    int el[MM], jk[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int f = tid + B * m;
        if (f < epi * nn) {
            el[m] = f / nn;
            jk[m] = f - el[m] * nn;
#pragma unroll
            for (int r = 0; r < NT; ++r) R[m][r] = a.tables[r * nn + jk[m]];
        } else {
            el[m] = 1 << 30;
            jk[m] = 0;
#pragma unroll
            for (int r = 0; r < NT; ++r) R[m][r] = 0.0;
        }
    }

    // coordinates of this thread's element in group g (registers)
    double v[NVD];
    bool have = false;
    auto fetch = [&](int64_t g) {
        const int64_t L = g * S + tid / epi;
        const int64_t e = ((b + (L / T) * G) * T + L % T) * epi + tid % epi;
        have = tid < GE && L < K && e < a.E;
        if (have) {
#pragma unroll
            for (int i = 0; i < NVD; ++i) v[i] = a.coords[e * NVD + i];
        }
    };
    auto geometry = [&](double* dst) {
        if (have) {
            double c[NT];
            if (preeval_coeffs<FORM, CELL>(v, c)) {
#pragma unroll
                for (int r = 0; r < NT; ++r) c[r] = __builtin_nan("");
                if (a.status) atomicAdd(a.status, 1);
            }
#pragma unroll
            for (int r = 0; r < NT; ++r) dst[tid * NT + r] = c[r];
        }
    };

    fetch(0);
    geometry(sG);
    __syncthreads();
    for (int64_t g = 0; g * S < K; ++g) {
        fetch(g + 1);
        const double* g0 = sG + (g & 1) * GE * NT;
        const int ns_here = (int)(K - g * S < S ? K - g * S : S);
        // visit and step within it of the group's first local step
        int64_t vq = (g * S) / T;
        int vr = (int)((g * S) % T);
        for (int i = 0; i < ns_here; ++i) {
            const int64_t e0 = ((b + vq * G) * T + vr) * epi;
            if (++vr == T) {
                vr = 0;
                ++vq;
            }
            if (e0 >= a.E) continue;
            const int64_t rem = a.E - e0;
            const int lim = rem < epi ? (int)rem : epi;
            double* o = a.out + e0 * nn;
            const double* gi = g0 + i * epi * NT;
            if (epi == 1) {
                double gg[NT];
#pragma unroll
                for (int r = 0; r < NT; ++r) gg[r] = gi[r];
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    if (el[m] == 0) {
                        double x = gg[0] * R[m][0];
#pragma unroll
                        for (int r = 1; r < NT; ++r) x = fma(gg[r], R[m][r], x);
                        store_out(o + jk[m], x, a.nt);
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    if (el[m] < lim) {
                        const double* gm = gi + el[m] * NT;
                        double x = gm[0] * R[m][0];
#pragma unroll
                        for (int r = 1; r < NT; ++r) x = fma(gm[r], R[m][r], x);
                        store_out(o + el[m] * nn + jk[m], x, a.nt);
                    }
                }
            }
        }
        geometry(sG + ((g + 1) & 1) * GE * NT);
        __syncthreads();
    }
}

}  // namespace fe
