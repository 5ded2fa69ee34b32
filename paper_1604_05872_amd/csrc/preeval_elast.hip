// Pre-evaluated linear elasticity (Sec. 3.3 with the coefficient expansion
// of Sec. 4.2): the Lame fields are P1, lambda(X) = sum_l lambda_l psi_l(X)
// and likewise mu, so with g_{j,c} = sum_a K[a][c] dphi_{j,a} every
// monomial's coefficient is a polynomial and the reduction over points
// hoists into reference tables
//     T_{l,a,b}[j][k] = sum_q W_q psi_l(X_q) dphi_{q,j,a} dphi_{q,k,b}
// (iota = n_c = the P1 basis size, rho = d^2 per table set).  Block (c, e)
// of the element matrix is then
//     A[(c,j),(e,k)] = sum_{l,a,b} C^{ce}_{l,a,b} T_{l,a,b}[j][k],
//     C^{ce}_{l,a,b} = |det J| (lambda_l K_ac K_be + mu_l K_ae K_bc
//                               + delta_ce mu_l (K K^T)_ab):
// dense products of a coefficient matrix with the table matrix on the FP64
// matrix cores (v_mfma_f64_16x16x4_f64).
//
// On triangles and tetrahedra the kernel is shaped by the order of its
// stores more than by its arithmetic: the output (88 KB per element at tet
// P4) is written far faster when each wavefront walks a few element matrices
// front to back than when many wavefronts write interleaved pieces of the
// same matrices (a store-only kernel with the 4.3 GB of tet P4 takes 0.85 ms
// in the first order and 1.1-1.3 ms in the second on MI355X).  So a unit of
// work is (floor(16 / d) elements, block row c) and belongs to one
// wavefront: the 16 rows of each MFMA tile are the (element, e) pairs of the
// unit (15 of 16 used in 3D, all 16 in 2D), its columns 16 consecutive (j, k)
// entries, and as the wavefront walks the table columns in order it fills
// block row c of its elements row after row.  Prisms, whose tables do not
// stay in the L2, use a column-group kernel that reads each table value once
// per 16 elements and d^2 blocks.
#include <algorithm>
#include <mutex>

#include "device_common.hpp"
#include "internal.hpp"

namespace fe {

typedef double v4d_e __attribute__((ext_vector_type(4)));
typedef unsigned u2_e __attribute__((ext_vector_type(2)));
// buffer resource word 3 on gfx950: a raw (stride 0) byte buffer whose
// accesses are range-checked against num_records; stores beyond it are
// dropped
constexpr int BUFFER_WORD3 = 0x00020000;

namespace {

constexpr int elast_nt(int cell) { return cell_nv(cell) * cell_dim(cell) * cell_dim(cell); }
// the contraction length in MFMA steps of 4 (tet 9, triangle 3, prism 14)
constexpr int elast_nk(int cell) { return (elast_nt(cell) + 3) / 4; }
__host__ __device__ constexpr unsigned elast_table_doubles_dev(int cell, int ns)
{
    return (unsigned)((ns * ns + 15) / 16) * 64u * (unsigned)elast_nk(cell);
}

// Table layout: Tb[g][kk][kq][i] = T_{t = 4 kk + kq}[column 16 g + i] (zero
// for t >= n_c d^2 or a column past n_s^2): the operand values of one
// contraction step of a column group are 64 consecutive doubles, one per lane.
__global__ void k_elast_tables(int nq, int ns, int d, int nc, int nk, const double* __restrict__ W,
                               const double* __restrict__ psi, const double* __restrict__ dphi, double* __restrict__ T)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nn = ns * ns, nt = nc * d * d, ng = (nn + 15) / 16;
    if (tid >= (int64_t)ng * 64 * nk) return;
    const int lane = (int)(tid % 64), i = lane % 16, kq = lane / 16;
    const int kk = (int)((tid / 64) % nk), g = (int)(tid / (64 * nk));
    const int t = 4 * kk + kq, col = 16 * g + i;
    double x = 0.0;
    if (t < nt && col < nn) {
        const int j = col / ns, k = col % ns;
        const int l = t / (d * d), a = (t / d) % d, b = t % d;
        for (int q = 0; q < nq; ++q)
            x = fma(W[q] * psi[q * nc + l], dphi[(q * ns + j) * d + a] * dphi[(q * ns + k) * d + b], x);
    }
    T[tid] = x;
}

struct ElastArgs {
    const double* coords;
    const double* coeff;   // [E][2][nc]: lambda, then mu, at the vertices
    double* out;
    int* status;
    const double* T;       // blocked tables (k_elast_tables)
    int64_t E;
    int ns;
    int parts;             // column-group kernel: column-group ranges per tile
};

// a byte offset past every unit's records: an invalid row plus an invalid
// column stays below 2^32 and above the buffer's range
constexpr unsigned OFF_NONE = 0x40000000u;
constexpr int GP = 2;       // column groups per step (independent accumulator chains)
constexpr int NSLOT = 4;    // steps of table operands in LDS

__device__ __forceinline__ void lds_barrier()
{
    // orders LDS only: nothing here waits for the global stores
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Unit kernel (triangles, tetrahedra): four compute wavefronts, each taking
// units (EPU elements, block row c), and one loader wavefront.
//  * On gfx950 a global store is counted with the loads it precedes, so a
//    wavefront that both loads and stores waits for its stores whenever it
//    needs a load.  Here only the loader reads global memory: the table
//    operands of each step (the same for every unit, so read once per
//    workgroup and step) and the element data of the next unit round, into
//    LDS.  The compute wavefronts read LDS and write the output; they never
//    wait for memory, and their stores stay in flight.
//  * An FP64 MFMA and a VALU instruction of any wavefront on the same SIMD
//    do not overlap (a 16x16x4 product takes about 64 cycles, a VALU
//    instruction 4 to 8 more), so the step loop keeps its VALU work small:
//    the column part of every store offset comes from an LDS table built
//    once, and units without flagged elements store their values unselected.
//  * All five wavefronts take one workgroup barrier per step.  In step s the
//    loader writes the operands of step s + NSLOT - 1 to LDS (read during
//    step s - 1) and reads those of step s + NSLOT; a compute wavefront
//    multiplies step s (two column groups, two accumulator chains), reads
//    the operands of step s + 1 from LDS into registers and stores the tiles
//    of step s - 1, each lane its rows kq + 4 r at its column.
template <int CELL>
__global__ __launch_bounds__(320) void k_preeval_elast(ElastArgs a)
{
    constexpr int D = cell_dim(CELL), NC = cell_nv(CELL), NVD = NC * D;
    constexpr int NT = elast_nt(CELL), NK = elast_nk(CELL);
    constexpr int EPU = 16 / D;               // elements per unit
    constexpr int ED = NVD + 2 * NC;          // element record: vertices, then lambda and mu at the vertices
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i16 = lane & 15, kq = lane >> 4;
    const int ns = a.ns, nn = ns * ns, n = D * ns, ng = (nn + 15) / 16;
    const int nst = (ng + GP - 1) / GP;       // steps per unit
    const unsigned nn_e = (unsigned)n * (unsigned)n;
    const int units = (int)((a.E + EPU - 1) / EPU * D);
    const int stride = gridDim.x * 4, first = blockIdx.x * 4;
    // unit rounds of this workgroup (its compute wavefront 0 has the most)
    const int rounds = first < units ? (units - first + stride - 1) / stride : 0;
    const int total = rounds * nst;           // steps with work
    extern __shared__ double lds_elast[];
    double* bring = lds_elast;                               // [NSLOT][GP][NK][64]
    double* ering = bring + NSLOT * GP * NK * 64;            // [2][4][EPU][ED]
    unsigned* coff = reinterpret_cast<unsigned*>(ering + 2 * 4 * EPU * ED);   // [nst GP][16]

    // byte offset of column 16 g + i of a block row within a block (j n + k),
    // OFF_NONE past n_s^2
    for (int i = threadIdx.x; i < nst * GP * 16; i += blockDim.x) {
        const int j = i / ns, k = i - j * ns;
        coff[i] = i < nn ? (unsigned)(j * n + k) * 8u : OFF_NONE;
    }

    if (w == 4) {
        // ---------------------------------------------------------------- loader
        // Every read is issued one step before its values go to LDS, so the
        // loader waits for reads that had a whole step to arrive.
        double x[GP][NK];                     // table operands of one step, in flight
        auto fetch = [&](int st) {
#pragma unroll
            for (int q = 0; q < GP; ++q) {
                const int g = GP * st + q < ng ? GP * st + q : ng - 1;
#pragma unroll
                for (int kk = 0; kk < NK; ++kk) x[q][kk] = a.T[((size_t)g * NK + kk) * 64 + lane];
            }
        };
        auto put = [&](int sl) {
#pragma unroll
            for (int q = 0; q < GP; ++q)
#pragma unroll
                for (int kk = 0; kk < NK; ++kk) bring[((sl * GP + q) * NK + kk) * 64 + lane] = x[q][kk];
        };
        // element records of a unit round: [4 wavefronts][EPU][ED], NE per lane
        constexpr int NE = (4 * EPU * ED + 63) / 64;
        double ex[NE];
        auto fetch_elems = [&](int r) {
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                const int idx = lane + 64 * i;
                const int wv = idx / (EPU * ED), m = (idx / ED) % EPU, f = idx % ED;
                const int u = first + wv + r * stride;
                const int64_t e = (int64_t)(u / D) * EPU + m;
                double v = 0.0;
                if (idx < 4 * EPU * ED && u < units && e < a.E)
                    v = f < NVD ? a.coords[e * NVD + f] : a.coeff[e * 2 * NC + (f - NVD)];
                ex[i] = v;
            }
        };
        auto put_elems = [&](int r) {
            double* dst = ering + (r & 1) * 4 * EPU * ED;
#pragma unroll
            for (int i = 0; i < NE; ++i)
                if (lane + 64 * i < 4 * EPU * ED) dst[lane + 64 * i] = ex[i];
        };
        // steps 0, 1 and 2 in place, step 3 in flight, round 0's records in place
#pragma unroll
        for (int g = 0; g < NSLOT - 1; ++g) {
            fetch(g % nst);
            put(g);
        }
        fetch((NSLOT - 1) % nst);
        fetch_elems(0);
        put_elems(0);
        lds_barrier();
        int stn = NSLOT % nst, r = 0, st = 0;  // unit step of global step gs + NSLOT; round and step of gs
        bool epend = false;                    // round r + 1's records in flight
        for (int gs = 0; gs < total; ++gs) {
            put((gs + NSLOT - 1) % NSLOT);     // step gs + NSLOT - 1
            fetch(stn);
            if (epend) {
                put_elems(r + 1);
                epend = false;
            }
            if (st == 0 && r + 1 < rounds) {
                // the next round's records: in place before it begins
                fetch_elems(r + 1);
                if (nst == 1) put_elems(r + 1);
                else epend = true;
            }
            if (++stn == nst) stn = 0;
            if (++st == nst) {
                st = 0;
                ++r;
            }
            lds_barrier();
        }
        return;
    }

    // -------------------------------------------------------------------- compute
    const int er = i16 / D, e2r = i16 - er * D;   // the operand row this lane forms
    double A[NK];
    // store state: the unit whose tiles are being stored
    unsigned ro[4] = {OFF_NONE, OFF_NONE, OFF_NONE, OFF_NONE};
    bool nanr[4] = {false, false, false, false};
    bool anybad = false;
    __amdgpu_buffer_rsrc_t out_rsrc = __builtin_amdgcn_make_buffer_rsrc(a.out, 0, 0, BUFFER_WORD3);
    double B[2][GP][NK];
    v4d_e acc[2][GP];
#pragma unroll
    for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
        for (int q = 0; q < GP; ++q) acc[p2][q] = (v4d_e){0.0, 0.0, 0.0, 0.0};
    auto read_ops = [&](double (&Bs)[GP][NK], int sl) {
#pragma unroll
        for (int q = 0; q < GP; ++q)
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) Bs[q][kk] = bring[((sl * GP + q) * NK + kk) * 64 + lane];
    };
    lds_barrier();
    read_ops(B[0], 0);
    int r = 0, st = 0, stp = 0;               // round and unit step of gs; unit step of gs - 1
    // new store state, taking effect after the previous unit's last tiles
    unsigned nro[4];
    bool nnanr[4], nanybad = false;
    __amdgpu_buffer_rsrc_t nrsrc = out_rsrc;
    // global steps in pairs: the register slot (ps) is a constant
    for (int g0 = 0; g0 < total + 1; g0 += 2) {
#pragma unroll
        for (int ps = 0; ps < 2; ++ps) {
            const int gs = g0 + ps;
            if (gs <= total) {
                const bool work = gs < total;
                if (work && st == 0) {
                    // a new unit: its coefficient operand from the element
                    // records, A[i16][4 kk + kq] = C^{c e2r}_{t}(element er)
                    const int u = first + w + r * stride;
                    const int64_t e0 = (int64_t)(u / D) * EPU;
                    const int c = u - u / D * D;
                    const int ne = u < units ? (a.E - e0 < EPU ? (int)(a.E - e0) : EPU) : 0;
                    int bad = 0;
#pragma unroll
                    for (int kk = 0; kk < NK; ++kk) A[kk] = 0.0;
                    if (er < ne) {
                        const double* rec = ering + (((r & 1) * 4 + w) * EPU + er) * ED;
                        double v[NVD], lm[2 * NC];
#pragma unroll
                        for (int i = 0; i < NVD; ++i) v[i] = rec[i];
#pragma unroll
                        for (int i = 0; i < 2 * NC; ++i) lm[i] = rec[NVD + i];
                        double K[3][3], adet;
                        bad = affine_map<CELL>(v, K, adet);
                        // columns c (uniform) and e2r (per lane) of K, selected
                        // rather than indexed so that K stays in registers
                        double Kc[D], Ke[D];
#pragma unroll
                        for (int m = 0; m < D; ++m) {
                            Kc[m] = K[m][0];
                            Ke[m] = K[m][0];
#pragma unroll
                            for (int x = 1; x < D; ++x) {
                                Kc[m] = c == x ? K[m][x] : Kc[m];
                                Ke[m] = e2r == x ? K[m][x] : Ke[m];
                            }
                        }
                        const bool diag = c == e2r;
                        // every t = (l, aa, b) with compile-time indices; lane
                        // kq keeps t = 4 kk + kq
#pragma unroll
                        for (int kk = 0; kk < NK; ++kk) {
                            double xs[4];
#pragma unroll
                            for (int q4 = 0; q4 < 4; ++q4) {
                                const int t = 4 * kk + q4;
                                xs[q4] = 0.0;
                                if (t < NT) {
                                    const int l = t / (D * D), aa = (t / D) % D, b = t % D;
                                    const double lam = lm[l], mu = lm[NC + l];
                                    double x = lam * (Kc[aa] * Ke[b]) + mu * (Ke[aa] * Kc[b]);
                                    double g = 0.0;
#pragma unroll
                                    for (int m = 0; m < D; ++m) g = fma(K[aa][m], K[b][m], g);
                                    x = diag ? fma(mu, g, x) : x;
                                    xs[q4] = x * adet;
                                }
                            }
                            A[kk] = kq == 0 ? xs[0] : kq == 1 ? xs[1] : kq == 2 ? xs[2] : xs[3];
                        }
                        // each flagged element is reported once, by its block row 0
                        if (bad && c == 0 && e2r == 0 && kq == 0 && a.status) atomicAdd(a.status, 1);
                    }
                    // flagged elements' rows are stored as NaN (a rare, separate path)
                    nanybad = __builtin_amdgcn_readfirstlane(__ballot(bad) != 0 ? 1 : 0) != 0;
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int i = kq + 4 * rr, ei = i / D, ci = i - ei * D;
                        nnanr[rr] = __shfl(bad, i) != 0;
                        nro[rr] = ei < ne ? ((unsigned)ei * nn_e + (unsigned)((c * ns) * n + ci * ns)) * 8u : OFF_NONE;
                    }
                    nrsrc = __builtin_amdgcn_make_buffer_rsrc(a.out + (u < units ? e0 * (int64_t)nn_e : 0), 0,
                                                              (int)((unsigned)ne * nn_e * 8u), BUFFER_WORD3);
                }
                // the tiles of step gs - 1, with the state of its unit: values
                // and byte offsets (in step 0 they go to an empty buffer)
                double sv[GP * 4];
                unsigned so[GP * 4];
#pragma unroll
                for (int q = 0; q < GP; ++q) {
                    const unsigned co = coff[(GP * stp + q) * 16 + i16];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        // through a scalar: a bit cast of the vector element
                        // itself is compiled as a cast of element 0 here
                        const double v = acc[1 - ps][q][rr];
                        sv[q * 4 + rr] = v;
                        so[q * 4 + rr] = ro[rr] + co;
                    }
                }
                if (anybad) {
                    // flagged elements' rows are stored as NaN (a rare path)
#pragma unroll
                    for (int i = 0; i < GP * 4; ++i) sv[i] = nanr[i % 4] ? __builtin_nan("") : sv[i];
                }
                auto store1 = [&](int i) {
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_e, sv[i]), out_rsrc, so[i], 0, 0);
                };
                if (work) {
                    // step gs: its operands are in B[ps]; those of gs + 1 into B[1 - ps]
                    read_ops(B[1 - ps], (gs + 1) % NSLOT);
#pragma unroll
                    for (int q = 0; q < GP; ++q) acc[ps][q] = (v4d_e){0.0, 0.0, 0.0, 0.0};
                    // the stores of step gs - 1 between the products of step gs,
                    // so that the matrix core keeps working while they issue
#pragma unroll
                    for (int kk = 0; kk < NK; ++kk) {
#pragma unroll
                        for (int q = 0; q < GP; ++q)
                            acc[ps][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[kk], B[ps][q][kk], acc[ps][q], 0, 0, 0);
                        if (kk < GP * 4) store1(kk);
                    }
#pragma unroll
                    for (int i = NK; i < GP * 4; ++i) store1(i);
#pragma unroll
                    for (int kk = 0; kk < NK; ++kk) {
                        __builtin_amdgcn_sched_group_barrier(0x008, GP, 0);   // MFMA
                        if (kk < GP * 4) __builtin_amdgcn_sched_group_barrier(0x040, 1, 0);   // VMEM write
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < GP * 4; ++i) store1(i);
                }
                if (work && st == 0) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        ro[rr] = nro[rr];
                        nanr[rr] = nnanr[rr];
                    }
                    anybad = nanybad;
                    out_rsrc = nrsrc;
                }
                stp = st;
                if (++st == nst) {
                    st = 0;
                    ++r;
                }
                if (work) lds_barrier();
            }
        }
    }
}

// Column-group kernel (prisms).  At n_s = 75 the tables (2.5 MB) do not
// stay in the L2 while the output streams through it, so each table value
// read must feed as many products as possible: a workgroup takes a 16-element
// tile, forms the coefficient rows of all d^2 blocks (c, e) in LDS (rows
// padded to an odd number of doubles), and its eight wavefronts split the
// 16-entry column groups, each group's table operand feeding the d^2 blocks
// as independent accumulator chains.  A tile's column groups are split into
// ranges run by consecutive workgroups.
__host__ __device__ constexpr int pe_waves(int cell) { return cell == PRISM ? 8 : 4; }

template <int CELL>
__global__ __launch_bounds__(64 * pe_waves(CELL)) __attribute__((amdgpu_waves_per_eu(2))) void k_preeval_elast_cols(ElastArgs a)
{
    constexpr int PE_WAVES = pe_waves(CELL);
    constexpr int D = cell_dim(CELL), NC = cell_nv(CELL), NVD = NC * D;
    constexpr int NT = NC * D * D, NTP = (NT + 7) / 8 * 8, NB = D * D, NK = NTP / 4;
    static_assert(NK == elast_nk(CELL), "table padding");
    // coefficient rows [block][element][(l, a, b)], rows NTP + 1 doubles apart
    // so that the 16 rows of an operand read fall in distinct LDS banks
    constexpr int LDA = NTP + 1;
    __shared__ double sA[NB * 16 * LDA];
    __shared__ double sG[16 * 12];           // K [9], |det J|, flag
    __shared__ double sL[16 * 2 * NC];       // Lame nodal values
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const __amdgpu_buffer_rsrc_t trsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(a.T), 0, (int)(elast_table_doubles_dev(CELL, a.ns) * 8u), BUFFER_WORD3);
    const unsigned tvo = (unsigned)(tid & 63) * 8u;
    const int i16 = lane & 15, kq = lane >> 4;
    const int ns = a.ns, nn = ns * ns, n = D * ns;
    const int64_t ntiles = (a.E + 15) / 16;
    const int ncb = (nn + 15) / 16;
    const int parts = a.parts;                 // column-group ranges per tile
    const int64_t units = ntiles * parts;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t tile = u / parts;
        const int part = (int)(u - tile * parts);
        const int64_t e0 = tile * 16;
        const int ne = a.E - e0 < 16 ? (int)(a.E - e0) : 16;
        // geometry and Lame values of the tile's elements
        if (tid < 16) {
            double K[3][3], adet;
            int bad = 0;
            if (tid < ne) {
                double v[NVD];
#pragma unroll
                for (int i = 0; i < NVD; ++i) v[i] = a.coords[(e0 + tid) * NVD + i];
                bad = affine_map<CELL>(v, K, adet);
            } else {
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int q = 0; q < 3; ++q) K[r][q] = 0.0;
                adet = 0.0;
            }
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int q = 0; q < D; ++q) sG[tid * 12 + r * 3 + q] = K[r][q];
            sG[tid * 12 + 9] = adet;
            sG[tid * 12 + 10] = bad ? 1.0 : 0.0;
            // the tile's first unit reports flagged elements
            if (bad && part == 0 && a.status) atomicAdd(a.status, 1);
        }
        for (int i = tid; i < 16 * 2 * NC; i += blockDim.x) sL[i] = i < ne * 2 * NC ? a.coeff[e0 * 2 * NC + i] : 0.0;
        __syncthreads();
        // coefficient rows C^{c e2}[e][(l, a, b)] of every block, zero-padded to
        // NTP: one work item per (block, element, l) forms its D^2 entries with
        // compile-time (a, b), so the setup of a unit stays short against its
        // products (it is repeated by each of the tile's column-group ranges)
        for (int it = tid; it < NB * 16 * NC; it += blockDim.x) {
            const int blk = it / (16 * NC), r = it - blk * 16 * NC, e = r / NC, l = r - e * NC;
            const int c = blk / D, e2 = blk - c * D;
            const double* K = sG + e * 12;
            const double lam = sL[e * 2 * NC + l] * K[9], mu = sL[e * 2 * NC + NC + l] * K[9];
            double Kc[D], Ke[D];
#pragma unroll
            for (int m = 0; m < D; ++m) {
                Kc[m] = K[m * 3 + c];
                Ke[m] = K[m * 3 + e2];
            }
            double* dst = sA + (blk * 16 + e) * LDA + l * D * D;
            if (c == e2) {
#pragma unroll
                for (int aa = 0; aa < D; ++aa)
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        double g = 0.0;
#pragma unroll
                        for (int m = 0; m < D; ++m) g = fma(K[aa * 3 + m], K[b * 3 + m], g);
                        dst[aa * D + b] = fma(mu, g, lam * (Kc[aa] * Kc[b]) + mu * (Kc[aa] * Kc[b]));
                    }
            } else {
#pragma unroll
                for (int aa = 0; aa < D; ++aa)
#pragma unroll
                    for (int b = 0; b < D; ++b) dst[aa * D + b] = lam * (Kc[aa] * Ke[b]) + mu * (Ke[aa] * Kc[b]);
            }
        }
        for (int i = tid; i < NB * 16 * (NTP - NT); i += blockDim.x) {
            const int row = i / (NTP - NT);
            sA[row * LDA + NT + (i - row * (NTP - NT))] = 0.0;
        }
        __syncthreads();
        // the tile's output as a buffer of ne element matrices (byte records)
        const int nn_e = n * n;
        const __amdgpu_buffer_rsrc_t out_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            a.out + e0 * (int64_t)nn_e, 0, (int)((unsigned)ne * (unsigned)nn_e * 8u), BUFFER_WORD3);
        bool bad_row[4];
        // the lane's rows (elements kq + 4 r) as byte offsets in the tile's
        // records, past them for elements beyond the tile
        unsigned rowo[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bad_row[r] = sG[(kq + 4 * r) * 12 + 10] != 0.0;
            rowo[r] = kq + 4 * r < ne ? (unsigned)(kq + 4 * r) * (unsigned)nn_e * 8u : OFF_NONE;
        }
        // flagged elements' rows are stored as NaN (a rare, separate path)
        const bool anybad = __builtin_amdgcn_readfirstlane(__ballot(bad_row[0] || bad_row[1] || bad_row[2] || bad_row[3]) != 0 ? 1 : 0) != 0;
        // this unit's column groups, wavefront w taking every PE_WAVES-th; a
        // group's table values feed all NB blocks, loaded one group ahead
        // into the other of two register sets
        const int cb_lo = (int)((int64_t)ncb * part / parts), cb_hi = (int)((int64_t)ncb * (part + 1) / parts);
        double B[2][NK];
        auto load_b = [&](double (&Bs)[NK], int cb) {
            // the blocked tables: this lane's NK operand values of group cb
            // (buffer loads: a scalar group offset and constant lane offsets)
            const int soff = cb * 64 * NK * 8;
#pragma unroll
            for (int kk = 0; kk < NK; ++kk)
                Bs[kk] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(trsrc, tvo + 512u * kk, soff, 0));
        };
        auto group = [&](const double (&Bc)[NK], int cb) {
            // the lane's column (j, k) of every block: a per-lane byte offset
            // (past the records beyond n_s^2); block (c, e2) adds a scalar one
            const int col = 16 * cb + i16;
            const unsigned cog = col < nn ? (unsigned)((col / ns) * n + col % ns) * 8u : OFF_NONE;
            unsigned vo[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) vo[r] = rowo[r] + cog;
            // blocks in groups of D (D independent accumulator chains per
            // group, few registers live), each group stored before the next
#pragma unroll 1
            for (int c = 0; c < D; ++c) {
                v4d_e acc[D];
#pragma unroll
                for (int e2 = 0; e2 < D; ++e2) acc[e2] = (v4d_e){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < NK; ++kk)
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2)
                        acc[e2] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            sA[((c * D + e2) * 16 + i16) * LDA + 4 * kk + kq], Bc[kk], acc[e2], 0, 0, 0);
                // lane holds elements kq + 4 r at column (j, k) of blocks
                // (c, e2).  Every store is issued; the buffer unit drops those
                // past the tile's records
                if (anybad) {
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2) {
                        const int soff = ((c * ns) * n + e2 * ns) * 8;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double v = bad_row[r] ? __builtin_nan("") : acc[e2][r];
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_e, v), out_rsrc, vo[r], soff, 0);
                        }
                    }
                } else {
#pragma unroll
                    for (int e2 = 0; e2 < D; ++e2) {
                        const int soff = ((c * ns) * n + e2 * ns) * 8;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            // through a scalar: a bit cast of the vector element
                            // itself is compiled as a cast of element 0 here
                            const double v = acc[e2][r];
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2_e, v), out_rsrc, vo[r], soff, 0);
                        }
                    }
                }
            }
        };
        int cb = cb_lo + w;
        if (cb < cb_hi) load_b(B[0], cb);
        for (; cb < cb_hi; cb += 2 * PE_WAVES) {
            if (cb + PE_WAVES < cb_hi) load_b(B[1], cb + PE_WAVES);
            group(B[0], cb);
            if (cb + PE_WAVES >= cb_hi) break;
            if (cb + 2 * PE_WAVES < cb_hi) load_b(B[0], cb + 2 * PE_WAVES);
            group(B[1], cb + PE_WAVES);
        }
        __syncthreads();
    }
}

// raise the kernel's dynamic LDS limit to `bytes` once per (device, cell)
// (a host-side attribute, so it is also safe while a stream is captured)
hipError_t allow_dynamic_lds(const void* fn, int cell, size_t bytes)
{
    static std::mutex mu;
    static size_t done[64][3] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) return e != hipSuccess ? e : hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (done[dev][cell] >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done[dev][cell] = bytes;
    return e;
}

}  // namespace

size_t elast_table_doubles(int cell, int ns)
{
    return elast_table_doubles_dev(cell, ns);
}

hipError_t launch_elast_tables(int nq, int ns, int d, int nc, const double* W, const double* psi, const double* dphi,
                               double* T, hipStream_t s)
{
    const int cell = d == 2 ? TRI : nc == 4 ? TET : PRISM;
    const int64_t n = (int64_t)elast_table_doubles(cell, ns);
    hipLaunchKernelGGL(k_elast_tables, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, nq, ns, d, nc,
                       elast_nk(cell), W, psi, dphi, T);
    return hipGetLastError();
}

hipError_t launch_preeval_elast(int cell, const double* coords, const double* coeff, double* out, int* status,
                                const double* T, int64_t E, int ns, int grid_per_cu, int cus, hipStream_t s)
{
    ElastArgs a;
    a.coords = coords;
    a.coeff = coeff;
    a.out = out;
    a.status = status;
    a.T = T;
    a.E = E;
    a.ns = ns;
    if (cell == PRISM) {
        // a workgroup per (tile, column-group range).  A tile's ranges are
        // consecutive units, so they run at the same time: splitting a large
        // tile into ranges of about 20 column groups narrows the span of
        // output that the grid writes at once, and the L2 merges more of its
        // partial lines before they are evicted.  Small problems split their
        // tiles so that every CU gets two units.
        const int64_t tiles = (E + 15) / 16;
        const int64_t want = (int64_t)cus * 2;
        const int ncb = (ns * ns + 15) / 16;
        const int by_width = std::min(16, (ncb + 19) / 20);
        const int by_count = (int)std::max<int64_t>(1, std::min<int64_t>(4, (want + tiles - 1) / tiles));
        a.parts = std::max(1, std::min(ncb, std::max(by_width, by_count)));
        const int64_t units = tiles * a.parts;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)cus * grid_per_cu));
        hipLaunchKernelGGL((k_preeval_elast_cols<PRISM>), dim3(grid), dim3(64 * pe_waves(PRISM)), 0, s, a);
        return hipGetLastError();
    }
    a.parts = 1;
    // four compute wavefronts (a unit each) and a loader per workgroup
    const int d = cell_dim(cell), epu = 16 / d;
    const int64_t units = (E + epu - 1) / epu * d;
    if (units >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const int64_t blocks = (units + 3) / 4;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)cus * grid_per_cu));
    // LDS: the operand ring, the element records and the column offsets
    const int nk = elast_nk(cell), nvd = cell_nv(cell) * d, ed = nvd + 2 * cell_nv(cell);
    const int nst = ((ns * ns + 15) / 16 + GP - 1) / GP;
    const size_t lds = sizeof(double) * ((size_t)NSLOT * GP * nk * 64 + 2 * 4 * (size_t)epu * ed) +
                       sizeof(unsigned) * (size_t)nst * GP * 16;
    const void* fn = cell == TRI ? (const void*)k_preeval_elast<TRI> : (const void*)k_preeval_elast<TET>;
    hipError_t e = allow_dynamic_lds(fn, cell, lds);
    if (e != hipSuccess) return e;
    if (cell == TRI) hipLaunchKernelGGL((k_preeval_elast<TRI>), dim3(grid), dim3(320), lds, s, a);
    else hipLaunchKernelGGL((k_preeval_elast<TET>), dim3(grid), dim3(320), lds, s, a);
    return hipGetLastError();
}

int preeval_elast_grid_per_cu(int cell, int ns)
{
    // unit kernel: one wavefront per SIMD (more resident wavefronts write more
    // element matrices at once, which the HBM absorbs less well).
    // Column-group kernel: wide element matrices (48 or more column groups)
    // one resident workgroup per CU, narrow ones two
    if (cell != PRISM) return 1;
    return (ns * ns + 15) / 16 >= 48 ? 1 : 2;
}

}  // namespace fe
