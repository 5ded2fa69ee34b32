// The compressed-row pattern of a global matrix (fe_csr_t) and what its
// insertion kernels share.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace fe {

constexpr int CSR_WAVE = 64;
// Rows of an insertion visit: their pointers sit in one lane each (lane
// VISIT_ROWS holds the end), and their element lists are staged in LDS once
// per visit.
constexpr int VISIT_ROWS = 32;
// round lengths kept for 1, 2, 4, ..., 32 rows per round
constexpr int CSR_RR_LEVELS = 6;

// LDS of one insertion wavefront: the values of a round plus the visit's
// element lists
inline size_t insert_lds(int round_cap, int visit_pairs)
{
    return sizeof(double) * (size_t)round_cap + sizeof(uint32_t) * (size_t)visit_pairs;
}

}  // namespace fe

struct fe_csr {
    int64_t E = 0, N = 0, nnz = 0;
    int n = 0, max_row = 0, max_pairs = 0;
    int round_len[fe::CSR_RR_LEVELS] = {0};   // longest aligned run of 1, 2, 4, ... rows (entries)
    int visit_pairs = 0;                      // most element pairs of an insertion visit
    int64_t* row_ptr = nullptr;    // [N + 1]
    int32_t* cols = nullptr;       // [nnz]
    int64_t* pair_ptr = nullptr;   // [N + 1]
    uint32_t* list = nullptr;      // [E * n] pairs e * n + j of each row, increasing
    uint16_t* pos = nullptr;       // [E * n][n] for list entry t = (e, j): position of column dofs[e][k]
                                   // within row dofs[e][j]
    double* geo = nullptr;         // [E][8] geometry workspace of fe_assemble_csr (first use)
};

namespace fe {
void csr_free(fe_csr* c);
}
