// Shared host/device definitions of the local-assembly library: cell traits,
// space dimensions and table layouts.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define FE_HD __host__ __device__
#else
#define FE_HD
#endif

namespace fe {

enum CellId { TRI = 0, TET = 1, PRISM = 2 };
enum FormId { MASS = 0, HELMHOLTZ = 1, ELASTICITY = 2, HYPERELASTIC = 3 };

// topological / geometric dimension and vertex count of each reference cell
FE_HD constexpr int cell_dim(int cell) { return cell == TRI ? 2 : 3; }
FE_HD constexpr int cell_nv(int cell) { return cell == TRI ? 3 : (cell == TET ? 4 : 6); }

// scalar Lagrange DOFs of degree p (equispaced lattice; prism = tri x interval)
FE_HD constexpr int n_scalar(int cell, int p)
{
    return cell == TRI ? (p + 1) * (p + 2) / 2
         : cell == TET ? (p + 1) * (p + 2) * (p + 3) / 6
                       : (p + 1) * (p + 2) / 2 * (p + 1);
}

FE_HD constexpr bool is_vector_form(int form) { return form == ELASTICITY || form == HYPERELASTIC; }

// rows of the element matrix
FE_HD constexpr int n_rows(int form, int cell, int p)
{
    return is_vector_form(form) ? cell_dim(cell) * n_scalar(cell, p) : n_scalar(cell, p);
}

// Pre-evaluated reference tensors of the scalar forms (Sec. 2.3 / Alg. 2):
//   r = 0           mass table  Mhat[j][k] = sum_q W phi_j phi_k
//   r = 1 .. d      Khat_aa[j][k] = sum_q W dphi_j/dX_a dphi_k/dX_a
//   r = d+1 ..      Khat_ab + Khat_ba for a < b, pairs (0,1),(0,2),(1,2)
// The geometry tensor multiplying table r is |detJ| for r = 0 and
// G'_ab = |detJ| sum_b K[a][b] K[b'][b] for the stiffness tables.
FE_HD constexpr int n_tables(int form, int cell)
{
    return form == MASS ? 1 : 1 + cell_dim(cell) * (cell_dim(cell) + 1) / 2;
}

// points per collapsed direction for an exact rule of degree qdeg
FE_HD constexpr int rule_m(int qdeg) { return qdeg < 1 ? 1 : (qdeg + 2) / 2; }

FE_HD constexpr int rule_size(int cell, int qdeg)
{
    return cell == TRI   ? (qdeg <= 2 ? 3 : rule_m(qdeg) * rule_m(qdeg))
         : cell == TET   ? rule_m(qdeg) * rule_m(qdeg) * rule_m(qdeg)
                         : (qdeg <= 2 ? 3 : rule_m(qdeg) * rule_m(qdeg)) * rule_m(qdeg);
}

// exact degree (the hyperelastic integrand is not a polynomial: degree 4);
// every form gains p per pre-multiplying coefficient function of degree p
// (nf, Sec. 7.1)
FE_HD constexpr int default_qdeg(int form, int cell, int p, int nf = 0)
{
    return (form == MASS || form == HELMHOLTZ) ? (2 + nf) * p
         : form == ELASTICITY ? (cell == PRISM ? 2 * p + 1 : 2 * p - 1) + nf * p
                              : 4 + nf * p;
}

// the form's own coefficient DOFs per element (elasticity: the Lame DOFs
// [2][nv]; hyperelastic: the displacement DOFs [d][n_s]); nf pre-multiplying
// functions follow them in the element's record, [nf][n_s]
FE_HD constexpr int own_coeff(int form, int cell, int p)
{
    return form == ELASTICITY ? 2 * cell_nv(cell) : form == HYPERELASTIC ? cell_dim(cell) * n_scalar(cell, p) : 0;
}

constexpr int MAX_DEGREE = 4;
constexpr int MAX_QDEG = 20;
constexpr int MAX_NS = 75;     // prism P4

}  // namespace fe
