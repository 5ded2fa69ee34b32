/*
 * felocal.h -- finite-element local assembly on AMD Instinct MI355X (gfx950).
 *
 * Computes per-element matrices
 *     A_e[i][j] = sum_q W_q |det J_e| * integrand(phi_i, phi_j, coefficients)(X_q)
 * (Luporini, Ham, Kelly, "An algorithm for the optimization of finite element
 * integration loops": quadrature mode Sec. 2.2 Eq. (7), tensor-contraction
 * mode Sec. 2.3 Eqs. (8)-(9)) in the flop-reduced form selected by the
 * transformation algorithm of Sec. 4.1 (Algorithm 3): pre-evaluated reference
 * tensors (Sec. 3.3, Algorithm 2) or sharing-eliminated quadrature
 * (Sec. 3.2, Algorithm 1), under the memory threshold T_H (Sec. 3.4,
 * Constraint 2).
 *
 * Conventions
 *   Reference cells: triangle (0,0),(1,0),(0,1); tetrahedron adds (0,0,1);
 *   prism = triangle x [0,1], vertices 0..2 at Z=0 and 3..5 = 0..2 + e_Z.
 *   Affine map x = v0 + J X, columns of J = v1-v0, v2-v0 (, v3-v0); prisms
 *   must be affine (v4-v1 = v5-v2 = v3-v0).
 *   Basis: Lagrange P_p on the equispaced lattice (i,j,k)/p, node loop order
 *   k, j, i with i fastest; prism node (t,l) has index l*n_tri + t.  Vector
 *   spaces are component-blocked: DOF (c, j) has index c*n_s + j.
 *   Output rows are test functions, columns trial functions.
 *
 * Memory layouts (row-major, element-major, float64):
 *   coords      [E][nv][gdim]     nv = 3 / 4 / 6, gdim = 2 / 3 / 3
 *   coeff_dofs  elasticity   [E][2][nc]   P1 (prism: P1 x P1) Lame lambda
 *                            DOFs then mu DOFs, nc = nv
 *               hyperelastic [E][gdim*n_s] displacement DOFs, component-blocked
 *               mass, Helmholtz: unused (may be NULL)
 *   out_A       [E][n][n]         n = n_s (scalar forms) or gdim*n_s (vector
 *                                 forms); fully overwritten
 *
 * Environment
 *   FE_TH_BYTES        T_H in bytes where fe_options_t.th_bytes is 0 (read
 *                      at every plan)
 *   FE_AUTOTUNE_CACHE  JSON file of autotuned launch shapes (fe_autotune)
 *   FE_LOG=1           one line on stderr per fe_assemble_local call: the
 *                      mode, precision and launch configuration used (read
 *                      at every call)
 *   FE_NT_STORES=1     non-temporal output stores in the kernels that offer
 *                      them (ordinary stores otherwise; read once)
 *
 * Forms (integrands summed with weight W_q |det J|; g = J^{-T} grad_X phi):
 *   FE_MASS          phi_i phi_j
 *   FE_HELMHOLTZ     g_i . g_j + phi_i phi_j
 *   FE_ELASTICITY    2 mu eps(v):eps(u) + lambda div v div u, lambda and mu
 *                    interpolated from their P1 DOFs at each point
 *   FE_HYPERELASTIC  tangent of the compressible neo-Hookean first Piola
 *                    stress P = mu (F - F^{-T}) + lambda ln(det F) F^{-T},
 *                    F = I + grad u, with constants mu, lambda from the options
 *
 * Errors: every entry point returns FE_OK (0) or a negative FE_E* code and
 * never aborts.  fe_strerror() describes a code; after FE_EHIP it also holds
 * the HIP runtime message of the failing call.
 *
 * Threading: entry points may be called from several host threads on
 * different streams; library caches are guarded by a mutex.
 */
#ifndef FELOCAL_H
#define FELOCAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FE_TRIANGLE = 0, FE_TETRAHEDRON = 1, FE_PRISM = 2 } fe_cell_t;
typedef enum { FE_MASS = 0, FE_HELMHOLTZ = 1, FE_ELASTICITY = 2, FE_HYPERELASTIC = 3 } fe_form_t;

/* Arithmetic of the element contraction.  Geometry (J, det J, J^{-1}) and the
 * per-point kinematics always run in float64.
 *   FE_FP64          float64 everywhere (all forms)
 *   FE_SPLIT_FP32    contraction on MFMA with float32 operands and float32
 *                    accumulation; the three terms of an entry (the two
 *                    products and the trace term) are added in float32 and
 *                    the sum is stored as float64
 *   FE_SPLIT_BF16X3  contraction on MFMA with each operand split into a
 *                    bf16 high and low part (three products hi*hi + hi*lo +
 *                    lo*hi), float32 accumulation, the same float32
 *                    three-term combination, stored as float64
 * The split precisions apply to FE_ELASTICITY and FE_HYPERELASTIC when the
 * element matrix fits one 32x32 tile (gdim*n_s <= 32) and the rule has at most
 * 32 points; otherwise FE_ENOTSUP.  At degree 1 on triangles and tetrahedra
 * (every gradient constant, the point loop hoisted) a split precision without
 * a shape override runs the float64 hoisted kernel (shape kernel 5), which is
 * faster there and meets the float64 bound.  Stated error bounds (normwise per element,
 * max|A - A_exact| / max|A_exact|): FE_SPLIT_BF16X3 <= 1e-4,
 * FE_SPLIT_FP32 <= 2e-6; FE_FP64 agrees with the float64 oracle to 1e-12. */
typedef enum { FE_FP64 = 0, FE_SPLIT_FP32 = 1, FE_SPLIT_BF16X3 = 2 } fe_precision_t;

/* Contraction mode (Sec. 4.1, Algorithm 3 chooses it when FE_MODE_AUTO).
 * FE_MODE_PREEVAL serves mass, Helmholtz and elasticity (its P1 Lame fields
 * expanded out of the reduction, FE_FP64 only); the hyperelastic form's
 * coefficient is not a polynomial, so it is FE_ENOTSUP there. */
typedef enum {
    FE_MODE_AUTO = 0,      /* planner decides from theta and T_H           */
    FE_MODE_PREEVAL = 1,   /* pre-evaluated reference tensors (Alg. 2)     */
    FE_MODE_QUADRATURE = 2 /* sharing-eliminated quadrature (Alg. 1)       */
} fe_mode_t;

enum {
    FE_OK = 0,
    FE_EINVAL = -1,     /* invalid argument (NULL pointer, degree, size ...)  */
    FE_ENOTSUP = -2,    /* valid but unsupported combination               */
    FE_EHIP = -3,       /* HIP runtime error; see fe_strerror              */
    FE_ENONAFFINE = -4, /* a prism is not affine (host-side validation)    */
    FE_ENOMEM = -5      /* allocation failed, or a size limit exceeded     */
};

/* Launch shape override.  Every field 0 = automatic (the autotuner's choice
 * for the variant when one is cached, else the built-in default); a nonzero
 * field replaces that field of the automatic shape.
 *   kernel       pre-evaluated mode (nf = 0; with nf > 0 one kernel
 *                serves the mode and only grid_per_cu applies): 1 = tiled kernel (tiles of `chunk`
 *                consecutive elements staged through LDS), 2 = streaming
 *                kernel (table entries held in registers for the whole
 *                launch, which needs epi * n^2 <= 8 * block, 16 * block for
 *                the mass form; visits of `chunk` consecutive elements);
 *                quadrature mode: 3 = VALU kernel (any size), 4 = matrix-
 *                core Gram kernel (vector forms with n <= 32, n_s <= 16 and
 *                at most 32 points, the only kernel of the split
 *                precisions; mass and Helmholtz with n <= 48 except a mixed
 *                plan without coefficient functions), 5 = the hoisted
 *                degree-1 kernel (elasticity and hyperelastic at degree 1 on
 *                triangles and tetrahedra, float64: every gradient is
 *                constant, one record per element, rows stored whole; the
 *                default there).  A kernel that does not serve the call's
 *                mode and precision is rejected.
 *   block        threads of the pre-evaluated kernels (multiple of 64, <= 512)
 *   epi          pre-evaluated: elements per step (1 <= epi <= block)
 *   chunk        pre-evaluated: elements per tile or visit, a multiple of
 *                epi (streaming: 0 = automatic, about 256 KiB of output)
 *   eb, qc       quadrature kernel: elements per tile, points per LDS chunk
 *   grid_per_cu  any kernel: at most this many resident blocks per CU
 * A shape that the kernel cannot take (or whose LDS exceeds the device's
 * per-block limit) is rejected with FE_EINVAL before any launch.  Fields
 * that do not apply to the selected kernel are ignored. */
typedef struct {
    int kernel, block, epi, chunk, eb, qc, grid_per_cu;
} fe_shape_t;

typedef struct {
    int            qdeg;       /* -1: form default (mass, Helmholtz 2p;
                                  elasticity 2p-1, prisms 2p+1; hyperelastic 4);
                                  else the exact degree of the rule          */
    fe_precision_t precision;  /* FE_FP64 by default                        */
    fe_mode_t      mode;       /* FE_MODE_AUTO by default                   */
    void*          stream;     /* hipStream_t; NULL = the null stream       */
    double         mu, lambda; /* hyperelastic constants (default 1, 10)    */
    int*           d_status;   /* optional device int32: atomically
                                  incremented once per flagged element
                                  (degenerate map, non-affine prism, or
                                  det F <= 0 at a point); the element's block
                                  is filled with NaN.  NULL = not counted.    */
    size_t         th_bytes;   /* T_H (Constraint 2); 0 = FE_TH_BYTES from
                                  the environment if set, else the device's
                                  L2 capacity (one XCD's 4 MiB on MI355X),
                                  the cache the pre-evaluated kernels stream
                                  their tables through                      */
    int            validate;   /* nonzero: synchronously copy coords to the
                                  host and reject non-affine prisms with
                                  FE_ENONAFFINE before launching            */
    fe_shape_t     shape;      /* launch shape override; zero = automatic   */
    int            nf;         /* the form is pre-multiplied by nf (0..3)
                                  coefficient functions f_i of the same
                                  Lagrange degree as the test and trial
                                  functions (the experiment matrix of
                                  Sec. 7.1, every form).  An element's
                                  coeff_dofs record is then the form's own
                                  DOFs (none for mass and Helmholtz, the Lame
                                  DOFs [2][nc] for elasticity, the
                                  displacement DOFs [gdim][n_s] for the
                                  hyperelastic form) followed by the
                                  functions' DOFs [nf][n_s]; the default rule
                                  gains nf * degree (mass and Helmholtz
                                  (2 + nf) * degree).  FE_FP64 only; the
                                  vector forms then run the VALU quadrature
                                  kernel (shape kernel 3) and, where
                                  Algorithm 3 pre-evaluates, the coefficient-
                                  expanded pre-evaluated kernels (elasticity;
                                  the hyperelastic trace monomial is added to
                                  the diagonal blocks after the quadrature
                                  kernel).  Default 0 */
    int            pointgeo;   /* prisms: nonzero lifts the affine assumption
                                  of Sec. 2.2.  The element map is the vertex
                                  map x(X) = sum_v psi_v(X) v (P1 x P1 basis
                                  psi), and J, det J and J^{-1} are evaluated
                                  at every quadrature point, so prisms need
                                  not be affine.  The geometry then varies
                                  over the element, which makes pre-
                                  evaluation illegal (Sec. 3.3): every
                                  monomial is evaluated by a float64
                                  quadrature kernel (FE_MODE_PREEVAL, nf > 0
                                  and the split precisions are FE_ENOTSUP;
                                  fe_autotune and batches refuse it), and the
                                  default rule gains one degree.  An element
                                  whose det J is zero, not finite, or changes
                                  sign between points is flagged.  No effect
                                  on triangles and tetrahedra (their vertex
                                  map is affine).  Default 0 */
    int            coord_degree; /* degree of the coordinate field: 0 or 1
                                  (default) coords holds the vertices, the
                                  map affine (Sec. 2.2); 2 (triangles and
                                  tetrahedra) coords is [E][n_2][gdim], the
                                  element's six or ten P2 nodes in the
                                  lattice order, and the element map is the
                                  isoparametric x(X) = sum_m psi2_m(X) x_m,
                                  so the element is curved: J, det J and
                                  J^{-1} are evaluated at every quadrature
                                  point, pre-evaluation is illegal
                                  (Sec. 3.3) and every monomial is
                                  evaluated by a float64 quadrature kernel
                                  (the VALU kernel, or for mass and
                                  Helmholtz the matrix-core kernel), and the
                                  default rule gains gdim degrees (det J of
                                  a P2 map has degree gdim, so the mass form
                                  stays exact).  FE_MODE_PREEVAL, nf > 0,
                                  the split precisions, prisms, batches,
                                  fe_autotune and fe_assemble_form are
                                  FE_ENOTSUP.  Flagged as with pointgeo.
                                  Lame fields stay P1 in the reference
                                  coordinates. */
} fe_options_t;

/* Fills *opt with the defaults listed above. */
void fe_options_init(fe_options_t* opt);

/* Reference tabulation (Sec. 2.2: the local basis Phi_i on the reference cell
 * K_0 and the quadrature rule; Sec. 7.1: exact Gauss-Legendre-Jacobi rule).
 * Rules are collapsed conical products (Gauss-Legendre x Gauss-Jacobi with
 * weights (1-t), (1-u)^2) with m = ceil((qdeg+1)/2) points per direction,
 * exact to total degree 2m-1; triangles with qdeg <= 2 use the three-point
 * interior rule (1/6,1/6), (2/3,1/6), (1/6,2/3); prisms use the triangle
 * rule times m-point Gauss-Legendre in Z.
 * All arrays are HOST pointers owned by the caller.  With points == NULL the
 * call only fills info = {nq, nb, tdim}.  Otherwise points [nq][tdim],
 * weights [nq], phi [nq][nb] and dphi [nq][nb][tdim] must all be non-NULL.
 * The basis values are computed by a HIP kernel; the call is synchronous.
 * Errors: FE_EINVAL (degree not in 1..4, qdeg not in 0..20, info NULL),
 * FE_EHIP. */
int fe_tabulate(fe_cell_t cell, int degree, int qdeg,
                double* points, double* weights, double* phi, double* dphi,
                int* info);

/* Sizes of the element tensor A^K of Sec. 2 (one row and one column per
 * local basis function of the test and trial space, Sec. 2.2) and of the
 * coefficient DOFs each element carries (the local DOFs of the coefficient
 * functions of Eq. (7)) for (form, cell, degree): n (rows) and the
 * coefficient DOFs per element (0 for mass and Helmholtz without nf).
 * Host pointers; either may be NULL.  Errors: FE_EINVAL. */
int fe_local_dims(fe_form_t form, fe_cell_t cell, int degree, int* n_rows, int* n_coeff);

/* Local assembly (Sec. 2: element tensor A^K of Eq. (7); evaluated in the
 * mode chosen by Algorithm 3, Sec. 4.1).  coords, coeff_dofs and out_A are
 * DEVICE pointers owned by the caller, in the layouts above; out_A must not
 * alias the inputs.  The call is asynchronous on opt->stream (reference
 * tables are built on first use of a (cell, degree, qdeg) and cached).
 * n_elems = 0 returns FE_OK without work.  opt = NULL uses the defaults.
 * Errors (returned synchronously, nothing launched): FE_EINVAL for NULL
 * pointers with n_elems > 0, n_elems < 0, degree not in 1..4, bad enums or
 * qdeg; FE_ENOTSUP for an unsupported precision/form/size combination;
 * FE_ENONAFFINE (opt->validate only); FE_ENOMEM; FE_EHIP for launch
 * failures.  Flagged elements are reported through opt->d_status. */
int fe_assemble_local(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems,
                      const double* coords, const double* coeff_dofs, double* out_A,
                      const fe_options_t* opt);

/* Geometry of the affine maps (Sec. 2.2, Eq. (7): dX/dx and det F_K').
 * DEVICE pointers: coords [E][nv][gdim] in; out_detJ [E] (signed det J) and
 * out_Kinv [E][gdim][gdim] (Kinv[a][b] = dX_a/dx_b) out.  Asynchronous on
 * stream.  Errors: FE_EINVAL, FE_EHIP. */
int fe_geometry(fe_cell_t cell, int64_t n_elems, const double* coords,
                double* out_detJ, double* out_Kinv, void* stream);

/* Plan of the transformation algorithm (Sec. 4.1, Algorithm 3) with the cost
 * function theta = theta_pre - theta_se (Sec. 4.2; increase factor iota and
 * term count rho) for one form.  Host-only; no GPU needed. */
typedef struct {
    int    n_monomials;        /* monomials of the form (Sec. 2.1)           */
    int    preevaluated[4];    /* 1 if monomial m is pre-evaluated            */
    double theta_se[4];        /* operation count of monomial m after sharing
                                  elimination, per element                   */
    double theta_pre[4];       /* operation count after pre-evaluation, per
                                  element (infinite when illegal)            */
    int    iota[4], rho[4];    /* increase factor and pre-evaluable terms    */
    size_t table_bytes[4];     /* bytes of the tables of monomial m          */
    size_t th_bytes;           /* the T_H used                               */
    double cost;               /* D[b] of the chosen bipartition             */
    fe_mode_t mode;            /* FE_MODE_PREEVAL if every monomial is
                                  pre-evaluated, else FE_MODE_QUADRATURE     */
} fe_plan_t;

/* qdeg = -1 for the form default; th_bytes = 0 for FE_TH_BYTES from the
 * environment if set, else the device's L2 capacity (4 MiB when no device is
 * present); nf as in fe_options_t
 * (iota = C(n_s + nf - 1, nf), Sec. 4.2; times n_c for elasticity, whose
 * P1 Lame fields are expanded as well).  A plan may
 * pre-evaluate only some monomials (Fig. 5): mode is then
 * FE_MODE_QUADRATURE and, with nf = 0, the quadrature kernel adds the
 * pre-evaluated monomials' tables; with nf > 0 such a mixed plan is executed
 * in quadrature mode.  Elasticity (P1 Lame fields, iota = n_c) has two
 * monomials that share one set of tables T_{l,a,b}[j][k] =
 * sum_q W_q psi_l dphi_{j,a} dphi_{k,b}; its pre-evaluated kernel takes both,
 * so its plans are both-or-neither (each must have theta <= 0 and the
 * tables must fit T_H).  The hyperelastic form has two monomials: the terms in
 * F (never pre-evaluable) and the trace term mu |det J| g_j . g_k (constant
 * coefficient); its matrix-core kernels (split precisions, float64 shape
 * kernel 4) pre-evaluate the trace term, the VALU kernel integrates both.
 * With nf > 0 the trace term's coefficient is mu prod_i f_i (iota =
 * C(n_s + nf - 1, nf)); where the plan pre-evaluates it, the VALU kernel
 * integrates the terms in F and the coefficient kernel adds the trace term.
 * Errors: FE_EINVAL. */
int fe_plan(fe_form_t form, fe_cell_t cell, int degree, int nf, int qdeg, size_t th_bytes,
            fe_plan_t* plan);

/* Mixed batches: several (form, cell, degree) sub-batches in one HIP graph,
 * replayed by fe_batch_run with one graph launch.  Every sub-batch uses
 * FE_FP64, the mode Algorithm 3 chooses for it, and the kernel and launch
 * shape that a single fe_assemble_local call with the same options would use
 * (the autotuner's, fe_autotune, when it has tuned the variant, else the
 * built-in default), so the batch's output equals those single calls bit
 * for bit.  Sub-batches whose kernel is the tiled pre-evaluated or the VALU
 * quadrature tile are grouped by kernel variant; each group runs as one
 * persistent kernel, specialised for the variant, whose workgroups take
 * element tiles from the group's device work queue.  The groups run on
 * parallel branches of the graph; after their join the other sub-batches
 * (streaming pre-evaluated, float64 matrix-core and hoisted degree-1
 * quadrature kernels) run as single launches one after another, and then
 * the elasticity sub-batches that Algorithm 3 pre-evaluates, one launch
 * each.
 * All sub-batch pointers are DEVICE pointers owned by the caller and must
 * stay valid until fe_batch_destroy.  Sub-batches with no elements are
 * allowed and do nothing.  Replays on one stream are ordered; replays of
 * one batch on different streams at once race on its work queues.
 * Coefficient functions (fe_options_t.nf), per-point geometry and curved
 * elements are not supported in batches.
 * Errors: FE_EINVAL, FE_ENOTSUP (hyperelastic, nf > 0), FE_ENOMEM, FE_EHIP. */
typedef struct fe_subbatch {
    fe_form_t     form;
    fe_cell_t     cell;
    int           degree;
    int           qdeg;        /* -1 = form default */
    int64_t       n_elems;
    const double* coords;
    const double* coeff_dofs;
    double*       out_A;
} fe_subbatch_t;

typedef struct fe_batch fe_batch_t;

int fe_batch_create(const fe_subbatch_t* subs, int n_subs, const fe_options_t* opt,
                    fe_batch_t** batch);
int fe_batch_run(fe_batch_t* batch, void* stream);
int fe_batch_destroy(fe_batch_t* batch);
/* Number of work tiles and the total workgroups of the persistent group
 * kernels of a batch (sub-batches launched as single calls or as
 * pre-evaluated elasticity are not counted). */
int fe_batch_info(const fe_batch_t* batch, int64_t* n_tiles, int* grid);

/* Autotuner: times the candidate launch shapes of the variant that serves
 * (form, cell, degree) on the given DEVICE inputs (n_elems >= 1; out_A is
 * overwritten) and stores the fastest in the in-memory cache (and in the
 * JSON file named by the environment variable FE_AUTOTUNE_CACHE, if set).
 * Synchronous.  *best_ms and *best_shape (either may be NULL) receive the
 * best time per launch and its shape (kernel 1 or 2 for the pre-evaluated
 * mode, 0 otherwise; chunk 0 = automatic visit length), which the caller can
 * also pass back through fe_options_t.shape.  opt->shape is ignored.
 * With opt->mode = FE_MODE_AUTO and a form that has two legal modes (mass,
 * Helmholtz, elasticity in FE_FP64), the other mode is tuned and timed as
 * well, and later FE_MODE_AUTO calls of the variant (fe_assemble_local,
 * batches) run the measured faster mode, the whole form in it; fe_plan keeps
 * reporting Algorithm 3's choice, and fe_autotune_clear forgets the choice.
 * The returned time and shape are those of the faster mode.
 * Errors: FE_EINVAL, FE_ENOTSUP, FE_EHIP. */
int fe_autotune(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems,
                const double* coords, const double* coeff_dofs, double* out_A,
                const fe_options_t* opt, double* best_ms, fe_shape_t* best_shape);

/* Empties the in-memory autotune cache, measured modes included (the JSON
 * file is left as it is; it is not read again in this process).  Host-only,
 * thread-safe. */
void fe_autotune_clear(void);

/* Global assembly (Sec. 2): the element matrices are coupled by adding them
 * into the matrix of the continuous space, A_ij = a(phi_i, phi_j), at the
 * global numbers of their DOFs (Sec. 7.1 times local assembly together with
 * this insertion).  The global matrix is held in compressed sparse rows with
 * sorted column indices.
 *
 * fe_csr_create builds the pattern on the device from
 *   cell_dofs  DEVICE int32 [n_elems][n], owned by the caller and read only
 *              during the call: the global number of local DOF j of element
 *              e, in the local numbering of the element matrices (vector
 *              forms: component c of scalar DOF j is local c*n_s + j); every
 *              number in [0, n_rows), distinct within an element
 *   n_rows     rows (and columns) of the global matrix; rows no element
 *              touches are empty
 * Entry (r, c) is stored when some element holds both r and c.  The call is
 * synchronous on stream; the handle owns the device memory of the pattern
 * (about 12 B per stored entry, 2 B per element-matrix entry and 12 B per
 * row).  Limits: n <= 256, n_elems * n < 2^32, n_rows < 2^31; for every
 * row, (elements holding it) * n <= 8192; and 8 B per entry of the longest
 * row plus 128 B per element of the row held by the most elements must fit
 * the LDS of one workgroup (64 KiB at least).
 * Errors: FE_EINVAL (NULL pointers, negative sizes, a number out of range or
 * repeated within an element: checked on the device before anything else),
 * FE_ENOTSUP (a limit exceeded), FE_ENOMEM, FE_EHIP. */
typedef struct fe_csr fe_csr_t;

int fe_csr_create(int64_t n_elems, int n, const int32_t* cell_dofs, int64_t n_rows, void* stream,
                  fe_csr_t** csr);
/* Sizes of the pattern (HOST outputs; any may be NULL): rows, stored entries
 * and the longest row.  Errors: FE_EINVAL. */
int fe_csr_info(const fe_csr_t* csr, int64_t* n_rows, int64_t* nnz, int* max_row_len);
/* Copies the pattern into DEVICE buffers owned by the caller: row_ptr
 * [n_rows + 1] int64 (row_ptr[0] = 0, row r holds entries row_ptr[r] ..
 * row_ptr[r+1]-1) and col_idx [nnz] int32.  Asynchronous on stream.
 * Errors: FE_EINVAL, FE_EHIP. */
int fe_csr_pattern(const fe_csr_t* csr, int64_t* row_ptr, int32_t* col_idx, void* stream);
/* values [nnz] (DEVICE float64, overwritten): for every stored (r, c), the sum
 * of local_A[e][j][k] over the elements e with cell_dofs[e][j] = r and
 * cell_dofs[e][k] = c, added in increasing e starting from zero, so the
 * result does not depend on the launch and equals that sequential sum bit
 * for bit.  local_A is DEVICE [n_elems][n][n] (the out_A layout of
 * fe_assemble_local) and must not alias values.  Asynchronous on stream.
 * Errors: FE_EINVAL (NULL pointers), FE_EHIP. */
int fe_csr_insert(const fe_csr_t* csr, const double* local_A, double* values, void* stream);
/* Frees the pattern (waits for the device first).  Errors: FE_EINVAL. */
int fe_csr_destroy(fe_csr_t* csr);

/* Local and global assembly in one pass for the pre-evaluated forms (Sec. 2
 * with the pre-evaluated contraction of Sec. 3.3, Algorithm 2): values [nnz]
 * (DEVICE float64, overwritten) = fe_csr_insert applied to the element
 * matrices that fe_assemble_local computes for the same arguments, bit for
 * bit, without storing them: each entry is formed from the element's
 * geometry tensor and the reference tables where it is added.  csr must come
 * from fe_csr_create with n_elems elements and n = the element matrix size;
 * coords as in fe_assemble_local (DEVICE).  Supported: FE_MASS and
 * FE_HELMHOLTZ in FE_FP64 with nf = 0, in the pre-evaluated mode (what
 * Algorithm 3 chooses for these forms, or FE_MODE_PREEVAL), with reference
 * tables of at most 96 KiB (every triangle and tetrahedron degree; prisms up
 * to P4 for mass and P3 for Helmholtz); other calls, and meshes where one
 * row's entries and the tables together exceed a workgroup's LDS, return
 * FE_ENOTSUP (use fe_assemble_local, then fe_csr_insert).  opt->shape is
 * ignored.  The
 * handle keeps a geometry workspace of 64 B per element, allocated on first
 * use, so calls on one handle must not overlap.  Asynchronous on
 * opt->stream; flagged elements are counted through opt->d_status and make
 * the entries they touch NaN.
 * Errors: FE_EINVAL (as fe_assemble_local, or csr sized for other
 * elements), FE_ENOTSUP, FE_ENOMEM, FE_EHIP. */
int fe_assemble_csr(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                    fe_csr_t* csr, double* values, const fe_options_t* opt);

/* fe_assemble_csr without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result (bit for bit) and errors as
 * fe_assemble_csr, and the same kernels; only the geometry workspace differs:
 * instead of the handle's (allocated on first use), a file-scope device array
 * of the library, 64 B per element, at most 1,048,576 elements (64 MiB that
 * every GPU the library runs on holds until the process ends).  The call
 * performs no hipMalloc, hipFree or other allocating call:
 *   - n_elems above 1,048,576 returns FE_ENOMEM;
 *   - the reference tables of (cell, degree, rule) are not built here: an
 *     earlier call on this device must have built them (any fe_assemble_local
 *     or fe_assemble_csr call with the same cell, degree and rule), else
 *     FE_EINVAL.
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents (every element's entry is rewritten before it is read, so nothing
 * needs clearing): calls that overlap on one GPU (different streams or host
 * threads) race and must be serialised by the caller.  Asynchronous on
 * opt->stream. */
int fe_assemble_csr_noalloc(fe_form_t form, fe_cell_t cell, int degree, int64_t n_elems, const double* coords,
                            fe_csr_t* csr, double* values, const fe_options_t* opt);

/* Automatic sharing elimination (Sec. 3.2, Algorithm 1) and code generation
 * for generic bilinear forms, scalar or on a vector-valued space.  A form is a
 * sum of terms
 *     scale * c(x) * s_test(phi_j) * s_trial(phi_k),
 * s_test and s_trial being the basis function (FE_SYM_VALUE) or one of its
 * physical derivatives d/dx_1..3 (FE_SYM_DX, _DY, _DZ), and c = 1 (field =
 * -1) or the P1 field `field` interpolated from its vertex values.  Rows are
 * test functions, columns trial functions, as for fe_assemble_local.
 * Vector-valued spaces (n_comp = the cell dimension): the basis functions are
 * phi_j e_c, numbered component-blocked (row c * n_s + j) as for the
 * elasticity form, and a term adds to block (test_comp, trial_comp) only;
 * e.g. linear elasticity is mu d_b v_a d_b u_a on the diagonal blocks plus
 * mu d_b v_a d_a u_b and lambda d_a v_a d_b u_b on every block (a, b). */
typedef enum { FE_SYM_VALUE = 0, FE_SYM_DX = 1, FE_SYM_DY = 2, FE_SYM_DZ = 3 } fe_symbol_t;
#define FE_MAX_TERMS 64
#define FE_MAX_FIELDS 4
#define FE_MAX_VERTICES 72   /* 9 component blocks of at most 8 symbols */
typedef struct {
    int    test, trial;   /* fe_symbol_t; derivatives up to the cell dimension */
    int    field;         /* -1 (constant) or the index of a P1 field         */
    double scale;
    int    test_comp, trial_comp;   /* components coupled; 0 for a scalar form */
} fe_term_t;
typedef struct {
    int       n_terms;    /* 1 .. FE_MAX_TERMS */
    fe_term_t terms[FE_MAX_TERMS];
    int       n_fields;   /* 0 .. FE_MAX_FIELDS */
    int       n_comp;     /* 0 or 1: scalar form; the cell dimension: vector-valued space */
} fe_form_spec_t;

/* Result of Algorithm 1 for one form.  Each component block (test_comp,
 * trial_comp) of the element matrix is its own (j, k) loop nest; a scalar
 * form has one block.  Per block: terms with the same pair of symbols are
 * merged into one product (step 1); the sharing graph (step 3) has one vertex
 * per distinct symbol of each side (test vertices first) and one edge per
 * product; the ILP of step 5 (minimise the factorised symbols so that every
 * product is grouped under exactly one factorised endpoint, i.e. a minimum
 * vertex cover with an orientation) is solved exactly.  A block's
 * factorisation is kept only if it lowers the block's operation count (steps
 * 2 and 4); otherwise none of its symbols is factorised, its edge_owner
 * entries are -1 and its expanded nest is used.  Vertices are listed block
 * by block (block index test_comp * n_comp + trial_comp).  Operation counts
 * are per element for the rule of degree qdeg, summed over the blocks. */
typedef struct {
    int    n_vertices;
    int    vertex_side[FE_MAX_VERTICES];      /* 0 test, 1 trial */
    int    vertex_symbol[FE_MAX_VERTICES];    /* fe_symbol_t */
    int    factorized[FE_MAX_VERTICES];       /* x_i: the symbol is factorised (Strategy 2) */
    int    n_edges;
    int    edge_test[FE_MAX_TERMS], edge_trial[FE_MAX_TERMS];   /* vertex indices */
    int    edge_owner[FE_MAX_TERMS];   /* y: the factorised vertex a product is grouped under */
    double theta_expanded;      /* every product in the innermost (j, k) body */
    double theta_se;            /* after sharing elimination */
    int    n_comp;              /* 1 for a scalar form */
    int    vertex_block[FE_MAX_VERTICES];     /* test_comp * n_comp + trial_comp */
} fe_sharing_t;

/* qdeg = -1: 2 * degree, plus one when a term carries a field.  Host only.
 * Errors: FE_EINVAL (bad spec, cell, degree or qdeg). */
int fe_sharing_plan(const fe_form_spec_t* spec, fe_cell_t cell, int degree, int qdeg, fe_sharing_t* plan);

/* HIP source of the kernel fe_assemble_form generates (expanded != 0: the
 * loop nest without sharing elimination).  For a vector-valued form whose
 * blocks' register tiles fit together, this is the fused nest (one point
 * loop, every block accumulated from it); fe_assemble_form replaces it by the
 * per-block nest where the fused kernel would hold less than two wavefronts
 * per SIMD on the device.  buf may be NULL; *len receives the size including
 * the terminating zero and, on input, is the capacity of buf.  Host only.
 * Errors: FE_EINVAL. */
int fe_form_source(const fe_form_spec_t* spec, fe_cell_t cell, int degree, int expanded, char* buf, size_t* len);

/* Element matrices of a generic form (affine cells) by a quadrature kernel
 * generated from Algorithm 1's result, compiled at run time with hipRTC for
 * the current device on first use and cached (the compilation is
 * synchronous).  coords as in fe_assemble_local; out_A DEVICE
 * [n_elems][n][n] with n = n_comp * n_s (n_s for a scalar form), fully
 * overwritten; fields DEVICE [n_elems][n_fields][nv] (may be NULL without
 * fields).  Options used: qdeg,
 * stream, d_status, and shape.kernel (0 = sharing-eliminated nest, 5 = the
 * expanded nest, for comparison).  Degenerate and non-affine elements are
 * flagged (NaN block, d_status).  n_s <= 64.
 * Errors: FE_EINVAL, FE_ENOTSUP, FE_EHIP (including a failed compilation). */
int fe_assemble_form(const fe_form_spec_t* spec, fe_cell_t cell, int degree, int64_t n_elems,
                     const double* coords, const double* fields, double* out_A, const fe_options_t* opt);

/* Human-readable text for an FE_* code. */
const char* fe_strerror(int code);

/* Frees the reference-table, coefficient-table and autotune caches (device
 * memory included) and unloads the kernels fe_assemble_form compiled (a later
 * call compiles its kernel again).  No call may be in flight. */
void fe_release_caches(void);

/* Library version string. */
const char* fe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FELOCAL_H */
