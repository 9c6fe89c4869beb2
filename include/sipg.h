/*
 * sipg.h -- C ABI of the MI355X (gfx950) library for the matrix-free
 * symmetric interior penalty (SIPG) discontinuous Galerkin Laplacian on
 * hexahedra in the Hermite-like basis (Kronbichler, Kormann, Pasichnyk,
 * Allalen: "A Hermite-like basis for faster matrix-free evaluation of interior
 * penalty discontinuous Galerkin operators").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns a sipg_status (0 = success, < 0 = error).  No C++
 *    exception crosses this boundary.  sipg_last_error() returns a
 *    thread-local text for the most recent failure of the calling thread.
 *  - Vectors are device pointers to ndofs contiguous elements of the
 *    operator's precision (double for SIPG_F64, float for SIPG_F32), in the
 *    cell-wise layout of Section 5: dof = cell * n^3 + i1 + n*i2 + n^2*i3 with
 *    n = degree + 1, cell = ix + nx*(iy + ny*iz), xi_1 varying fastest.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Unless stated,
 *    calls are stream ordered and do not synchronise the host.
 *  - A sipg_op is immutable after sipg_setup: several streams may apply the
 *    same operator concurrently as long as their output buffers differ.
 */
#ifndef SIPG_H
#define SIPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIPG_OK = 0,
    SIPG_E_ARG = -1,         /* invalid argument (null pointer, bad size, aliasing, ...) */
    SIPG_E_OOM = -2,         /* device allocation failed */
    SIPG_E_HIP = -3,         /* a HIP runtime call failed; text in sipg_last_error() */
    SIPG_E_UNSUPPORTED = -4, /* valid request the library does not provide */
    SIPG_E_NOTREADY = -5,    /* asynchronous result not finished yet */
    SIPG_E_NOCONV = -6,      /* iterative solve hit its iteration limit */
    SIPG_E_BUDGET = -7       /* request exceeds the configured memory budget */
} sipg_status;

/* Bases (Section 4.1): the Hermite-like basis, and for comparison the nodal
 * Lagrange bases in the Gauss-Lobatto points and in the Gauss points (the
 * latter collocated with the quadrature: S = I, dense face rows). */
typedef enum { SIPG_BASIS_HERMITE_LIKE = 0, SIPG_BASIS_NODAL_GL = 1, SIPG_BASIS_NODAL_GAUSS = 2 } sipg_basis;
typedef enum { SIPG_F64 = 0, SIPG_F32 = 1 } sipg_dtype;

/* How metric terms are stored (Section 3 and Section 4.2):
 *  SIPG_GEOM_AUTO   : SIPG_GEOM_CELL on undeformed meshes, else SIPG_GEOM_QPOINT.
 *  SIPG_GEOM_CELL   : one merged tensor J^-1 J^-T det J per cell and one
 *                     7-value record per face; the kernel multiplies by the
 *                     quadrature weights.  Only valid for affine cells.
 *  SIPG_GEOM_QPOINT : the merged tensor at every cell quadrature point
 *                     (6 values) and a 7-value record at every face
 *                     quadrature point, as for general (deformed) cells. */
typedef enum { SIPG_GEOM_AUTO = 0, SIPG_GEOM_CELL = 1, SIPG_GEOM_QPOINT = 2 } sipg_geometry;

/* Structured brick of n[0] x n[1] x n[2] hexahedra.  Cell (ix,iy,iz) is
 * mapped from the reference cube [0,1]^3 by
 *     X = lo + ((ix,iy,iz) + xi) * (hi - lo) / n,
 *     Y = L X                 (L = lin, row major; all zeros means identity),
 *     x = Y + deform_amp * sin(pi Y1) sin(pi Y2) sin(pi Y3) * (1,1,1).
 * The first two steps give the affine benchmark geometry of Section 5; the
 * last one is a smooth deformation that keeps the unit cube's boundary.
 * A graded brick sets width (all three entries > 0; all zero means the
 * uniform brick above): in direction d, cells 0 .. n[d]-2 have width
 * width[d] and the last cell ends at hi[d], so its width
 * hi[d] - lo[d] - (n[d]-1) width[d] must lie in (0, width[d]].  The
 * multigrid hierarchy uses such bricks for its coarse levels of meshes whose
 * cell counts are odd. */
typedef struct {
    int32_t n[3];
    double lo[3];
    double hi[3];
    double lin[9];
    double deform_amp;
    double width[3];
} sipg_mesh;

/*
 * Device memory provider.  The operator's own arrays (1D tables, metric
 * terms, preconditioner data), solver hierarchies and workspaces live in
 * memory obtained from `alloc(bytes, ctx)`: device memory of the current
 * device, at least 256-byte aligned, or NULL when none is available (the
 * call then fails with SIPG_E_OOM).  `free(ptr, ctx)` returns it.  The
 * library calls `free` only for blocks no device work it queued still uses
 * (it waits for that work first); both callbacks may be called from the
 * request loop's worker threads.  Every entry point that takes a
 * `const sipg_allocator*` accepts NULL, meaning hipMalloc / hipFree.  With a
 * caching allocator (for example PyTorch's) the set-up and solver calls then
 * allocate no device memory of their own.
 */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} sipg_allocator;

typedef struct sipg_op sipg_op;

/*
 * Build the operator of the weak form of Section 2 (eq. discrete_laplace):
 * cell term, interior-penalty face terms, homogeneous Dirichlet boundaries
 * by the mirror principle (u+ = -u-, grad u+ = grad u-), tensor Gauss
 * quadrature with degree+1 points per direction (Section 3), basis of
 * Section 4.1 (or the nodal Gauss-Lobatto basis for comparison).
 * Penalty: sigma_F = penalty_factor * (degree+1)^2 * max(|F|/|K-|, |F|/|K+|),
 * which is penalty_factor * (degree+1)^2 / h on a Cartesian cell of size h
 * (Section 2 uses penalty_factor = 1).
 *
 *   mesh            brick description (host memory, read during the call).
 *   degree          polynomial degree k, 1 <= k <= 8.
 *   penalty_factor  > 0.
 *   basis, dtype, geometry   see the enums above.
 *   allocator       device memory provider of the operator (NULL: hipMalloc);
 *                   the operator keeps a copy of the struct and uses it for
 *                   every later allocation of its own (the diagonal of
 *                   sipg_compute_gl_diagonal, the workspace of sipg_cg_solve)
 *                   and to free everything in sipg_destroy.
 *   stream          stream for the set-up kernels; the call synchronises
 *                   that stream before it returns.
 *   out             receives the operator handle (owned by the caller, freed
 *                   with sipg_destroy).
 * Errors: SIPG_E_ARG (null pointers, k out of range, non-positive n or
 * penalty, SIPG_GEOM_CELL on a deformed mesh, a non-invertible map, an
 * allocator with only one of its callbacks), SIPG_E_OOM, SIPG_E_HIP.
 */
int sipg_setup(const sipg_mesh* mesh, int degree, double penalty_factor, int basis,
               int dtype, int geometry, const sipg_allocator* allocator, void* stream, sipg_op** out);

/* Release an operator and its device memory through its allocator (NULL is
 * accepted).  The caller must make sure no work that uses it is still
 * queued. */
int sipg_destroy(sipg_op* op);

/* Number of unknowns n_cells * (degree+1)^3, or -1 for NULL. */
int64_t sipg_ndofs(const sipg_op* op);

/* Description of the operator (host memory).  `geometry` is the resolved
 * storage mode; `device_bytes` the operator's own device memory;
 * `diagonal_metric` is 1 when the storage is per cell and every cell's
 * merged tensor J^-1 J^-T det J is diagonal (an affine map with a diagonal
 * linear part), in which case the cell term of the product is evaluated in
 * reference coordinates with the 1D mass and stiffness matrices (Section 3,
 * affine cells); such operators form their own group in a batch. */
typedef struct {
    int32_t degree, basis, dtype, geometry;
    int32_t n[3];
    int64_t ndofs;
    int64_t device_bytes;
    int32_t cells_per_block, threads_per_block;
    int32_t diagonal_metric;
} sipg_op_info;
int sipg_get_info(const sipg_op* op, sipg_op_info* info);

/*
 * y = A x, matrix-free (Section 3): per cell, sum factorization of the cell
 * integral (eq. tensor_cell and its transpose), the six face integrals
 * evaluated element-wise with the neighbour's value and derivative layers
 * (eq. tensor_face; Section 4.2), and one write of y per cell.
 *   x, y  device pointers, ndofs elements each, operator precision; they
 *         must not overlap (SIPG_E_ARG).
 * Allocates nothing; stream ordered.
 */
int sipg_apply(const sipg_op* op, const void* x, void* y, void* stream);

/*
 * Batched product y_i = A_i x_i of nops independent operators (the same
 * element-wise evaluation as sipg_apply, Section 3), for many small problems
 * at once.  Operators of equal degree, basis, precision, geometry mode and
 * diagonal_metric (sipg_op_info) share one grid, so a batch runs as one
 * launch per such group.
 *   sipg_batch_create  ops[i], x[i], y[i] (host arrays of nops entries; x, y
 *                      device pointers of ops[i]'s size and precision) are
 *                      bound at creation.  The batch stores device pointers
 *                      only: operators and vectors must outlive it.  All
 *                      operators on one device.  Inputs may be shared; an
 *                      output that overlaps any input or other output ->
 *                      SIPG_E_ARG.  Allocates one small device table
 *                      (kernel parameters, workgroup -> operator map) and
 *                      copies it synchronously.
 *   sipg_batch_apply   launches the groups, spread over `stream` and up to
 *                      three streams of the batch that start after the work
 *                      queued on `stream` and that `stream` waits for
 *                      (events), so groups run concurrently; allocates
 *                      nothing, stream ordered with respect to `stream`.
 *                      Each y_i is bit-identical to sipg_apply(ops[i], x[i],
 *                      y[i]).  Calls on one batch must not overlap.
 *   sipg_batch_destroy frees the table (NULL accepted); no queued work may
 *                      still use it.
 */
typedef struct sipg_batch sipg_batch;
typedef struct {
    int32_t nops, launches;      /* launches = groups of equal degree/basis/precision/geometry */
    int64_t ndofs, ncells, workgroups;
    int64_t device_bytes;
    int32_t per_operator_groups; /* groups that sipg_batch_tune set to one launch per operator */
    int32_t streams;             /* streams the groups are spread over (the caller's included) */
} sipg_batch_info;
int sipg_batch_create(int nops, const sipg_op* const* ops, const void* const* x, void* const* y,
                      sipg_batch** out);
int sipg_batch_apply(const sipg_batch* batch, void* stream);
/* Schedule autotuning: for every group, time `reps` applications as one grid
 * and as one launch per operator on `stream` (HIP events) and keep the faster
 * schedule for later sipg_batch_apply calls.  Runs the products, so the
 * outputs are overwritten; synchronises the stream.  Results are the same in
 * both schedules (same kernel body). */
int sipg_batch_tune(sipg_batch* batch, int reps, void* stream);
int sipg_batch_get_info(const sipg_batch* batch, sipg_batch_info* info);
int sipg_batch_destroy(sipg_batch* batch);

/*
 * Cell-wise tensor-product basis change between the operator's basis and the
 * nodal Gauss-Lobatto basis, and the element-wise preconditioners of the
 * form of eq. (jacobi) (Sections 6.3, 6.4).  With E_ij = phi_i(x^GL_j),
 * T = E^-1:
 *   SIPG_BC_T        out = (T x T x T) in        : HL residual -> GL residual
 *   SIPG_BC_TT       out = (T^T x T^T x T^T) in  : GL coefficients -> HL coefficients
 *   SIPG_BC_VALUES   out = (E^T x E^T x E^T) in  : HL coefficients -> values at GL nodes
 *   SIPG_BC_PJACOBI  out = (T^T)^{x3} diag(A_GL)^-1 T^{x3} in, the point-Jacobi
 *                    preconditioner of the nodal GL basis expressed in the
 *                    operator's basis (needs sipg_compute_gl_diagonal first).
 *   SIPG_BC_FDM      out = P_K^-1 in per cell, the block-Jacobi preconditioner
 *                    of Section 6.4: P_K = M (x) M (x) L + M (x) L (x) M +
 *                    L (x) M (x) M (eq. KDlaplace_dg) with the 1D SIPG matrix
 *                    L of an interior element and the mass matrix M on
 *                    intervals of lengths h_d = |J(cell centre) e_d| (exact
 *                    for interior cells of Cartesian meshes; interior-element
 *                    matrices also at the boundary, as in the paper), inverted
 *                    by fast diagonalization: Z^{x3} (vol Lambda_sum)^-1
 *                    (Z^T)^{x3} with L z = lambda M z on the unit interval.
 * in, out: device pointers, ndofs elements, must not overlap.  Allocates
 * nothing; stream ordered.  SIPG_E_ARG for a bad mode or missing diagonal.
 */
enum { SIPG_BC_T = 0, SIPG_BC_TT = 1, SIPG_BC_VALUES = 2, SIPG_BC_PJACOBI = 3, SIPG_BC_FDM = 4 };
int sipg_basis_change(const sipg_op* op, int mode, const void* in, void* out, void* stream);

/*
 * y = A x and z = P^-1 y in one pass, with P^-1 the point-Jacobi
 * preconditioner of eq. (jacobi) as in SIPG_BC_PJACOBI: the product of
 * sipg_apply, then, cell by cell in the same workgroup, (T^T)^{x3}
 * diag(A_GL)^-1 T^{x3} of that cell's y.  y equals sipg_apply's output bit
 * for bit; z equals sipg_basis_change(SIPG_BC_PJACOBI, y) up to rounding.
 * Saves the second read of y and a launch.
 *   x, y, z  device pointers, ndofs elements each, operator precision; they
 *            must not overlap (SIPG_E_ARG).
 * Needs sipg_compute_gl_diagonal first (else SIPG_E_ARG).  Allocates nothing;
 * stream ordered.
 */
int sipg_apply_pjacobi(const sipg_op* op, const void* x, void* y, void* z, void* stream);

/*
 * Measurement aid, not part of the method: moves exactly the bytes of
 * sipg_apply_pjacobi (x, the operator's metric terms and 1/diag(A_GL) read
 * once, y and z written once) with no arithmetic, every workgroup reading one
 * contiguous share of each array in 16-byte pieces.  Its duration is the
 * step's duration if it were bound by HBM alone for that mix of reads and
 * writes; the contents written to y and z are meaningless.  x, y, z: device
 * pointers, ndofs elements, 16-byte aligned, not overlapping.  Needs
 * sipg_compute_gl_diagonal first (SIPG_E_ARG).  Allocates nothing; stream
 * ordered.
 */
int sipg_stream_bound(const sipg_op* op, const void* x, void* y, void* z, void* stream);

/*
 * One GPU's share of a partition of the mesh into z-slabs (Section 5: in a
 * distributed run only the value and derivative layers of the cells next to
 * a partition boundary travel between processes, 2 n^2 values per face in
 * the Hermite-like basis against n^3 for a nodal one).
 *
 * sipg_setup_slab: the operator of the cells z0 <= iz < z1 of `mesh` (0 <=
 * z0 < z1 <= mesh->n[2]; other arguments and errors as sipg_setup).  Its
 * metric terms are those of the whole mesh: the faces on the planes z0 (if
 * z0 > 0) and z1 (if z1 < n[2]) are interior faces, whose neighbour cells
 * belong to the slabs below and above.  A slab with a neighbouring slab is
 * applied only through sipg_apply_slab (sipg_apply, sipg_apply_pjacobi, the
 * solvers and batches reject it: SIPG_E_ARG); sipg_basis_change and
 * sipg_compute_gl_diagonal work on it as on any operator.  Vectors are the
 * slab's own cells, in the usual cell-wise layout (ndofs = nx ny (z1-z0) n^3).
 *
 * sipg_ghost_size: values of one ghost buffer, nx ny NL n^2 with NL = 2
 * (Hermite-like) or n (nodal bases); -1 for a null operator.
 *
 * sipg_pack_ghost: out = the layers that the neighbouring slab reads from
 * this one: side 0, of the bottom row of cells (for the slab below, whose
 * ghost_hi it is); side 1, of the top row (the ghost_lo of the slab above).
 * Layout [column ix + nx iy][layer j][point i1 + n i2]: in the Hermite-like
 * basis the value and derivative layers, 0 and 1 of the bottom row (side 0)
 * or n-2 and n-1 of the top row (side 1); in the nodal bases all n layers,
 * bottom up.
 * x: this slab's vector; out: device, sipg_ghost_size values, not
 * overlapping x.  Stream ordered; allocates nothing.
 *
 * sipg_apply_slab: y = A x for the slab, the neighbour layers across its
 * lower and upper z planes read from ghost_lo and ghost_hi (the packed
 * buffers of the slabs below and above); a ghost buffer is required exactly
 * where the slab has a neighbour (SIPG_E_ARG otherwise).  With z non-null,
 * also z = P^-1 y of eq. (jacobi) in the same pass (needs
 * sipg_compute_gl_diagonal on this operator).  x, y, z: device, ndofs
 * values of the operator's dtype, not overlapping.  Stream ordered; the
 * results equal the rows of these cells of the whole mesh's operator.
 */
int sipg_setup_slab(const sipg_mesh* mesh, int z0, int z1, int degree, double penalty_factor, int basis,
                    int dtype, int geometry, const sipg_allocator* allocator, void* stream, sipg_op** out);
int64_t sipg_ghost_size(const sipg_op* op);
int sipg_pack_ghost(const sipg_op* op, int side, const void* x, void* out, void* stream);
int sipg_apply_slab(const sipg_op* op, const void* x, const void* ghost_lo, const void* ghost_hi, void* y,
                    void* z, void* stream);

/*
 * Compute diag(A) of the operator in the nodal Gauss-Lobatto basis, i.e. the
 * element-wise diagonal P_d of eq. (jacobi), and keep its inverse inside the
 * operator for SIPG_BC_PJACOBI.  Computed on the device by the same weak form.
 * If `diag_out` is not NULL it also receives diag(A_GL) (ndofs elements,
 * operator precision, device memory).  Synchronises `stream`.
 */
int sipg_compute_gl_diagonal(sipg_op* op, void* diag_out, void* stream);

/*
 * Conjugate gradient solve of A x = b in FP64 (the outer solver of Section
 * 6.2).  b, x: device pointers (double, ndofs); x holds the initial guess
 * on entry and the solution on exit.  Stops when ||b - A x||_2 <= rel_tol *
 * ||b||_2 (recursive CG residual) or after max_iter iterations
 * (SIPG_E_NOCONV, info still filled).  Blocks the host: it reads one scalar
 * per iteration.  Its workspace (3 vectors and a few scalars) comes from the
 * operator's allocator and is returned before the call ends (with no
 * allocator: stream-ordered memory on `stream`, hipMallocAsync and
 * hipFreeAsync, so no device-wide synchronisation).  Requires an SIPG_F64
 * operator.
 */
typedef struct {
    int32_t iterations;
    double initial_residual;    /* ||b - A x0||_2 */
    double final_residual;      /* recursive residual at exit */
    double true_residual;       /* ||b - A x||_2 recomputed at exit */
} sipg_solve_info;
int sipg_cg_solve(const sipg_op* op, const double* b, double* x, double rel_tol,
                  int max_iter, sipg_solve_info* info, void* stream);

/*
 * sipg_cg_solve for callers that cannot allocate device memory: code under
 * HIP stream capture (the solve itself still reads one scalar per iteration,
 * so the capture has to end before it is called), tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, same kernels and the same
 * results, bit for bit, as sipg_cg_solve; the work arrays are a fixed array
 * of the library in device memory, one per GPU (held from the first call on
 * that GPU until the process ends), which holds operators of up to
 * sipg_cg_static_max_dofs() = 2^20 unknowns (24 MiB of work vectors):
 * SIPG_E_ARG beyond that.  Calls no hipMalloc, hipFree or allocating routine.
 * Every call on one GPU uses that GPU's array, so calls that overlap in time
 * on one GPU (from several threads or streams) race and must not be made.
 */
int sipg_cg_solve_static(const sipg_op* op, const double* b, double* x, double rel_tol,
                         int max_iter, sipg_solve_info* info, void* stream);
int64_t sipg_cg_static_max_dofs(void);

/* Host-only: the order in which the single-operator product kernel visits
 * its blocks of cells_per_block consecutive cells: workgroup b (in dispatch
 * order) handles block order[b].  layer_blocks = round(nx ny / cells_per_block)
 * is the number of blocks of one z-layer of cells.  Each of the 8 XCDs of the
 * GPU (workgroups are dispatched to them round robin) gets a contiguous range
 * of blocks and visits it z-layers interleaved, so that the two cells of a
 * z-face are processed close together in time (data reuse in the XCD's L2,
 * Section 4.2's data-access argument on this GPU).  order: nblocks entries,
 * caller-owned host memory. */
int sipg_host_block_order(int nblocks, int layer_blocks, int32_t* order);

/* Host-only: launch shape of the matrix-free kernel for a degree and precision:
 * cells per workgroup, threads per workgroup and dynamic LDS bytes. */
int sipg_launch_shape(int degree, int dtype, int32_t* cells_per_block, int32_t* threads_per_block,
                      int64_t* lds_bytes);

/*
 * Geometric multigrid solver of Section 6: FP64 conjugate gradient
 * preconditioned by one V-cycle per iteration.  On every level of the brick
 * coarsened by two in each direction (while all cell counts are even and at
 * least min_coarse_cells coarse cells remain; or graded, see
 * graded_coarsening) the V-cycle smooths with a
 * Chebyshev iteration (eq. chebyshev) around P^-1 of the form of eq. (jacobi)
 * (point Jacobi in the nodal Gauss-Lobatto basis through the basis change,
 * or the block Jacobi of Section 6.4 by fast diagonalization).  Optionally
 * the first levels lower the polynomial degree on the fine mesh
 * (p_coarsening); the transfer between degrees is the exact embedding of the
 * lower-degree space and its transpose.  The smoothing range is
 * [range_lo, range_hi] times the largest eigenvalue of
 * P^-1 A estimated by lanczos_steps conjugate-gradient (Lanczos) steps from
 * [-5.5, -4.5, ..., 5.5, -5.5, ...] (Section 6.2); the coarsest level is
 * solved by a Chebyshev iteration whose degree guarantees a residual
 * reduction of coarse_reduction, or, when small, by its dense inverse
 * (coarse_direct_max_dofs).  Grid transfer: exact embedding of the
 * coarse space and its transpose.
 *   precision 0: the V-cycle runs in FP32 (mixed precision, Section 6.2);
 *   precision 1: everything in FP64.
 */
typedef struct {
    int32_t smoother_degree;     /* Chebyshev degree per smoothing (5) */
    int32_t lanczos_steps;       /* eigenvalue estimate steps (15; at most 512) */
    double range_lo, range_hi;   /* smoothing range factors (0.06, 1.2) */
    double coarse_reduction;     /* coarse solve residual reduction (1e5) */
    int32_t min_coarse_cells;    /* stop coarsening below this many cells (1) */
    int32_t precision;           /* 0 mixed, 1 FP64 */
    int32_t smoother;            /* P^-1 inside the Chebyshev smoother: 0 point Jacobi in the
                                    nodal Gauss-Lobatto basis (SIPG_BC_PJACOBI), 1 the block
                                    Jacobi of Section 6.4 (SIPG_BC_FDM) */
    int32_t p_coarsening;        /* levels that lower the degree on the fine mesh before the
                                    mesh is coarsened: 0 none, 1 k -> max(1, k/2), 2 k -> k-1.
                                    Needed for meshes with odd cell counts, which cannot be
                                    coarsened by two */
    int32_t fused_smoother;      /* 1 (default): on Hermite-like levels each Chebyshev step is
                                    one launch, the product with the residual, P^-1 and the
                                    update fused (the "merged" arrangement of Section 6); 0: the
                                    product, then one merged pass.  Same results up to rounding */
    int32_t lanczos_start;       /* start of the eigenvalue estimate: 0 (default) the right-hand
                                    side [-5.5, ..., 5.5, ...] in the level's own coefficients
                                    (Section 6.2); 1 the right-hand side A u of the function u
                                    whose nodal Gauss-Lobatto values are that sequence, the same
                                    start in every basis, so that hierarchies in the Hermite-like
                                    and the nodal basis get the same estimates (Section 6.3) */
    int32_t graded_coarsening;   /* 0 (default): the mesh is coarsened by two while every cell
                                    count is even (the paper's 2^L bricks).  1: every direction
                                    with more than one cell goes from n to ceil(n/2) cells, the
                                    cells paired from lo on; for odd n the last cell stays alone,
                                    so coarse levels are graded bricks (sipg_mesh.width) and
                                    every mesh coarsens down to one cell */
    int32_t coarse_direct_max_dofs; /* 0 (default): the coarsest level is solved by the Chebyshev
                                    iteration above.  n in [1, 1024]: a coarsest level of at most
                                    n unknowns is solved exactly instead, by a dense inverse of
                                    its matrix formed at set-up (n products with the level's
                                    FP64 operator, then a Cholesky inverse on the host: about
                                    10 ms at 256, 1 s at 1024) and applied in one launch per
                                    V-cycle.  Coarsening stops at the first level that small */
} sipg_mg_opts;
typedef struct {
    int32_t levels;
    int64_t ndofs;
    int32_t precision;
    double lambda_max_fine;      /* estimated largest eigenvalue of P^-1 A, finest level */
    double lambda_min_coarse, lambda_max_coarse;
    int32_t coarse_steps;        /* Chebyshev degree of the coarse solve (0: dense inverse) */
    int64_t device_bytes;        /* device memory owned by the solver */
} sipg_mg_info;
typedef struct sipg_mg sipg_mg;

/* Fill *opts with the defaults above. */
int sipg_mg_default_opts(sipg_mg_opts* opts);
/* Build the hierarchy (operators, diagonals, eigenvalue estimates) for the
 * same problem as sipg_setup; opts may be NULL (defaults).  Synchronises
 * `stream`.  The solver owns all its device memory: the level operators,
 * vectors and CG work vectors come from `allocator` (NULL: hipMalloc) and are
 * returned in sipg_mg_destroy. */
int sipg_mg_setup(const sipg_mesh* mesh, int degree, double penalty_factor, int basis,
                  const sipg_mg_opts* opts, const sipg_allocator* allocator, void* stream, sipg_mg** out);
int sipg_mg_destroy(sipg_mg* mg);
int sipg_mg_get_info(const sipg_mg* mg, sipg_mg_info* info);
/* z = V-cycle(r): one application of the preconditioner (device, double, ndofs). */
int sipg_mg_apply_vcycle(sipg_mg* mg, const double* r, double* z, void* stream);
/* Solve A x = b (device, double) to ||b - A x|| <= rel_tol ||b|| with the
 * preconditioned CG; x holds the initial guess, b and x must not overlap.
 * The stopping test is taken on the device after every iteration and read by
 * the host with a lag (the device does not wait for the host); x is the
 * iterate of the first iteration that meets the tolerance.  Blocks the host
 * until then.  Uses the FP64 work vectors allocated by sipg_mg_setup (so
 * concurrent solves on one hierarchy are not allowed).  SIPG_E_NOCONV after
 * max_iter iterations (info still filled). */
int sipg_mg_solve(sipg_mg* mg, const double* b, double* x, double rel_tol, int max_iter,
                  sipg_solve_info* info, void* stream);
/* nrhs right-hand sides of the same problem solved together (Section 6's
 * solver; several requests for one operator co-scheduled): one iteration
 * loop for all of them, in which every product, smoothing step, transfer,
 * coarse solve, dot product and vector update is one launch covering all
 * right-hand sides.
 *   nrhs        1 .. 16
 *   b, x        device, double, nrhs * ndofs each: right-hand side v at
 *               b + v * ndofs, x likewise (initial guesses in, solutions out);
 *               b and x must not overlap
 *   info        host array of nrhs results
 * Each right-hand side stops being updated at the first iteration where its
 * residual meets rel_tol ||b_v||: its iterate and iteration count are those
 * sipg_mg_solve gives for it alone.  The call returns when all have stopped.  A workspace of the level vectors of nrhs right-hand sides and
 * four FP64 CG vectors per right-hand side is taken from the solver's
 * allocator for the call (without one: stream-ordered hipMallocAsync /
 * hipFreeAsync).  Blocks the host; not concurrent with other solves on the
 * same hierarchy.  SIPG_E_ARG for bad sizes or overlapping b and x,
 * SIPG_E_OOM when the workspace cannot be had, SIPG_E_NOCONV when some
 * right-hand side did not converge within max_iter (info still filled). */
int sipg_mg_solve_many(sipg_mg* mg, int nrhs, const double* b, double* x, double rel_tol, int max_iter,
                       sipg_solve_info* info, void* stream);

/* Grid transfer between level `level` and level+1 of the hierarchy (0 =
 * finest), in the V-cycle's precision (float for precision 0, double for 1):
 * mode 0 prolongation out_fine = P in_coarse, mode 1 restriction
 * out_coarse = P^T in_fine.  Device pointers, stream ordered. */
int sipg_mg_transfer(sipg_mg* mg, int level, int mode, const void* in, void* out, void* stream);
/* Unknowns and cell counts of a level. */
int sipg_mg_level_ndofs(const sipg_mg* mg, int level, int64_t* ndofs, int32_t cells[3]);
/* Polynomial degree of a level (host). */
int sipg_mg_level_degree(const sipg_mg* mg, int level, int32_t* degree);

/* b_i = sum_K sum_q f(F_K(xi_q)) phi_i(xi_q) det J w_q for
 * f(x) = sum_m amps[m] sin(w[3m] pi x1) sin(w[3m+1] pi x2) sin(w[3m+2] pi x3),
 * 1 <= nmodes <= 16 (amps, waves in host memory; b device, operator
 * precision).  Stream ordered.  The manufactured solution sin sin sin is the
 * single mode (1,1,1) with amplitude 3 pi^2. */
int sipg_assemble_rhs_sines(const sipg_op* op, int nmodes, const double* amps, const int* waves,
                            void* b, void* stream);

/*
 * Request loop for Poisson solves on one GPU (continuous batching).
 * A request names the problem (mesh, degree, penalty, basis), a smooth source
 * f = sum of sine modes (as for sipg_assemble_rhs_sines) and a tolerance; the
 * server assembles b on the device and solves A x = b with the multigrid
 * solver (precision of the server).  Requests wait in a FIFO; `workers`
 * threads with one HIP stream each take the oldest request whose memory fits
 * the budget, so solves of different requests overlap on the device and new
 * arrivals are admitted as soon as a worker and memory are free.  Solver
 * hierarchies stay resident in a cache keyed by the problem (reused by later
 * requests, evicted least-recently-used when memory is needed).
 */
typedef struct {
    int64_t hbm_budget_bytes;    /* device memory the server may hold (64 GiB) */
    int32_t workers;             /* concurrent solves, 1..16 (8) */
    int32_t precision;           /* 0 mixed FP32 V-cycle, 1 FP64 (0) */
    int32_t smoother;            /* sipg_mg_opts.smoother of every solve (1: block Jacobi) */
    int32_t p_coarsening;        /* sipg_mg_opts.p_coarsening of every solve (1: halve the
                                    degree; requests have odd cell counts too) */
    double coarse_reduction;     /* sipg_mg_opts.coarse_reduction of every solve (10).  An
                                    odd or prime cell count cannot be coarsened, so the
                                    coarse level of such a request is its whole mesh at
                                    the reduced degree; inside the V-cycle preconditioner
                                    a reduction of 10 there (instead of the 1e5 of the
                                    plain solver) halves the solve time of the served mix
                                    for the same final residual, at 3% more CG steps */
    int32_t graded_coarsening;   /* sipg_mg_opts.graded_coarsening of every solve (0: on the
                                    served mix the graded levels cost more CG steps than their
                                    cheaper coarse solves save) */
    int32_t coarse_direct_max_dofs; /* sipg_mg_opts.coarse_direct_max_dofs of every solve (256) */
    int32_t batch_max_rhs;       /* requests of one problem (same mesh, degree, basis, penalty,
                                    rel_tol and max_iter) among the next 2 x workers queued
                                    ones are solved together by one sipg_mg_solve_many, at
                                    most this many (1..16; 8; 1: each request alone) */
    int64_t batch_max_dofs;      /* ... while their unknowns add up to at most this (2^20:
                                    small problems, whose solves are bound by launch latency
                                    and gain most; a group of larger ones delays each member
                                    by the whole group's solve) */
} sipg_server_opts;
typedef struct {
    sipg_mesh mesh;
    int32_t degree;
    double penalty_factor;
    int32_t basis;
    int32_t nmodes;              /* 1..16 */
    double amps[16];
    int32_t waves[16][3];
    double rel_tol;
    int32_t max_iter;
    double* x_out;               /* device buffer (ndofs doubles) for the solution, or NULL:
                                    the server then owns it until sipg_release */
} sipg_request;
typedef struct {
    int32_t status;              /* SIPG_OK, SIPG_E_NOCONV, ... of the solve */
    int32_t iterations;
    double true_residual;        /* ||b - A x||_2 */
    double rel_residual;         /* true_residual / ||b||_2 */
    double queue_s, solve_s, total_s;   /* wait, run, submit-to-done (seconds) */
    int64_t ndofs;
    const double* x;             /* device pointer of the solution */
} sipg_result;
typedef struct {
    int64_t queued, completed, cached_hierarchies, used_bytes, peak_bytes;
    int64_t batched_solves;      /* sipg_mg_solve_many calls over 2 or more requests */
    int64_t batched_requests;    /* requests solved in those */
} sipg_server_stats_t;
typedef struct sipg_server sipg_server;

int sipg_server_default_opts(sipg_server_opts* opts);
/* opts may be NULL (defaults).  Hierarchies and server-owned result buffers
 * come from `allocator` (NULL: hipMalloc), whose callbacks are then called
 * from the worker threads too. */
int sipg_server_create(const sipg_server_opts* opts, const sipg_allocator* allocator, sipg_server** out);
/* Non-blocking.  *ticket identifies the request.  SIPG_E_BUDGET if the
 * request alone can never fit the budget, SIPG_E_ARG for an invalid one. */
int sipg_submit(sipg_server* s, const sipg_request* req, uint64_t* ticket);
/* SIPG_E_NOTREADY until the request finished; then fills *res. */
int sipg_poll(sipg_server* s, uint64_t ticket, sipg_result* res);
/* Blocks until the request finished, then fills *res. */
int sipg_wait(sipg_server* s, uint64_t ticket, sipg_result* res);
/* Forget a finished request.  A server-owned solution buffer is freed after
 * the work queued on `stream` so far (for example a copy of the solution made
 * with sipg_copy_device on that stream) has finished: the call waits for it. */
int sipg_release(sipg_server* s, uint64_t ticket, void* stream);
int sipg_server_stats(sipg_server* s, sipg_server_stats_t* stats);
/* Finishes every submitted request, then frees the server. */
int sipg_server_destroy(sipg_server* s);

/* Stream-ordered device-to-device copy of `bytes` bytes (e.g. a result's solution). */
int sipg_copy_device(void* dst, const void* src, size_t bytes, void* stream);

/* Text of the calling thread's last error ("" if none). */
const char* sipg_last_error(void);

/*
 * Host-only: the 1D tables the kernels use, computed in double precision on
 * the CPU (no GPU needed).  With n = degree + 1 and Gauss points x_q:
 *   points[n], weights[n]     Gauss-Legendre rule on (0,1)
 *   shape[n*n]                S[q*n + j]  = phi_j(x_q)
 *   shape_grad[n*n]           S'[q*n + j] = phi_j'(x_q)
 *   colloc_grad[n*n]          D[q*n + j]  = l_j'(x_q), Lagrange basis in the Gauss points
 *   face_value0[n], face_grad0[n], face_value1[n], face_grad1[n]
 *                             phi_j(0), phi_j'(0), phi_j(1), phi_j'(1)
 *   to_gl[n*n]                T = E^-1 with E[i*n + j] = phi_i(x^GL_j), row major
 * Any pointer may be NULL.  SIPG_E_ARG for a bad degree or basis.
 */
typedef struct {
    double* points;
    double* weights;
    double* shape;
    double* shape_grad;
    double* colloc_grad;
    double* face_value0;
    double* face_grad0;
    double* face_value1;
    double* face_grad1;
    double* to_gl;
} sipg_tables1d;
int sipg_host_tables(int degree, int basis, sipg_tables1d* out);

/* Host-only: the 1D tables of SIPG_BC_FDM (Section 6.4) that the library
 * builds for (degree, basis, penalty_factor): zt[m*n + j] = z_m[j], the
 * generalized eigenvectors of L z = lambda M z on the unit interval (L the
 * interior-element SIPG matrix with penalty penalty_factor (degree+1)^2, M the
 * mass matrix), normalised to Z^T M Z = I, and lam[m].  zt: n*n doubles, lam:
 * n doubles, n = degree + 1 (caller-owned host memory). */
int sipg_host_fdm_tables(int degree, int basis, double penalty_factor, double* zt, double* lam);

#ifdef __cplusplus
}
#endif
#endif /* SIPG_H */
