// Internal interfaces between the C-ABI front end and the device code.
#pragma once

#include <vector>

#include "sipg_common.hpp"

namespace sipg {

template <typename T>
int build_geometry(sipg_op* op, const std::vector<double>& xq, const std::vector<double>& wq,
                   hipStream_t st);

// Neighbour layers across the z boundaries of a slab operator (null: none).
struct Ghosts {
    const void* lo = nullptr;
    const void* hi = nullptr;
};

// y = A x for the operator (dispatch over degree, basis, precision, geometry);
// with nv > 1 (no ghosts) for nv right-hand sides stored one after another
// (op->ndofs apart), all in one grid.
int launch_matvec(const sipg_op* op, const void* x, void* y, hipStream_t st, Ghosts g = {}, int nv = 1);
// Per-degree launchers (one translation unit each).
template <int N>
int launch_matvec_n(const sipg_op* op, const void* x, void* y, hipStream_t st, Ghosts g, int nv);
// y = A x and z = P^-1 y of eq. (jacobi) in one pass (needs op->gl_inv_diag).
int launch_matvec_pjacobi(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st, Ghosts g = {});
template <int N>
int launch_matvec_pjacobi_n(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st, Ghosts g);
// The layers of the slab's bottom (side 0) or top (side 1) cells that the
// neighbouring slab reads as its ghost layers.
int launch_pack_ghost(const sipg_op* op, int side, const void* x, void* out, hipStream_t st);
// One Chebyshev smoothing step fused into the product, Hermite-like basis
// only: uo = u + sigma (u - uo) + theta P^-1 (b - A u), P^-1 by mode
// (SIPG_BC_PJACOBI or SIPG_BC_FDM); sigma = 0 does not read uo.  u, uo, b
// distinct.  SIPG_E_UNSUPPORTED for other bases.  nv right-hand sides as in
// launch_matvec.
int launch_matvec_cheb(const sipg_op* op, int mode, const void* b, const void* u, void* uo, double sigma,
                       double theta, hipStream_t st, int nv = 1);
template <int N>
int launch_matvec_cheb_n(const sipg_op* op, int mode, const void* b, const void* u, void* uo, double sigma,
                         double theta, hipStream_t st, int nv);

// Operators of one degree, basis, precision and geometry mode applied by one
// grid (sipg_batch_apply).  Device arrays: `params` holds one kernel
// parameter block per operator, `blk_first[o]` the first workgroup of
// operator o, `blk_op[b]` the operator of workgroup b.
struct BatchGroup {
    int n = 0, basis = 0, dtype = 0, geom = 0;
    int nops = 0;
    int64_t nblocks = 0;
    int64_t ndofs = 0;
    const void* params = nullptr;
    const int* blk_op = nullptr;
    const int* blk_first = nullptr;
};
int launch_matvec_batched(const BatchGroup& g, hipStream_t st);
template <int N>
int launch_matvec_batched_n(const BatchGroup& g, hipStream_t st);

// Cell-wise basis change / preconditioner (see sipg_basis_change).
int launch_basis_change(const sipg_op* op, int mode, const void* in, void* out, hipStream_t st);

// One Chebyshev step merged with the residual and the preconditioner
// (mode SIPG_BC_PJACOBI or SIPG_BC_FDM): uo = u + sigma (u - uo) + theta P^-1
// (b - au); au null means au = 0, u null means u = 0, sigma = 0 does not read uo.
// zero, when set, is zeroed where uo is written (a zero start's u_old, without
// a fill launch).  nv right-hand sides as in launch_matvec.
int launch_precond_cheb(const sipg_op* op, int mode, const void* b, const void* au, const void* u, void* uo,
                        double sigma, double theta, hipStream_t st, void* zero = nullptr, int nv = 1);

// Bandwidth bound of the fused step (see sipg_stream_bound).
int launch_stream_bound(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st);

// Right-hand side of a sum of sine modes (see sipg_assemble_rhs_sines).
int launch_rhs_sines(const sipg_op* op, int nmodes, const double* amps, const int* waves, void* b, hipStream_t st);

// diag(A) in the nodal Gauss-Lobatto basis, written to `diag` (operator precision).
int launch_gl_diagonal(const sipg_op* op, void* diag, hipStream_t st);

// FP64 conjugate gradient method: work arrays from the operator's allocator
// (cg_solve_device) or from the fixed per-device array (cg_solve_static,
// at most cg_static_max_dofs() unknowns).
int cg_solve_device(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                    sipg_solve_info* info, hipStream_t st);
int cg_solve_static(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                    sipg_solve_info* info, hipStream_t st);
int64_t cg_static_max_dofs();

// Device bytes a multigrid solver for this problem will hold.
int64_t mg_estimate_bytes(const sipg_mesh& mesh, int degree, const sipg_mg_opts& o);

// nrhs right-hand sides of one multigrid solver in lockstep (sipg_mg_solve_many);
// bnorm (null or nrhs values) receives ||b_v||, conv (null or nrhs) whether
// right-hand side v converged.  mg_many_bytes / mg_many_estimate: the device
// bytes of its workspace for a solver, or for the solver of (mesh, degree, o).
int mg_solve_many(sipg_mg* mg, int nrhs, const double* b, double* x, double rel_tol, int max_iter,
                  sipg_solve_info* info, double* bnorm, int* conv, hipStream_t st);
int64_t mg_many_bytes(const sipg_mg* mg, int nv);
int64_t mg_many_estimate(const sipg_mesh& mesh, int degree, const sipg_mg_opts& o, int nv);
constexpr int kMaxSolveRhs = 16;

// Accessors of the multigrid solver used by the request loop.
sipg_op* mg_fine_operator(sipg_mg* mg);
double* mg_rhs_buffer(sipg_mg* mg);
double mg_last_rhs_norm(const sipg_mg* mg);

}  // namespace sipg
