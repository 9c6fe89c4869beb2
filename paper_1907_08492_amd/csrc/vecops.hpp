// Vector kernels (FP32 / FP64) used by the solvers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sipg {

constexpr int kVecPartials = 2048;   // size of the partial-sum buffer of vec_dot_async

template <typename T> int vec_cheb(const T* u, T* u_old, const T* z, double sigma, double theta, int64_t n, hipStream_t st);
template <typename T> int vec_sub(const T* b, const T* a, T* r, int64_t n, hipStream_t st);
template <typename T> int vec_axpby(double alpha, const T* x, double beta, T* y, int64_t n, hipStream_t st);
template <typename T> int vec_scale(double alpha, const T* x, T* y, int64_t n, hipStream_t st);
template <typename TO, typename TI> int vec_convert(const TI* x, TO* y, int64_t n, hipStream_t st);
// x_i = -5.5 + (i mod 12)
template <typename T> int vec_sawtooth(T* x, int64_t n, hipStream_t st);
// Updates whose coefficient c = sign * num[0] / den[0] is read from device
// memory:  y = c x + y  and  y = x + c y  (sign = +1); out[0] = num[0] / den[0]
// (or num[0] when den is null).
template <typename T> int vec_axpy_dev(const double* num, const double* den, double sign, const T* x, T* y, int64_t n, hipStream_t st);
template <typename T> int vec_xpby_dev(const T* x, const double* num, const double* den, T* y, int64_t n, hipStream_t st);
int scalar_ratio(const double* num, const double* den, double* out, hipStream_t st);
// y = A x for a dense n x n matrix A (row major); for nv vectors x (and y)
// stored one after another
template <typename T> int vec_dense_mv(const T* A, const T* x, T* y, int n, hipStream_t st, int nv = 1);
// *out = sum a_i b_i (device scalar, double); partial holds kVecPartials doubles
template <typename T> int vec_dot_async(const T* a, const T* b, double* partial, double* out, int64_t n, hipStream_t st);

// Several right-hand sides advanced together (nv vectors of n entries stored
// one after another; per-vector device scalars num[v], den[v], active[v]):
// out[v] = a_v . b_v (partial holds nv * kVecPartials doubles);
// y_v = sign num[v]/den[v] x_v + y_v and y_v = x_v + num[v]/den[v] y_v for
// the vectors with active[v] != 0; out[v] = num[v] for those.
template <typename T> int vec_dot_many(const T* a, const T* b, double* partial, double* out, int64_t n, int nv, hipStream_t st);
template <typename T> int vec_axpy_many(const double* num, const double* den, const double* active, double sign, const T* x,
                                        T* y, int64_t n, int nv, hipStream_t st);
template <typename T> int vec_xpby_many(const T* x, const double* num, const double* den, const double* active, T* y,
                                        int64_t n, int nv, hipStream_t st);
int scalar_copy_many(const double* num, const double* active, double* out, int nv, hipStream_t st);
// Stopping test of the conjugate gradient method per right-hand side (nv <= 64):
// target[v] = rel_tol ||b_v|| (rel_tol when b_v = 0) from bb[v], active[v] =
// (||r_v|| > target[v]) from rr[v], iters[v] = 0; after each iteration an
// active vector counts it and stops once ||r_v|| <= target[v].
int cg_start_many(const double* bb, const double* rr, double rel_tol, double* target, double* active, double* iters,
                  int nv, hipStream_t st);
int cg_mask_many(const double* rr, const double* target, double* active, double* iters, int nv, hipStream_t st);

// Grid transfer between a mesh and its coarsening in every direction (fine
// cells paired from the low end, the last coarse cell of an odd count with one
// child): tensor-product embedding of each coarse cell into its children.
// emb: M_0, M_1 of two halves, then per direction the pair of the last coarse
// cell (8 n x n matrices).  Prolongation: fine += P coarse.  Restriction:
// coarse = P^T fine.
// nv > 1: nv vectors stored one after another on each side.
template <typename T>
int transfer_prolongate_add(int n, const int nc_fine[3], const T* coarse, T* fine, const T* emb, hipStream_t st,
                            int nv = 1);
template <typename T>
int transfer_restrict(int n, const int nc_fine[3], const T* fine, T* coarse, const T* emb, hipStream_t st, int nv = 1);
// Between degrees on one mesh: restriction out = (E^T)^{x3} in (Et: nc x nf),
// or prolongation out += E^{x3} in (E: nf x nc); nf, nc = degree + 1.
template <typename T>
int transfer_degree(int nf, int nc, int64_t ncells, bool restrict_, const T* in, T* out, const T* E, const T* Et,
                    hipStream_t st, int nv = 1);

}  // namespace sipg
