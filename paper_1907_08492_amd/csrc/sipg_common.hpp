// Shared definitions of the device code and the host library: operator
// record, packed 1D tables, launch shapes, error helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "../../include/sipg.h"

namespace sipg {

// ---------------------------------------------------------------------------
// Launch shape per n = k + 1: cells per workgroup and threads per workgroup.
// Three 64-wide wavefronts per workgroup.  In the cell steps one thread owns
// one n-long pencil of a cell (n^2 threads per cell); in the face steps
// wavefront d owns the faces of normal direction d, one lane per face row,
// so cells_per_block * 2n <= 64 and cells_per_block * n^2 <= 192.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cells_per_block(int n) {
    return n == 2 ? 16 : n == 3 ? 10 : n == 4 ? 8 : n == 5 ? 6 : n == 6 ? 5 : n == 7 ? 3 : n == 8 ? 3 : 2;
}
__host__ __device__ constexpr int threads_per_block(int) { return 192; }

// Row stride of the face arrays in LDS.  A face array row holds the same row
// of every (cell, side) face of one direction, 2 n cells_per_block words,
// padded so that row-wise accesses of a wavefront hit distinct banks.
__host__ __device__ constexpr int face_row_stride(int n) {
    return n == 2 ? 65 : n == 3 ? 61 : n == 4 ? 65 : n == 5 ? 65 : n == 6 ? 65 : n == 7 ? 49 : n == 8 ? 49 : 37;
}

// Dynamic LDS bytes of the matrix-free kernel (must match Shape<N> in
// matvec.hpp): the x/work array of every cell plus 9 face arrays (3 per
// direction) of n rows; the cell arrays B, C start at the seventh face array.
__host__ __device__ constexpr size_t matvec_lds_bytes_rt(int n, int esz) {
    const int rs = (n % 2 == 0) ? n + 1 : n;
    const int cs = rs * n * n;
    const int cells = cells_per_block(n) * cs, farr = n * face_row_stride(n);
    const int faces = 9 * farr > 6 * farr + 2 * cells ? 9 * farr : 6 * farr + 2 * cells;
    return size_t(cells + faces) * esz;
}

// ---------------------------------------------------------------------------
// Even-odd packed form of an n x n matrix M with M[n-1-q][n-1-j] = eps M[q][j]
// (all 1D matrices here have this symmetry because phi_i(xi) =
// phi_{p-i}(1-xi) and the point sets are symmetric, Section 4.1).
// Layout, h = n/2:  A[h][h], B[h][h], C[h], R[h], M_center  (2h^2 + 2h + 1).
//   A[q][j] = (M[q][j] + M[q][n-1-j]) / 2,  B[q][j] = (M[q][j] - M[q][n-1-j]) / 2,
//   C[q] = M[q][h] (odd n), R = middle row (A-type for eps=+1, B-type for eps=-1).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int eo_size(int n) { return 2 * (n / 2) * (n / 2) + 2 * (n / 2) + 1; }

// Offsets (in elements) of the packed tables of an operator.
struct TableLayout {
    int n, es;
    int S, ST, D, DT, SG, T, TT, ET;   // even-odd packed matrices
    int df0, df1, w;                   // face derivative rows at 0 and 1, Gauss weights
    int Sgl, SGgl, df0gl, df1gl;       // plain row-major tables of the nodal GL basis
    int FZP, FLAM;                     // block preconditioner: parity-split eigenvectors, eigenvalues
    int FV0, FV1;                      // face value rows S_f at 0 and 1
    int MM, CT, CS, LL;                // even-odd packed 1D M = S^T W S, Ct = S^T W S', Cs = S'^T W S, L = S'^T W S'
    int total;
    __host__ __device__ constexpr TableLayout(int n_)
        : n(n_), es(eo_size(n_)), S(0), ST(es), D(2 * es), DT(3 * es), SG(4 * es),
          T(5 * es), TT(6 * es), ET(7 * es), df0(8 * es), df1(8 * es + n_), w(8 * es + 2 * n_),
          Sgl(8 * es + 3 * n_), SGgl(8 * es + 3 * n_ + n_ * n_), df0gl(8 * es + 3 * n_ + 2 * n_ * n_),
          df1gl(8 * es + 4 * n_ + 2 * n_ * n_), FZP(8 * es + 5 * n_ + 2 * n_ * n_),
          FLAM(8 * es + 5 * n_ + 3 * n_ * n_), FV0(8 * es + 6 * n_ + 3 * n_ * n_),
          FV1(8 * es + 7 * n_ + 3 * n_ * n_), MM(8 * es + 8 * n_ + 3 * n_ * n_), CT(9 * es + 8 * n_ + 3 * n_ * n_),
          CS(10 * es + 8 * n_ + 3 * n_ * n_), LL(11 * es + 8 * n_ + 3 * n_ * n_), total(12 * es + 8 * n_ + 3 * n_ * n_ + 1) {}
};

// Geometry storage modes (GEOM_CELL, GEOM_QPOINT as in the C ABI).  The
// product kernel has a third variant for per-cell storage whose metric
// tensors are all diagonal (affine map with a diagonal linear part).
enum GeomMode { GEOM_CELL = 1, GEOM_QPOINT = 2, GEOM_CELL_DIAG = 3 };

// Number of stored values per cell / per face for each geometry mode.
__host__ __device__ constexpr int cell_geom_stride(int mode, int n) { return mode == GEOM_QPOINT ? 6 * n * n * n : 8; }
__host__ __device__ constexpr int face_geom_stride(int mode, int n) { return mode == GEOM_QPOINT ? 7 * n * n : 8; }

// Offset, inside a cell's per-point record of 6 n^3 values, of metric
// component m at point q = q1 + n (q2 + n q3), with `chunk` = 16 / sizeof
// (element) points per load.  The points of one (q1, q2) pencil along q3
// are stored in chunks next to each other, so that the thread of a pencil
// reads them with 16-byte loads and a wavefront's load is one contiguous,
// 16-byte aligned range per cell: first the chunks of every component
// ([m][q3 / chunk][pencil][chunk]), then the remaining points of every pencil
// ([m][pencil][rest]).
__host__ __device__ constexpr int cell_metric_offset(int n, int chunk, int m, int q) {
    const int n2 = n * n, t = q % n2, k = q / n2, J = n / chunk, R = n % chunk;
    return k < J * chunk ? (m * J + k / chunk) * chunk * n2 + chunk * t + k % chunk
                         : 6 * J * chunk * n2 + m * R * n2 + R * t + (k - J * chunk);
}

// Offset of stored value k (0..6) at face point (qa along t1, qb along t2) of
// face f among the nf faces of one direction, per-point storage, with
// `chunk` = 16 / sizeof(element) points per load.  The records of a
// direction are stored plane by plane: plane (k, j) holds, for every face in
// order, the points qb = chunk j, ..., chunk j + chunk - 1 of every qa
// ([face][qa][chunk]); for n not a multiple of the chunk, the remaining
// points of every qa follow in planes k ([face][qa][rest]).  The lanes of a
// face step that own consecutive columns qa of the faces of consecutive
// cells then read one contiguous, 16-byte aligned range per plane.
__host__ __device__ constexpr int64_t face_rec_offset(int n, int chunk, int64_t nf, int64_t f, int k, int qa,
                                                      int qb) {
    const int J = n / chunk, R = n % chunk;
    return qb < J * chunk ? ((int64_t(k) * J + qb / chunk) * nf + f) * (chunk * n) + chunk * qa + qb % chunk
                          : int64_t(7) * J * chunk * n * nf + (int64_t(k) * nf + f) * (R * n) + R * qa + (qb - J * chunk);
}

// Offset, inside a cell's n^3 values of the inverse diagonal kept for
// P^-1 of eq. (jacobi), of unknown i = i1 + n (i2 + n i3).  The kernels read
// it by x pencils (thread t = i2 + n i3 takes i1 = 0..n-1), so each pencil's
// values are stored in chunks of `chunk` = 16 / sizeof(element) consecutive
// i1 next to each other ([i1 / chunk][t][chunk]), then the remaining i1 of
// every pencil ([t][rest]): a pencil is read with 16-byte loads, and the
// pencils of a cell read one contiguous range per load.
__host__ __device__ constexpr int inv_diag_offset(int n, int chunk, int i) {
    const int n2 = n * n, t = i / n, k = i % n, J = n / chunk, R = n % chunk;
    return k < J * chunk ? (k / chunk) * chunk * n2 + chunk * t + k % chunk : J * chunk * n2 + R * t + (k - J * chunk);
}

// Device memory of the library's objects: through the caller's allocator
// (sipg_allocator) when one was given, else hipMalloc / hipFree.
struct DevAlloc {
    sipg_allocator a{nullptr, nullptr, nullptr};
    DevAlloc() = default;
    explicit DevAlloc(const sipg_allocator* p) {
        if (p) a = *p;
    }
    // *out = `bytes` bytes of device memory; SIPG_OK or SIPG_E_OOM / SIPG_E_HIP
    // with the error text naming `what`
    int alloc(void** out, size_t bytes, const char* what) const;
    void release(void* p) const;
};
// An allocator argument is valid when it is NULL or sets both callbacks or
// neither (neither: hipMalloc / hipFree).
inline bool allocator_valid(const sipg_allocator* a) { return !a || (a->alloc != nullptr) == (a->free != nullptr); }

// Mesh description in the form the device kernels take it: in direction d
// cell i spans [lo + i h, lo + i h + w] with w = h, except the last cell,
// whose width is hl (hl = h on a uniform brick).  An operator on a z-slab of
// a mesh holds the cells z0 <= iz < z0 + n[2] of a mesh of nzg cells along z:
// local cell iz is mesh cell z0 + iz (z0 = 0, nzg = n[2] otherwise).
struct MeshDev {
    int n[3];
    double lo[3], h[3], hl[3];
    double L[9];
    double a;
    int z0, nzg;
};

}  // namespace sipg

// The operator handle (opaque in the C ABI).
struct sipg_op {
    int degree = 0, n = 0, basis = 0, dtype = 0, geom = 0;
    int diag_metric = 0;             // per-cell storage and every metric tensor diagonal
    int nc[3] = {0, 0, 0};
    int64_t ncells = 0, ndofs = 0;
    double eta = 0.0;
    sipg::MeshDev mesh{};
    int device = 0;
    sipg::DevAlloc mem;              // provider of the memory below
    // device memory owned by the operator
    void* tables = nullptr;          // packed 1D tables, operator precision
    void* cell_geom = nullptr;       // [ncells][cell_geom_stride]
    void* face_geom[3] = {nullptr, nullptr, nullptr};   // [nfaces_d][face_geom_stride]
    int64_t nfaces[3] = {0, 0, 0};
    void* gl_inv_diag = nullptr;     // 1 / diag(A_GL) for SIPG_BC_PJACOBI (optional; inv_diag_offset layout)
    void* fdm_cell = nullptr;        // [ncells][4]: 1/h_1^2, 1/h_2^2, 1/h_3^2, 1/(h_1 h_2 h_3)
    int64_t device_bytes = 0;
};

namespace sipg {
// Geometry variant of the product kernel for this operator.
inline int matvec_geom(const sipg_op* op) { return op->geom == GEOM_CELL && op->diag_metric ? GEOM_CELL_DIAG : op->geom; }
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);
}  // namespace sipg

#define SIPG_HIP(call)                                                 \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return sipg::hip_fail(e_, #call);        \
    } while (0)
