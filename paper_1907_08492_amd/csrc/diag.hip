// diag(A) of the SIPG operator in the nodal Gauss-Lobatto basis: the
// element-wise diagonal P_d of the preconditioner of eq. (jacobi), Section 6.3.
// Evaluated directly from the weak form of Section 2 at the quadrature points
// with the operator's stored metric terms (set-up time kernel: one workgroup
// per cell, one thread per unknown).
//   cell:  sum_q grad_xi phi_i^T G_q grad_xi phi_i
//   face:  only unknowns on the face layer (phi_i(face) != 0):
//          sum_q JxW sigma phi_i^2 - phi_i (g- . grad_xi phi_i),  doubled on
//          boundary faces (mirror principle).
#include "sipg_common.hpp"
#include "setup.hpp"

namespace sipg {

template <typename T, int GEOM>
__global__ void gl_diagonal_kernel(const T* __restrict__ tab, int n, const T* __restrict__ cgeom,
                                   const T* __restrict__ fg0, const T* __restrict__ fg1,
                                   const T* __restrict__ fg2, int nx, int ny, int nz, int z0, int nzg,
                                   T* __restrict__ diag, T* __restrict__ inv_diag) {
    const TableLayout TL(n);
    const int cell = blockIdx.x;
    const int n2 = n * n, n3 = n2 * n;
    const int i = threadIdx.x;
    if (i >= n3) return;
    const int ii[3] = {i % n, (i / n) % n, i / n2};
    const T* S = tab + TL.Sgl;     // S[q*n + j] = l_j(x_q)
    const T* Sg = tab + TL.SGgl;   // l_j'(x_q)
    const T* w = tab + TL.w;
    double acc = 0.0;
    // cell term
    for (int q3 = 0; q3 < n; ++q3)
        for (int q2 = 0; q2 < n; ++q2)
            for (int q1 = 0; q1 < n; ++q1) {
                const int qq[3] = {q1, q2, q3};
                double v[3], dv[3];
                for (int t = 0; t < 3; ++t) {
                    v[t] = S[qq[t] * n + ii[t]];
                    dv[t] = Sg[qq[t] * n + ii[t]];
                }
                const double g[3] = {dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]};
                double G[6];
                if (GEOM == GEOM_CELL) {
                    const double wq = double(w[q1]) * double(w[q2]) * double(w[q3]);
                    for (int m = 0; m < 6; ++m) G[m] = double(cgeom[size_t(cell) * 8 + m]) * wq;
                } else {
                    const int q = q1 + n * (q2 + n * q3);
                    for (int m = 0; m < 6; ++m)
                        G[m] = double(cgeom[size_t(cell) * 6 * n3 + cell_metric_offset(n, 16 / int(sizeof(T)), m, q)]);
                }
                acc += G[0] * g[0] * g[0] + G[3] * g[1] * g[1] + G[5] * g[2] * g[2] +
                       2.0 * (G[1] * g[0] * g[1] + G[2] * g[0] * g[2] + G[4] * g[1] * g[2]);
            }
    // face terms
    const int idx[3] = {cell % nx, (cell / nx) % ny, cell / (nx * ny)};
    const int nd[3] = {nx, ny, nz};
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, s = f & 1;
        const int layer = s ? n - 1 : 0;
        if (ii[d] != layer) continue;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        // on a z-slab the faces at its z boundaries are interior faces of the mesh
        const int gi = d == 2 ? idx[2] + z0 : idx[d], gn = d == 2 ? nzg : nd[d];
        const bool interior = s ? gi + 1 < gn : gi > 0;
        int fi[3] = {idx[0], idx[1], idx[2]};
        fi[d] += s;
        int64_t fidx, nf;
        const T* fg;
        if (d == 0) { fidx = fi[0] + int64_t(nx + 1) * (fi[1] + int64_t(ny) * fi[2]); fg = fg0; nf = int64_t(nx + 1) * ny * nz; }
        else if (d == 1) { fidx = fi[0] + int64_t(nx) * (fi[1] + int64_t(ny + 1) * fi[2]); fg = fg1; nf = int64_t(nx) * (ny + 1) * nz; }
        else { fidx = fi[0] + int64_t(nx) * (fi[1] + int64_t(ny) * fi[2]); fg = fg2; nf = int64_t(nx) * ny * (nz + 1); }
        const double dfl = double((s ? tab + TL.df1gl : tab + TL.df0gl)[layer]);
        double fs = 0.0;
        for (int qb = 0; qb < n; ++qb)
            for (int qa = 0; qa < n; ++qa) {
                double rec[7];
                if (GEOM == GEOM_CELL) {
                    const double wq = double(w[qa]) * double(w[qb]);
                    for (int k = 0; k < 7; ++k) rec[k] = double(fg[fidx * 8 + k]) * wq;
                } else {
                    for (int k = 0; k < 7; ++k) rec[k] = double(fg[face_rec_offset(n, 16 / int(sizeof(T)), nf, fidx, k, qa, qb)]);
                }
                double gm[3];
                for (int k = 0; k < 3; ++k) gm[k] = s ? rec[1 + k] : -rec[4 + k];
                const double va = S[qa * n + ii[t1]], vb = S[qb * n + ii[t2]];
                const double da = Sg[qa * n + ii[t1]], db = Sg[qb * n + ii[t2]];
                const double phi = va * vb;
                double grad[3];
                grad[d] = dfl * phi;
                grad[t1] = da * vb;
                grad[t2] = va * db;
                fs += rec[0] * phi * phi - phi * (gm[0] * grad[0] + gm[1] * grad[1] + gm[2] * grad[2]);
            }
        acc += interior ? fs : 2.0 * fs;
    }
    const size_t o = size_t(cell) * n3;
    if (diag) diag[o + i] = T(acc);
    inv_diag[o + inv_diag_offset(n, 16 / int(sizeof(T)), i)] = T(1.0 / acc);
}

int launch_gl_diagonal(const sipg_op* op, void* diag, hipStream_t st) {
    const int n3 = op->n * op->n * op->n;
    const int bs = ((n3 + 63) / 64) * 64;
    const unsigned nb = unsigned(op->ncells);
    if (op->dtype == SIPG_F64) {
        using T = double;
        auto k = op->geom == GEOM_CELL ? gl_diagonal_kernel<T, GEOM_CELL> : gl_diagonal_kernel<T, GEOM_QPOINT>;
        k<<<nb, bs, 0, st>>>(static_cast<const T*>(op->tables), op->n, static_cast<const T*>(op->cell_geom),
                             static_cast<const T*>(op->face_geom[0]), static_cast<const T*>(op->face_geom[1]),
                             static_cast<const T*>(op->face_geom[2]), op->nc[0], op->nc[1], op->nc[2],
                             op->mesh.z0, op->mesh.nzg, static_cast<T*>(diag), static_cast<T*>(op->gl_inv_diag));
    } else {
        using T = float;
        auto k = op->geom == GEOM_CELL ? gl_diagonal_kernel<T, GEOM_CELL> : gl_diagonal_kernel<T, GEOM_QPOINT>;
        k<<<nb, bs, 0, st>>>(static_cast<const T*>(op->tables), op->n, static_cast<const T*>(op->cell_geom),
                             static_cast<const T*>(op->face_geom[0]), static_cast<const T*>(op->face_geom[1]),
                             static_cast<const T*>(op->face_geom[2]), op->nc[0], op->nc[1], op->nc[2],
                             op->mesh.z0, op->mesh.nzg, static_cast<T*>(diag), static_cast<T*>(op->gl_inv_diag));
    }
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

}  // namespace sipg
