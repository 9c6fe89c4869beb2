// Operator set-up on the device: metric terms of the cells and the faces
// (Section 3, eq. integral_laplace; Section 4.2 for the per-point storage),
// computed in double precision from the analytic mesh map and stored in the
// operator's precision.
#include "sipg_common.hpp"
#include "sumfac.hpp"
#include "setup.hpp"
#include "basis1d.hpp"

namespace sipg {

// Brick point X of cell (ix, iy, iz) at reference point xi, and the cell's
// widths w.
__device__ void brick_point(const MeshDev& m, const int i[3], const double xi[3], double X[3], double w[3]) {
    for (int d = 0; d < 3; ++d) {
        const int gi = d == 2 ? i[2] + m.z0 : i[d], gn = d == 2 ? m.nzg : m.n[d];   // index in the mesh
        w[d] = gi == gn - 1 ? m.hl[d] : m.h[d];
        X[d] = m.lo[d] + gi * m.h[d] + xi[d] * w[d];
    }
}

// J[a][b] = dx_a / dxi_b of the map of cell (ix, iy, iz) at reference point xi.
__device__ void map_jacobian(const MeshDev& m, int ix, int iy, int iz, double x0, double x1,
                             double x2, double J[9]) {
    const int ci[3] = {ix, iy, iz};
    const double xi[3] = {x0, x1, x2};
    double X[3], w[3];
    brick_point(m, ci, xi, X, w);
    double LH[9], Y[3];
    for (int i = 0; i < 3; ++i) {
        Y[i] = m.L[3 * i] * X[0] + m.L[3 * i + 1] * X[1] + m.L[3 * i + 2] * X[2];
        for (int j = 0; j < 3; ++j) LH[3 * i + j] = m.L[3 * i + j] * w[j];
    }
    if (m.a == 0.0) {
        for (int i = 0; i < 9; ++i) J[i] = LH[i];
        return;
    }
    const double pi = 3.14159265358979323846;
    double sn[3], cs[3];
    for (int i = 0; i < 3; ++i) sincos(pi * Y[i], &sn[i], &cs[i]);
    const double gs[3] = {pi * cs[0] * sn[1] * sn[2], pi * sn[0] * cs[1] * sn[2],
                          pi * sn[0] * sn[1] * cs[2]};
    // J = (I + a (1,1,1) grad s^T) L diag(w)
    double t[3];
    for (int j = 0; j < 3; ++j) t[j] = gs[0] * LH[j] + gs[1] * LH[3 + j] + gs[2] * LH[6 + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[3 * i + j] = LH[3 * i + j] + m.a * t[j];
}

// Physical point of cell (ix, iy, iz) at reference point xi (same map).
__device__ void map_point(const MeshDev& m, int ix, int iy, int iz, double x0, double x1, double x2,
                          double x[3]) {
    const int ci[3] = {ix, iy, iz};
    const double xi[3] = {x0, x1, x2};
    double X[3], w[3];
    brick_point(m, ci, xi, X, w);
    double Y[3];
    for (int i = 0; i < 3; ++i) Y[i] = m.L[3 * i] * X[0] + m.L[3 * i + 1] * X[1] + m.L[3 * i + 2] * X[2];
    double s = 0.0;
    if (m.a != 0.0) {
        const double pi = 3.14159265358979323846;
        s = m.a * sin(pi * Y[0]) * sin(pi * Y[1]) * sin(pi * Y[2]);
    }
    for (int i = 0; i < 3; ++i) x[i] = Y[i] + s;
}

__device__ double inverse3(const double J[9], double Ji[9]) {
    const double c00 = J[4] * J[8] - J[5] * J[7];
    const double c01 = J[5] * J[6] - J[3] * J[8];
    const double c02 = J[3] * J[7] - J[4] * J[6];
    const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
    const double id = 1.0 / det;
    Ji[0] = c00 * id;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) * id;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) * id;
    Ji[3] = c01 * id;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) * id;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) * id;
    Ji[6] = c02 * id;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) * id;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) * id;
    return det;
}

struct Rule {
    double x[16], w[16];
    int n;
};

// Cell metric: G = J^-1 J^-T det J (times w_q for per-point storage), and the
// cell measure |K| = sum_q det J w_q.  One thread per cell.
template <typename T, int MODE>
__global__ void cell_geometry_kernel(MeshDev m, Rule r, T* __restrict__ out,
                                     double* __restrict__ vol, int* __restrict__ bad, int64_t ncells) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int ix = c % m.n[0], iy = (c / m.n[0]) % m.n[1], iz = c / (int64_t(m.n[0]) * m.n[1]);
    const int n = r.n, n3 = n * n * n;
    double v = 0.0;
    for (int q = 0; q < n3; ++q) {
        const int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
        double J[9], Ji[9];
        map_jacobian(m, ix, iy, iz, r.x[q1], r.x[q2], r.x[q3], J);
        const double det = inverse3(J, Ji);
        if (!(det > 0.0)) atomicOr(bad, 1);
        const double w = r.w[q1] * r.w[q2] * r.w[q3];
        v += det * w;
        if (MODE == GEOM_QPOINT || q == 0) {
            double G[6];
            int k = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = a; b < 3; ++b)
                    G[k++] = (Ji[3 * a] * Ji[3 * b] + Ji[3 * a + 1] * Ji[3 * b + 1] + Ji[3 * a + 2] * Ji[3 * b + 2]) * det;
            if (MODE == GEOM_QPOINT) {
                for (int k2 = 0; k2 < 6; ++k2)
                    out[c * 6 * n3 + cell_metric_offset(n, 16 / int(sizeof(T)), k2, q)] = T(G[k2] * w);
            } else {
                for (int k2 = 0; k2 < 6; ++k2) out[c * 8 + k2] = T(G[k2]);
                out[c * 8 + 6] = T(0);
                out[c * 8 + 7] = T(0);
            }
        }
    }
    vol[c] = v;
}

// Volumes of the cells across a slab's z boundaries, summed in the order of
// cell_geometry_kernel: below the slab gvol[column], above it
// gvol[nx ny + column] (column = ix + nx iy).  One thread per cell.
__global__ void ghost_volume_kernel(MeshDev m, Rule r, double* __restrict__ gvol) {
    const int64_t ncol = int64_t(m.n[0]) * m.n[1];
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= 2 * ncol) return;
    const int64_t col = t % ncol;
    const int ix = int(col % m.n[0]), iy = int(col / m.n[0]), iz = t < ncol ? -1 : m.n[2];
    const int n = r.n, n3 = n * n * n;
    double v = 0.0;
    for (int q = 0; q < n3; ++q) {
        const int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
        double J[9], Ji[9];
        map_jacobian(m, ix, iy, iz, r.x[q1], r.x[q2], r.x[q3], J);
        const double det = inverse3(J, Ji);
        v += det * (r.w[q1] * r.w[q2] * r.w[q3]);
    }
    gvol[t] = v;
}

// Face records for the faces normal to direction d, one thread per face.
// Record = {JxW sigma, JxW J_L^-1 n, JxW J_R^-1 n} with n the unit normal
// pointing from the lower cell L to the upper cell R; on boundary faces the
// missing side takes the present cell's values (mirror principle).  Per-point
// storage multiplies by the face quadrature weights and stores the records
// of a direction plane by plane (face_rec_offset); per-face storage keeps the
// weight-free constant of an affine face.
template <typename T, int MODE>
__global__ void face_geometry_kernel(MeshDev m, Rule r, int d, double sigma0, T* __restrict__ out,
                                     const double* __restrict__ vol, const double* __restrict__ gvol, int64_t nfaces) {
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= nfaces) return;
    int ext[3] = {m.n[0], m.n[1], m.n[2]};
    ext[d] += 1;
    int idx[3];
    idx[0] = f % ext[0];
    idx[1] = (f / ext[0]) % ext[1];
    idx[2] = f / (int64_t(ext[0]) * ext[1]);
    // a side exists if its cell is in the mesh; on a slab, the cells across
    // its z boundaries are in the mesh but not in the slab: their volumes are
    // gvol[column] (below) and gvol[nx ny + column] (above)
    const int gz = d == 2 ? idx[2] + m.z0 : idx[d], gn = d == 2 ? m.nzg : m.n[d];
    const bool hasL = gz > 0, hasR = gz < gn;
    int cl[3] = {idx[0], idx[1], idx[2]}, cr[3] = {idx[0], idx[1], idx[2]};
    cl[d] -= 1;
    const int64_t col = idx[0] + int64_t(m.n[0]) * idx[1];
    const bool ghostL = d == 2 && hasL && cl[2] < 0, ghostR = d == 2 && hasR && cr[2] >= m.n[2];
    const int64_t cellL = hasL && !ghostL ? cl[0] + int64_t(m.n[0]) * (cl[1] + int64_t(m.n[1]) * cl[2]) : -1;
    const int64_t cellR = hasR && !ghostR ? cr[0] + int64_t(m.n[0]) * (cr[1] + int64_t(m.n[1]) * cr[2]) : -1;
    const double volL = ghostL ? gvol[col] : hasL ? vol[cellL] : 0.0;
    const double volR = ghostR ? gvol[int64_t(m.n[0]) * m.n[1] + col] : hasR ? vol[cellR] : 0.0;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int n = r.n, n2 = n * n;
    const int npts = MODE == GEOM_QPOINT ? n2 : 1;
    double area = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        double sigma = 0.0;
        if (pass == 1) {
            double ih = 0.0;
            if (hasL) ih = fmax(ih, area / volL);
            if (hasR) ih = fmax(ih, area / volR);
            sigma = sigma0 * ih;
        }
        for (int q = 0; q < npts; ++q) {
            const int qa = q % n, qb = q / n;
            double xiL[3], xiR[3];
            xiL[d] = 1.0;
            xiR[d] = 0.0;
            const double xa = MODE == GEOM_QPOINT ? r.x[qa] : 0.5, xb = MODE == GEOM_QPOINT ? r.x[qb] : 0.5;
            const double wq = MODE == GEOM_QPOINT ? r.w[qa] * r.w[qb] : 1.0;
            xiL[t1] = xiR[t1] = xa;
            xiL[t2] = xiR[t2] = xb;
            double JL[9], JLi[9], JR[9], JRi[9];
            double detL = 0.0, detR = 0.0;
            if (hasL) { map_jacobian(m, cl[0], cl[1], cl[2], xiL[0], xiL[1], xiL[2], JL); detL = inverse3(JL, JLi); }
            if (hasR) { map_jacobian(m, cr[0], cr[1], cr[2], xiR[0], xiR[1], xiR[2], JR); detR = inverse3(JR, JRi); }
            if (!hasL) { for (int i = 0; i < 9; ++i) JLi[i] = JRi[i]; detL = detR; }
            if (!hasR) { for (int i = 0; i < 9; ++i) JRi[i] = JLi[i]; detR = detL; }
            // own side for the measure and the normal: L if present, else R
            const double* Ji = hasL ? JLi : JRi;
            const double det = hasL ? detL : detR;
            // J^-T e_d = column d of J^-1 seen as a row: (J^-T)_{a d} = Ji[d][a]
            double nv[3] = {Ji[3 * d], Ji[3 * d + 1], Ji[3 * d + 2]};
            const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            for (int k = 0; k < 3; ++k) nv[k] /= nn;
            const double jxw = det * nn * wq;
            if (pass == 0) { area += jxw; continue; }
            double rec[7];
            rec[0] = jxw * sigma;
            for (int a = 0; a < 3; ++a) {
                rec[1 + a] = jxw * (JLi[3 * a] * nv[0] + JLi[3 * a + 1] * nv[1] + JLi[3 * a + 2] * nv[2]);
                rec[4 + a] = jxw * (JRi[3 * a] * nv[0] + JRi[3 * a + 1] * nv[1] + JRi[3 * a + 2] * nv[2]);
            }
            if (MODE == GEOM_QPOINT) {
                for (int k = 0; k < 7; ++k) out[face_rec_offset(n, 16 / int(sizeof(T)), nfaces, f, k, qa, qb)] = T(rec[k]);
            } else {
                for (int k = 0; k < 7; ++k) out[f * 8 + k] = T(rec[k]);
                out[f * 8 + 7] = T(0);
            }
        }
    }
}

// Right-hand side for f = sum_m a_m sin(p_m pi x1) sin(q_m pi x2) sin(r_m pi x3):
// b_i = sum_q f(F_K(xi_q)) phi_i(xi_q) det J w_q on every cell, the source at
// the mapped Gauss points followed by the transposed sweeps S^T x S^T x S^T.
struct Modes {
    int count;
    double a[16];
    int w[16][3];
};

template <int N, typename T>
__global__ void __launch_bounds__(128) rhs_kernel(MeshDev m, Rule r, Modes md, const T* __restrict__ tab,
                                                  T* __restrict__ b) {
    constexpr int N2 = N * N, N3 = N2 * N;
    constexpr TableLayout TL(N);
    __shared__ T F[N3];
    const int cell = blockIdx.x;
    const int ix = cell % m.n[0], iy = (cell / m.n[0]) % m.n[1], iz = cell / (m.n[0] * m.n[1]);
    const double pi = 3.14159265358979323846;
    for (int q = threadIdx.x; q < N3; q += blockDim.x) {
        const int q1 = q % N, q2 = (q / N) % N, q3 = q / N2;
        double x[3], J[9], Ji[9];
        map_point(m, ix, iy, iz, r.x[q1], r.x[q2], r.x[q3], x);
        map_jacobian(m, ix, iy, iz, r.x[q1], r.x[q2], r.x[q3], J);
        const double det = inverse3(J, Ji);
        double f = 0.0;
        for (int k = 0; k < md.count; ++k)
            f += md.a[k] * sin(md.w[k][0] * pi * x[0]) * sin(md.w[k][1] * pi * x[1]) * sin(md.w[k][2] * pi * x[2]);
        F[q] = T(f * det * r.w[q1] * r.w[q2] * r.w[q3]);
    }
    __syncthreads();
    const int t = threadIdx.x;
    const bool act = t < N2;
    const int ta = t % N, tb = t / N;
    T v[N];
    auto sweep = [&](int dir) {
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k)
                v[k] = F[dir == 0 ? k + N * (ta + N * tb) : dir == 1 ? ta + N * (k + N * tb) : ta + N * (tb + N * k)];
            eo_apply<N, +1>(tab + TL.ST, v, v);
#pragma unroll
            for (int k = 0; k < N; ++k)
                F[dir == 0 ? k + N * (ta + N * tb) : dir == 1 ? ta + N * (k + N * tb) : ta + N * (tb + N * k)] = v[k];
        }
        __syncthreads();
    };
    sweep(0);
    sweep(1);
    sweep(2);
    for (int e = threadIdx.x; e < N3; e += blockDim.x) b[size_t(cell) * N3 + e] = F[e];
}

template <typename T>
static int launch_rhs_t(const sipg_op* op, const Modes& md, void* b, hipStream_t st) {
    std::vector<double> xq, wq;
    gauss_rule(op->n, xq, wq);
    Rule r{};
    r.n = op->n;
    for (int i = 0; i < op->n; ++i) { r.x[i] = xq[i]; r.w[i] = wq[i]; }
    const T* tab = static_cast<const T*>(op->tables);
    T* bp = static_cast<T*>(b);
    const unsigned nb = unsigned(op->ncells);
    switch (op->n) {
#define SIPG_RHS_CASE(NN) \
    case NN: rhs_kernel<NN, T><<<nb, 128, 0, st>>>(op->mesh, r, md, tab, bp); break;
        SIPG_RHS_CASE(2) SIPG_RHS_CASE(3) SIPG_RHS_CASE(4) SIPG_RHS_CASE(5)
        SIPG_RHS_CASE(6) SIPG_RHS_CASE(7) SIPG_RHS_CASE(8) SIPG_RHS_CASE(9)
#undef SIPG_RHS_CASE
        default: set_error("rhs: unsupported degree"); return SIPG_E_UNSUPPORTED;
    }
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

int launch_rhs_sines(const sipg_op* op, int nmodes, const double* amps, const int* waves, void* b, hipStream_t st) {
    Modes md{};
    md.count = nmodes;
    for (int k = 0; k < nmodes; ++k) {
        md.a[k] = amps[k];
        for (int d = 0; d < 3; ++d) md.w[k][d] = waves[3 * k + d];
    }
    return op->dtype == SIPG_F64 ? launch_rhs_t<double>(op, md, b, st) : launch_rhs_t<float>(op, md, b, st);
}

// Cell scalars of the separable block preconditioner (Section 6.4): with
// h_d = |J(1/2,1/2,1/2) e_d| (the cell extents on a Cartesian mesh) the
// values 1/h_1^2, 1/h_2^2, 1/h_3^2 and 1/(h_1 h_2 h_3).  One thread per cell.
template <typename T>
__global__ void fdm_cell_kernel(MeshDev m, T* __restrict__ out, int64_t ncells) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int ix = c % m.n[0], iy = (c / m.n[0]) % m.n[1], iz = c / (int64_t(m.n[0]) * m.n[1]);
    double J[9];
    map_jacobian(m, ix, iy, iz, 0.5, 0.5, 0.5, J);
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = sqrt(J[d] * J[d] + J[3 + d] * J[3 + d] + J[6 + d] * J[6 + d]);
    for (int d = 0; d < 3; ++d) out[c * 4 + d] = T(1.0 / (h[d] * h[d]));
    out[c * 4 + 3] = T(1.0 / (h[0] * h[1] * h[2]));
}

template <typename T>
int build_geometry(sipg_op* op, const std::vector<double>& xq, const std::vector<double>& wq,
                   hipStream_t st) {
    Rule r{};
    r.n = op->n;
    for (int i = 0; i < op->n; ++i) { r.x[i] = xq[i]; r.w[i] = wq[i]; }
    // stream-ordered temporaries: a plain free would wait for the whole device
    double* vol = nullptr;
    double* gvol = nullptr;
    int* bad = nullptr;
    const int64_t ncol = int64_t(op->nc[0]) * op->nc[1];
    SIPG_HIP(hipMallocAsync(reinterpret_cast<void**>(&vol), sizeof(double) * op->ncells, st));
    SIPG_HIP(hipMallocAsync(reinterpret_cast<void**>(&gvol), sizeof(double) * 2 * ncol, st));
    SIPG_HIP(hipMallocAsync(reinterpret_cast<void**>(&bad), sizeof(int), st));
    SIPG_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    const int bs = 128;
    const unsigned gc = unsigned((op->ncells + bs - 1) / bs);
    T* cg = static_cast<T*>(op->cell_geom);
    if (op->geom == GEOM_QPOINT)
        cell_geometry_kernel<T, GEOM_QPOINT><<<gc, bs, 0, st>>>(op->mesh, r, cg, vol, bad, op->ncells);
    else
        cell_geometry_kernel<T, GEOM_CELL><<<gc, bs, 0, st>>>(op->mesh, r, cg, vol, bad, op->ncells);
    SIPG_HIP(hipGetLastError());
    fdm_cell_kernel<T><<<gc, bs, 0, st>>>(op->mesh, static_cast<T*>(op->fdm_cell), op->ncells);
    SIPG_HIP(hipGetLastError());
    if (op->mesh.z0 > 0 || op->mesh.z0 + op->nc[2] < op->mesh.nzg) {
        ghost_volume_kernel<<<unsigned((2 * ncol + bs - 1) / bs), bs, 0, st>>>(op->mesh, r, gvol);
        SIPG_HIP(hipGetLastError());
    }
    const double sigma0 = op->eta * double(op->degree + 1) * double(op->degree + 1);
    for (int d = 0; d < 3; ++d) {
        const unsigned gf = unsigned((op->nfaces[d] + bs - 1) / bs);
        T* fg = static_cast<T*>(op->face_geom[d]);
        if (op->geom == GEOM_QPOINT)
            face_geometry_kernel<T, GEOM_QPOINT><<<gf, bs, 0, st>>>(op->mesh, r, d, sigma0, fg, vol, gvol, op->nfaces[d]);
        else
            face_geometry_kernel<T, GEOM_CELL><<<gf, bs, 0, st>>>(op->mesh, r, d, sigma0, fg, vol, gvol, op->nfaces[d]);
        SIPG_HIP(hipGetLastError());
    }
    int hbad = 0;
    SIPG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    SIPG_HIP(hipFreeAsync(vol, st));
    SIPG_HIP(hipFreeAsync(gvol, st));
    SIPG_HIP(hipFreeAsync(bad, st));
    SIPG_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error("sipg_setup: the mesh map has a non-positive Jacobian determinant");
        return SIPG_E_ARG;
    }
    return SIPG_OK;
}

template int build_geometry<double>(sipg_op*, const std::vector<double>&, const std::vector<double>&, hipStream_t);
template int build_geometry<float>(sipg_op*, const std::vector<double>&, const std::vector<double>&, hipStream_t);

}  // namespace sipg
