// C ABI front end (include/sipg.h): argument checks, operator set-up on the
// host side (1D tables), device memory ownership, dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "basis1d.hpp"
#include "matvec.hpp"
#include "setup.hpp"
#include "sipg_common.hpp"

namespace sipg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SIPG_E_OOM : SIPG_E_HIP;
}

int DevAlloc::alloc(void** out, size_t bytes, const char* what) const {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (a.alloc) {
        *out = a.alloc(bytes, a.ctx);
        if (!*out) {
            g_last_error = std::string(what) + ": the allocator returned no memory";
            return SIPG_E_OOM;
        }
        return SIPG_OK;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        return hip_fail(e, what);
    }
    return SIPG_OK;
}

void DevAlloc::release(void* p) const {
    if (!p) return;
    if (a.free) a.free(p, a.ctx);
    else (void)hipFree(p);
}

// Even-odd packing of an n x n row-major matrix (layout in sipg_common.hpp).
template <typename T>
static void pack_eo(const std::vector<double>& M, int n, int eps, T* out) {
    const int h = n / 2;
    const int oA = 0, oB = h * h, oC = 2 * h * h, oR = 2 * h * h + h, oM = 2 * h * h + 2 * h;
    for (int i = 0; i < eo_size(n); ++i) out[i] = T(0);
    for (int q = 0; q < h; ++q)
        for (int j = 0; j < h; ++j) {
            out[oA + q * h + j] = T(0.5 * (M[q * n + j] + M[q * n + n - 1 - j]));
            out[oB + q * h + j] = T(0.5 * (M[q * n + j] - M[q * n + n - 1 - j]));
        }
    if (n % 2 == 1) {
        for (int q = 0; q < h; ++q) out[oC + q] = T(M[q * n + h]);
        for (int j = 0; j < h; ++j)
            out[oR + j] = T(eps > 0 ? 0.5 * (M[h * n + j] + M[h * n + n - 1 - j])
                                    : 0.5 * (M[h * n + j] - M[h * n + n - 1 - j]));
        out[oM] = T(M[h * n + h]);
    }
}

static std::vector<double> transpose(const std::vector<double>& M, int n) {
    std::vector<double> t(n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) t[j * n + i] = M[i * n + j];
    return t;
}

template <typename T>
static std::vector<T> make_table(const Tables1D& t, const Tables1D& gl, const std::vector<double>& fzp,
                                 const std::vector<double>& lam) {
    const int n = t.n;
    const TableLayout L(n);
    std::vector<T> tab(L.total + 1, T(0));
    pack_eo<T>(t.S, n, +1, &tab[L.S]);
    pack_eo<T>(transpose(t.S, n), n, +1, &tab[L.ST]);
    pack_eo<T>(t.D, n, -1, &tab[L.D]);
    pack_eo<T>(transpose(t.D, n), n, -1, &tab[L.DT]);
    pack_eo<T>(t.Sg, n, -1, &tab[L.SG]);
    pack_eo<T>(t.T, n, +1, &tab[L.T]);
    pack_eo<T>(transpose(t.T, n), n, +1, &tab[L.TT]);
    pack_eo<T>(transpose(t.E, n), n, +1, &tab[L.ET]);
    for (int j = 0; j < n; ++j) {
        tab[L.df0 + j] = T(t.g0[j]);
        tab[L.df1 + j] = T(t.g1[j]);
        tab[L.w + j] = T(t.weights[j]);
        tab[L.df0gl + j] = T(gl.g0[j]);
        tab[L.df1gl + j] = T(gl.g1[j]);
    }
    for (int i = 0; i < n * n; ++i) {
        tab[L.Sgl + i] = T(gl.S[i]);
        tab[L.SGgl + i] = T(gl.Sg[i]);
    }
    for (int i = 0; i < n; ++i) {
        tab[L.FLAM + i] = T(lam[i]);
        tab[L.FV0 + i] = T(t.v0[i]);
        tab[L.FV1 + i] = T(t.v1[i]);
    }
    for (size_t i = 0; i < fzp.size(); ++i) tab[L.FZP + i] = T(fzp[i]);
    // 1D face matrices of the affine (reference-coordinate) face terms, by
    // the n-point Gauss rule, which integrates these degree <= 2p products
    // exactly: M_ij = (phi_i, phi_j), Ct_ij = (phi_i, phi_j'), Cs_ij = (phi_i', phi_j)
    // and the 1D stiffness L_ij = (phi_i', phi_j') of the cell term with a
    // diagonal metric
    std::vector<double> M(size_t(n) * n, 0.0), Ct(size_t(n) * n, 0.0), Cs(size_t(n) * n, 0.0),
        Lk(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int q = 0; q < n; ++q) {
                const double w = t.weights[q];
                M[i * n + j] += w * t.S[q * n + i] * t.S[q * n + j];
                Ct[i * n + j] += w * t.S[q * n + i] * t.Sg[q * n + j];
                Cs[i * n + j] += w * t.Sg[q * n + i] * t.S[q * n + j];
                Lk[i * n + j] += w * t.Sg[q * n + i] * t.Sg[q * n + j];
            }
    pack_eo<T>(M, n, +1, &tab[L.MM]);
    pack_eo<T>(Ct, n, -1, &tab[L.CT]);
    pack_eo<T>(Cs, n, -1, &tab[L.CS]);
    pack_eo<T>(Lk, n, +1, &tab[L.LL]);
    return tab;
}

static int free_op(sipg_op* op) {
    if (!op) return SIPG_OK;
    void* ptrs[] = {op->tables, op->cell_geom, op->face_geom[0], op->face_geom[1], op->face_geom[2], op->gl_inv_diag,
                    op->fdm_cell};
    for (void* p : ptrs) op->mem.release(p);
    delete op;
    return SIPG_OK;
}

int launch_matvec(const sipg_op* op, const void* x, void* y, hipStream_t st, Ghosts g, int nv) {
    if (nv < 1 || (nv > 1 && (g.lo || g.hi))) {
        set_error("product: one right-hand side with ghost layers, at least one otherwise");
        return SIPG_E_ARG;
    }
    switch (op->n) {
        case 2: return launch_matvec_n<2>(op, x, y, st, g, nv);
        case 3: return launch_matvec_n<3>(op, x, y, st, g, nv);
        case 4: return launch_matvec_n<4>(op, x, y, st, g, nv);
        case 5: return launch_matvec_n<5>(op, x, y, st, g, nv);
        case 6: return launch_matvec_n<6>(op, x, y, st, g, nv);
        case 7: return launch_matvec_n<7>(op, x, y, st, g, nv);
        case 8: return launch_matvec_n<8>(op, x, y, st, g, nv);
        case 9: return launch_matvec_n<9>(op, x, y, st, g, nv);
    }
    set_error("unsupported degree");
    return SIPG_E_UNSUPPORTED;
}

int launch_matvec_pjacobi(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st, Ghosts g) {
    switch (op->n) {
        case 2: return launch_matvec_pjacobi_n<2>(op, x, y, z, st, g);
        case 3: return launch_matvec_pjacobi_n<3>(op, x, y, z, st, g);
        case 4: return launch_matvec_pjacobi_n<4>(op, x, y, z, st, g);
        case 5: return launch_matvec_pjacobi_n<5>(op, x, y, z, st, g);
        case 6: return launch_matvec_pjacobi_n<6>(op, x, y, z, st, g);
        case 7: return launch_matvec_pjacobi_n<7>(op, x, y, z, st, g);
        case 8: return launch_matvec_pjacobi_n<8>(op, x, y, z, st, g);
        case 9: return launch_matvec_pjacobi_n<9>(op, x, y, z, st, g);
    }
    set_error("unsupported degree");
    return SIPG_E_UNSUPPORTED;
}

int launch_matvec_cheb(const sipg_op* op, int mode, const void* b, const void* u, void* uo, double sigma,
                       double theta, hipStream_t st, int nv) {
    if (op->basis != SIPG_BASIS_HERMITE_LIKE) {
        set_error("fused Chebyshev step: Hermite-like basis only");
        return SIPG_E_UNSUPPORTED;
    }
    if ((mode == SIPG_BC_PJACOBI && !op->gl_inv_diag) || (mode == SIPG_BC_FDM && !op->fdm_cell) ||
        (mode != SIPG_BC_PJACOBI && mode != SIPG_BC_FDM)) {
        set_error("fused Chebyshev step: preconditioner mode or its data missing");
        return SIPG_E_ARG;
    }
    if (nv < 1) {
        set_error("fused Chebyshev step: at least one right-hand side");
        return SIPG_E_ARG;
    }
    switch (op->n) {
        case 2: return launch_matvec_cheb_n<2>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 3: return launch_matvec_cheb_n<3>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 4: return launch_matvec_cheb_n<4>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 5: return launch_matvec_cheb_n<5>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 6: return launch_matvec_cheb_n<6>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 7: return launch_matvec_cheb_n<7>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 8: return launch_matvec_cheb_n<8>(op, mode, b, u, uo, sigma, theta, st, nv);
        case 9: return launch_matvec_cheb_n<9>(op, mode, b, u, uo, sigma, theta, st, nv);
    }
    set_error("unsupported degree");
    return SIPG_E_UNSUPPORTED;
}

static bool ranges_overlap(const void* a, const void* b, size_t bytes) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + bytes && pb < pa + bytes;
}

// [a, a + la) and [b, b + lb) share a byte
static bool ranges_overlap(const void* a, size_t la, const void* b, size_t lb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + lb && pb < pa + la;
}

// A slab of a z-partition with a neighbouring slab: its product needs ghost layers.
static bool is_inner_slab(const sipg_op* op) { return op->mesh.z0 > 0 || op->mesh.z0 + op->nc[2] < op->mesh.nzg; }

}  // namespace sipg

using namespace sipg;

extern "C" {

const char* sipg_last_error(void) { return g_last_error.c_str(); }

int sipg_host_tables(int degree, int basis, sipg_tables1d* out) {
    if (degree < 1 || degree > 15 || basis < 0 || basis > 2 || !out) {
        set_error("sipg_host_tables: degree must be in [1,15], basis 0, 1 or 2, out non-null");
        return SIPG_E_ARG;
    }
    Tables1D t;
    if (!build_tables(basis, degree, t)) {
        set_error("sipg_host_tables: singular basis-change matrix");
        return SIPG_E_ARG;
    }
    const int n = degree + 1;
    auto cp = [](double* dst, const std::vector<double>& src) {
        if (dst) std::memcpy(dst, src.data(), sizeof(double) * src.size());
    };
    cp(out->points, t.points);
    cp(out->weights, t.weights);
    cp(out->shape, t.S);
    cp(out->shape_grad, t.Sg);
    cp(out->colloc_grad, t.D);
    cp(out->face_value0, t.v0);
    cp(out->face_grad0, t.g0);
    cp(out->face_value1, t.v1);
    cp(out->face_grad1, t.g1);
    cp(out->to_gl, t.T);
    (void)n;
    return SIPG_OK;
}

int sipg_host_fdm_tables(int degree, int basis, double penalty_factor, double* zt, double* lam) {
    if (degree < 1 || degree > 15 || basis < 0 || basis > 2 || !zt || !lam || !(penalty_factor > 0.0)) {
        set_error("sipg_host_fdm_tables: degree in [1,15], basis 0, 1 or 2, penalty > 0, non-null outputs");
        return SIPG_E_ARG;
    }
    std::vector<double> z, l;
    if (!fdm_1d(basis, degree, penalty_factor, z, l)) {
        set_error("sipg_host_fdm_tables: 1D eigenproblem failed");
        return SIPG_E_ARG;
    }
    std::memcpy(zt, z.data(), sizeof(double) * z.size());
    std::memcpy(lam, l.data(), sizeof(double) * l.size());
    return SIPG_OK;
}

// The operator of the cells z0 <= iz < z1 of `mesh` (the whole mesh: z0 = 0,
// z1 = mesh->n[2]).
static int setup_impl(const sipg_mesh* mesh, int z0, int z1, int degree, double penalty_factor, int basis,
                      int dtype, int geometry, const sipg_allocator* allocator, void* stream, sipg_op** out) {
    if (!mesh || !out) { set_error("sipg_setup: null mesh or out"); return SIPG_E_ARG; }
    *out = nullptr;
    if (!allocator_valid(allocator)) { set_error("sipg_setup: allocator needs both callbacks"); return SIPG_E_ARG; }
    if (degree < 1 || degree > 8) { set_error("sipg_setup: degree must be in [1,8]"); return SIPG_E_ARG; }
    if (!(penalty_factor > 0.0) || !std::isfinite(penalty_factor)) { set_error("sipg_setup: penalty_factor must be > 0"); return SIPG_E_ARG; }
    if (basis != SIPG_BASIS_HERMITE_LIKE && basis != SIPG_BASIS_NODAL_GL && basis != SIPG_BASIS_NODAL_GAUSS) {
        set_error("sipg_setup: bad basis");
        return SIPG_E_ARG;
    }
    if (dtype != SIPG_F64 && dtype != SIPG_F32) { set_error("sipg_setup: bad dtype"); return SIPG_E_ARG; }
    if (geometry < SIPG_GEOM_AUTO || geometry > SIPG_GEOM_QPOINT) { set_error("sipg_setup: bad geometry mode"); return SIPG_E_ARG; }
    for (int d = 0; d < 3; ++d) {
        if (mesh->n[d] <= 0) { set_error("sipg_setup: cell counts must be positive"); return SIPG_E_ARG; }
        if (!(mesh->hi[d] > mesh->lo[d])) { set_error("sipg_setup: need hi > lo in every direction"); return SIPG_E_ARG; }
    }
    const bool graded = mesh->width[0] != 0.0 || mesh->width[1] != 0.0 || mesh->width[2] != 0.0;
    if (graded) {
        for (int d = 0; d < 3; ++d) {
            const double w = mesh->width[d], last = mesh->hi[d] - mesh->lo[d] - (mesh->n[d] - 1) * w;
            if (!(w > 0.0) || !std::isfinite(w) || !(last > 0.0) || last > w * (1.0 + 1e-12)) {
                set_error("sipg_setup: graded brick needs width > 0 and a last cell of width in (0, width]");
                return SIPG_E_ARG;
            }
        }
    }
    if (z0 < 0 || z1 > mesh->n[2] || z0 >= z1) {
        set_error("sipg_setup_slab: need 0 <= z0 < z1 <= n[2]");
        return SIPG_E_ARG;
    }
    const int nloc[3] = {mesh->n[0], mesh->n[1], z1 - z0};   // cells of this operator
    const int64_t ncells = int64_t(nloc[0]) * nloc[1] * nloc[2];
    const int n = degree + 1;
    if (ncells * n * n * n > (int64_t(1) << 31) - 1 || ncells > (int64_t(1) << 30)) {
        set_error("sipg_setup: mesh too large (dofs must fit in 31 bits)");
        return SIPG_E_ARG;
    }
    if (geometry == SIPG_GEOM_CELL && mesh->deform_amp != 0.0) {
        set_error("sipg_setup: per-cell geometry requires an undeformed (affine) mesh");
        return SIPG_E_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    sipg_op* op = new (std::nothrow) sipg_op();
    if (!op) { set_error("sipg_setup: out of host memory"); return SIPG_E_OOM; }
    op->mem = DevAlloc(allocator);
    op->degree = degree;
    op->n = n;
    op->basis = basis;
    op->dtype = dtype;
    op->geom = geometry == SIPG_GEOM_AUTO ? (mesh->deform_amp != 0.0 ? GEOM_QPOINT : GEOM_CELL) : geometry;
    // Per-cell storage of an affine map whose linear part is diagonal (or the
    // identity, all zero): J = L diag(h) is diagonal, so is every J^-1 J^-T det J.
    {
        const double* Lm = mesh->lin;
        const bool offdiag_zero = Lm[1] == 0.0 && Lm[2] == 0.0 && Lm[3] == 0.0 && Lm[5] == 0.0 && Lm[6] == 0.0 &&
                                  Lm[7] == 0.0;
        op->diag_metric = op->geom == GEOM_CELL && offdiag_zero ? 1 : 0;
    }
    op->eta = penalty_factor;
    for (int d = 0; d < 3; ++d) op->nc[d] = nloc[d];
    op->ncells = ncells;
    op->ndofs = ncells * n * n * n;
    MeshDev& m = op->mesh;
    bool lin_zero = true;
    for (int i = 0; i < 9; ++i) lin_zero = lin_zero && mesh->lin[i] == 0.0;
    m.z0 = z0;
    m.nzg = mesh->n[2];
    for (int d = 0; d < 3; ++d) {
        m.n[d] = nloc[d];
        m.lo[d] = mesh->lo[d];
        m.h[d] = graded ? mesh->width[d] : (mesh->hi[d] - mesh->lo[d]) / mesh->n[d];
        m.hl[d] = graded ? mesh->hi[d] - mesh->lo[d] - (mesh->n[d] - 1) * mesh->width[d] : m.h[d];
    }
    for (int i = 0; i < 9; ++i) m.L[i] = lin_zero ? (i % 4 == 0 ? 1.0 : 0.0) : mesh->lin[i];
    m.a = mesh->deform_amp;
    {
        const double* L = m.L;
        const double det = L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                           L[2] * (L[3] * L[7] - L[4] * L[6]);
        if (!(det > 0.0)) { free_op(op); set_error("sipg_setup: linear map must have a positive determinant"); return SIPG_E_ARG; }
    }
    hipError_t e = hipGetDevice(&op->device);
    if (e != hipSuccess) { free_op(op); return hip_fail(e, "hipGetDevice"); }

    Tables1D t, tgl;
    std::vector<double> fzt, flam, fzp;
    if (!build_tables(basis, degree, t) || !build_tables(SIPG_BASIS_NODAL_GL, degree, tgl) ||
        !fdm_1d(basis, degree, penalty_factor, fzt, flam, &fzp)) {
        free_op(op);
        set_error("sipg_setup: singular basis change or 1D eigenproblem");
        return SIPG_E_ARG;
    }
    const size_t esz = dtype == SIPG_F64 ? 8 : 4;
    const TableLayout L(n);
    const size_t tab_bytes = esz * (L.total + 1);
    for (int d = 0; d < 3; ++d) {
        int64_t nf = 1;
        for (int k = 0; k < 3; ++k) nf *= (k == d ? nloc[k] + 1 : nloc[k]);
        op->nfaces[d] = nf;
    }
    const size_t cg_bytes = esz * size_t(ncells) * cell_geom_stride(op->geom, n);
    auto fail = [&](hipError_t err, const char* what) { free_op(op); return hip_fail(err, what); };
    auto take = [&](void** p, size_t bytes, const char* what) {
        const int rc = op->mem.alloc(p, bytes, what);
        if (rc != SIPG_OK) free_op(op);
        return rc;
    };
    int arc;
    if ((arc = take(&op->tables, tab_bytes, "sipg_setup: tables")) != SIPG_OK) return arc;
    if ((arc = take(&op->cell_geom, cg_bytes, "sipg_setup: cell geometry")) != SIPG_OK) return arc;
    const size_t fdm_bytes = esz * size_t(ncells) * 4;
    if ((arc = take(&op->fdm_cell, fdm_bytes, "sipg_setup: block preconditioner")) != SIPG_OK) return arc;
    op->device_bytes = int64_t(tab_bytes + cg_bytes + fdm_bytes);
    for (int d = 0; d < 3; ++d) {
        const size_t fb = esz * size_t(op->nfaces[d]) * face_geom_stride(op->geom, n);
        if ((arc = take(&op->face_geom[d], fb, "sipg_setup: face geometry")) != SIPG_OK) return arc;
        op->device_bytes += int64_t(fb);
    }
    if (dtype == SIPG_F64) {
        std::vector<double> tab = make_table<double>(t, tgl, fzp, flam);
        if ((e = hipMemcpyAsync(op->tables, tab.data(), tab_bytes, hipMemcpyHostToDevice, st)) != hipSuccess) return fail(e, "hipMemcpy(tables)");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e, "hipStreamSynchronize");
        const int rc = build_geometry<double>(op, t.points, t.weights, st);
        if (rc != SIPG_OK) { free_op(op); return rc; }
    } else {
        std::vector<float> tab = make_table<float>(t, tgl, fzp, flam);
        if ((e = hipMemcpyAsync(op->tables, tab.data(), tab_bytes, hipMemcpyHostToDevice, st)) != hipSuccess) return fail(e, "hipMemcpy(tables)");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e, "hipStreamSynchronize");
        const int rc = build_geometry<float>(op, t.points, t.weights, st);
        if (rc != SIPG_OK) { free_op(op); return rc; }
    }
    *out = op;
    return SIPG_OK;
}

int sipg_setup(const sipg_mesh* mesh, int degree, double penalty_factor, int basis, int dtype,
               int geometry, const sipg_allocator* allocator, void* stream, sipg_op** out) {
    return setup_impl(mesh, 0, mesh ? mesh->n[2] : 1, degree, penalty_factor, basis, dtype, geometry, allocator, stream,
                      out);
}

int sipg_setup_slab(const sipg_mesh* mesh, int z0, int z1, int degree, double penalty_factor, int basis, int dtype,
                    int geometry, const sipg_allocator* allocator, void* stream, sipg_op** out) {
    return setup_impl(mesh, z0, z1, degree, penalty_factor, basis, dtype, geometry, allocator, stream, out);
}

int sipg_destroy(sipg_op* op) { return free_op(op); }

int sipg_copy_device(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src) { set_error("sipg_copy_device: null pointer"); return SIPG_E_ARG; }
    SIPG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    return SIPG_OK;
}

int sipg_launch_shape(int degree, int dtype, int32_t* cpb, int32_t* nt, int64_t* lds) {
    if (degree < 1 || degree > 8 || (dtype != SIPG_F64 && dtype != SIPG_F32)) {
        set_error("sipg_launch_shape: degree must be in [1,8], dtype SIPG_F64 or SIPG_F32");
        return SIPG_E_ARG;
    }
    const int n = degree + 1;
    if (cpb) *cpb = cells_per_block(n);
    if (nt) *nt = threads_per_block(n);
    if (lds) *lds = int64_t(matvec_lds_bytes_rt(n, dtype == SIPG_F64 ? 8 : 4));
    return SIPG_OK;
}

int sipg_host_block_order(int nblocks, int layer_blocks, int32_t* order) {
    if (nblocks < 1 || layer_blocks < 0 || !order) {
        set_error("sipg_host_block_order: nblocks >= 1, layer_blocks >= 0, order non-null");
        return SIPG_E_ARG;
    }
    for (int b = 0; b < nblocks; ++b) order[b] = xcd_block_zinterleaved(b, nblocks, layer_blocks);
    return SIPG_OK;
}

int64_t sipg_ndofs(const sipg_op* op) { return op ? op->ndofs : -1; }

int sipg_get_info(const sipg_op* op, sipg_op_info* info) {
    if (!op || !info) { set_error("sipg_get_info: null argument"); return SIPG_E_ARG; }
    info->degree = op->degree;
    info->basis = op->basis;
    info->dtype = op->dtype;
    info->geometry = op->geom;
    for (int d = 0; d < 3; ++d) info->n[d] = op->nc[d];
    info->ndofs = op->ndofs;
    info->device_bytes = op->device_bytes;
    info->cells_per_block = cells_per_block(op->n);
    info->threads_per_block = threads_per_block(op->n);
    info->diagonal_metric = op->diag_metric;
    return SIPG_OK;
}

int64_t sipg_ghost_size(const sipg_op* op) {
    if (!op) return -1;
    const int64_t nl = op->basis == SIPG_BASIS_HERMITE_LIKE ? 2 : op->n;
    return int64_t(op->nc[0]) * op->nc[1] * nl * op->n * op->n;
}

int sipg_pack_ghost(const sipg_op* op, int side, const void* x, void* out, void* stream) {
    if (!op || !x || !out || (side != 0 && side != 1)) {
        set_error("sipg_pack_ghost: null argument or side not 0 / 1");
        return SIPG_E_ARG;
    }
    const size_t esz = op->dtype == SIPG_F64 ? 8 : 4;
    if (ranges_overlap(x, size_t(op->ndofs) * esz, out, size_t(sipg_ghost_size(op)) * esz)) {
        set_error("sipg_pack_ghost: x and out overlap");
        return SIPG_E_ARG;
    }
    return launch_pack_ghost(op, side, x, out, static_cast<hipStream_t>(stream));
}

int sipg_apply_slab(const sipg_op* op, const void* x, const void* ghost_lo, const void* ghost_hi, void* y, void* z,
                    void* stream) {
    if (!op || !x || !y) { set_error("sipg_apply_slab: null argument"); return SIPG_E_ARG; }
    const bool below = op->mesh.z0 > 0, above = op->mesh.z0 + op->nc[2] < op->mesh.nzg;
    if (bool(ghost_lo) != below || bool(ghost_hi) != above) {
        set_error("sipg_apply_slab: a ghost buffer is needed exactly for each side with a neighbouring slab");
        return SIPG_E_ARG;
    }
    const size_t bytes = size_t(op->ndofs) * (op->dtype == SIPG_F64 ? 8 : 4);
    if (ranges_overlap(x, y, bytes) || (z && (ranges_overlap(x, z, bytes) || ranges_overlap(y, z, bytes)))) {
        set_error("sipg_apply_slab: x, y and z must not overlap");
        return SIPG_E_ARG;
    }
    const Ghosts g{ghost_lo, ghost_hi};
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!z) return launch_matvec(op, x, y, st, g);
    if (!op->gl_inv_diag) {
        set_error("sipg_apply_slab: z = P^-1 y needs sipg_compute_gl_diagonal first");
        return SIPG_E_ARG;
    }
    return launch_matvec_pjacobi(op, x, y, z, st, g);
}

int sipg_apply(const sipg_op* op, const void* x, void* y, void* stream) {
    if (!op || !x || !y) { set_error("sipg_apply: null argument"); return SIPG_E_ARG; }
    if (is_inner_slab(op)) { set_error("sipg_apply: a slab with neighbours needs sipg_apply_slab"); return SIPG_E_ARG; }
    const size_t bytes = size_t(op->ndofs) * (op->dtype == SIPG_F64 ? 8 : 4);
    if (ranges_overlap(x, y, bytes)) { set_error("sipg_apply: x and y overlap"); return SIPG_E_ARG; }
    return launch_matvec(op, x, y, static_cast<hipStream_t>(stream));
}

int sipg_apply_pjacobi(const sipg_op* op, const void* x, void* y, void* z, void* stream) {
    if (!op || !x || !y || !z) { set_error("sipg_apply_pjacobi: null argument"); return SIPG_E_ARG; }
    if (is_inner_slab(op)) {
        set_error("sipg_apply_pjacobi: a slab with neighbours needs sipg_apply_slab");
        return SIPG_E_ARG;
    }
    if (!op->gl_inv_diag) {
        set_error("sipg_apply_pjacobi: needs sipg_compute_gl_diagonal first");
        return SIPG_E_ARG;
    }
    const size_t bytes = size_t(op->ndofs) * (op->dtype == SIPG_F64 ? 8 : 4);
    if (ranges_overlap(x, y, bytes) || ranges_overlap(x, z, bytes) || ranges_overlap(y, z, bytes)) {
        set_error("sipg_apply_pjacobi: x, y and z must not overlap");
        return SIPG_E_ARG;
    }
    return launch_matvec_pjacobi(op, x, y, z, static_cast<hipStream_t>(stream));
}

int sipg_stream_bound(const sipg_op* op, const void* x, void* y, void* z, void* stream) {
    if (!op || !x || !y || !z) { set_error("sipg_stream_bound: null argument"); return SIPG_E_ARG; }
    if (!op->gl_inv_diag) { set_error("sipg_stream_bound: needs sipg_compute_gl_diagonal first"); return SIPG_E_ARG; }
    const size_t bytes = size_t(op->ndofs) * (op->dtype == SIPG_F64 ? 8 : 4);
    if (ranges_overlap(x, y, bytes) || ranges_overlap(x, z, bytes) || ranges_overlap(y, z, bytes)) {
        set_error("sipg_stream_bound: x, y and z must not overlap");
        return SIPG_E_ARG;
    }
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(z)) % 16) {
        set_error("sipg_stream_bound: x, y and z must be 16-byte aligned");
        return SIPG_E_ARG;
    }
    return launch_stream_bound(op, x, y, z, static_cast<hipStream_t>(stream));
}

int sipg_basis_change(const sipg_op* op, int mode, const void* in, void* out, void* stream) {
    if (!op || !in || !out) { set_error("sipg_basis_change: null argument"); return SIPG_E_ARG; }
    if (mode < SIPG_BC_T || mode > SIPG_BC_FDM) { set_error("sipg_basis_change: bad mode"); return SIPG_E_ARG; }
    if (mode == SIPG_BC_PJACOBI && !op->gl_inv_diag) {
        set_error("sipg_basis_change: SIPG_BC_PJACOBI needs sipg_compute_gl_diagonal first");
        return SIPG_E_ARG;
    }
    const size_t bytes = size_t(op->ndofs) * (op->dtype == SIPG_F64 ? 8 : 4);
    if (ranges_overlap(in, out, bytes)) { set_error("sipg_basis_change: in and out overlap"); return SIPG_E_ARG; }
    return launch_basis_change(op, mode, in, out, static_cast<hipStream_t>(stream));
}

int sipg_compute_gl_diagonal(sipg_op* op, void* diag_out, void* stream) {
    if (!op) { set_error("sipg_compute_gl_diagonal: null operator"); return SIPG_E_ARG; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = size_t(op->ndofs) * (op->dtype == SIPG_F64 ? 8 : 4);
    if (!op->gl_inv_diag) {
        const int rc = op->mem.alloc(&op->gl_inv_diag, bytes, "sipg_compute_gl_diagonal");
        if (rc != SIPG_OK) return rc;
        op->device_bytes += int64_t(bytes);
    }
    const int rc = launch_gl_diagonal(op, diag_out, st);
    if (rc != SIPG_OK) return rc;
    SIPG_HIP(hipStreamSynchronize(st));
    return SIPG_OK;
}

int sipg_cg_solve(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                  sipg_solve_info* info, void* stream) {
    if (!op || !b || !x || !info) { set_error("sipg_cg_solve: null argument"); return SIPG_E_ARG; }
    if (op->dtype != SIPG_F64) { set_error("sipg_cg_solve: needs an SIPG_F64 operator"); return SIPG_E_ARG; }
    if (is_inner_slab(op)) { set_error("sipg_cg_solve: not for a slab with neighbours"); return SIPG_E_ARG; }
    if (!(rel_tol > 0.0) || max_iter < 0) { set_error("sipg_cg_solve: rel_tol must be > 0, max_iter >= 0"); return SIPG_E_ARG; }
    if (ranges_overlap(b, x, size_t(op->ndofs) * 8)) { set_error("sipg_cg_solve: b and x overlap"); return SIPG_E_ARG; }
    std::memset(info, 0, sizeof(*info));
    return cg_solve_device(op, b, x, rel_tol, max_iter, info, static_cast<hipStream_t>(stream));
}

int sipg_cg_solve_static(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                         sipg_solve_info* info, void* stream) {
    if (!op || !b || !x || !info) { set_error("sipg_cg_solve_static: null argument"); return SIPG_E_ARG; }
    if (op->dtype != SIPG_F64) { set_error("sipg_cg_solve_static: needs an SIPG_F64 operator"); return SIPG_E_ARG; }
    if (is_inner_slab(op)) { set_error("sipg_cg_solve_static: not for a slab with neighbours"); return SIPG_E_ARG; }
    if (!(rel_tol > 0.0) || max_iter < 0) {
        set_error("sipg_cg_solve_static: rel_tol must be > 0, max_iter >= 0");
        return SIPG_E_ARG;
    }
    if (ranges_overlap(b, x, size_t(op->ndofs) * 8)) { set_error("sipg_cg_solve_static: b and x overlap"); return SIPG_E_ARG; }
    std::memset(info, 0, sizeof(*info));
    return cg_solve_static(op, b, x, rel_tol, max_iter, info, static_cast<hipStream_t>(stream));
}

int64_t sipg_cg_static_max_dofs(void) { return cg_static_max_dofs(); }

}  // extern "C"
