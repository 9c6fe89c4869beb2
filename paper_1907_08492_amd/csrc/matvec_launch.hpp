// Launchers of the matrix-free product for one degree (included by the
// per-degree translation units matvec_n<N>.hip).
#pragma once

#include <mutex>

#include "matvec.hpp"
#include "setup.hpp"

namespace sipg {

template <int N, int BASIS, typename T, int GEOM, int KIND, typename K>
static int set_lds_limit(K kernel) {
    // once per kernel (the request loop's workers launch concurrently)
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [&] {
        err = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(matvec_lds_bytes<N, T>()));
    });
    if (err != hipSuccess) return hip_fail(err, "hipFuncSetAttribute(dynamic LDS)");
    return SIPG_OK;
}

// nv right-hand sides stored one after another (op->ndofs apart): grid row
// blockIdx.y = v works on right-hand side v.
template <int N, int BASIS, typename T, int GEOM>
static int launch_one(const sipg_op* op, const void* x, void* y, hipStream_t st, Ghosts g, int nv) {
    auto kern = &sipg_matvec_kernel<N, BASIS, T, GEOM>;
    if (int rc = set_lds_limit<N, BASIS, T, GEOM, 0>(kern)) return rc;
    const unsigned nblk = unsigned((op->ncells + cells_per_block(N) - 1) / cells_per_block(N));
    MatvecParams<T> p = matvec_params<T>(op, x, y);
    p.ghost_lo = static_cast<const T*>(g.lo);
    p.ghost_hi = static_cast<const T*>(g.hi);
    kern<<<dim3(nblk, unsigned(nv)), threads_per_block(N), matvec_lds_bytes<N, T>(), st>>>(p);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

// y = A x and z = P^-1 y (eq. (jacobi)) in one pass; op->gl_inv_diag is set.
template <int N, int BASIS, typename T, int GEOM>
static int launch_one_pjacobi(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st, Ghosts g) {
    auto kern = &sipg_matvec_pjacobi_kernel<N, BASIS, T, GEOM>;
    if (int rc = set_lds_limit<N, BASIS, T, GEOM, 2>(kern)) return rc;
    const unsigned nblk = unsigned((op->ncells + cells_per_block(N) - 1) / cells_per_block(N));
    MatvecParams<T> p = matvec_params<T>(op, x, y);
    p.ghost_lo = static_cast<const T*>(g.lo);
    p.ghost_hi = static_cast<const T*>(g.hi);
    p.dinv = static_cast<const T*>(op->gl_inv_diag);
    p.z = static_cast<T*>(z);
    kern<<<nblk, threads_per_block(N), matvec_lds_bytes<N, T>(), st>>>(p);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

// One Chebyshev smoothing step fused into the product (Hermite-like basis):
// uo = u + sigma (u - uo) + theta P^-1 (b - A u), P^-1 by `mode`
// (SIPG_BC_PJACOBI with op->gl_inv_diag, SIPG_BC_FDM with op->fdm_cell);
// nv right-hand sides as in launch_one.
template <int N, typename T, int GEOM>
static int launch_one_cheb(const sipg_op* op, int mode, const void* b, const void* u, void* uo, double sigma,
                           double theta, hipStream_t st, int nv) {
    MatvecParams<T> p = matvec_params<T>(op, u, uo);   // y is not written by this epilogue
    p.b = static_cast<const T*>(b);
    p.uo = static_cast<T*>(uo);
    p.sigma = sigma;
    p.theta = theta;
    const dim3 grid = dim3(unsigned((op->ncells + cells_per_block(N) - 1) / cells_per_block(N)), unsigned(nv));
    if (mode == SIPG_BC_PJACOBI) {
        auto kern = &sipg_matvec_cheb_kernel<N, 0, T, GEOM, EPI_CHEB_PJ>;
        if (int rc = set_lds_limit<N, 0, T, GEOM, 3>(kern)) return rc;
        p.dinv = static_cast<const T*>(op->gl_inv_diag);
        kern<<<grid, threads_per_block(N), matvec_lds_bytes<N, T>(), st>>>(p);
    } else {
        auto kern = &sipg_matvec_cheb_kernel<N, 0, T, GEOM, EPI_CHEB_FDM>;
        if (int rc = set_lds_limit<N, 0, T, GEOM, 4>(kern)) return rc;
        p.dinv = static_cast<const T*>(op->fdm_cell);
        kern<<<grid, threads_per_block(N), matvec_lds_bytes<N, T>(), st>>>(p);
    }
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

template <int N, int BASIS, typename T, int GEOM>
static int launch_group(const BatchGroup& g, hipStream_t st) {
    auto kern = &sipg_matvec_batched_kernel<N, BASIS, T, GEOM>;
    if (int rc = set_lds_limit<N, BASIS, T, GEOM, 1>(kern)) return rc;
    kern<<<unsigned(g.nblocks), threads_per_block(N), matvec_lds_bytes<N, T>(), st>>>(
        static_cast<const MatvecParams<T>*>(g.params), g.blk_op, g.blk_first);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

// Calls launch<N, BASIS, T, GEOM>() for the run-time (basis, dtype, kernel
// geometry variant, matvec_geom).
template <int N, typename F>
static int dispatch(int basis, int dtype, int geom, F&& launch) {
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using GC = std::integral_constant<int, GEOM_CELL>;
    using GQ = std::integral_constant<int, GEOM_QPOINT>;
    using GD = std::integral_constant<int, GEOM_CELL_DIAG>;
    auto by_geom = [&](auto b, auto t) {
        if (geom == GEOM_CELL) return launch(b, t, GC{});
        if (geom == GEOM_CELL_DIAG) return launch(b, t, GD{});
        return launch(b, t, GQ{});
    };
    auto by_basis = [&](auto t) {
        if (basis == SIPG_BASIS_HERMITE_LIKE) return by_geom(I0{}, t);
        if (basis == SIPG_BASIS_NODAL_GL) return by_geom(I1{}, t);
        return by_geom(I2{}, t);
    };
    return dtype == SIPG_F64 ? by_basis(double{}) : by_basis(float{});
}

// The same for the Hermite-like basis only: launch<T, GEOM>().
template <int N, typename F>
static int dispatch_hl(int dtype, int geom, F&& launch) {
    using GC = std::integral_constant<int, GEOM_CELL>;
    using GQ = std::integral_constant<int, GEOM_QPOINT>;
    using GD = std::integral_constant<int, GEOM_CELL_DIAG>;
    auto by_geom = [&](auto t) {
        if (geom == GEOM_CELL) return launch(t, GC{});
        if (geom == GEOM_CELL_DIAG) return launch(t, GD{});
        return launch(t, GQ{});
    };
    return dtype == SIPG_F64 ? by_geom(double{}) : by_geom(float{});
}

}  // namespace sipg

// Defines the four per-degree entry points of setup.hpp for degree NV - 1.
#define SIPG_MATVEC_DEGREE(NV)                                                                          \
    namespace sipg {                                                                                    \
    template <>                                                                                         \
    int launch_matvec_n<NV>(const sipg_op* op, const void* x, void* y, hipStream_t st, Ghosts gh, int nv) { \
        return dispatch<NV>(op->basis, op->dtype, matvec_geom(op), [&](auto b, auto t, auto g) {        \
            return launch_one<NV, decltype(b)::value, decltype(t), decltype(g)::value>(op, x, y, st, gh, nv); \
        });                                                                                             \
    }                                                                                                   \
    template <>                                                                                         \
    int launch_matvec_pjacobi_n<NV>(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st,  \
                                    Ghosts gh) {                                                        \
        return dispatch<NV>(op->basis, op->dtype, matvec_geom(op), [&](auto b, auto t, auto g) {        \
            return launch_one_pjacobi<NV, decltype(b)::value, decltype(t), decltype(g)::value>(op, x, y, z, \
                                                                                                 st, gh); \
        });                                                                                             \
    }                                                                                                   \
    template <>                                                                                         \
    int launch_matvec_cheb_n<NV>(const sipg_op* op, int mode, const void* b, const void* u, void* uo,   \
                                 double sigma, double theta, hipStream_t st, int nv) {                  \
        return dispatch_hl<NV>(op->dtype, matvec_geom(op), [&](auto t, auto g) {                        \
            return launch_one_cheb<NV, decltype(t), decltype(g)::value>(op, mode, b, u, uo, sigma, theta, st, nv); \
        });                                                                                             \
    }                                                                                                   \
    template <>                                                                                         \
    int launch_matvec_batched_n<NV>(const BatchGroup& grp, hipStream_t st) {                            \
        return dispatch<NV>(grp.basis, grp.dtype, grp.geom, [&](auto b, auto t, auto g) {               \
            return launch_group<NV, decltype(b)::value, decltype(t), decltype(g)::value>(grp, st);      \
        });                                                                                             \
    }                                                                                                   \
    }
