// Geometric multigrid solver of Section 6: conjugate gradient in FP64
// preconditioned by one V-cycle per iteration.  The V-cycle runs in FP32
// (mixed precision, Section 6.2) or FP64; on every level it smooths with a
// Chebyshev iteration (eq. chebyshev, degree 5 by default) around the
// preconditioner of eq. (jacobi): point Jacobi in the nodal Gauss-Lobatto
// basis reached by the tensor-product basis change.  The smoothing range is
// [0.06, 1.2] times the largest eigenvalue of P^-1 A estimated by 15 Lanczos
// steps from the vector [-5.5, -4.5, ..., 5.5, -5.5, ...]; the coarsest level
// is solved by a Chebyshev iteration whose degree guarantees a residual
// reduction of 1e5 by the a-priori Chebyshev bound.  Levels coarsen the brick
// by two in every direction while all cell counts are even; the transfer is
// the exact embedding of the coarse space (the coarse map differs from the
// fine one by an affine map per child).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "basis1d.hpp"
#include "setup.hpp"
#include "sipg_common.hpp"
#include "vecops.hpp"

namespace sipg {

// Largest and smallest eigenvalue of the symmetric tridiagonal matrix
// (diag d, off-diagonal e) by Sturm-sequence bisection.
static void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double& lmin, double& lmax) {
    const int n = int(d.size());
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    auto count_below = [&](double x) {   // eigenvalues < x
        int c = 0;
        double q = d[0] - x;
        if (q < 0) ++c;
        for (int i = 1; i < n; ++i) {
            const double qq = q != 0.0 ? q : 1e-300;
            q = d[i] - x - e[i - 1] * e[i - 1] / qq;
            if (q < 0) ++c;
        }
        return c;
    };
    auto kth = [&](int k) {   // k-th smallest (0-based)
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (a + b);
            if (count_below(m) > k) b = m; else a = m;
        }
        return 0.5 * (a + b);
    };
    lmin = kth(0);
    lmax = kth(n - 1);
}

// A device array of the solver, from the solver's allocator (which outlives
// every buffer of the solver).
template <typename T>
struct DevBuf {
    T* p = nullptr;
    const DevAlloc* a = nullptr;
    ~DevBuf() { if (p) a->release(p); }
    int alloc(int64_t n, const DevAlloc& from) {
        a = &from;
        void* q = nullptr;
        const int rc = from.alloc(&q, sizeof(T) * size_t(std::max<int64_t>(n, 1)), "multigrid");
        p = static_cast<T*>(q);
        return rc;
    }
};

template <typename T>
struct Level {
    sipg_op* op = nullptr;
    int nc[3] = {0, 0, 0};
    int np = 0;                         // degree + 1
    int next = 0;                       // transfer to level l+1: 0 mesh coarsening, 1 lower degree
    int64_t n = 0;                      // unknowns
    DevBuf<T> b, u, uo, r, z;
    DevBuf<T> emb;                      // h: child embedding M_0, M_1; p: E then E^T
    double lmin = 0.0, lmax = 0.0;
    int steps = 0;                      // Lanczos steps of its eigenvalue estimate
    std::vector<double> key;            // what defines the level operator (eigenvalue cache)
    std::vector<double> sigma, theta;   // Chebyshev coefficients per step
    bool direct = false;                // coarsest level solved by its dense inverse
    DevBuf<T> ainv;                     // that inverse (n x n)
    // b, u, uo, r of several right-hand sides stored one after another (n
    // apart), set for the duration of sipg_mg_solve_many (its workspace)
    T *mb = nullptr, *mu = nullptr, *muo = nullptr, *mr = nullptr;
    int64_t ncells() const { return int64_t(nc[0]) * nc[1] * nc[2]; }
    ~Level() { if (op) sipg_destroy(op); }
};

// Level sequence of the hierarchy: first the degree is lowered on the fine
// mesh (p_coarsening 1: k -> max(1, k/2); 2: k -> k-1), then the brick is
// coarsened while at least min_coarse_cells coarse cells remain (at most 16
// levels): by two while every cell count is even, or with graded_coarsening
// from n to ceil(n/2) cells in every direction with n > 1 (fine cells paired
// from lo on, the last one alone for odd n: a graded brick of twice the
// regular width).  With coarse_direct_max_dofs, coarsening stops at the
// first level of at most that many unknowns.
struct LevelSpec {
    int nc[3];
    double width[3];   // sipg_mesh.width of the level (all zero: uniform brick)
    int degree;
    int next;
};
std::vector<LevelSpec> mg_level_sequence(const sipg_mesh& mesh, int degree, const sipg_mg_opts& o) {
    std::vector<LevelSpec> seq;
    LevelSpec cur{{mesh.n[0], mesh.n[1], mesh.n[2]}, {mesh.width[0], mesh.width[1], mesh.width[2]}, degree, 0};
    for (;;) {
        seq.push_back(cur);
        if (seq.size() >= 16) break;
        if (o.p_coarsening != 0 && cur.degree > 1) {
            seq.back().next = 1;
            cur.degree = o.p_coarsening == 1 ? std::max(1, cur.degree / 2) : cur.degree - 1;
            continue;
        }
        const int64_t np = cur.degree + 1;
        if (o.coarse_direct_max_dofs > 0 &&
            int64_t(cur.nc[0]) * cur.nc[1] * cur.nc[2] * np * np * np <= o.coarse_direct_max_dofs)
            break;
        const bool even = cur.nc[0] % 2 == 0 && cur.nc[1] % 2 == 0 && cur.nc[2] % 2 == 0;
        const bool uniform = cur.width[0] == 0.0 && cur.width[1] == 0.0 && cur.width[2] == 0.0;
        int nn[3];
        if (o.graded_coarsening) {
            for (int d = 0; d < 3; ++d) nn[d] = (cur.nc[d] + 1) / 2;
        } else {
            if (!even) break;
            for (int d = 0; d < 3; ++d) nn[d] = cur.nc[d] / 2;
        }
        const int64_t cells = int64_t(cur.nc[0]) * cur.nc[1] * cur.nc[2];
        if (cells == 1 || int64_t(nn[0]) * nn[1] * nn[2] < o.min_coarse_cells) break;
        seq.back().next = 0;
        // an even uniform brick coarsens to a uniform one (the paper's case);
        // otherwise every regular width doubles where cells are paired
        if (!(uniform && even)) {
            for (int d = 0; d < 3; ++d) {
                const double w = uniform ? (mesh.hi[d] - mesh.lo[d]) / cur.nc[d] : cur.width[d];
                cur.width[d] = cur.nc[d] > 1 ? 2.0 * w : w;
            }
        }
        for (int d = 0; d < 3; ++d) cur.nc[d] = nn[d];
    }
    return seq;
}

// Regular and last cell widths of a level in every direction.
static void level_widths(const sipg_mesh& mesh, const LevelSpec& sp, double w[3], double last[3]) {
    const bool uniform = sp.width[0] == 0.0 && sp.width[1] == 0.0 && sp.width[2] == 0.0;
    for (int d = 0; d < 3; ++d) {
        w[d] = uniform ? (mesh.hi[d] - mesh.lo[d]) / sp.nc[d] : sp.width[d];
        last[d] = uniform ? w[d] : mesh.hi[d] - mesh.lo[d] - (sp.nc[d] - 1) * sp.width[d];
    }
}

// Inverse of the symmetric positive definite n x n matrix a (row major), in
// place, through its Cholesky factor a = L L^T; false when a is not positive
// definite.
static bool spd_inverse(int n, std::vector<double>& a) {
    for (int j = 0; j < n; ++j) {
        double d = a[size_t(j) * n + j];
        for (int k = 0; k < j; ++k) d -= a[size_t(j) * n + k] * a[size_t(j) * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        d = std::sqrt(d);
        a[size_t(j) * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = a[size_t(i) * n + j];
            for (int k = 0; k < j; ++k) s -= a[size_t(i) * n + k] * a[size_t(j) * n + k];
            a[size_t(i) * n + j] = s / d;
        }
    }
    std::vector<double> inv(size_t(n) * n), y(n);
    for (int c = 0; c < n; ++c) {
        // L y = e_c (y_i = 0 for i < c), then L^T x = y
        for (int i = 0; i < c; ++i) y[i] = 0.0;
        for (int i = c; i < n; ++i) {
            double s = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= a[size_t(i) * n + k] * y[k];
            y[i] = s / a[size_t(i) * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= a[size_t(k) * n + i] * y[k];
            y[i] = s / a[size_t(i) * n + i];
        }
        for (int i = 0; i < n; ++i) inv[size_t(i) * n + c] = y[i];
    }
    a.swap(inv);
    return true;
}

// Lanczos steps are bounded so that their coefficients fit the scratch.
constexpr int kMaxLanczos = 512;
// Right-hand sides of one sipg_mg_solve_many call, at most.
constexpr int kMaxRhs = kMaxSolveRhs;

struct Scratch {
    DevBuf<double> partial, scal, coef;
    double* host = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};   // residual copies of the lagged stopping test
    ~Scratch() {
        if (host) (void)hipHostFree(host);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    int init(const DevAlloc& mem) {
        int rc;
        if ((rc = partial.alloc(kVecPartials, mem)) != SIPG_OK) return rc;
        if ((rc = scal.alloc(8 * kMaxRhs, mem)) != SIPG_OK) return rc;
        if ((rc = coef.alloc(2 * kMaxLanczos, mem)) != SIPG_OK) return rc;
        SIPG_HIP(hipHostMalloc(&host, sizeof(double) * (8 + 6 * kMaxRhs), hipHostMallocDefault));
        for (hipEvent_t& e : ev) SIPG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return SIPG_OK;
    }
    // scal[slot] = a . b on the device (no host synchronisation)
    template <typename T>
    int dot_dev(const T* a, const T* b, int64_t n, int slot, hipStream_t st) {
        return vec_dot_async<T>(a, b, partial.p, scal.p + slot, n, st);
    }
};

// Chebyshev coefficients (Saad, Chebyshev acceleration, written in the
// three-term form of eq. chebyshev) for eigenvalues in [a, b], m steps.
static void chebyshev_coefficients(double a, double b, int m, std::vector<double>& sig, std::vector<double>& th) {
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
    const double s1 = theta / delta;
    sig.assign(m, 0.0);
    th.assign(m, 0.0);
    double rho_old = 1.0 / s1;
    th[0] = 1.0 / theta;
    for (int j = 1; j < m; ++j) {
        const double rho = 1.0 / (2.0 * s1 - rho_old);
        sig[j] = rho * rho_old;
        th[j] = 2.0 * rho / delta;
        rho_old = rho;
    }
}

// Byte sizes of the pieces of a workspace, rounded to 256 bytes.
static inline int64_t many_align(int64_t bytes) { return (bytes + 255) / 256 * 256; }

template <typename T>
struct Hierarchy {
    std::vector<std::unique_ptr<Level<T>>> lv;
    int smooth_steps = 5;
    int coarse_steps = 1;
    int pmode = SIPG_BC_PJACOBI;   // P^-1 of the smoother: SIPG_BC_PJACOBI or SIPG_BC_FDM
    bool fused = true;             // Chebyshev steps fused into the product (Hermite-like levels)
    int lanczos_start = 0;         // sipg_mg_opts.lanczos_start

    // Level vectors b, u, uo, r: the level's own (nv = 1), or those of nv
    // right-hand sides stored one after another (sipg_mg_solve_many).
    T*& vec_u(int l, int nv) { return nv > 1 ? lv[l]->mu : lv[l]->u.p; }
    T*& vec_uo(int l, int nv) { return nv > 1 ? lv[l]->muo : lv[l]->uo.p; }
    T* vec_b(int l, int nv) { return nv > 1 ? lv[l]->mb : lv[l]->b.p; }
    T* vec_r(int l, int nv) { return nv > 1 ? lv[l]->mr : lv[l]->r.p; }

    // u = S^m(b; u) on level l (u = 0 on entry when zero_init), for nv
    // right-hand sides at once (stored one after another, n apart).
    int smooth(int l, bool zero_init, int steps, const std::vector<double>& sig, const std::vector<double>& th,
               hipStream_t st, int nv = 1) {
        Level<T>& L = *lv[l];
        T*& u = vec_u(l, nv);
        T*& uo = vec_uo(l, nv);
        T* b = vec_b(l, nv);
        T* r = vec_r(l, nv);
        int rc;
        for (int j = 0; j < steps; ++j) {
            if (j == 0 && zero_init) {
                // u_0 = 0 (written into uo for the next step by the same
                // launch), u_1 = theta_0 P^-1 b
                if ((rc = launch_precond_cheb(L.op, pmode, b, nullptr, nullptr, u, 0.0, th[0], st,
                                              steps > 1 ? uo : nullptr, nv)) != SIPG_OK)
                    return rc;
                continue;
            }
            // u_{j+1} = u_j + sigma_j (u_j - u_{j-1}) + theta_j P^-1 (b - A u_j)
            // into uo, then swap: one launch (product, residual, preconditioner
            // and update fused) on Hermite-like levels, else the product and
            // one merged pass
            const double sj = j == 0 ? 0.0 : sig[j];
            if (fused && L.op->basis == SIPG_BASIS_HERMITE_LIKE) {
                if ((rc = launch_matvec_cheb(L.op, pmode, b, u, uo, sj, th[j], st, nv)) != SIPG_OK) return rc;
            } else {
                if ((rc = launch_matvec(L.op, u, r, st, {}, nv)) != SIPG_OK) return rc;
                if ((rc = launch_precond_cheb(L.op, pmode, b, r, u, uo, sj, th[j], st, nullptr, nv)) != SIPG_OK)
                    return rc;
            }
            std::swap(u, uo);
        }
        return SIPG_OK;
    }

    // u_l = V-cycle(b_l) with zero initial guess (nv right-hand sides).
    int vcycle(int l, hipStream_t st, int nv = 1) {
        Level<T>& L = *lv[l];
        int rc;
        if (l + 1 == int(lv.size()))
            return L.direct ? vec_dense_mv<T>(L.ainv.p, vec_b(l, nv), vec_u(l, nv), int(L.n), st, nv)
                            : smooth(l, true, coarse_steps, L.sigma, L.theta, st, nv);
        if ((rc = smooth(l, true, smooth_steps, L.sigma, L.theta, st, nv)) != SIPG_OK) return rc;
        T* r = vec_r(l, nv);
        if ((rc = launch_matvec(L.op, vec_u(l, nv), r, st, {}, nv)) != SIPG_OK) return rc;
        if ((rc = vec_sub<T>(vec_b(l, nv), r, r, L.n * nv, st)) != SIPG_OK) return rc;
        if ((rc = restrict_to(l, r, vec_b(l + 1, nv), st, nv)) != SIPG_OK) return rc;
        if ((rc = vcycle(l + 1, st, nv)) != SIPG_OK) return rc;
        if ((rc = prolongate_add(l, vec_u(l + 1, nv), vec_u(l, nv), st, nv)) != SIPG_OK) return rc;
        return smooth(l, false, smooth_steps, L.sigma, L.theta, st, nv);
    }

    // coarse = R fine  from level l to level l+1
    int restrict_to(int l, const T* fine, T* coarse, hipStream_t st, int nv = 1) {
        Level<T>& L = *lv[l];
        const Level<T>& C = *lv[l + 1];
        if (L.next == 0) return transfer_restrict<T>(L.np, L.nc, fine, coarse, L.emb.p, st, nv);
        return transfer_degree<T>(L.np, C.np, L.ncells(), true, fine, coarse, L.emb.p, L.emb.p + L.np * C.np, st, nv);
    }
    // fine += P coarse  from level l+1 to level l
    int prolongate_add(int l, const T* coarse, T* fine, hipStream_t st, int nv = 1) {
        Level<T>& L = *lv[l];
        const Level<T>& C = *lv[l + 1];
        if (L.next == 0) return transfer_prolongate_add<T>(L.np, L.nc, coarse, fine, L.emb.p, st, nv);
        return transfer_degree<T>(L.np, C.np, L.ncells(), false, coarse, fine, L.emb.p, L.emb.p + L.np * C.np, st,
                                  nv);
    }

    // Device bytes of the level vectors of nv right-hand sides.
    int64_t many_bytes(int nv) const {
        int64_t b = 0;
        for (const auto& L : lv) b += 4 * many_align(int64_t(sizeof(T)) * L->n * nv);
        return b;
    }
    // Points the levels' multi-right-hand-side vectors into `ws` (many_bytes(nv)
    // bytes), or back to null.
    void set_many(char* ws, int nv) {
        for (auto& L : lv) {
            const int64_t sz = many_align(int64_t(sizeof(T)) * L->n * nv);
            T** v[4] = {&L->mb, &L->mu, &L->muo, &L->mr};
            for (T** q : v) {
                *q = ws ? reinterpret_cast<T*>(ws) : nullptr;
                if (ws) ws += sz;
            }
        }
    }

    // Extreme eigenvalues of P^-1 A on level l from `steps` conjugate gradient
    // (Lanczos) steps started from the vector [-5.5, -4.5, ..., 5.5, ...].
    // The CG coefficients stay on the device (scalar slots 0: r.z, 1: p.Ap,
    // 2: new r.z) and are read once at the end.
    int lanczos(int l, int steps, Scratch& sc, hipStream_t st) {
        Level<T>& L = *lv[l];
        int rc;
        if (lanczos_start == 0) {
            if ((rc = vec_sawtooth<T>(L.r.p, L.n, st)) != SIPG_OK) return rc;
        } else {
            // r = A u for the function u whose nodal Gauss-Lobatto values are
            // the sawtooth: the same start in every basis (u's coefficients
            // in the level's basis are (T^T)^{x3} of the values)
            if ((rc = vec_sawtooth<T>(L.z.p, L.n, st)) != SIPG_OK) return rc;
            if ((rc = launch_basis_change(L.op, SIPG_BC_TT, L.z.p, L.uo.p, st)) != SIPG_OK) return rc;
            if ((rc = launch_matvec(L.op, L.uo.p, L.r.p, st)) != SIPG_OK) return rc;
        }
        steps = std::min(steps, kMaxLanczos);
        double* da = sc.coef.p;               // alpha_k
        double* db = sc.coef.p + steps;       // beta_k
        double* s_rz = sc.scal.p;
        double* s_pap = sc.scal.p + 1;
        double* s_rzn = sc.scal.p + 2;
        // x = 0, r = b; z = P^-1 r; p = z  (p in uo, Ap in b)
        if ((rc = launch_basis_change(L.op, pmode, L.r.p, L.z.p, st)) != SIPG_OK) return rc;
        SIPG_HIP(hipMemcpyAsync(L.uo.p, L.z.p, sizeof(T) * L.n, hipMemcpyDeviceToDevice, st));
        if ((rc = sc.dot_dev<T>(L.r.p, L.z.p, L.n, 0, st)) != SIPG_OK) return rc;
        for (int k = 0; k < steps; ++k) {
            if ((rc = launch_matvec(L.op, L.uo.p, L.b.p, st)) != SIPG_OK) return rc;
            if ((rc = sc.dot_dev<T>(L.uo.p, L.b.p, L.n, 1, st)) != SIPG_OK) return rc;
            if ((rc = scalar_ratio(s_rz, s_pap, da + k, st)) != SIPG_OK) return rc;          // alpha
            if ((rc = vec_axpy_dev<T>(s_rz, s_pap, -1.0, L.b.p, L.r.p, L.n, st)) != SIPG_OK) return rc;
            if ((rc = launch_basis_change(L.op, pmode, L.r.p, L.z.p, st)) != SIPG_OK) return rc;
            if ((rc = sc.dot_dev<T>(L.r.p, L.z.p, L.n, 2, st)) != SIPG_OK) return rc;
            if ((rc = scalar_ratio(s_rzn, s_rz, db + k, st)) != SIPG_OK) return rc;          // beta
            if ((rc = vec_xpby_dev<T>(L.z.p, s_rzn, s_rz, L.uo.p, L.n, st)) != SIPG_OK) return rc;
            if ((rc = scalar_ratio(s_rzn, nullptr, s_rz, st)) != SIPG_OK) return rc;
        }
        std::vector<double> ab(2 * steps);
        SIPG_HIP(hipMemcpyAsync(ab.data(), sc.coef.p, sizeof(double) * ab.size(), hipMemcpyDeviceToHost, st));
        SIPG_HIP(hipStreamSynchronize(st));
        // keep the steps before the first breakdown (zero residual or a
        // non-positive curvature)
        std::vector<double> alpha, beta;
        for (int k = 0; k < steps; ++k) {
            const double a = ab[k], bt = ab[steps + k];
            if (!(a > 0.0) || !std::isfinite(a)) break;
            alpha.push_back(a);
            beta.push_back(std::isfinite(bt) && bt >= 0.0 ? bt : 0.0);
            if (!(bt > 0.0) || !std::isfinite(bt)) break;
        }
        const int m = int(alpha.size());
        if (m == 0) { set_error("multigrid: Lanczos breakdown"); return SIPG_E_NOCONV; }
        std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
        for (int k = 0; k < m; ++k) {
            d[k] = 1.0 / alpha[k] + (k > 0 ? beta[k - 1] / alpha[k - 1] : 0.0);
            if (k + 1 < m) e[k] = std::sqrt(beta[k]) / alpha[k];
        }
        tridiag_extremes(d, e, L.lmin, L.lmax);
        return SIPG_OK;
    }
};

}  // namespace sipg

using namespace sipg;

struct sipg_mg;
namespace sipg {
sipg_op* mg_fine_operator(sipg_mg* mg);
double* mg_rhs_buffer(sipg_mg* mg);
double mg_last_rhs_norm(const sipg_mg* mg);
}  // namespace sipg

struct sipg_mg {
    DevAlloc mem;                        // provider of all device memory below (declared first:
                                         // destroyed after the buffers it provided)
    sipg_allocator user_alloc{nullptr, nullptr, nullptr};
    int precision = 0;                   // 0: FP32 V-cycle, 1: FP64 V-cycle
    sipg_op* fine64 = nullptr;           // FP64 operator of the outer iteration
    Hierarchy<float> h32;
    Hierarchy<double> h64;
    Scratch sc;
    int64_t ndofs = 0;
    DevBuf<double> wb, wr, wz, wp, wap;  // right-hand side and CG work vectors (FP64)
    double last_bnorm = 0.0;
    int64_t device_bytes = 0;            // operators, diagonals and level vectors
    int levels = 0;
    double lmax0 = 0.0, lmin_coarse = 0.0, lmax_coarse = 0.0;
    int coarse_steps = 0;
    ~sipg_mg() { if (fine64) sipg_destroy(fine64); }
};

namespace sipg {
// Device bytes of a solver for (mesh, degree) with options o: the FP64 fine
// operator and CG vectors plus, per level, metric terms, block-preconditioner
// scalars, the GL diagonal and five level vectors.
int64_t mg_estimate_bytes(const sipg_mesh& mesh, int degree, const sipg_mg_opts& o) {
    const bool deformed = mesh.deform_amp != 0.0;
    auto geo = [&](int n) -> int64_t { return (deformed ? int64_t(6 * n * n * n + 3 * 7 * n * n) : 32) + 4; };
    const int esz = o.precision == 0 ? 4 : 8;
    const int n0 = degree + 1;
    const int64_t cells0 = int64_t(mesh.n[0]) * mesh.n[1] * mesh.n[2];
    int64_t bytes = 8 * (geo(n0) * cells0 + 6 * cells0 * n0 * n0 * n0) + (int64_t(1) << 20);
    const std::vector<LevelSpec> seq = mg_level_sequence(mesh, degree, o);
    for (const LevelSpec& sp : seq) {
        const int n = sp.degree + 1;
        const int64_t cells = int64_t(sp.nc[0]) * sp.nc[1] * sp.nc[2];
        bytes += esz * (geo(n) * cells + 6 * cells * n * n * n) + 4096 * 8;
    }
    const LevelSpec& c = seq.back();
    const int64_t nc = int64_t(c.nc[0]) * c.nc[1] * c.nc[2] * (c.degree + 1) * (c.degree + 1) * (c.degree + 1);
    if (nc <= o.coarse_direct_max_dofs) bytes += esz * nc * nc;
    return bytes;
}

sipg_op* mg_fine_operator(sipg_mg* mg) { return mg->fine64; }
double* mg_rhs_buffer(sipg_mg* mg) { return mg->wb.p; }
double mg_last_rhs_norm(const sipg_mg* mg) { return mg->last_bnorm; }
}  // namespace sipg

// Eigenvalue estimates of P^-1 A per level operator, shared by every
// hierarchy of the process.  The Lanczos run is deterministic for a given
// level (mesh, degree, penalty, basis, precision, preconditioner, number of
// steps), so a level estimated before is not estimated again: a stream of
// solves sets up many hierarchies whose levels coincide.
static std::mutex g_lambda_mu;
static std::map<std::vector<double>, std::pair<double, double>> g_lambda;

static std::vector<double> level_key(const sipg_mesh& m, int degree, double penalty, int basis, int dtype,
                                     int pmode, int steps, int start) {
    std::vector<double> k = {double(m.n[0]), double(m.n[1]), double(m.n[2])};
    for (int d = 0; d < 3; ++d) { k.push_back(m.lo[d]); k.push_back(m.hi[d]); k.push_back(m.width[d]); }
    for (int i = 0; i < 9; ++i) k.push_back(m.lin[i]);
    k.insert(k.end(), {m.deform_amp, double(degree), penalty, double(basis), double(dtype), double(pmode),
                       double(steps), double(start)});
    return k;
}

template <typename T>
static int build_hierarchy(sipg_mg* mg, Hierarchy<T>& H, const sipg_mesh* mesh, int degree, double penalty,
                           int basis, const sipg_mg_opts& o, hipStream_t st) {
    const int dt = std::is_same<T, double>::value ? SIPG_F64 : SIPG_F32;
    H.smooth_steps = o.smoother_degree;
    H.pmode = o.smoother == 1 ? SIPG_BC_FDM : SIPG_BC_PJACOBI;
    H.fused = o.fused_smoother != 0;
    H.lanczos_start = o.lanczos_start;
    const std::vector<LevelSpec> seq = mg_level_sequence(*mesh, degree, o);
    int rc;
    for (size_t l = 0; l < seq.size(); ++l) {
        const LevelSpec& sp = seq[l];
        auto L = std::make_unique<Level<T>>();
        sipg_mesh m = *mesh;
        for (int d = 0; d < 3; ++d) { m.n[d] = sp.nc[d]; m.width[d] = sp.width[d]; L->nc[d] = sp.nc[d]; }
        L->np = sp.degree + 1;
        L->next = sp.next;
        {
            // the coarse solve needs both ends of the spectrum: more Lanczos
            // steps, bounded well below the level size so that the FP32
            // recurrence does not lose orthogonality into spurious extreme values
            const bool coarsest = l + 1 == seq.size();
            const int64_t nl = int64_t(sp.nc[0]) * sp.nc[1] * sp.nc[2] * L->np * L->np * L->np;
            L->steps = coarsest ? int(std::min<int64_t>(nl / 4 + 2, 120)) : o.lanczos_steps;
            L->key = level_key(m, sp.degree, penalty, basis, dt, H.pmode, L->steps, o.lanczos_start);
        }
        if ((rc = sipg_setup(&m, sp.degree, penalty, basis, dt, SIPG_GEOM_AUTO, &mg->user_alloc, st, &L->op)) != SIPG_OK)
            return rc;
        if (H.pmode == SIPG_BC_PJACOBI && (rc = sipg_compute_gl_diagonal(L->op, nullptr, st)) != SIPG_OK) return rc;
        L->n = L->op->ndofs;
        if ((rc = L->b.alloc(L->n, mg->mem)) || (rc = L->u.alloc(L->n, mg->mem)) || (rc = L->uo.alloc(L->n, mg->mem)) ||
            (rc = L->r.alloc(L->n, mg->mem)) || (rc = L->z.alloc(L->n, mg->mem)))
            return rc;
        // transfer matrices to the next level
        if (l + 1 < seq.size()) {
            std::vector<T> e;
            if (sp.next == 0) {
                // two halves, then per direction the children of the last
                // coarse cell: the last two fine cells (unequal on a graded
                // brick) or, for an odd count, the last fine cell alone
                std::vector<double> M0, M1;
                if (!child_embedding(basis, sp.degree, 0.5, M0, M1)) { set_error("multigrid: singular embedding"); return SIPG_E_ARG; }
                const int nn = L->np * L->np;
                e.assign(8 * nn, T(0));
                for (int i = 0; i < nn; ++i) { e[i] = T(M0[i]); e[nn + i] = T(M1[i]); }
                double w[3], last[3];
                level_widths(*mesh, sp, w, last);
                for (int d = 0; d < 3; ++d) {
                    T* dst = e.data() + (2 + 2 * d) * nn;
                    if (sp.nc[d] % 2 == 1) {
                        for (int i = 0; i < L->np; ++i) dst[i * L->np + i] = T(1);
                        continue;
                    }
                    if (!child_embedding(basis, sp.degree, w[d] / (w[d] + last[d]), M0, M1)) {
                        set_error("multigrid: singular embedding");
                        return SIPG_E_ARG;
                    }
                    for (int i = 0; i < nn; ++i) { dst[i] = T(M0[i]); dst[nn + i] = T(M1[i]); }
                }
            } else {
                std::vector<double> E;
                const int nf = L->np, ncd = seq[l + 1].degree + 1;
                if (!degree_embedding(basis, sp.degree, seq[l + 1].degree, E)) {
                    set_error("multigrid: singular degree embedding");
                    return SIPG_E_ARG;
                }
                e.resize(2 * nf * ncd);
                for (int i = 0; i < nf; ++i)
                    for (int j = 0; j < ncd; ++j) {
                        e[i * ncd + j] = T(E[i * ncd + j]);               // E  (nf x nc)
                        e[nf * ncd + j * nf + i] = T(E[i * ncd + j]);     // E^T (nc x nf)
                    }
            }
            if ((rc = L->emb.alloc(int64_t(e.size()), mg->mem)) != SIPG_OK) return rc;
            SIPG_HIP(hipMemcpyAsync(L->emb.p, e.data(), sizeof(T) * e.size(), hipMemcpyHostToDevice, st));
            SIPG_HIP(hipStreamSynchronize(st));
        }
        H.lv.push_back(std::move(L));
    }
    // a small coarsest level: its matrix, column by column (A e_i with the
    // FP64 operator of the level), inverted on the host
    {
        Level<T>& C = *H.lv.back();
        const LevelSpec& sp = seq.back();
        if (C.n <= o.coarse_direct_max_dofs) {
            const int n = int(C.n);
            sipg_mesh m = *mesh;
            for (int d = 0; d < 3; ++d) { m.n[d] = sp.nc[d]; m.width[d] = sp.width[d]; }
            sipg_op* op64 = nullptr;
            if ((rc = sipg_setup(&m, sp.degree, penalty, basis, SIPG_F64, SIPG_GEOM_AUTO, &mg->user_alloc, st, &op64)) != SIPG_OK)
                return rc;
            std::unique_ptr<sipg_op, int (*)(sipg_op*)> own(op64, sipg_destroy);
            // columns e_i and A e_i at a 32-byte aligned stride
            const size_t ld = (size_t(n) + 3) & ~size_t(3);
            DevBuf<double> X, Y;
            if ((rc = X.alloc(int64_t(ld) * n, mg->mem)) || (rc = Y.alloc(int64_t(ld) * n, mg->mem))) return rc;
            std::vector<double> a(ld * n, 0.0);
            for (int i = 0; i < n; ++i) a[size_t(i) * ld + i] = 1.0;
            SIPG_HIP(hipMemcpyAsync(X.p, a.data(), sizeof(double) * a.size(), hipMemcpyHostToDevice, st));
            for (int i = 0; i < n && rc == SIPG_OK; ++i)
                rc = launch_matvec(op64, X.p + size_t(i) * ld, Y.p + size_t(i) * ld, st);
            if (rc != SIPG_OK) {
                (void)hipStreamSynchronize(st);   // nothing in flight on X, Y when they go back
                return rc;
            }
            SIPG_HIP(hipMemcpyAsync(a.data(), Y.p, sizeof(double) * a.size(), hipMemcpyDeviceToHost, st));
            SIPG_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) a[size_t(i) * n + j] = a[size_t(i) * ld + j];   // close the stride
            a.resize(size_t(n) * n);
            // row i holds A e_i; A is symmetric: average out the rounding
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < i; ++j) {
                    const double s = 0.5 * (a[size_t(i) * n + j] + a[size_t(j) * n + i]);
                    a[size_t(i) * n + j] = a[size_t(j) * n + i] = s;
                }
            if (!spd_inverse(n, a)) { set_error("multigrid: coarse matrix not positive definite"); return SIPG_E_NOCONV; }
            std::vector<T> at(a.size());
            for (size_t i = 0; i < a.size(); ++i) at[i] = T(a[i]);
            if ((rc = C.ainv.alloc(int64_t(n) * n, mg->mem)) != SIPG_OK) return rc;
            SIPG_HIP(hipMemcpyAsync(C.ainv.p, at.data(), sizeof(T) * at.size(), hipMemcpyHostToDevice, st));
            SIPG_HIP(hipStreamSynchronize(st));
            C.direct = true;
        }
    }
    // eigenvalue estimates and Chebyshev coefficients
    for (size_t l = 0; l < H.lv.size(); ++l) {
        const bool coarsest = l + 1 == H.lv.size();
        Level<T>& L = *H.lv[l];
        if (coarsest && L.direct) {
            H.coarse_steps = 0;
            mg->lmin_coarse = mg->lmax_coarse = 0.0;
            mg->coarse_steps = 0;
            continue;
        }
        bool known = false;
        {
            std::lock_guard<std::mutex> g(g_lambda_mu);
            auto it = g_lambda.find(L.key);
            if (it != g_lambda.end()) { L.lmin = it->second.first; L.lmax = it->second.second; known = true; }
        }
        if (!known) {
            if ((rc = H.lanczos(int(l), L.steps, mg->sc, st)) != SIPG_OK) return rc;
            std::lock_guard<std::mutex> g(g_lambda_mu);
            g_lambda.emplace(L.key, std::make_pair(L.lmin, L.lmax));
        }
        if (!coarsest) {
            chebyshev_coefficients(o.range_lo * L.lmax, o.range_hi * L.lmax, H.smooth_steps, L.sigma, L.theta);
        } else {
            // degree with 2 c^m / (1 + c^2m) <= 1 / coarse_reduction
            const double a = 0.9 * L.lmin, b = 1.1 * L.lmax;
            const double kap = b / a, c = (std::sqrt(kap) - 1.0) / (std::sqrt(kap) + 1.0);
            int m = 1;
            while (m < 2000) {
                const double cm = std::pow(c, m);
                if (2.0 * cm / (1.0 + cm * cm) <= 1.0 / o.coarse_reduction) break;
                ++m;
            }
            H.coarse_steps = m;
            chebyshev_coefficients(a, b, m, L.sigma, L.theta);
            mg->lmin_coarse = L.lmin;
            mg->lmax_coarse = L.lmax;
            mg->coarse_steps = m;
        }
    }
    mg->lmax0 = H.lv[0]->lmax;
    mg->levels = int(H.lv.size());
    int64_t bytes = mg->fine64 ? mg->fine64->device_bytes : 0;
    for (auto& L : H.lv) bytes += L->op->device_bytes + int64_t(5 * sizeof(T)) * L->n + (L->direct ? int64_t(sizeof(T)) * L->n * L->n : 0);
    mg->device_bytes = bytes + int64_t(sizeof(double)) * (kVecPartials + 8 + 2 * kMaxLanczos + 5 * mg->ndofs);
    return SIPG_OK;
}

namespace sipg {

// z = V-cycle(r) for nv right-hand sides stored one after another (FP64 in
// and out; the hierarchy's multi-right-hand-side vectors are set).
static int mg_vcycle_many(sipg_mg* mg, const double* r, double* z, int nv, hipStream_t st) {
    int rc;
    const int64_t n = mg->ndofs * nv;
    if (mg->precision == 0) {
        auto& H = mg->h32;
        if ((rc = vec_convert<float, double>(r, H.vec_b(0, nv), n, st)) != SIPG_OK) return rc;
        if ((rc = H.vcycle(0, st, nv)) != SIPG_OK) return rc;
        return vec_convert<double, float>(H.vec_u(0, nv), z, n, st);
    }
    auto& H = mg->h64;
    SIPG_HIP(hipMemcpyAsync(H.vec_b(0, nv), r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    if ((rc = H.vcycle(0, st, nv)) != SIPG_OK) return rc;
    SIPG_HIP(hipMemcpyAsync(z, H.vec_u(0, nv), sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    return SIPG_OK;
}

// Workspace of sipg_mg_solve_many: the level vectors of nv right-hand sides,
// the FP64 vectors r, z, p, Ap of each, per-vector scalars and dot partials.
struct ManyWork {
    sipg_mg* mg = nullptr;
    char* base = nullptr;
    hipStream_t st = nullptr;
    ~ManyWork() {
        if (!base) return;
        mg->h32.set_many(nullptr, 0);
        mg->h64.set_many(nullptr, 0);
        if (mg->mem.a.alloc) {
            (void)hipStreamSynchronize(st);
            mg->mem.release(base);
        } else {
            (void)hipFreeAsync(base, st);
        }
    }
};

// Device bytes of the workspace of nv right-hand sides: of an existing solver,
// or of the solver sipg_mg_setup would build for (mesh, degree, o).
int64_t mg_many_estimate(const sipg_mesh& mesh, int degree, const sipg_mg_opts& o, int nv) {
    const int esz = o.precision == 0 ? 4 : 8;
    auto dofs = [](const int nc[3], int deg) { return int64_t(nc[0]) * nc[1] * nc[2] * (deg + 1) * (deg + 1) * (deg + 1); };
    int64_t bytes = 4 * many_align(8 * dofs(mesh.n, degree) * nv) + many_align(int64_t(sizeof(double)) * 8 * kMaxRhs) +
                    many_align(int64_t(sizeof(double)) * kVecPartials * nv);
    for (const LevelSpec& sp : mg_level_sequence(mesh, degree, o)) bytes += 4 * many_align(esz * dofs(sp.nc, sp.degree) * nv);
    return bytes;
}

int64_t mg_many_bytes(const sipg_mg* mg, int nv) {
    const int64_t vec = many_align(int64_t(sizeof(double)) * mg->ndofs * nv);
    return (mg->precision == 0 ? mg->h32.many_bytes(nv) : mg->h64.many_bytes(nv)) + 4 * vec +
           many_align(int64_t(sizeof(double)) * 8 * kMaxRhs) +
           many_align(int64_t(sizeof(double)) * kVecPartials * nv);
}

// FP64 preconditioned conjugate gradient with one V-cycle per iteration for
// nrhs right-hand sides of one hierarchy advanced in lockstep: every product,
// smoothing step, transfer, coarse solve, dot product and vector update is
// one launch for all of them.  Vector v stops (its x, r and p are no longer updated) at the first
// iteration whose residual meets its tolerance (decided on the device, so
// no vector takes an iteration beyond it); the loop ends when every vector
// has stopped.
int mg_solve_many(sipg_mg* mg, int nrhs, const double* b, double* x, double rel_tol, int max_iter,
                  sipg_solve_info* info, double* bnorm, int* conv, hipStream_t st) {
    if (!mg || !b || !x || !info) { set_error("multigrid solve: null argument"); return SIPG_E_ARG; }
    if (nrhs < 1 || nrhs > kMaxRhs) { set_error("multigrid solve: nrhs must lie in [1, 16]"); return SIPG_E_ARG; }
    if (!(rel_tol > 0.0) || max_iter < 0) {
        set_error("multigrid solve: rel_tol must be > 0, max_iter >= 0");
        return SIPG_E_ARG;
    }
    const int nv = nrhs;
    const int64_t n = mg->ndofs;
    const size_t vbytes = sizeof(double) * size_t(n) * nv;
    {
        const char *b0 = reinterpret_cast<const char*>(b), *x0 = reinterpret_cast<const char*>(x);
        if (b0 < x0 + vbytes && x0 < b0 + vbytes) { set_error("multigrid solve: b and x overlap"); return SIPG_E_ARG; }
    }
    std::memset(info, 0, sizeof(*info) * size_t(nv));
    Scratch& sc = mg->sc;
    ManyWork w;
    double *r, *z, *p, *ap, *scal, *partial;
    if (nv == 1) {
        // one right-hand side: the solver's own vectors and scalars
        r = mg->wr.p;
        z = mg->wz.p;
        p = mg->wp.p;
        ap = mg->wap.p;
        scal = sc.scal.p;
        partial = sc.partial.p;
    } else {
        w.mg = mg;
        w.st = st;
        const int64_t total = mg_many_bytes(mg, nv);
        void* q = nullptr;
        if (mg->mem.a.alloc) {
            if (int rc = mg->mem.alloc(&q, size_t(total), "sipg_mg_solve_many workspace")) return rc;
        } else if (hipMallocAsync(&q, size_t(total), st) != hipSuccess) {
            (void)hipGetLastError();
            set_error("sipg_mg_solve_many: out of device memory for the workspace");
            return SIPG_E_OOM;
        }
        w.base = static_cast<char*>(q);
        char* ws = w.base;
        if (mg->precision == 0) {
            mg->h32.set_many(ws, nv);
            ws += mg->h32.many_bytes(nv);
        } else {
            mg->h64.set_many(ws, nv);
            ws += mg->h64.many_bytes(nv);
        }
        const int64_t vec = many_align(int64_t(vbytes));
        r = reinterpret_cast<double*>(ws);
        z = reinterpret_cast<double*>(ws + vec);
        p = reinterpret_cast<double*>(ws + 2 * vec);
        ap = reinterpret_cast<double*>(ws + 3 * vec);
        ws += 4 * vec;
        scal = reinterpret_cast<double*>(ws);
        ws += many_align(int64_t(sizeof(double)) * 8 * kMaxRhs);
        partial = reinterpret_cast<double*>(ws);
    }
    // per-vector scalars (kMaxRhs apart): r.z, p.Ap, new r.z, r.r, active
    // flag (r.r and the flags adjacent: one copy to the host), b.b, target,
    // iterations
    double *s_rz = scal, *s_pap = scal + kMaxRhs, *s_rzn = scal + 2 * kMaxRhs, *s_rr = scal + 3 * kMaxRhs;
    double *s_act = scal + 4 * kMaxRhs, *s_bb = scal + 5 * kMaxRhs, *s_tgt = scal + 6 * kMaxRhs,
           *s_it = scal + 7 * kMaxRhs;
    // pinned host memory: the start's and the end's scalars (one copy each),
    // and in between two lagged slots of (r.r, active flags), kMaxRhs each
    double* hb = sc.host + 8;
    int rc;
    // ||b_v||, r = b - A x, ||r_v||, targets and active flags
    if ((rc = vec_dot_many<double>(b, b, partial, s_bb, n, nv, st)) != SIPG_OK) return rc;
    if ((rc = launch_matvec(mg->fine64, x, ap, st, {}, nv)) != SIPG_OK) return rc;
    if ((rc = vec_sub<double>(b, ap, r, n * nv, st)) != SIPG_OK) return rc;
    if ((rc = vec_dot_many<double>(r, r, partial, s_rr, n, nv, st)) != SIPG_OK) return rc;
    if ((rc = cg_start_many(s_bb, s_rr, rel_tol, s_tgt, s_act, s_it, nv, st)) != SIPG_OK) return rc;
    SIPG_HIP(hipMemcpyAsync(hb, s_rr, sizeof(double) * 3 * kMaxRhs, hipMemcpyDeviceToHost, st));   // r.r, flags, b.b
    SIPG_HIP(hipStreamSynchronize(st));
    std::vector<double> rr(hb, hb + nv), act(hb + kMaxRhs, hb + kMaxRhs + nv),
        bb(hb + 2 * kMaxRhs, hb + 2 * kMaxRhs + nv);
    std::vector<double> target(nv);
    for (int v = 0; v < nv; ++v) {
        info[v].initial_residual = std::sqrt(rr[v]);
        target[v] = rel_tol * (bb[v] > 0.0 ? std::sqrt(bb[v]) : 1.0);
    }
    auto all_stopped = [&](const double* a) {
        for (int v = 0; v < nv; ++v)
            if (a[v] != 0.0) return false;
        return true;
    };
    // The stopping test is decided on the device (the flags) and read by the
    // host with a lag: r.r and the flags of iteration it are copied to pinned
    // host memory behind its work, and before queueing iteration it + 2 the
    // host reads those of iteration it while iteration it + 1 runs, so the
    // device does not wait for the host between iterations.  Only when the
    // observed reduction rates predict that every running vector stops in
    // iteration it + 1 does the host wait for that iteration too.  Iterations
    // queued after every vector stopped change nothing (the flags gate every
    // update), so the lag costs at most device time, never the result.
    std::vector<double> rr_prev = rr;
    int it = 0;
    bool done = all_stopped(act.data());
    while (!done && it < max_iter) {
        if (it >= 2) {
            SIPG_HIP(hipEventSynchronize(sc.ev[it % 2]));
            const double* h = hb + kMaxRhs + (it % 2) * 2 * kMaxRhs;   // r.r, flags of iteration it - 2
            if (all_stopped(h + kMaxRhs)) { done = true; break; }
            bool likely = true;
            for (int v = 0; v < nv; ++v) {
                if (h[kMaxRhs + v] == 0.0) continue;
                const double rate = rr_prev[v] > 0.0 ? std::min(1.0, h[v] / rr_prev[v]) : 1.0;
                likely = likely && std::sqrt(h[v] * rate) <= 1.5 * target[v];
            }
            for (int v = 0; v < nv; ++v) rr_prev[v] = h[v];
            if (likely) {
                SIPG_HIP(hipEventSynchronize(sc.ev[(it - 1) % 2]));
                if (all_stopped(hb + kMaxRhs + ((it - 1) % 2) * 2 * kMaxRhs + kMaxRhs)) { done = true; break; }
            }
        }
        if ((rc = mg_vcycle_many(mg, r, z, nv, st)) != SIPG_OK) return rc;
        if ((rc = vec_dot_many<double>(r, z, partial, s_rzn, n, nv, st)) != SIPG_OK) return rc;
        if (it == 0) {
            SIPG_HIP(hipMemcpyAsync(p, z, vbytes, hipMemcpyDeviceToDevice, st));
        } else {
            if ((rc = vec_xpby_many<double>(z, s_rzn, s_rz, s_act, p, n, nv, st)) != SIPG_OK) return rc;
        }
        if ((rc = scalar_copy_many(s_rzn, s_act, s_rz, nv, st)) != SIPG_OK) return rc;
        if ((rc = launch_matvec(mg->fine64, p, ap, st, {}, nv)) != SIPG_OK) return rc;
        if ((rc = vec_dot_many<double>(p, ap, partial, s_pap, n, nv, st)) != SIPG_OK) return rc;
        if ((rc = vec_axpy_many<double>(s_rz, s_pap, s_act, 1.0, p, x, n, nv, st)) != SIPG_OK) return rc;
        if ((rc = vec_axpy_many<double>(s_rz, s_pap, s_act, -1.0, ap, r, n, nv, st)) != SIPG_OK) return rc;
        if ((rc = vec_dot_many<double>(r, r, partial, s_rr, n, nv, st)) != SIPG_OK) return rc;
        if ((rc = cg_mask_many(s_rr, s_tgt, s_act, s_it, nv, st)) != SIPG_OK) return rc;
        double* h = hb + kMaxRhs + (it % 2) * 2 * kMaxRhs;
        SIPG_HIP(hipMemcpyAsync(h, s_rr, sizeof(double) * 2 * kMaxRhs, hipMemcpyDeviceToHost, st));
        SIPG_HIP(hipEventRecord(sc.ev[it % 2], st));
        ++it;
    }
    // per-vector results: the true residual ||b - A x|| (into the r.z slots),
    // the residual at which each stopped, its flag and its iterations, in one
    // copy
    if ((rc = launch_matvec(mg->fine64, x, ap, st, {}, nv)) != SIPG_OK) return rc;
    if ((rc = vec_sub<double>(b, ap, r, n * nv, st)) != SIPG_OK) return rc;
    if ((rc = vec_dot_many<double>(r, r, partial, s_rzn, n, nv, st)) != SIPG_OK) return rc;
    SIPG_HIP(hipMemcpyAsync(hb, s_rzn, sizeof(double) * 6 * kMaxRhs, hipMemcpyDeviceToHost, st));
    SIPG_HIP(hipStreamSynchronize(st));
    std::vector<double> tr(hb, hb + nv), its(hb + 5 * kMaxRhs, hb + 5 * kMaxRhs + nv);
    rr.assign(hb + kMaxRhs, hb + kMaxRhs + nv);
    act.assign(hb + 2 * kMaxRhs, hb + 2 * kMaxRhs + nv);
    bool all_converged = true;
    for (int v = 0; v < nv; ++v) {
        info[v].iterations = int(its[v]);
        info[v].final_residual = std::sqrt(rr[v]);
        info[v].true_residual = std::sqrt(tr[v]);
        all_converged = all_converged && act[v] == 0.0;
        if (conv) conv[v] = act[v] == 0.0;
    }
    if (bnorm)
        for (int v = 0; v < nv; ++v) bnorm[v] = std::sqrt(bb[v]);
    if (!all_converged) {
        set_error("multigrid solve: no convergence within max_iter");
        return SIPG_E_NOCONV;
    }
    return SIPG_OK;
}

}  // namespace sipg

extern "C" {

int sipg_mg_default_opts(sipg_mg_opts* o) {
    if (!o) { set_error("sipg_mg_default_opts: null"); return SIPG_E_ARG; }
    o->smoother_degree = 5;
    o->lanczos_steps = 15;
    o->range_lo = 0.06;
    o->range_hi = 1.2;
    o->coarse_reduction = 1e5;
    o->min_coarse_cells = 1;
    o->precision = 0;
    o->smoother = 0;
    o->p_coarsening = 0;
    o->fused_smoother = 1;
    o->lanczos_start = 0;
    o->graded_coarsening = 0;
    o->coarse_direct_max_dofs = 0;
    return SIPG_OK;
}

int sipg_mg_setup(const sipg_mesh* mesh, int degree, double penalty, int basis, const sipg_mg_opts* opts,
                  const sipg_allocator* allocator, void* stream, sipg_mg** out) {
    if (!mesh || !out) { set_error("sipg_mg_setup: null argument"); return SIPG_E_ARG; }
    *out = nullptr;
    if (!allocator_valid(allocator)) { set_error("sipg_mg_setup: allocator needs both callbacks"); return SIPG_E_ARG; }
    sipg_mg_opts o;
    sipg_mg_default_opts(&o);
    if (opts) o = *opts;
    if (o.smoother_degree < 1 || o.smoother_degree > 64 || o.lanczos_steps < 2 || o.lanczos_steps > kMaxLanczos || !(o.range_lo > 0.0) ||
        !(o.range_hi > o.range_lo) || !(o.coarse_reduction > 1.0) || (o.precision != 0 && o.precision != 1) ||
        o.min_coarse_cells < 1 || (o.smoother != 0 && o.smoother != 1) || o.p_coarsening < 0 || o.p_coarsening > 2 ||
        (o.fused_smoother != 0 && o.fused_smoother != 1) || (o.lanczos_start != 0 && o.lanczos_start != 1) ||
        (o.graded_coarsening != 0 && o.graded_coarsening != 1) || o.coarse_direct_max_dofs < 0 ||
        o.coarse_direct_max_dofs > 1024) {
        set_error("sipg_mg_setup: invalid options");
        return SIPG_E_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::unique_ptr<sipg_mg> mg(new (std::nothrow) sipg_mg());
    if (!mg) { set_error("sipg_mg_setup: out of host memory"); return SIPG_E_OOM; }
    mg->mem = DevAlloc(allocator);
    if (allocator) mg->user_alloc = *allocator;
    mg->precision = o.precision;
    int rc = sipg_setup(mesh, degree, penalty, basis, SIPG_F64, SIPG_GEOM_AUTO, &mg->user_alloc, stream, &mg->fine64);
    if (rc != SIPG_OK) return rc;
    mg->ndofs = mg->fine64->ndofs;
    if ((rc = mg->sc.init(mg->mem)) != SIPG_OK) return rc;
    if ((rc = mg->wb.alloc(mg->ndofs, mg->mem)) || (rc = mg->wr.alloc(mg->ndofs, mg->mem)) ||
        (rc = mg->wz.alloc(mg->ndofs, mg->mem)) || (rc = mg->wp.alloc(mg->ndofs, mg->mem)) ||
        (rc = mg->wap.alloc(mg->ndofs, mg->mem)))
        return rc;
    rc = o.precision == 0 ? build_hierarchy<float>(mg.get(), mg->h32, mesh, degree, penalty, basis, o, st)
                          : build_hierarchy<double>(mg.get(), mg->h64, mesh, degree, penalty, basis, o, st);
    if (rc != SIPG_OK) return rc;
    SIPG_HIP(hipStreamSynchronize(st));
    *out = mg.release();
    return SIPG_OK;
}

int sipg_mg_destroy(sipg_mg* mg) {
    delete mg;
    return SIPG_OK;
}

int sipg_mg_get_info(const sipg_mg* mg, sipg_mg_info* info) {
    if (!mg || !info) { set_error("sipg_mg_get_info: null argument"); return SIPG_E_ARG; }
    info->levels = mg->levels;
    info->ndofs = mg->ndofs;
    info->precision = mg->precision;
    info->lambda_max_fine = mg->lmax0;
    info->lambda_min_coarse = mg->lmin_coarse;
    info->lambda_max_coarse = mg->lmax_coarse;
    info->coarse_steps = mg->coarse_steps;
    info->device_bytes = mg->device_bytes;
    return SIPG_OK;
}

int sipg_mg_apply_vcycle(sipg_mg* mg, const double* r, double* z, void* stream) {
    if (!mg || !r || !z) { set_error("sipg_mg_apply_vcycle: null argument"); return SIPG_E_ARG; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc;
    if (mg->precision == 0) {
        auto& L = *mg->h32.lv[0];
        if ((rc = vec_convert<float, double>(r, L.b.p, L.n, st)) != SIPG_OK) return rc;
        if ((rc = mg->h32.vcycle(0, st)) != SIPG_OK) return rc;
        return vec_convert<double, float>(L.u.p, z, L.n, st);
    }
    auto& L = *mg->h64.lv[0];
    SIPG_HIP(hipMemcpyAsync(L.b.p, r, sizeof(double) * L.n, hipMemcpyDeviceToDevice, st));
    if ((rc = mg->h64.vcycle(0, st)) != SIPG_OK) return rc;
    SIPG_HIP(hipMemcpyAsync(z, L.u.p, sizeof(double) * L.n, hipMemcpyDeviceToDevice, st));
    return SIPG_OK;
}

// FP64 preconditioned conjugate gradient with one V-cycle per iteration: the
// lockstep solve of one right-hand side, on the solver's own vectors.
int sipg_mg_solve(sipg_mg* mg, const double* b, double* x, double rel_tol, int max_iter, sipg_solve_info* info,
                  void* stream) {
    double bn = 0.0;
    const int rc = mg_solve_many(mg, 1, b, x, rel_tol, max_iter, info, &bn, nullptr, static_cast<hipStream_t>(stream));
    if (mg) mg->last_bnorm = bn;
    return rc;
}

// nrhs right-hand sides of one hierarchy solved in lockstep (see mg_solve_many).
int sipg_mg_solve_many(sipg_mg* mg, int nrhs, const double* b, double* x, double rel_tol, int max_iter,
                       sipg_solve_info* info, void* stream) {
    return mg_solve_many(mg, nrhs, b, x, rel_tol, max_iter, info, nullptr, nullptr, static_cast<hipStream_t>(stream));
}

int sipg_mg_transfer(sipg_mg* mg, int level, int mode, const void* in, void* out, void* stream) {
    if (!mg || !in || !out || level < 0 || level + 1 >= mg->levels || (mode != 0 && mode != 1)) {
        set_error("sipg_mg_transfer: bad argument (level must have a coarser level, mode 0 or 1)");
        return SIPG_E_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto run = [&](auto& H) -> int {
        using T = typename std::remove_reference<decltype(*H.lv[0]->emb.p)>::type;
        auto& L = *H.lv[level];
        if (mode == 1) return H.restrict_to(level, static_cast<const T*>(in), static_cast<T*>(out), st);
        SIPG_HIP(hipMemsetAsync(out, 0, sizeof(T) * size_t(L.n), st));
        return H.prolongate_add(level, static_cast<const T*>(in), static_cast<T*>(out), st);
    };
    return mg->precision == 0 ? run(mg->h32) : run(mg->h64);
}

int sipg_mg_level_ndofs(const sipg_mg* mg, int level, int64_t* ndofs, int32_t cells[3]) {
    if (!mg || level < 0 || level >= mg->levels) { set_error("sipg_mg_level_ndofs: bad level"); return SIPG_E_ARG; }
    auto get = [&](const auto& H) {
        const auto& L = *H.lv[level];
        if (ndofs) *ndofs = L.n;
        if (cells) for (int d = 0; d < 3; ++d) cells[d] = L.nc[d];
    };
    if (mg->precision == 0) get(mg->h32); else get(mg->h64);
    return SIPG_OK;
}

int sipg_mg_level_degree(const sipg_mg* mg, int level, int32_t* degree) {
    if (!mg || !degree || level < 0 || level >= mg->levels) { set_error("sipg_mg_level_degree: bad argument"); return SIPG_E_ARG; }
    *degree = mg->precision == 0 ? mg->h32.lv[level]->np - 1 : mg->h64.lv[level]->np - 1;
    return SIPG_OK;
}

int sipg_assemble_rhs_sines(const sipg_op* op, int nmodes, const double* amps, const int* waves, void* b,
                            void* stream) {
    if (!op || !amps || !waves || !b || nmodes < 1 || nmodes > 16) {
        set_error("sipg_assemble_rhs_sines: null argument or nmodes outside [1,16]");
        return SIPG_E_ARG;
    }
    return launch_rhs_sines(op, nmodes, amps, waves, b, static_cast<hipStream_t>(stream));
}

}  // extern "C"
