// Cell-wise tensor-product basis change and the preconditioners of the form
// of eq. (jacobi), Sections 6.3 and 6.4:  out = (M3 x M2 x M1) in  with the
// same 1D matrix M in every direction, or  (T^T)^{x3} P_d^-1 T^{x3} in  with
// P_d the Gauss-Lobatto point-Jacobi diagonal (T = E^-1) or the diagonal of
// the fast diagonalization (T = Z^T, generalized eigenvectors of the 1D
// SIPG and mass matrices).  One thread per pencil, sweeps through LDS,
// coalesced loads and stores of whole cells.
#include "sipg_common.hpp"
#include "sumfac.hpp"
#include "setup.hpp"

namespace sipg {

template <int N>
struct BcShape {
    static constexpr int RS = (N % 2 == 0) ? N + 1 : N;
    static constexpr int CS = RS * N * N;
    static constexpr int CPB = cells_per_block(N);
    static constexpr int NT = threads_per_block(N);
    __device__ static constexpr int idx(int i1, int i2, int i3) { return i1 + RS * (i2 + N * i3); }
};

// MODE: 0 = apply M (table offset moff) in all directions; 1 = P^-1 with
// T (table TL.T), the inverse diagonal inv_diag (one value per unknown),
// then T^T (table TL.TT); 2 = block preconditioner of Section 6.4 with Z^T
// (TL.FZP, parity-split), 1 / (vol (lambda_i/h_1^2 + lambda_j/h_2^2 +
// lambda_k/h_3^2)) from the eigenvalues TL.FLAM and the four cell scalars in
// inv_diag, then Z.
//
// MERGE (modes 1 and 2 only): one step of the Chebyshev iteration of eq.
// (chebyshev) in the same pass (the "merged" arrangement of Section 6): the
// input is the residual b - A u formed while loading (au = A u; au null:
// r = b), and the output u_old is overwritten by
//     u + sigma (u - u_old) + theta P^-1 r
// (u null: u = 0; sigma = 0: u_old is not read).
template <typename T>
struct BcMerge {
    const T* au;
    const T* u;
    T sigma, theta;
    T* zero;   // when set, zeroed at the positions written (the next step's u_old)
};

template <int N, typename T, int MODE, bool MERGE>
__global__ void __launch_bounds__(BcShape<N>::NT)
basis_change_kernel(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ tab,
                    int moff, const T* __restrict__ inv_diag, int ncells, BcMerge<T> mg) {
    using Sh = BcShape<N>;
    constexpr int N2 = N * N, N3 = N2 * N, CPB = Sh::CPB, NT = Sh::NT, CS = Sh::CS;
    constexpr TableLayout TL(N);
    static_assert(!MERGE || MODE != 0, "the merged step needs a preconditioner mode");
    __shared__ T lds[CPB * CS];
    const int tid = threadIdx.x;
    const int cell0 = blockIdx.x * CPB;
    if constexpr (MERGE) {
        // several right-hand sides stored one after another: blockIdx.y
        // picks one (the preconditioner's data are shared)
        const size_t voff = size_t(blockIdx.y) * size_t(ncells) * N3;
        in += voff;
        out += voff;
        if (mg.au) mg.au += voff;
        if (mg.u) mg.u += voff;
        if (mg.zero) mg.zero += voff;
    }
    const int ncb = min(CPB, ncells - cell0);
    const T* __restrict__ src = in + size_t(cell0) * N3;
    // all loads of the workgroup's input tile issued back to back
    constexpr int XPER = (CPB * N3 + NT - 1) / NT;
    T xv[XPER];
#pragma unroll
    for (int j = 0; j < XPER; ++j) {
        const int e = tid + j * NT;
        xv[j] = e < ncb * N3 ? src[e] : T(0);
    }
    if constexpr (MERGE) {
        if (mg.au) {
            const T* __restrict__ asrc = mg.au + size_t(cell0) * N3;
#pragma unroll
            for (int j = 0; j < XPER; ++j) {
                const int e = tid + j * NT;
                if (e < ncb * N3) xv[j] -= asrc[e];
            }
        }
    }
    const int c = tid / N2, t = tid % N2, ta = t % N, tb = t / N;
    const bool act = c < ncb;
    // the block preconditioner's four cell scalars, loaded with the tile
    T cs[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (MODE == 2) {
        if (act) {
#pragma unroll
            for (int m = 0; m < 4; ++m) cs[m] = inv_diag[size_t(cell0 + c) * 4 + m];
        }
    }
#pragma unroll
    for (int j = 0; j < XPER; ++j) {
        const int e = tid + j * NT;
        if (e < ncb * N3) {
            const int cc = e / N3, i = e % N3;
            lds[cc * CS + Sh::idx(i % N, (i / N) % N, i / N2)] = xv[j];
        }
    }
    __syncthreads();
    T* A = lds + (act ? c : 0) * CS;
    const T* M = tab + (MODE == 0 ? moff : MODE == 1 ? TL.T : TL.FZP);
    // forward sweeps (M, T or Z^T) and backward sweeps (T^T or Z)
    auto fwd = [&](T* v) {
        if constexpr (MODE == 2) fdm_fwd<N>(M, v);
        else eo_apply<N, +1>(M, v, v);
    };
    auto bwd = [&](T* v) {
        if constexpr (MODE == 2) fdm_bwd<N>(M, v);
        else eo_apply<N, +1>(tab + TL.TT, v, v);
    };
    T v[N];
    // z
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::idx(ta, tb, k)];
        fwd(v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::idx(ta, tb, k)] = v[k];
    }
    __syncthreads();
    // y
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::idx(ta, k, tb)];
        fwd(v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::idx(ta, k, tb)] = v[k];
    }
    __syncthreads();
    // x (and for the preconditioners: diagonal scaling, then the backward
    // sweep along x)
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::idx(k, ta, tb)];
        fwd(v);
        if constexpr (MODE == 1) {
            T dg[N];
            load_chunked_pencil<N>(inv_diag + size_t(cell0 + c) * N3, ta + N * tb, dg);
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] *= dg[k];
        }
        if constexpr (MODE == 2) {
            const T* lam = tab + TL.FLAM;
            const T yz = pick<N>(lam, ta) * cs[1] + pick<N>(lam, tb) * cs[2];
            // 1/d by the hardware reciprocal refined with two Newton steps
            // (d > 0): independent per k, unlike the full division sequence
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const T d = fma(lam[k], cs[0], yz);
                T r;
                if constexpr (sizeof(T) == 8) r = __builtin_amdgcn_rcp(d);
                else r = __builtin_amdgcn_rcpf(d);
                r = fma(r, fma(-d, r, T(1)), r);
                r = fma(r, fma(-d, r, T(1)), r);
                v[k] = v[k] * cs[3] * r;
            }
        }
        if constexpr (MODE != 0) bwd(v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::idx(k, ta, tb)] = v[k];
    }
    __syncthreads();
    if constexpr (MODE != 0) {
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::idx(ta, k, tb)];
            bwd(v);
#pragma unroll
            for (int k = 0; k < N; ++k) A[Sh::idx(ta, k, tb)] = v[k];
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::idx(ta, tb, k)];
            bwd(v);
            const size_t off = size_t(cell0 + c) * N3 + ta + N * tb;
            T* __restrict__ dst = out + off;
            if constexpr (MERGE) {
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const T ui = mg.u ? mg.u[off + k * N2] : T(0);
                    const T uo = mg.sigma != T(0) ? dst[k * N2] : ui;
                    dst[k * N2] = ui + mg.sigma * (ui - uo) + mg.theta * v[k];
                    if (mg.zero) mg.zero[off + k * N2] = T(0);
                }
            } else {
#pragma unroll
                for (int k = 0; k < N; ++k) dst[k * N2] = v[k];
            }
        }
        return;
    }
    T* __restrict__ dst = out + size_t(cell0) * N3;
    for (int e = tid; e < ncb * N3; e += NT) {
        const int cc = e / N3, i = e % N3;
        dst[e] = lds[cc * CS + Sh::idx(i % N, (i / N) % N, i / N2)];
    }
}

template <int N, typename T>
static int launch_bc_t(const sipg_op* op, int mode, const void* in, void* out, hipStream_t st) {
    constexpr TableLayout TL(N);
    const int ncells = int(op->ncells);
    const unsigned nblk = unsigned((ncells + cells_per_block(N) - 1) / cells_per_block(N));
    const T* tab = static_cast<const T*>(op->tables);
    const T* i_ = static_cast<const T*>(in);
    T* o_ = static_cast<T*>(out);
    constexpr int NT = threads_per_block(N);
    const BcMerge<T> none{nullptr, nullptr, T(0), T(0), nullptr};
    if (mode == SIPG_BC_PJACOBI) {
        basis_change_kernel<N, T, 1, false><<<nblk, NT, 0, st>>>(i_, o_, tab, 0, static_cast<const T*>(op->gl_inv_diag), ncells, none);
    } else if (mode == SIPG_BC_FDM) {
        basis_change_kernel<N, T, 2, false><<<nblk, NT, 0, st>>>(i_, o_, tab, 0, static_cast<const T*>(op->fdm_cell), ncells, none);
    } else {
        const int off = mode == SIPG_BC_T ? TL.T : mode == SIPG_BC_TT ? TL.TT : TL.ET;
        basis_change_kernel<N, T, 0, false><<<nblk, NT, 0, st>>>(i_, o_, tab, off, nullptr, ncells, none);
    }
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

template <int N, typename T>
static int launch_cheb_t(const sipg_op* op, int mode, const void* b, const void* au, const void* u, void* uo,
                         double sigma, double theta, void* zero, hipStream_t st, int nv) {
    const int ncells = int(op->ncells);
    const dim3 nblk = dim3(unsigned((ncells + cells_per_block(N) - 1) / cells_per_block(N)), unsigned(nv));
    constexpr int NT = threads_per_block(N);
    const T* tab = static_cast<const T*>(op->tables);
    const BcMerge<T> m{static_cast<const T*>(au), static_cast<const T*>(u), T(sigma), T(theta), static_cast<T*>(zero)};
    if (mode == SIPG_BC_PJACOBI)
        basis_change_kernel<N, T, 1, true><<<nblk, NT, 0, st>>>(static_cast<const T*>(b), static_cast<T*>(uo), tab, 0,
                                                                static_cast<const T*>(op->gl_inv_diag), ncells, m);
    else
        basis_change_kernel<N, T, 2, true><<<nblk, NT, 0, st>>>(static_cast<const T*>(b), static_cast<T*>(uo), tab, 0,
                                                                static_cast<const T*>(op->fdm_cell), ncells, m);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

template <int N>
static int launch_cheb_n(const sipg_op* op, int mode, const void* b, const void* au, const void* u, void* uo,
                         double sigma, double theta, void* zero, hipStream_t st, int nv) {
    return op->dtype == SIPG_F64 ? launch_cheb_t<N, double>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv)
                                 : launch_cheb_t<N, float>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
}

int launch_precond_cheb(const sipg_op* op, int mode, const void* b, const void* au, const void* u, void* uo,
                        double sigma, double theta, hipStream_t st, void* zero, int nv) {
    if ((mode != SIPG_BC_PJACOBI && mode != SIPG_BC_FDM) || nv < 1) {
        set_error("merged Chebyshev step: preconditioner mode and at least one right-hand side expected");
        return SIPG_E_ARG;
    }
    switch (op->n) {
        case 2: return launch_cheb_n<2>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 3: return launch_cheb_n<3>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 4: return launch_cheb_n<4>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 5: return launch_cheb_n<5>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 6: return launch_cheb_n<6>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 7: return launch_cheb_n<7>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 8: return launch_cheb_n<8>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
        case 9: return launch_cheb_n<9>(op, mode, b, au, u, uo, sigma, theta, zero, st, nv);
    }
    set_error("merged Chebyshev step: unsupported degree");
    return SIPG_E_UNSUPPORTED;
}

template <int N>
static int launch_bc_n(const sipg_op* op, int mode, const void* in, void* out, hipStream_t st) {
    return op->dtype == SIPG_F64 ? launch_bc_t<N, double>(op, mode, in, out, st)
                                 : launch_bc_t<N, float>(op, mode, in, out, st);
}

int launch_basis_change(const sipg_op* op, int mode, const void* in, void* out, hipStream_t st) {
    switch (op->n) {
        case 2: return launch_bc_n<2>(op, mode, in, out, st);
        case 3: return launch_bc_n<3>(op, mode, in, out, st);
        case 4: return launch_bc_n<4>(op, mode, in, out, st);
        case 5: return launch_bc_n<5>(op, mode, in, out, st);
        case 6: return launch_bc_n<6>(op, mode, in, out, st);
        case 7: return launch_bc_n<7>(op, mode, in, out, st);
        case 8: return launch_bc_n<8>(op, mode, in, out, st);
        case 9: return launch_bc_n<9>(op, mode, in, out, st);
    }
    set_error("basis change: unsupported degree");
    return SIPG_E_UNSUPPORTED;
}

}  // namespace sipg
