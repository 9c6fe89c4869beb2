// Device building blocks for sum factorization on gfx950: even-odd 1D
// contractions on register pencils and small helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace sipg {

// Read-only coefficient tables seen through the constant address space: the
// compiler then always reads wavefront-uniform entries with scalar loads into
// scalar registers (for global pointers it has to prove that no store of the
// kernel may reach them first, and with many LDS stores it may not).
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ const_ptr<T> ctab(const T* p) {
    return (const_ptr<T>)p;
}

// out = M in for an n x n matrix in even-odd packed form (sipg_common.hpp),
// with M[n-1-q][n-1-j] = EPS M[q][j].  Costs about n^2/2 multiply-adds
// instead of n^2 (even-odd decomposition, Section 4.1 / Section 5).
// `in` and `out` may be the same array.  P must be a wavefront-uniform
// pointer so that the coefficients come through scalar loads (a pointer to
// the constant address space, ctab(), guarantees them).
template <int N, int EPS, typename T, typename PT>
__device__ __forceinline__ void eo_apply(PT P, const T* in, T* out) {
    constexpr int H = N / 2;
    constexpr int oA = 0, oB = H * H, oC = 2 * H * H, oR = 2 * H * H + H, oM = 2 * H * H + 2 * H;
    T e[H], o[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        e[j] = in[j] + in[N - 1 - j];
        o[j] = in[j] - in[N - 1 - j];
    }
    T mid = T(0);
    if constexpr (N % 2 == 1) mid = in[H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
        T ev = T(0), od = T(0);
        if constexpr (N % 2 == 1) ev = P[oC + q] * mid;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            ev = fma(P[oA + q * H + j], e[j], ev);
            od = fma(P[oB + q * H + j], o[j], od);
        }
        if constexpr (EPS > 0) {
            out[q] = ev + od;
            out[N - 1 - q] = ev - od;
        } else {
            out[q] = ev + od;
            out[N - 1 - q] = od - ev;
        }
    }
    if constexpr (N % 2 == 1) {
        T m = T(0);
        if constexpr (EPS > 0) {
            m = P[oM] * mid;
#pragma unroll
            for (int j = 0; j < H; ++j) m = fma(P[oR + j], e[j], m);
        } else {
#pragma unroll
            for (int j = 0; j < H; ++j) m = fma(P[oR + j], o[j], m);
        }
        out[H] = m;
    }
}

// An interpolation-type sweep (S or S^T) that is the identity for a basis
// collocated with the quadrature (nodal Gauss basis, S = I, Section 4.1).
template <int N, bool IDENTITY, typename T, typename PT>
__device__ __forceinline__ void s_apply(PT P, const T* in, T* out) {
    if constexpr (IDENTITY) {
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = in[i];
    } else {
        eo_apply<N, +1>(P, in, out);
    }
}

// Eigenvector transforms of the block preconditioner (Section 6.4) in the
// parity-split form (basis1d.hpp, fdm_1d): the ceil(n/2) reflection-even
// eigenvectors z_m store entries 0..h (h = n/2), the odd ones entries
// 0..h-1, so each transform costs about n^2/2 multiply-adds.
// fdm_fwd: v <- Z^T v (even coefficients first, then odd ones).
template <int N, typename T>
__device__ __forceinline__ void fdm_fwd(const T* __restrict__ P, T* v) {
    constexpr int H = N / 2, NE = N - H, NO = H;
    T e[H > 0 ? H : 1], o[H > 0 ? H : 1], r[N];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        e[j] = v[j] + v[N - 1 - j];
        o[j] = v[j] - v[N - 1 - j];
    }
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        T acc = (N % 2 == 1) ? P[m * (H + 1) + H] * v[H] : T(0);
#pragma unroll
        for (int j = 0; j < H; ++j) acc = fma(P[m * (H + 1) + j], e[j], acc);
        r[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < NO; ++m) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < H; ++j) acc = fma(P[NE * (H + 1) + m * H + j], o[j], acc);
        r[NE + m] = acc;
    }
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = r[m];
}
// fdm_bwd: v <- Z v for v ordered as fdm_fwd leaves it.
template <int N, typename T>
__device__ __forceinline__ void fdm_bwd(const T* __restrict__ P, T* v) {
    constexpr int H = N / 2, NE = N - H, NO = H;
    T r[N];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        T ev = T(0), od = T(0);
#pragma unroll
        for (int m = 0; m < NE; ++m) ev = fma(P[m * (H + 1) + j], v[m], ev);
#pragma unroll
        for (int m = 0; m < NO; ++m) od = fma(P[NE * (H + 1) + m * H + j], v[NE + m], od);
        r[j] = ev + od;
        r[N - 1 - j] = ev - od;
    }
    if constexpr (N % 2 == 1) {
        T mid = T(0);
#pragma unroll
        for (int m = 0; m < NE; ++m) mid = fma(P[m * (H + 1) + H], v[m], mid);
        r[H] = mid;
    }
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = r[m];
}

// dst[0..M) = src[0..M) with 16-byte loads where possible (global memory on
// gfx950 takes them at element alignment), fewer load instructions and cache
// accesses for a lane's run of consecutive values.
template <int M, typename T>
__device__ __forceinline__ void load_run(const T* __restrict__ src, T* dst) {
    constexpr int V = 16 / int(sizeof(T));
    typedef T vec __attribute__((ext_vector_type(V), aligned(sizeof(T))));
    int i = 0;
#pragma unroll
    for (; i + V <= M; i += V) {
        const vec v = *reinterpret_cast<const vec*>(src + i);
#pragma unroll
        for (int j = 0; j < V; ++j) dst[i + j] = v[j];
    }
#pragma unroll
    for (; i < M; ++i) dst[i] = src[i];
}

// The N values of pencil t of a cell stored in chunks of 16 bytes
// (inv_diag_offset): `cell` points to the cell's N^3 values.
template <int N, typename T>
__device__ __forceinline__ void load_chunked_pencil(const T* __restrict__ cell, int t, T* dst) {
    constexpr int CH = 16 / int(sizeof(T)), J = N / CH, R = N % CH;
#pragma unroll
    for (int j = 0; j < J; ++j) load_run<CH>(cell + j * CH * N * N + CH * t, dst + j * CH);
    if constexpr (R > 0) load_run<R>(cell + J * CH * N * N + R * t, dst + J * CH);
}

// P[i] for a lane-varying index 0 <= i < N, from uniform (scalar) loads.
template <int N, typename PT>
__device__ __forceinline__ auto pick(PT P, int i) {
    auto r = P[0];
#pragma unroll
    for (int j = 1; j < N; ++j) r = (i == j) ? P[j] : r;
    return r;
}

}  // namespace sipg
