// Geometric multigrid transfer between a brick of cells and its coarsening:
// in every direction the fine cells are paired from the low end on, coarse
// cell i owning fine cells 2i and 2i+1; for an odd fine count the last coarse
// cell owns only the last fine cell.  The coarse and fine maps differ by an
// affine map per child, so the coarse space is a subspace of the fine one and
// the prolongation is the exact embedding: on child (s1,s2,s3) the fine
// coefficients are (M_s3 x M_s2 x M_s1) times the coarse ones, with the 1D
// matrices M_s of the child intervals within the coarse interval.  The
// matrices (emb, N x N each, row major): M_0, M_1 of the two halves, then for
// each direction d the pair of the last coarse cell of that direction (its
// children may be unequal on a graded brick; with one child the first matrix
// is the identity).  Restriction is the transpose.  One workgroup per coarse
// cell, one thread per pencil; the 1D contractions are shared between
// children with the same sides.
#include "sipg_common.hpp"
#include "vecops.hpp"

namespace sipg {

template <int N>
struct TrShape {
    static constexpr int N2 = N * N, N3 = N2 * N;
    static constexpr int NT = ((N2 + 63) / 64) * 64;
    __device__ static constexpr int idx(int i1, int i2, int i3) { return i1 + N * (i2 + N * i3); }
};

// out[i] = sum_j M[i][j] in[j]  (TRANS: out[j] = sum_i M[i][j] in[i])
template <int N, bool TRANS, typename T>
__device__ __forceinline__ void mat1d(const T* __restrict__ M, const T* in, T* out) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) acc = fma(TRANS ? M[j * N + i] : M[i * N + j], in[j], acc);
        out[i] = acc;
    }
}

// Children and embedding matrices of coarse cell index i in direction d.
struct ChildMap {
    int nf[3], nc[3], nl[3];   // fine and coarse counts, children of the last coarse cell
    __device__ int children(int d, int i) const { return i == nc[d] - 1 ? nl[d] : 2; }
    template <int N, typename T>
    __device__ const T* matrix(const T* emb, int d, int i, int s) const {
        return emb + (i == nc[d] - 1 ? 2 + 2 * d + s : s) * (N * N);
    }
};

template <int N, typename T>
__global__ void __launch_bounds__(TrShape<N>::NT)
prolongate_kernel(const T* __restrict__ coarse, T* __restrict__ fine, const T* __restrict__ emb, ChildMap cm) {
    using S = TrShape<N>;
    constexpr int N3 = S::N3;
    __shared__ T C[N3];
    __shared__ T Z[2][N3];
    __shared__ T Y[4][N3];
    const int cx = cm.nc[0], cy = cm.nc[1];
    const int cc = blockIdx.x;
    // several right-hand sides stored one after another: blockIdx.y picks one
    coarse += size_t(blockIdx.y) * gridDim.x * N3;
    fine += size_t(blockIdx.y) * (size_t(cm.nf[0]) * cm.nf[1] * cm.nf[2]) * N3;
    const int ix = cc % cx, iy = (cc / cx) % cy, iz = cc / (cx * cy);
    const int n1 = cm.children(0, ix), n2 = cm.children(1, iy), n3 = cm.children(2, iz);
    const int tid = threadIdx.x;
    const bool act = tid < S::N2;
    const int ta = tid % N, tb = tid / N;
    for (int e = tid; e < N3; e += S::NT) C[e] = coarse[size_t(cc) * N3 + e];
    __syncthreads();
    T v[N], r[N];
    if (act) {   // z: thread (j1, j2)
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = C[S::idx(ta, tb, k)];
        for (int s3 = 0; s3 < n3; ++s3) {
            mat1d<N, false>(cm.matrix<N>(emb, 2, iz, s3), v, r);
#pragma unroll
            for (int k = 0; k < N; ++k) Z[s3][S::idx(ta, tb, k)] = r[k];
        }
    }
    __syncthreads();
    if (act) {   // y: thread (j1, i3)
        for (int s3 = 0; s3 < n3; ++s3) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = Z[s3][S::idx(ta, k, tb)];
            for (int s2 = 0; s2 < n2; ++s2) {
                mat1d<N, false>(cm.matrix<N>(emb, 1, iy, s2), v, r);
#pragma unroll
                for (int k = 0; k < N; ++k) Y[s2 + 2 * s3][S::idx(ta, k, tb)] = r[k];
            }
        }
    }
    __syncthreads();
    if (act) {   // x: thread (i2, i3), add into the children
        for (int q = 0; q < 4; ++q) {
            const int s2 = q & 1, s3 = q >> 1;
            if (s2 >= n2 || s3 >= n3) continue;
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = Y[q][S::idx(k, ta, tb)];
            for (int s1 = 0; s1 < n1; ++s1) {
                mat1d<N, false>(cm.matrix<N>(emb, 0, ix, s1), v, r);
                const size_t child = size_t(2 * ix + s1) +
                                     size_t(cm.nf[0]) * (size_t(2 * iy + s2) + size_t(cm.nf[1]) * size_t(2 * iz + s3));
                T* __restrict__ dst = fine + child * N3 + N * (ta + N * tb);
#pragma unroll
                for (int k = 0; k < N; ++k) dst[k] += r[k];
            }
        }
    }
}

template <int N, typename T>
__global__ void __launch_bounds__(TrShape<N>::NT)
restrict_kernel(const T* __restrict__ fine, T* __restrict__ coarse, const T* __restrict__ emb, ChildMap cm) {
    using S = TrShape<N>;
    constexpr int N3 = S::N3;
    __shared__ T X[4][N3];
    __shared__ T Y[2][N3];
    const int cx = cm.nc[0], cy = cm.nc[1];
    const int cc = blockIdx.x;
    // several right-hand sides stored one after another: blockIdx.y picks one
    coarse += size_t(blockIdx.y) * gridDim.x * N3;
    fine += size_t(blockIdx.y) * (size_t(cm.nf[0]) * cm.nf[1] * cm.nf[2]) * N3;
    const int ix = cc % cx, iy = (cc / cx) % cy, iz = cc / (cx * cy);
    const int n1 = cm.children(0, ix), n2 = cm.children(1, iy), n3 = cm.children(2, iz);
    const int tid = threadIdx.x;
    const bool act = tid < S::N2;
    const int ta = tid % N, tb = tid / N;
    T v[N], r[N], acc[N];
    if (act) {   // x: thread (i2, i3); sum the children along x
        for (int q = 0; q < 4; ++q) {
            const int s2 = q & 1, s3 = q >> 1;
            if (s2 >= n2 || s3 >= n3) continue;
#pragma unroll
            for (int k = 0; k < N; ++k) acc[k] = T(0);
            for (int s1 = 0; s1 < n1; ++s1) {
                const size_t child = size_t(2 * ix + s1) +
                                     size_t(cm.nf[0]) * (size_t(2 * iy + s2) + size_t(cm.nf[1]) * size_t(2 * iz + s3));
                const T* __restrict__ src = fine + child * N3 + N * (ta + N * tb);
#pragma unroll
                for (int k = 0; k < N; ++k) v[k] = src[k];
                mat1d<N, true>(cm.matrix<N>(emb, 0, ix, s1), v, r);
#pragma unroll
                for (int k = 0; k < N; ++k) acc[k] += r[k];
            }
#pragma unroll
            for (int k = 0; k < N; ++k) X[q][S::idx(k, ta, tb)] = acc[k];
        }
    }
    __syncthreads();
    if (act) {   // y: thread (j1, i3)
        for (int s3 = 0; s3 < n3; ++s3) {
#pragma unroll
            for (int k = 0; k < N; ++k) acc[k] = T(0);
            for (int s2 = 0; s2 < n2; ++s2) {
#pragma unroll
                for (int k = 0; k < N; ++k) v[k] = X[s2 + 2 * s3][S::idx(ta, k, tb)];
                mat1d<N, true>(cm.matrix<N>(emb, 1, iy, s2), v, r);
#pragma unroll
                for (int k = 0; k < N; ++k) acc[k] += r[k];
            }
#pragma unroll
            for (int k = 0; k < N; ++k) Y[s3][S::idx(ta, k, tb)] = acc[k];
        }
    }
    __syncthreads();
    if (act) {   // z: thread (j1, j2)
#pragma unroll
        for (int k = 0; k < N; ++k) acc[k] = T(0);
        for (int s3 = 0; s3 < n3; ++s3) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = Y[s3][S::idx(ta, tb, k)];
            mat1d<N, true>(cm.matrix<N>(emb, 2, iz, s3), v, r);
#pragma unroll
            for (int k = 0; k < N; ++k) acc[k] += r[k];
        }
        T* __restrict__ dst = coarse + size_t(cc) * N3 + ta + N * tb;
#pragma unroll
        for (int k = 0; k < N; ++k) dst[k * S::N2] = acc[k];
    }
}

static ChildMap child_map(const int nf[3]) {
    ChildMap cm;
    for (int d = 0; d < 3; ++d) {
        cm.nf[d] = nf[d];
        cm.nc[d] = (nf[d] + 1) / 2;
        cm.nl[d] = nf[d] % 2 == 1 ? 1 : 2;
    }
    return cm;
}

template <typename T>
int transfer_prolongate_add(int n, const int nf[3], const T* coarse, T* fine, const T* emb, hipStream_t st, int nv) {
    const ChildMap cm = child_map(nf);
    const dim3 ncoarse = dim3(unsigned(cm.nc[0] * cm.nc[1] * cm.nc[2]), unsigned(nv));
    switch (n) {
#define SIPG_TR_CASE(NN)                                                                          \
    case NN:                                                                                      \
        prolongate_kernel<NN, T><<<ncoarse, TrShape<NN>::NT, 0, st>>>(coarse, fine, emb, cm);      \
        break;
        SIPG_TR_CASE(2) SIPG_TR_CASE(3) SIPG_TR_CASE(4) SIPG_TR_CASE(5)
        SIPG_TR_CASE(6) SIPG_TR_CASE(7) SIPG_TR_CASE(8) SIPG_TR_CASE(9)
#undef SIPG_TR_CASE
        default: set_error("transfer: unsupported degree"); return SIPG_E_UNSUPPORTED;
    }
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

template <typename T>
int transfer_restrict(int n, const int nf[3], const T* fine, T* coarse, const T* emb, hipStream_t st, int nv) {
    const ChildMap cm = child_map(nf);
    const dim3 ncoarse = dim3(unsigned(cm.nc[0] * cm.nc[1] * cm.nc[2]), unsigned(nv));
    switch (n) {
#define SIPG_TR_CASE(NN)                                                                        \
    case NN:                                                                                    \
        restrict_kernel<NN, T><<<ncoarse, TrShape<NN>::NT, 0, st>>>(fine, coarse, emb, cm);      \
        break;
        SIPG_TR_CASE(2) SIPG_TR_CASE(3) SIPG_TR_CASE(4) SIPG_TR_CASE(5)
        SIPG_TR_CASE(6) SIPG_TR_CASE(7) SIPG_TR_CASE(8) SIPG_TR_CASE(9)
#undef SIPG_TR_CASE
        default: set_error("transfer: unsupported degree"); return SIPG_E_UNSUPPORTED;
    }
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

// Transfer between two degrees on the same mesh (p-multigrid): per cell
// out (+)= (M x M x M) in with a rectangular 1D matrix M (NO x NI, row major):
// M = E (prolongation, degree embedding) or E^T (restriction).  One
// workgroup of 64 threads per cell; three sweeps through LDS.
template <int NI, int NO, typename T, bool ADD>
__global__ void __launch_bounds__(64)
ptransfer_kernel(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ M) {
    constexpr int I3 = NI * NI * NI, B = NI * NI * NO, C = NI * NO * NO, O3 = NO * NO * NO;
    __shared__ T a[I3];
    __shared__ T b[B];
    __shared__ T c[C];
    const size_t cell = blockIdx.x;
    const int tid = threadIdx.x;
    // several right-hand sides stored one after another: blockIdx.y picks one
    in += size_t(blockIdx.y) * gridDim.x * I3;
    out += size_t(blockIdx.y) * gridDim.x * O3;
    for (int e = tid; e < I3; e += 64) a[e] = in[cell * I3 + e];
    __syncthreads();
    for (int e = tid; e < B; e += 64) {   // b[i3][i2][o1]
        const int o1 = e % NO, r = e / NO;
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < NI; ++i) acc = fma(M[o1 * NI + i], a[r * NI + i], acc);
        b[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < C; e += 64) {   // c[i3][o2][o1]
        const int o1 = e % NO, o2 = (e / NO) % NO, i3 = e / (NO * NO);
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < NI; ++i) acc = fma(M[o2 * NI + i], b[(i3 * NI + i) * NO + o1], acc);
        c[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < O3; e += 64) {  // out[o3][o2][o1]
        const int r = e % (NO * NO), o3 = e / (NO * NO);
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < NI; ++i) acc = fma(M[o3 * NI + i], c[i * NO * NO + r], acc);
        if constexpr (ADD) out[cell * O3 + e] += acc;
        else out[cell * O3 + e] = acc;
    }
}

// Degree pairs (fine n, coarse n) of the two coarsening rules: halving the
// degree (k -> max(1, k/2)) and lowering it by one.
#define SIPG_PAIRS(X)                                                                     \
    X(3, 2) X(4, 2) X(4, 3) X(5, 3) X(5, 4) X(6, 3) X(6, 4) X(6, 5) X(7, 4) X(7, 6) X(8, 4) \
    X(8, 5) X(8, 7) X(9, 5) X(9, 8)

template <typename T>
int transfer_degree(int nf, int nc, int64_t ncells, bool restrict_, const T* in, T* out, const T* E,
                    const T* Et, hipStream_t st, int nv) {
    const dim3 g = dim3(unsigned(ncells), unsigned(nv));
#define SIPG_PCASE(F, C)                                                                     \
    if (nf == F && nc == C) {                                                                \
        if (restrict_) ptransfer_kernel<F, C, T, false><<<g, 64, 0, st>>>(in, out, Et);      \
        else ptransfer_kernel<C, F, T, true><<<g, 64, 0, st>>>(in, out, E);                  \
        SIPG_HIP(hipGetLastError());                                                         \
        return SIPG_OK;                                                                      \
    }
    SIPG_PAIRS(SIPG_PCASE)
#undef SIPG_PCASE
    set_error("transfer: unsupported pair of degrees");
    return SIPG_E_UNSUPPORTED;
}

template int transfer_degree<float>(int, int, int64_t, bool, const float*, float*, const float*, const float*, hipStream_t, int);
template int transfer_degree<double>(int, int, int64_t, bool, const double*, double*, const double*, const double*, hipStream_t, int);

template int transfer_prolongate_add<float>(int, const int[3], const float*, float*, const float*, hipStream_t, int);
template int transfer_prolongate_add<double>(int, const int[3], const double*, double*, const double*, hipStream_t, int);
template int transfer_restrict<float>(int, const int[3], const float*, float*, const float*, hipStream_t, int);
template int transfer_restrict<double>(int, const int[3], const double*, double*, const double*, hipStream_t, int);

}  // namespace sipg
