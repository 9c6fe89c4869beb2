// Vector kernels of the multigrid solver (Section 6): Chebyshev updates
// (eq. chebyshev), residuals, precision conversion and dot products, in
// FP32 and FP64.
#include "sipg_common.hpp"
#include "vecops.hpp"

namespace sipg {

constexpr int kVT = 256;
constexpr int kVB = 2048;   // max blocks of a grid-stride vector kernel

static unsigned vblocks(int64_t n) { return unsigned(std::min<int64_t>(kVB, (n + kVT - 1) / kVT)); }

// u_new = u + sigma (u - u_old) + theta z, written into u_old's storage (the
// three-term recurrence of eq. chebyshev; the caller swaps u and u_old).
template <typename T>
__global__ void __launch_bounds__(kVT) cheb_kernel(const T* __restrict__ u, T* __restrict__ u_old, const T* __restrict__ z,
                                                   T sigma, T theta, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) {
        const T ui = u[i];
        const T uo = sigma != T(0) ? u_old[i] : ui;   // first step: u_old is not read
        u_old[i] = ui + sigma * (ui - uo) + theta * z[i];
    }
}

// r = b - a
template <typename T>
__global__ void __launch_bounds__(kVT) sub_kernel(const T* __restrict__ b, const T* __restrict__ a, T* __restrict__ r, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) r[i] = b[i] - a[i];
}

// y = alpha x + beta y
template <typename T>
__global__ void __launch_bounds__(kVT) axpby_kernel(T alpha, const T* __restrict__ x, T beta, T* __restrict__ y, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = alpha * x[i] + beta * y[i];
}

// y = alpha x
template <typename T>
__global__ void __launch_bounds__(kVT) scale_kernel(T alpha, const T* __restrict__ x, T* __restrict__ y, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = alpha * x[i];
}

// x_i = -5.5 + (i mod 12): the start vector of the eigenvalue estimates
template <typename T>
__global__ void __launch_bounds__(kVT) sawtooth_kernel(T* __restrict__ x, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT)
        x[i] = T(-5.5 + double(i % 12));
}

template <typename TO, typename TI>
__global__ void __launch_bounds__(kVT) convert_kernel(const TI* __restrict__ x, TO* __restrict__ y, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = TO(x[i]);
}

// Coefficients held in device memory (no host round trip between a dot
// product and the update that uses it): c = sign * num[0] / den[0].
// y = c x + y
template <typename T>
__global__ void __launch_bounds__(kVT) axpy_dev_kernel(const double* __restrict__ num, const double* __restrict__ den,
                                                       double sign, const T* __restrict__ x, T* __restrict__ y, int64_t n) {
    const T c = T(sign * (num[0] / den[0]));
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = c * x[i] + y[i];
}
// y = x + c y
template <typename T>
__global__ void __launch_bounds__(kVT) xpby_dev_kernel(const T* __restrict__ x, const double* __restrict__ num,
                                                       const double* __restrict__ den, T* __restrict__ y, int64_t n) {
    const T c = T(num[0] / den[0]);
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = x[i] + c * y[i];
}
// out[0] = num[0] / den[0] (den = nullptr: out[0] = num[0])
__global__ void scalar_kernel(const double* __restrict__ num, const double* __restrict__ den, double* __restrict__ out) {
    if (threadIdx.x == 0) out[0] = den ? num[0] / den[0] : num[0];
}

__device__ __forceinline__ double vblock_sum(double v) {
    __shared__ double sh[kVT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kVT / 64; ++w) s += sh[w];
    return s;
}

// partial[block] = sum a_i b_i, accumulated in double
template <typename T>
__global__ void __launch_bounds__(kVT) vdot_kernel(const T* __restrict__ a, const T* __restrict__ b, double* __restrict__ partial, int64_t n) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) s += double(a[i]) * double(b[i]);
    s = vblock_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kVT) vfinish_kernel(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kVT) s += partial[i];
    s = vblock_sum(s);
    if (threadIdx.x == 0) *out = s;
}

template <typename T>
int vec_cheb(const T* u, T* u_old, const T* z, double sigma, double theta, int64_t n, hipStream_t st) {
    cheb_kernel<T><<<vblocks(n), kVT, 0, st>>>(u, u_old, z, T(sigma), T(theta), n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_sub(const T* b, const T* a, T* r, int64_t n, hipStream_t st) {
    sub_kernel<T><<<vblocks(n), kVT, 0, st>>>(b, a, r, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_axpby(double alpha, const T* x, double beta, T* y, int64_t n, hipStream_t st) {
    axpby_kernel<T><<<vblocks(n), kVT, 0, st>>>(T(alpha), x, T(beta), y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_scale(double alpha, const T* x, T* y, int64_t n, hipStream_t st) {
    scale_kernel<T><<<vblocks(n), kVT, 0, st>>>(T(alpha), x, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_sawtooth(T* x, int64_t n, hipStream_t st) {
    sawtooth_kernel<T><<<vblocks(n), kVT, 0, st>>>(x, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename TO, typename TI>
int vec_convert(const TI* x, TO* y, int64_t n, hipStream_t st) {
    convert_kernel<TO, TI><<<vblocks(n), kVT, 0, st>>>(x, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_dot_async(const T* a, const T* b, double* partial, double* out, int64_t n, hipStream_t st) {
    const unsigned nb = vblocks(n);
    vdot_kernel<T><<<nb, kVT, 0, st>>>(a, b, partial, n);
    vfinish_kernel<<<1, kVT, 0, st>>>(partial, int(nb), out);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

template <typename T>
int vec_axpy_dev(const double* num, const double* den, double sign, const T* x, T* y, int64_t n, hipStream_t st) {
    axpy_dev_kernel<T><<<vblocks(n), kVT, 0, st>>>(num, den, sign, x, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_xpby_dev(const T* x, const double* num, const double* den, T* y, int64_t n, hipStream_t st) {
    xpby_dev_kernel<T><<<vblocks(n), kVT, 0, st>>>(x, num, den, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
int scalar_ratio(const double* num, const double* den, double* out, hipStream_t st) {
    scalar_kernel<<<1, 64, 0, st>>>(num, den, out);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

// y = A x, A dense n x n row major: one wavefront per row, its lanes striding
// over the columns, then a shuffle reduction.
template <typename T>
__global__ void __launch_bounds__(kVT) dense_mv_kernel(const T* __restrict__ A, const T* __restrict__ x,
                                                       T* __restrict__ y, int n) {
    const int row = blockIdx.x * (kVT / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (row >= n) return;
    const T* __restrict__ a = A + size_t(row) * n;
    T acc = T(0);
    for (int j = lane; j < n; j += 64) acc = fma(a[j], x[j], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) y[row] = acc;
}

template <typename T>
int vec_dense_mv(const T* A, const T* x, T* y, int n, hipStream_t st) {
    const unsigned g = unsigned((n + kVT / 64 - 1) / (kVT / 64));
    dense_mv_kernel<T><<<g, kVT, 0, st>>>(A, x, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

#define SIPG_VEC_INST(T)                                                                        \
    template int vec_axpy_dev<T>(const double*, const double*, double, const T*, T*, int64_t, hipStream_t); \
    template int vec_xpby_dev<T>(const T*, const double*, const double*, T*, int64_t, hipStream_t); \
    template int vec_cheb<T>(const T*, T*, const T*, double, double, int64_t, hipStream_t);  \
    template int vec_sub<T>(const T*, const T*, T*, int64_t, hipStream_t);                   \
    template int vec_axpby<T>(double, const T*, double, T*, int64_t, hipStream_t);           \
    template int vec_scale<T>(double, const T*, T*, int64_t, hipStream_t);                   \
    template int vec_sawtooth<T>(T*, int64_t, hipStream_t);                                  \
    template int vec_dot_async<T>(const T*, const T*, double*, double*, int64_t, hipStream_t); \
    template int vec_dense_mv<T>(const T*, const T*, T*, int, hipStream_t);
SIPG_VEC_INST(float)
SIPG_VEC_INST(double)
template int vec_convert<float, double>(const double*, float*, int64_t, hipStream_t);
template int vec_convert<double, float>(const float*, double*, int64_t, hipStream_t);

}  // namespace sipg
