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

// partial[block] = sum a_i b_i, accumulated in double; blockIdx.y picks one
// of several vector pairs stored one after another (partials gridDim.x apart)
template <typename T>
__global__ void __launch_bounds__(kVT) vdot_kernel(const T* __restrict__ a, const T* __restrict__ b, double* __restrict__ partial, int64_t n) {
    a += size_t(blockIdx.y) * n;
    b += size_t(blockIdx.y) * n;
    partial += size_t(blockIdx.y) * gridDim.x;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) s += double(a[i]) * double(b[i]);
    s = vblock_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[block] = sum of the block's nb partials
__global__ void __launch_bounds__(kVT) vfinish_kernel(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    partial += size_t(blockIdx.x) * nb;
    out += blockIdx.x;
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
int vec_dot_many(const T* a, const T* b, double* partial, double* out, int64_t n, int nv, hipStream_t st) {
    const unsigned nb = vblocks(n);
    vdot_kernel<T><<<dim3(nb, unsigned(nv)), kVT, 0, st>>>(a, b, partial, n);
    vfinish_kernel<<<unsigned(nv), kVT, 0, st>>>(partial, int(nb), out);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

// Several right-hand sides of one conjugate gradient iteration, stored one
// after another (n apart), blockIdx.y picking one; vector v is updated only
// while active[v] != 0, with c = sign * num[v] / den[v]:  y = c x + y  and
// y = x + c y.
template <typename T>
__global__ void __launch_bounds__(kVT) axpy_many_kernel(const double* __restrict__ num, const double* __restrict__ den,
                                                        const double* __restrict__ active, double sign,
                                                        const T* __restrict__ x, T* __restrict__ y, int64_t n) {
    const int v = blockIdx.y;
    if (active[v] == 0.0) return;
    const T c = T(sign * (num[v] / den[v]));
    x += size_t(v) * n;
    y += size_t(v) * n;
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = c * x[i] + y[i];
}
template <typename T>
__global__ void __launch_bounds__(kVT) xpby_many_kernel(const T* __restrict__ x, const double* __restrict__ num,
                                                        const double* __restrict__ den, const double* __restrict__ active,
                                                        T* __restrict__ y, int64_t n) {
    const int v = blockIdx.y;
    if (active[v] == 0.0) return;
    const T c = T(num[v] / den[v]);
    x += size_t(v) * n;
    y += size_t(v) * n;
    for (int64_t i = int64_t(blockIdx.x) * kVT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kVT) y[i] = x[i] + c * y[i];
}
// out[v] = num[v] while active[v] != 0
__global__ void copy_many_kernel(const double* __restrict__ num, const double* __restrict__ active,
                                 double* __restrict__ out, int nv) {
    const int v = threadIdx.x;
    if (v < nv && active[v] != 0.0) out[v] = num[v];
}
// Start of the iteration: target[v] = rel_tol ||b_v|| (rel_tol for b_v = 0)
// from bb[v] = ||b_v||^2, active[v] = 1 while ||r_v|| > target[v], iters[v] = 0.
__global__ void cg_start_many_kernel(const double* __restrict__ bb, const double* __restrict__ rr, double rel_tol,
                                     double* __restrict__ target, double* __restrict__ active,
                                     double* __restrict__ iters, int nv) {
    const int v = threadIdx.x;
    if (v >= nv) return;
    const double t = rel_tol * (bb[v] > 0.0 ? sqrt(bb[v]) : 1.0);
    target[v] = t;
    active[v] = sqrt(rr[v]) <= t ? 0.0 : 1.0;
    iters[v] = 0.0;
}
// End of an iteration (rr[v] = r_v.r_v after it): an active vector counts
// the iteration and stops once ||r_v|| <= target[v].
__global__ void cg_mask_many_kernel(const double* __restrict__ rr, const double* __restrict__ target,
                                    double* __restrict__ active, double* __restrict__ iters, int nv) {
    const int v = threadIdx.x;
    if (v >= nv || active[v] == 0.0) return;
    iters[v] += 1.0;
    if (sqrt(rr[v]) <= target[v]) active[v] = 0.0;
}

template <typename T>
int vec_axpy_many(const double* num, const double* den, const double* active, double sign, const T* x, T* y, int64_t n,
                  int nv, hipStream_t st) {
    axpy_many_kernel<T><<<dim3(vblocks(n), unsigned(nv)), kVT, 0, st>>>(num, den, active, sign, x, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
template <typename T>
int vec_xpby_many(const T* x, const double* num, const double* den, const double* active, T* y, int64_t n, int nv,
                  hipStream_t st) {
    xpby_many_kernel<T><<<dim3(vblocks(n), unsigned(nv)), kVT, 0, st>>>(x, num, den, active, y, n);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
int scalar_copy_many(const double* num, const double* active, double* out, int nv, hipStream_t st) {
    copy_many_kernel<<<1, 64, 0, st>>>(num, active, out, nv);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
int cg_start_many(const double* bb, const double* rr, double rel_tol, double* target, double* active, double* iters,
                  int nv, hipStream_t st) {
    cg_start_many_kernel<<<1, 64, 0, st>>>(bb, rr, rel_tol, target, active, iters, nv);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}
int cg_mask_many(const double* rr, const double* target, double* active, double* iters, int nv, hipStream_t st) {
    cg_mask_many_kernel<<<1, 64, 0, st>>>(rr, target, active, iters, nv);
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
// over the columns, then a shuffle reduction; blockIdx.y picks one of several
// x (and y) stored one after another.
template <typename T>
__global__ void __launch_bounds__(kVT) dense_mv_kernel(const T* __restrict__ A, const T* __restrict__ x,
                                                       T* __restrict__ y, int n) {
    const int row = blockIdx.x * (kVT / 64) + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (row >= n) return;
    x += size_t(blockIdx.y) * n;
    y += size_t(blockIdx.y) * n;
    const T* __restrict__ a = A + size_t(row) * n;
    T acc = T(0);
    for (int j = lane; j < n; j += 64) acc = fma(a[j], x[j], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) y[row] = acc;
}

template <typename T>
int vec_dense_mv(const T* A, const T* x, T* y, int n, hipStream_t st, int nv) {
    const dim3 g = dim3(unsigned((n + kVT / 64 - 1) / (kVT / 64)), unsigned(nv));
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
    template int vec_dot_many<T>(const T*, const T*, double*, double*, int64_t, int, hipStream_t); \
    template int vec_axpy_many<T>(const double*, const double*, const double*, double, const T*, T*, int64_t, int, \
                                  hipStream_t);                                               \
    template int vec_xpby_many<T>(const T*, const double*, const double*, const double*, T*, int64_t, int, hipStream_t); \
    template int vec_dense_mv<T>(const T*, const T*, T*, int, hipStream_t, int);
SIPG_VEC_INST(float)
SIPG_VEC_INST(double)
template int vec_convert<float, double>(const double*, float*, int64_t, hipStream_t);
template int vec_convert<double, float>(const float*, double*, int64_t, hipStream_t);

}  // namespace sipg
