// FP64 conjugate gradient method for A x = b (outer solver of Section 6.2),
// with fused vector updates and two-stage dot products on the device.  The
// host reads one scalar per iteration to decide convergence.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "sipg_common.hpp"
#include "setup.hpp"

namespace sipg {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[kRedThreads / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    return s;
}

// partial[block] = sum a_i b_i
__global__ void __launch_bounds__(kRedThreads) dot_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                          double* __restrict__ partial, int64_t n) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRedThreads)
        s = fma(a[i], b[i], s);
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// r = b - Ax ; p = r ; partial = r.r
__global__ void __launch_bounds__(kRedThreads) residual_kernel(const double* __restrict__ b, const double* __restrict__ ax,
                                                               double* __restrict__ r, double* __restrict__ p,
                                                               double* __restrict__ partial, int64_t n) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRedThreads) {
        const double v = b[i] - ax[i];
        r[i] = v;
        if (p) p[i] = v;
        s = fma(v, v, s);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// alpha = rr / pAp (both reduced from partials); x += alpha p; r -= alpha Ap; partial = r.r
__global__ void __launch_bounds__(kRedThreads) update_kernel(double* __restrict__ x, double* __restrict__ r,
                                                             const double* __restrict__ p, const double* __restrict__ ap,
                                                             const double* __restrict__ scal, double* __restrict__ partial,
                                                             int64_t n) {
    const double alpha = scal[0] / scal[1];
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRedThreads) {
        x[i] = fma(alpha, p[i], x[i]);
        const double v = fma(-alpha, ap[i], r[i]);
        r[i] = v;
        s = fma(v, v, s);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// p = r + beta p with beta = rr_new / rr_old
__global__ void __launch_bounds__(kRedThreads) direction_kernel(double* __restrict__ p, const double* __restrict__ r,
                                                                const double* __restrict__ scal, int64_t n) {
    const double beta = scal[2] / scal[0];
    for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += int64_t(gridDim.x) * kRedThreads)
        p[i] = fma(beta, p[i], r[i]);
}

// scal[slot] = sum(partial[0..nb)); with `shift`, first scal[0] = scal[2] (rr_old <- rr_new)
__global__ void __launch_bounds__(kRedThreads) finish_kernel(const double* __restrict__ partial, int nb,
                                                             double* __restrict__ scal, int slot) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kRedThreads) s += partial[i];
    s = block_sum(s);
    if (threadIdx.x == 0) scal[slot] = s;
}

__global__ void copy_scalar_kernel(double* scal, int from, int to) {
    if (threadIdx.x == 0 && blockIdx.x == 0) scal[to] = scal[from];
}

// Work arrays of one solve: r, p, ap (ndofs each), kRedBlocks partial sums,
// 4 scalars.
struct CgWork {
    double *r, *p, *ap, *partial, *scal;
};

static int cg_iterate(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                      sipg_solve_info* info, const CgWork& w, hipStream_t st) {
    const int64_t n = op->ndofs;
    double *r = w.r, *p = w.p, *ap = w.ap, *partial = w.partial, *scal = w.scal;
    const int nb = int(std::min<int64_t>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads));
    int status = SIPG_OK;
    auto read = [&](int slot, double& v) -> int {
        if (hipMemcpyAsync(&v, scal + slot, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("sipg_cg_solve: device to host copy failed");
            return SIPG_E_HIP;
        }
        return SIPG_OK;
    };
    // ||b||
    dot_kernel<<<nb, kRedThreads, 0, st>>>(b, b, partial, n);
    finish_kernel<<<1, kRedThreads, 0, st>>>(partial, nb, scal, 3);
    double bb = 0.0;
    if ((status = read(3, bb)) != SIPG_OK) return status;
    const double bnorm = std::sqrt(bb);
    // r = b - A x, p = r
    if ((status = launch_matvec(op, x, ap, st)) != SIPG_OK) return status;
    residual_kernel<<<nb, kRedThreads, 0, st>>>(b, ap, r, p, partial, n);
    finish_kernel<<<1, kRedThreads, 0, st>>>(partial, nb, scal, 0);
    double rr = 0.0;
    if ((status = read(0, rr)) != SIPG_OK) return status;
    info->initial_residual = std::sqrt(rr);
    const double target = rel_tol * (bnorm > 0.0 ? bnorm : 1.0);
    int it = 0;
    double res = std::sqrt(rr);
    while (res > target && it < max_iter) {
        if ((status = launch_matvec(op, p, ap, st)) != SIPG_OK) break;
        dot_kernel<<<nb, kRedThreads, 0, st>>>(p, ap, partial, n);
        finish_kernel<<<1, kRedThreads, 0, st>>>(partial, nb, scal, 1);
        update_kernel<<<nb, kRedThreads, 0, st>>>(x, r, p, ap, scal, partial, n);
        finish_kernel<<<1, kRedThreads, 0, st>>>(partial, nb, scal, 2);
        direction_kernel<<<nb, kRedThreads, 0, st>>>(p, r, scal, n);
        copy_scalar_kernel<<<1, 64, 0, st>>>(scal, 2, 0);
        if ((status = read(0, rr)) != SIPG_OK) break;
        res = std::sqrt(rr);
        ++it;
    }
    if (status == SIPG_OK) {
        info->iterations = it;
        info->final_residual = res;
        // true residual
        if ((status = launch_matvec(op, x, ap, st)) == SIPG_OK) {
            residual_kernel<<<nb, kRedThreads, 0, st>>>(b, ap, r, nullptr, partial, n);
            finish_kernel<<<1, kRedThreads, 0, st>>>(partial, nb, scal, 3);
            double tr = 0.0;
            status = read(3, tr);
            info->true_residual = std::sqrt(tr);
        }
        if (status == SIPG_OK && res > target) {
            set_error("sipg_cg_solve: no convergence within max_iter");
            status = SIPG_E_NOCONV;
        }
    }
    return status;
}

int cg_solve_device(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                    sipg_solve_info* info, hipStream_t st) {
    const size_t n = size_t(op->ndofs);
    CgWork w{};
    void* blk[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    const size_t bytes[5] = {8 * n, 8 * n, 8 * n, 8 * size_t(kRedBlocks), 8 * 4};
    // without a caller allocator the workspace is stream-ordered memory (no
    // device-wide synchronisation when it goes back)
    const bool ordered = !op->mem.a.alloc;
    int status = SIPG_OK;
    for (int i = 0; i < 5 && status == SIPG_OK; ++i) {
        if (!ordered) {
            status = op->mem.alloc(&blk[i], bytes[i], "sipg_cg_solve: workspace");
        } else if (hipError_t e = hipMallocAsync(&blk[i], bytes[i], st); e != hipSuccess) {
            blk[i] = nullptr;
            status = hip_fail(e, "sipg_cg_solve: workspace");
        }
    }
    if (status == SIPG_OK) {
        w = CgWork{static_cast<double*>(blk[0]), static_cast<double*>(blk[1]), static_cast<double*>(blk[2]),
                   static_cast<double*>(blk[3]), static_cast<double*>(blk[4])};
        status = cg_iterate(op, b, x, rel_tol, max_iter, info, w, st);
        // a caller allocator's free is not stream-ordered: every launch of the
        // solve is finished before the blocks go back
        if (!ordered && hipStreamSynchronize(st) != hipSuccess && status == SIPG_OK) {
            set_error("sipg_cg_solve: stream synchronisation failed");
            status = SIPG_E_HIP;
        }
    }
    for (void* q : blk) {
        if (!q) continue;
        if (ordered) (void)hipFreeAsync(q, st);
        else op->mem.release(q);
    }
    return status;
}

// ---------------------------------------------------------------------------
// The same solve for callers that cannot allocate device memory (code under
// stream capture, tight serving loops): the work arrays are a fixed array in
// device memory, one per GPU, that holds up to kStaticCgDofs unknowns.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticCgDofs = int64_t(1) << 20;
constexpr size_t kStaticCgWords = size_t(3 * kStaticCgDofs) + size_t(kRedBlocks) + 64;
static __device__ __align__(256) double scratch[kStaticCgWords];

// Device address of `scratch` on each device, looked up once per device with
// that device current (the host-side name of the array is not a device
// address).
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_ptr;

static int static_scratch(double** out) {
    int dev = 0;
    SIPG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (int(g_scratch_ptr.size()) <= dev) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        SIPG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return SIPG_OK;
}

int64_t cg_static_max_dofs() { return kStaticCgDofs; }

int cg_solve_static(const sipg_op* op, const double* b, double* x, double rel_tol, int max_iter,
                    sipg_solve_info* info, hipStream_t st) {
    if (op->ndofs > kStaticCgDofs) {
        set_error("sipg_cg_solve_static: the operator has " + std::to_string(op->ndofs) +
                  " unknowns, more than the fixed work arrays hold (" + std::to_string(kStaticCgDofs) + ")");
        return SIPG_E_ARG;
    }
    double* base = nullptr;
    if (int rc = static_scratch(&base)) return rc;
    // every array is written before it is read: nothing to clear
    const CgWork w{base, base + kStaticCgDofs, base + 2 * kStaticCgDofs, base + 3 * kStaticCgDofs,
                   base + 3 * kStaticCgDofs + kRedBlocks};
    return cg_iterate(op, b, x, rel_tol, max_iter, info, w, st);
}

}  // namespace sipg
