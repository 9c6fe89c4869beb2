// Ghost layers of a z-slab partition of the mesh (the per-GPU share of the
// multi-GPU design): the face terms of Section 3 read only the value and
// derivative layers of a neighbour cell (two layers in the Hermite-like
// basis, every layer in the nodal ones), so a slab sends its neighbour just
// those layers of the cells next to the shared plane.
#include "sipg_common.hpp"
#include "setup.hpp"

namespace sipg {

// out[(column c, layer j, point r)] = x[cell (c, iz)][r + n^2 layer(j)] with iz
// the bottom (side 0) or top (side 1) cell row of the slab, c = ix + nx iy,
// r = i1 + n i2, and layer(j) the j-th layer of the derivative support at
// that side (Hermite-like: 0, 1 at the bottom and n-2, n-1 at the top;
// nodal: 0 .. n-1).  One thread per output value.
template <typename T>
__global__ void pack_ghost_kernel(const T* __restrict__ x, T* __restrict__ out, int nx, int ny, int nz, int n,
                                  int nl, int side, int hermite_like) {
    const int n2 = n * n;
    const int64_t total = int64_t(nx) * ny * nl * n2;
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int r = int(o % n2), j = int((o / n2) % nl);
    const int64_t c = o / (int64_t(nl) * n2);
    const int iz = side ? nz - 1 : 0;
    const int layer = hermite_like ? (side ? n - 2 + j : j) : j;
    const int64_t cell = c + int64_t(nx) * ny * iz;
    out[o] = x[cell * n2 * n + r + int64_t(n2) * layer];
}

int launch_pack_ghost(const sipg_op* op, int side, const void* x, void* out, hipStream_t st) {
    const int n = op->n, nl = op->basis == SIPG_BASIS_HERMITE_LIKE ? 2 : n;
    const int64_t total = int64_t(op->nc[0]) * op->nc[1] * nl * n * n;
    const int bs = 256;
    const unsigned g = unsigned((total + bs - 1) / bs);
    const int hl = op->basis == SIPG_BASIS_HERMITE_LIKE;
    if (op->dtype == SIPG_F64)
        pack_ghost_kernel<double><<<g, bs, 0, st>>>(static_cast<const double*>(x), static_cast<double*>(out),
                                                    op->nc[0], op->nc[1], op->nc[2], n, nl, side, hl);
    else
        pack_ghost_kernel<float><<<g, bs, 0, st>>>(static_cast<const float*>(x), static_cast<float*>(out), op->nc[0],
                                                   op->nc[1], op->nc[2], n, nl, side, hl);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

}  // namespace sipg
