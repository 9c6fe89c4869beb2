// Bandwidth bound of the product step: a kernel that moves exactly the bytes
// of sipg_apply_pjacobi -- x, the cell and face metric terms and 1/diag(A_GL)
// read once, y and z written once -- with no arithmetic, each workgroup
// reading one contiguous share of every array in 16-byte pieces.  Its time
// is what the step would take if it were limited by HBM alone, so the ratio
// of the two measures how far the step's access pattern and arithmetic are
// from the memory system's own limit for that mix of reads and writes
// (Section 5 relates throughput to the data each unknown moves).
#include "sipg_common.hpp"
#include "setup.hpp"

namespace sipg {

constexpr int kSbThreads = 256;
constexpr int kSbArrays = 6;   // x, cell metric, face metric (3 directions), 1/diag

struct SbArrays {
    const uint4* in[kSbArrays];
    int64_t in_units[kSbArrays];   // 16-byte pieces of each input
    uint4* out[2];                 // y, z
    int64_t out_units;
};

// Workgroup b streams pieces [n b / nb, n (b+1) / nb) of every array; each
// round issues one 16-byte load per input and thread before the sum of the
// round is formed, and the sum of all rounds is written to y and z.
__global__ void __launch_bounds__(kSbThreads) stream_bound_kernel(SbArrays a) {
    const int64_t b = blockIdx.x, nb = gridDim.x;
    int64_t lo[kSbArrays], hi[kSbArrays];
    int64_t rounds = 0;
#pragma unroll
    for (int k = 0; k < kSbArrays; ++k) {
        lo[k] = a.in_units[k] * b / nb;
        hi[k] = a.in_units[k] * (b + 1) / nb;
        const int64_t r = (hi[k] - lo[k] + kSbThreads - 1) / kSbThreads;
        rounds = r > rounds ? r : rounds;
    }
    uint32_t acc = 0;
    for (int64_t r = 0; r < rounds; ++r) {
        uint4 v[kSbArrays];
#pragma unroll
        for (int k = 0; k < kSbArrays; ++k) {
            const int64_t i = lo[k] + r * kSbThreads + threadIdx.x;
            v[k] = i < hi[k] ? a.in[k][i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < kSbArrays; ++k) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
    }
    const int64_t n = a.out_units;
    const int64_t olo = n * b / nb, ohi = n * (b + 1) / nb;
    for (int64_t i = olo + threadIdx.x; i < ohi; i += kSbThreads) {
        a.out[0][i] = make_uint4(acc, acc, acc, acc);
        a.out[1][i] = make_uint4(acc, 0, acc, 0);
    }
}

int launch_stream_bound(const sipg_op* op, const void* x, void* y, void* z, hipStream_t st) {
    const size_t esz = op->dtype == SIPG_F64 ? 8 : 4;
    const int n = op->n;
    SbArrays a{};
    const void* in[kSbArrays] = {x, op->cell_geom, op->face_geom[0], op->face_geom[1], op->face_geom[2],
                                 op->gl_inv_diag};
    const size_t bytes[kSbArrays] = {
        esz * size_t(op->ndofs), esz * size_t(op->ncells) * cell_geom_stride(op->geom, n),
        esz * size_t(op->nfaces[0]) * face_geom_stride(op->geom, n),
        esz * size_t(op->nfaces[1]) * face_geom_stride(op->geom, n),
        esz * size_t(op->nfaces[2]) * face_geom_stride(op->geom, n), esz * size_t(op->ndofs)};
    size_t total = 0;
    for (int k = 0; k < kSbArrays; ++k) {
        a.in[k] = static_cast<const uint4*>(in[k]);
        a.in_units[k] = int64_t(bytes[k] / 16);   // a tail below 16 bytes is left out
        total += bytes[k];
    }
    a.out[0] = static_cast<uint4*>(y);
    a.out[1] = static_cast<uint4*>(z);
    a.out_units = int64_t(esz * size_t(op->ndofs) / 16);
    // about 64 KiB of input per workgroup (16 rounds of 256 pieces)
    const int64_t nb = std::max<int64_t>(1, int64_t(total / 65536));
    stream_bound_kernel<<<unsigned(nb), kSbThreads, 0, st>>>(a);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

}  // namespace sipg
