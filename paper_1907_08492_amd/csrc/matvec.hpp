// Element-wise matrix-free SIPG product y = A x on gfx950 (Section 3).
//
// One workgroup of three wavefronts handles CPB consecutive cells.  Every
// step maps one thread to one n-long pencil (of a cell or of a face array)
// held in registers; the 1D contraction along the pencil is an even-odd
// multiply-add sweep with coefficients in scalar registers, and the change of
// pencil direction between sweeps goes through LDS.
//
// Face integrals (eq. tensor_face, element-wise arrangement): wavefront d
// works on the two faces of normal direction d of every cell, so the
// direction is a compile-time constant inside its code, and each lane owns
// one row (t1 direction) and one column (t2 direction) of one face:
//   G1  gather the own value/derivative layers (LDS), combine them with S_f
//       and D_f and interpolate along t1 (S, and S' for values); combine the
//       neighbour's layers (registers loaded at kernel start: two layers for
//       the Hermite-like basis, all n for the nodal bases) into its value
//       and derivative rows
//   F1  own side along t2 (S, and D for the tangential derivative), reduced
//       to u- and the normal flux at the face Gauss points, kept in registers
//   G2  neighbour side along t1, written over the own side's arrays
//   F2  neighbour side along t2, flux at the face Gauss points, transposed
//       sweeps along t2
//   I   transposed sweeps along t1 -> P (value test) and Q (normal-derivative
//       test) coefficient arrays of the face
// The face steps of a direction stay inside its wavefront (wavefront-level
// syncs); where a wavefront holds whole cells, so do the cell steps.
// Cell integral: S along z, y, x, collocation D along x, y, z (eq.
// tensor_cell), merged metric at the points (eq. integral_laplace),
// transposed sweeps back; the last sweep adds e_layer (x) P + D_f (x) Q of
// the six faces and writes y_K once.
// Affine cells (Section 3 notes the reduction): with per-cell records the
// face terms are Kronecker products in reference coordinates, and with a
// diagonal metric so is the cell term.
#pragma once

#include <type_traits>

#include "sipg_common.hpp"
#include "sumfac.hpp"

namespace sipg {

template <typename T>
struct MatvecParams {
    const T* __restrict__ x;
    T* __restrict__ y;
    const T* __restrict__ tab;
    const T* __restrict__ cgeom;
    const T* __restrict__ fgeom0;
    const T* __restrict__ fgeom1;
    const T* __restrict__ fgeom2;
    int nx, ny, nz;
    int ncells;
    // epilogues (see matvec_block): P^-1 data (1 / diag(A_GL) per unknown,
    // or the 4 block-Jacobi scalars per cell), output z, and the Chebyshev
    // step's right-hand side b, output uo and coefficients
    const T* __restrict__ dinv;
    T* __restrict__ z;
    const T* __restrict__ b;
    T* __restrict__ uo;
    double sigma, theta;   // double in both precisions: one parameter layout
    // slab of a z-partition: the neighbour layers across its lower / upper
    // z boundary (null: a boundary face of the mesh), NL layers of n^2 values
    // per (x, y) column
    const T* __restrict__ ghost_lo;
    const T* __restrict__ ghost_hi;
};

// Epilogues of the product kernel, applied per cell once y = A x is known:
// EPI_PJACOBI writes y and z = P^-1 y (eq. (jacobi), point Jacobi in the GL
// basis); EPI_CHEB_PJ / EPI_CHEB_FDM do not write y but one step of the
// Chebyshev iteration of eq. (chebyshev) with u = x:
//     uo <- u + sigma (u - uo) + theta P^-1 (b - A u)
// with P^-1 the point Jacobi or the block Jacobi of Section 6.4 (the
// "merged" arrangement of Section 6 fused into the product).
enum { EPI_NONE = 0, EPI_PJACOBI = 1, EPI_CHEB_PJ = 2, EPI_CHEB_FDM = 3 };

// Kernel parameters of operator `op` for the product y = A x.
template <typename T>
inline MatvecParams<T> matvec_params(const sipg_op* op, const void* x, void* y) {
    MatvecParams<T> p;
    p.x = static_cast<const T*>(x);
    p.y = static_cast<T*>(y);
    p.tab = static_cast<const T*>(op->tables);
    p.cgeom = static_cast<const T*>(op->cell_geom);
    p.fgeom0 = static_cast<const T*>(op->face_geom[0]);
    p.fgeom1 = static_cast<const T*>(op->face_geom[1]);
    p.fgeom2 = static_cast<const T*>(op->face_geom[2]);
    p.nx = op->nc[0];
    p.ny = op->nc[1];
    p.nz = op->nc[2];
    p.ncells = int(op->ncells);
    p.dinv = nullptr;
    p.z = nullptr;
    p.b = nullptr;
    p.uo = nullptr;
    p.sigma = 0.0;
    p.theta = 0.0;
    p.ghost_lo = nullptr;
    p.ghost_hi = nullptr;
    return p;
}

template <int N>
struct Shape {
    static constexpr int N2 = N * N, N3 = N * N * N;
    static constexpr int RS = (N % 2 == 0) ? N + 1 : N;   // LDS row stride (odd: no bank aliasing)
    static constexpr int CS = RS * N * N;                  // one cell array in LDS
    static constexpr int CPB = cells_per_block(N);
    static constexpr int NT = threads_per_block(N);
    static constexpr int FROWS = CPB * 2 * N;              // face rows (= columns) per direction
    static constexpr int FR = face_row_stride(N);          // row stride of a face array
    static constexpr int FARR = N * FR;                    // one face array (all faces of a direction)
    // words of T per workgroup: the x/work arrays, then 9 face arrays; in the
    // cell steps arrays FV, FT of every direction persist and the cell arrays
    // B, C start at the FN arrays
    static constexpr int WORDS = CPB * CS + (9 * FARR > 6 * FARR + 2 * CPB * CS ? 9 * FARR : 6 * FARR + 2 * CPB * CS);
    __host__ __device__ static constexpr int lds_idx(int i1, int i2, int i3) { return i1 + RS * (i2 + N * i3); }
};

template <int N, typename T>
constexpr size_t matvec_lds_bytes() {
    using S = Shape<N>;
    constexpr size_t b = size_t(S::WORDS) * sizeof(T);
    static_assert(b == matvec_lds_bytes_rt(N, sizeof(T)), "LDS size formula mismatch");
    static_assert(S::FR >= S::FROWS, "face row holds every face of a direction");
    static_assert(b <= 160 * 1024, "LDS budget of a gfx950 CU exceeded");
    static_assert(S::NT == 192 && S::CPB * N * N <= S::NT, "three wavefronts, one pencil per thread");
    static_assert(S::FROWS <= 64, "one face row per lane of a direction wavefront");
    return b;
}

// Coordinates of cell0 + c from those of cell0 (cells of a workgroup are
// consecutive in the lexicographic order; c is small).
__device__ __forceinline__ void cell_coords(int bx, int by, int bz, int c, int nx, int ny, int& ix, int& iy, int& iz) {
    ix = bx + c;
    iy = by;
    iz = bz;
    while (ix >= nx) {
        ix -= nx;
        if (++iy == ny) { iy = 0; ++iz; }
    }
}

// Neighbour cell across face f = 2d+s of the cell (ix,iy,iz) (-1 on the
// boundary) and the index of that face in the face arrays of direction d.
__device__ __forceinline__ void face_topology(int ix, int iy, int iz, int f, int nx, int ny, int nz, int& nb, int& fi) {
    const int d = f >> 1, s = f & 1;
    const int cell = ix + nx * (iy + ny * iz);
    int idx[3] = {ix, iy, iz};
    const int nd[3] = {nx, ny, nz};
    const int j = idx[d] + (s ? 1 : -1);
    nb = (j >= 0 && j < nd[d]) ? cell + (s ? 1 : -1) * (d == 0 ? 1 : d == 1 ? nx : nx * ny) : -1;
    idx[d] += s;
    if (d == 0) fi = idx[0] + (nx + 1) * (idx[1] + ny * idx[2]);
    else if (d == 1) fi = idx[0] + nx * (idx[1] + (ny + 1) * idx[2]);
    else fi = idx[0] + nx * (idx[1] + ny * idx[2]);
}

// basis: 0 Hermite-like (derivative rows touch layers {0,1} / {n-2,n-1}),
//        1 nodal Gauss-Lobatto (derivative rows touch every layer),
//        2 nodal Gauss (value and derivative rows touch every layer).
template <int N, int BASIS>
struct Layers {
    static constexpr int NL = (BASIS == 0) ? 2 : N;
    // j-th layer of the derivative support at side s
    __host__ __device__ static constexpr int layer(int s, int j) { return BASIS == 0 ? (s ? N - 2 + j : j) : j; }
};

// Index in a cell array of (layer l along direction D, tangential t1 = a, t2 = b).
template <int N, int D>
__device__ __forceinline__ constexpr int face_lidx(int l, int a, int b) {
    using Sh = Shape<N>;
    return D == 0 ? Sh::lds_idx(l, a, b) : D == 1 ? Sh::lds_idx(a, l, b) : Sh::lds_idx(a, b, l);
}
template <int N, int D>
__device__ __forceinline__ constexpr int face_gidx(int l, int a, int b) {
    return D == 0 ? l + N * (a + N * b) : D == 1 ? a + N * (l + N * b) : a + N * (b + N * l);
}

template <int D>
using DirC = std::integral_constant<int, D>;

// Calls fn(DirC<d>) with d the (wavefront-uniform) direction of this wave.
template <typename F>
__device__ __forceinline__ void by_direction(int wave, F&& fn) {
    if (wave == 0) fn(DirC<0>{});
    else if (wave == 1) fn(DirC<1>{});
    else fn(DirC<2>{});
}

// Orders the LDS accesses of one wavefront before and after it (the lanes of
// a wavefront exchange data through LDS without a workgroup barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Minimum wavefronts per SIMD requested from the register allocator: two for
// n >= 7 with per-cell metric terms, so that two workgroups share a compute
// unit (the few spilled registers cost less than the idle SIMD); with
// per-point metric terms the spill traffic would compete with the HBM
// stream, so those keep one.  The FP32 Hermite-like per-point kernels at
// n = 6 fit five wavefronts per SIMD without spills (95 registers instead of
// 100), which lets the LDS limit of six workgroups per compute unit bind.
template <int N, int BASIS, typename T, int GEOM>
constexpr int matvec_min_waves() {
    return (N >= 7 && GEOM != GEOM_QPOINT) ? 2 : (N == 6 && BASIS == 0 && sizeof(T) == 4 && GEOM == GEOM_QPOINT) ? 5 : 1;
}

// XCD-aware order: consecutive workgroups are dispatched round-robin over
// the 8 XCDs, so give each XCD a contiguous range of block indices (a range
// of consecutive cells, whose x- and y-neighbours then meet in that XCD's L2).
// Workgroup blk is the sl-th of its XCD, whose range starts at `start` and
// holds `len` blocks.
struct XcdSlot { int start, len, sl; };
__host__ __device__ __forceinline__ XcdSlot xcd_slot(int blk, int nblk) {
    const int per = (nblk + 7) / 8;
    const int xcd = blk % 8, sl = blk / 8;
    const int full = nblk % 8 == 0 ? 8 : nblk % 8;   // XCDs that get `per` blocks
    return {xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1), xcd < full ? per : per - 1, sl};
}
__host__ __device__ __forceinline__ int xcd_block(int blk, int nblk) {
    const XcdSlot x = xcd_slot(blk, nblk);
    return x.start + x.sl;
}

// The same, with the blocks of up to eight consecutive z-layers interleaved
// inside each XCD's range: with P blocks per layer, the range is cut into
// groups of TZ P blocks (TZ = min(8, layers in the range)), and a group is
// visited column by column: block j of its first, second, ... layer, then
// block j + 1 of each, and so on (a transpose of the TZ x P group; the last
// group, with fewer layers and a shorter last row, is transposed the same
// way).  In the lexicographic order a z-neighbour is P blocks away, beyond
// what one XCD's L2 holds while it streams the blocks in between;
// interleaved, the two cells of a z-face are read TZ - 1 or fewer blocks
// apart, and the two XCDs that share the plane between their ranges reach it
// at the same time.  y-neighbours, about TZ rows of blocks apart, are then
// read again from the memory-side cache rather than from HBM.
__host__ __device__ __forceinline__ int xcd_block_zinterleaved(int blk, int nblk, int P) {
    const XcdSlot x = xcd_slot(blk, nblk);
    if (P <= 0) return x.start + x.sl;
    const int TZ = (x.len + P - 1) / P < 8 ? (x.len + P - 1) / P : 8;
    const int G = TZ * P;
    const int g = x.sl / G, s = x.sl - g * G;
    const int m = G < x.len - g * G ? G : x.len - g * G;   // blocks of this group
    const int tz = (m + P - 1) / P;               // its layers
    const int r = m - (tz - 1) * P;               // blocks of its last layer
    int row, col;
    if (s < r * tz) {
        col = s / tz;
        row = s - col * tz;
    } else {                                      // tz > 1 here
        const int t = s - r * tz;
        col = r + t / (tz - 1);
        row = t - (col - r) * (tz - 1);
    }
    return x.start + g * G + row * P + col;
}

// The product on workgroup `blk` of the operator `p`: cells blk*CPB ...,
// followed by the epilogue EPI on each cell (EPI_NONE: y only).  voff moves
// every vector access (x, y, z, b, uo) by that many entries: one of several
// right-hand sides stored one after another.  (The parameter block itself is
// not changed: a modified copy of it would be kept in scratch memory.)
template <int N, int BASIS, typename T, int GEOM, int EPI = EPI_NONE>
__device__ __forceinline__ void matvec_block(const MatvecParams<T>& p, const int blk, const size_t voff = 0) {
    using Sh = Shape<N>;
    using Ly = Layers<N, BASIS>;
    constexpr int N2 = Sh::N2, N3 = Sh::N3, RS = Sh::RS, CS = Sh::CS, FR = Sh::FR;
    constexpr int CPB = Sh::CPB, NT = Sh::NT;
    constexpr TableLayout TL(N);
    // nodal Gauss basis: S = I, dense face value rows
    constexpr bool COLLOC = BASIS == 2;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    T* ldsX = lds;                                   // [CPB][CS]   x, later the cell work array A
    // Face arrays [3 arrays][3 directions][n rows][FR]: a row holds that row
    // of every (cell, side) face of the direction, (2 cell + side) n + column.
    // Arrays FV, FT (P, Q at the end of the face steps) persist; the cell
    // arrays B, C start at the FN arrays.
    T* ldsF = lds + CPB * CS;

    const auto tab = ctab(p.tab);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // = face direction in the face steps
    const int lane = tid & 63;
    const int cell0 = blk * CPB;
    const int ncb = min(CPB, p.ncells - cell0);      // cells in this workgroup
    const int bx = cell0 % p.nx, by = (cell0 / p.nx) % p.ny, bz = cell0 / (p.nx * p.ny);

    auto fel = [&](int m, int d, int c, int s) -> T* { return ldsF + (m * 3 + d) * Sh::FARR + (2 * c + s) * N; };

    // Face item of this lane (the same in the three face steps): cell fc,
    // side fs (face f = 2 wave + fs), row / column index fab.
    const int fc = lane / (2 * N), fs = (lane / N) & 1, fab = lane % N;
    const bool fact = lane < ncb * 2 * N;
    int fnb = -1, fidx = 0;
    int gcol = -1;                   // (x, y) column of a ghost neighbour (slab z boundary)
    if (fact) {
        int ix, iy, iz;
        cell_coords(bx, by, bz, fc, p.nx, p.ny, ix, iy, iz);
        face_topology(ix, iy, iz, 2 * wave + fs, p.nx, p.ny, p.nz, fnb, fidx);
        if (wave == 2 && fnb < 0 && (fs ? p.ghost_hi : p.ghost_lo)) gcol = ix + p.nx * iy;
    }

    // The workgroup's x tile, one contiguous range, as XPER loads per thread
    // issued back to back.
    constexpr int XPER = (CPB * N3 + NT - 1) / NT;
    T xv[XPER];
    {
        const T* __restrict__ xs = p.x + voff + size_t(cell0) * N3;
#pragma unroll
        for (int j = 0; j < XPER; ++j) {
            const int e = tid + j * NT;
            xv[j] = e < ncb * N3 ? xs[e] : T(0);
        }
    }

    // ------------------------------------------------------------ prefetch
    // Registers, before any LDS work: the metric terms of this lane's flux
    // column (used in F1, F2) and the neighbour layers of this lane's row
    // (used in G1).
    // For n >= 7 (FP64) the registers are needed by the sweeps: the face
    // records are then loaded in two parts, at the start of steps F1 and G2,
    // and the cell metric terms at the start of C4.
    constexpr bool EARLY = N <= 6 || sizeof(T) == 4;
    constexpr int NREC = GEOM != GEOM_QPOINT ? 7 : 7 * N;
    // frec: the penalty term, this lane's own side scaled normal (3
    // components), the neighbour side's (3); the side slots of the stored
    // record (lower cell first) are chosen here, by the load addresses.
    T frec[NREC];
    T nbv[Ly::NL][N];
    // part 1: own side normal (used from F1 on); part 2: penalty term and
    // neighbour side normal (used in F2)
    auto load_frec = [&](auto dc, int part) {
        constexpr int D = decltype(dc)::value;
        const T* __restrict__ fg = D == 0 ? p.fgeom0 : D == 1 ? p.fgeom1 : p.fgeom2;
        const int own = fs ? 1 : 4, nb = fs ? 4 : 1;
        if constexpr (GEOM != GEOM_QPOINT) {
            const T* __restrict__ r = fg + size_t(fidx) * 8;
            if (part & 1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) frec[1 + k] = r[own + k];
            }
            if (part & 2) {
                frec[0] = r[0];
#pragma unroll
                for (int k = 0; k < 3; ++k) frec[4 + k] = r[nb + k];
            }
        } else {
            // plane-major records (face_rec_offset): this lane's column a =
            // fab is read as CH-point chunks along t2, one plane per chunk;
            // the lanes of consecutive faces read consecutive 16-byte pieces
            constexpr int CH = 16 / int(sizeof(T)), J = N / CH, R = N % CH;
            const size_t nf = D == 0 ? size_t(p.nx + 1) * p.ny * p.nz
                              : D == 1 ? size_t(p.nx) * (p.ny + 1) * p.nz : size_t(p.nx) * p.ny * (p.nz + 1);
            const T* __restrict__ rc = fg + (size_t(fidx) * N + fab) * CH;
            const T* __restrict__ rt = fg + size_t(7 * J * CH * N) * nf + (size_t(fidx) * N + fab) * R;
            auto comp = [&](int k, T* dst) {
#pragma unroll
                for (int j = 0; j < J; ++j) load_run<CH>(rc + size_t(k * J + j) * nf * (CH * N), dst + j * CH);
                if constexpr (R > 0) load_run<R>(rt + size_t(k) * nf * (R * N), dst + J * CH);
            };
            if (part & 1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) comp(own + k, frec + (1 + k) * N);
            }
            if (part & 2) {
                comp(0, frec);
#pragma unroll
                for (int k = 0; k < 3; ++k) comp(nb + k, frec + (4 + k) * N);
            }
        }
    };
    by_direction(wave, [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        if (!fact) return;
        // x-neighbours inside the workgroup are read from the x tile in G1;
        // the neighbour layers go first, as G1 needs them before F1 needs
        // the face records
        if (fnb >= 0 && !(D == 0 && (fs ? fc + 1 < ncb : fc > 0))) {
            // runs of consecutive values: the layers (x faces, whose layers
            // are contiguous), else each layer's row
            const T* __restrict__ xn = p.x + voff + size_t(fnb) * N3;
            if constexpr (D == 0) {
                const int l0 = Ly::layer(1 - fs, 0);
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    T run[Ly::NL];
                    load_run<Ly::NL>(xn + face_gidx<N, 0>(l0, a, fab), run);
#pragma unroll
                    for (int j = 0; j < Ly::NL; ++j) nbv[j][a] = run[j];
                }
            } else {
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) load_run<N>(xn + face_gidx<N, D>(Ly::layer(1 - fs, j), 0, fab), nbv[j]);
            }
        }
        if constexpr (D == 2) {
            // a neighbour in another slab: its layers Ly::layer(1 - fs, j)
            // packed per column (sipg_pack_ghost), in the same row order
            if (gcol >= 0) {
                const T* __restrict__ xn = (fs ? p.ghost_hi : p.ghost_lo) + size_t(gcol) * (Ly::NL * N2);
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) load_run<N>(xn + face_gidx<N, D>(j, 0, fab), nbv[j]);
            }
        }
        if constexpr (EARLY) load_frec(dc, 3);
    });
    // --------------------------------------------------------------- x tile
    // (loaded into registers at kernel start, with every other load of the
    // workgroup in flight; written to LDS here)
#pragma unroll
    for (int j = 0; j < XPER; ++j) {
        const int e = tid + j * NT;
        if (e < ncb * N3) {
            const int c = e / N3, i = e % N3;
            ldsX[c * CS + Sh::lds_idx(i % N, (i / N) % N, i / N2)] = xv[j];
        }
    }
    __syncthreads();

    // Face steps G1, F1, G2, F2, I.  Wavefront d touches only the face arrays
    // of direction d, so the steps are separated by wavefront-level syncs; the
    // block barrier comes before the cell steps, which read every direction.
    // Array roles: FV value, FT t1 derivative, FN normal derivative; the own
    // side's arrays are consumed (F1) before the neighbour side's are written
    // (G2) into the same place.
    constexpr int FV = 0, FT = 1, FN = 2;
    // Per-cell (affine) records use the reference-coordinate face step below
    // in the Hermite-like basis.  The nodal bases keep the quadrature face
    // steps: the Gauss basis has no interpolation sweeps to save there, and
    // for both the dense n-layer face rows dominate (measured: no gain for
    // Gauss-Lobatto, a loss for Gauss).
    constexpr bool KRON = GEOM != GEOM_QPOINT && BASIS == 0;
    by_direction(wave, [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        constexpr int t1 = D == 0 ? 1 : 0, t2 = D == 2 ? 1 : 2;
        const int s = fs, c = fc, rc = fab;   // rc: this lane's row (G) / column (F)
        const bool interior = fnb >= 0 || gcol >= 0;
        T r[N];
        auto put_row = [&](int m, const T* v) {
            T* o = fel(m, D, c, s) + rc * FR;
#pragma unroll
            for (int q = 0; q < N; ++q) o[q] = v[q];
        };
        auto col = [&](int m, T* v) {
            const T* src = fel(m, D, c, s) + rc;
#pragma unroll
            for (int q = 0; q < N; ++q) v[q] = src[q * FR];
        };
        // Face record of this lane's face: penalty term, own side (g-) and
        // neighbour side (g+) scaled normals in the cell's reference
        // coordinates, at point b of the lane's column (per-point records) or
        // constant (per-cell records, without the point weights).  The stored
        // normal points from the lower to the upper cell of the face; sg turns
        // it outward for this side and is applied once per point.
        const T sg = s ? T(1) : T(-1);
        auto pen = [&](int b) -> T { return GEOM != GEOM_QPOINT ? frec[0] : frec[b]; };
        auto gmn = [&](int k, int b) -> T { return GEOM != GEOM_QPOINT ? frec[1 + k] : frec[(1 + k) * N + b]; };
        auto gpn = [&](int k, int b) -> T { return GEOM != GEOM_QPOINT ? frec[4 + k] : frec[(4 + k) * N + b]; };
        // Row rc (points a along t1) of the own value and normal-derivative
        // layers, combined with S_f and D_f from the LDS x tile.
        auto own_rows = [&](T* vm, T* nm) {
            const int b = rc;
            const T* Xc = ldsX + c * CS;
            const auto dfs = tab + (s ? TL.df1 : TL.df0);
            const auto fvs = tab + (s ? TL.FV1 : TL.FV0);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                T acc = T(0), val = T(0);
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) {
                    const int l = Ly::layer(s, j);
                    const T xl = Xc[face_lidx<N, D>(l, a, b)];
                    acc = fma(dfs[l], xl, acc);
                    if constexpr (COLLOC) val = fma(fvs[l], xl, val);
                }
                if constexpr (!COLLOC) val = Xc[face_lidx<N, D>(s ? N - 1 : 0, a, b)];
                vm[a] = val;
                nm[a] = acc;
            }
        };
        // The same rows of the neighbour (interior faces): its value layer
        // touches the face; its derivative row combines the layers loaded at
        // kernel start, or read from the x tile for an x-neighbour inside the
        // workgroup.
        auto neighbour_rows = [&](T* vp, T* np) {
            const int b = rc;
            if (D == 0 && (s ? c + 1 < ncb : c > 0)) {
                const T* Xn = ldsX + (s ? c + 1 : c - 1) * CS;
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) {
                    const int l = Ly::layer(1 - s, j);
#pragma unroll
                    for (int a = 0; a < N; ++a) nbv[j][a] = Xn[face_lidx<N, 0>(l, a, b)];
                }
            }
            const auto dfn = tab + (s ? TL.df0 : TL.df1);
            const auto fvn = tab + (s ? TL.FV0 : TL.FV1);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                T acc = T(0), val = T(0);
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) {
                    const int l = Ly::layer(1 - s, j);
                    acc = fma(dfn[l], nbv[j][a], acc);
                    if constexpr (COLLOC) val = fma(fvn[l], nbv[j][a], val);
                    else if (l == (s ? 0 : N - 1)) val = nbv[j][a];
                }
                vp[a] = val;
                np[a] = acc;
            }
        };
        if constexpr (KRON) {
            // ---- Affine face (constant J on the face and in both cells; the
            // per-cell records are weight-free constants).  The face terms in
            // reference coordinates are Kronecker products of the 1D matrices
            // M = S^T W S, Ct = S^T W S', Cs = S'^T W S (t1 factor first),
            // exact with the n-point Gauss rule (Section 3, affine cells):
            //   P = (M x M) A + (Ct x M) T1 + (M x Ct) T2 + h g1 (Cs x M) J + h g2 (M x Cs) J
            //   Q = h gn (M x M) J
            // with J = U- - U+, A = pen J + h (gn- N- + gn+ N+),
            // Tk = h (gk- U- + gk+ U+) and h = -sg/2; U, N the value and
            // normal-derivative layers, g the scaled normals (mirror principle
            // on the boundary: U+ = -U- in J, the gradient of u+ that of u-).
            // The t1 products run along this lane's row, the t2 products along
            // its column; no quadrature-point stage.
            const T hs = T(-0.5) * sg;
            if (fact) {
                if constexpr (!EARLY) load_frec(dc, 3);
                // gathered and combined point by point (fewer live registers)
                const int b = rc;
                const T* Xc = ldsX + c * CS;
                const bool inwg = D == 0 && (s ? c + 1 < ncb : c > 0);   // x-neighbour in the workgroup
                const T* Xn = ldsX + (inwg ? (s ? c + 1 : c - 1) : c) * CS;
                const auto dfs = tab + (s ? TL.df1 : TL.df0), fvs = tab + (s ? TL.FV1 : TL.FV0);
                const auto dfn = tab + (s ? TL.df0 : TL.df1), fvn = tab + (s ? TL.FV0 : TL.FV1);
                T jc[N], av[N], t1v[N], t2v[N], q[N];
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    T vm = T(0), nm = T(0), vp = T(0), np = T(0);
#pragma unroll
                    for (int j = 0; j < Ly::NL; ++j) {
                        const int l = Ly::layer(s, j), ln = Ly::layer(1 - s, j);
                        const T xl = Xc[face_lidx<N, D>(l, a, b)];
                        nm = fma(dfs[l], xl, nm);
                        if constexpr (COLLOC) vm = fma(fvs[l], xl, vm);
                        if (interior) {
                            const T xn = inwg ? Xn[face_lidx<N, 0>(ln, a, b)] : nbv[j][a];
                            np = fma(dfn[ln], xn, np);
                            if constexpr (COLLOC) vp = fma(fvn[ln], xn, vp);
                            else if (ln == (s ? 0 : N - 1)) vp = xn;
                        }
                    }
                    if constexpr (!COLLOC) vm = Xc[face_lidx<N, D>(s ? N - 1 : 0, a, b)];
                    const T ug = interior ? vp : vm;    // u+ in its gradient
                    const T ng = interior ? np : nm;
                    jc[a] = interior ? vm - vp : vm + vm;
                    av[a] = pen(0) * jc[a] + hs * (gmn(D, 0) * nm + gpn(D, 0) * ng);
                    t1v[a] = hs * (gmn(t1, 0) * vm + gpn(t1, 0) * ug);
                    t2v[a] = hs * (gmn(t2, 0) * vm + gpn(t2, 0) * ug);
                }
                eo_apply<N, +1>(tab + TL.MM, av, r);
                eo_apply<N, -1>(tab + TL.CT, t1v, q);
#pragma unroll
                for (int a = 0; a < N; ++a) r[a] += q[a];
                eo_apply<N, -1>(tab + TL.CS, jc, q);
                const T h1 = hs * gmn(t1, 0);
#pragma unroll
                for (int a = 0; a < N; ++a) r[a] = fma(h1, q[a], r[a]);
                put_row(FV, r);
                eo_apply<N, +1>(tab + TL.MM, t2v, r);
                put_row(FT, r);
                eo_apply<N, +1>(tab + TL.MM, jc, r);
                put_row(FN, r);
            }
            wave_sync();
            if (fact) {
                const int a = rc;                  // this lane's column
                T r1[N], r2[N], mj[N], pv[N], q[N];
                col(FV, r1);
                col(FT, r2);
                col(FN, mj);
                eo_apply<N, +1>(tab + TL.MM, r1, pv);
                eo_apply<N, -1>(tab + TL.CT, r2, q);
#pragma unroll
                for (int b = 0; b < N; ++b) pv[b] += q[b];
                eo_apply<N, -1>(tab + TL.CS, mj, q);
                const T h2 = hs * gmn(t2, 0);
#pragma unroll
                for (int b = 0; b < N; ++b) pv[b] = fma(h2, q[b], pv[b]);
                eo_apply<N, +1>(tab + TL.MM, mj, q);
                const T hn = hs * gmn(D, 0);
                T* s0 = fel(FV, D, c, s) + a;
                T* s1 = fel(FT, D, c, s) + a;
#pragma unroll
                for (int b = 0; b < N; ++b) { s0[b * FR] = pv[b]; s1[b * FR] = hn * q[b]; }
            }
        } else {
        // ---- G1: own value and normal-derivative layers of row rc, S and S'
        // along t1; the neighbour's layers combined into its value and
        // derivative rows (vp, np) for G2
        T vp[N], np[N];
        if (fact) {
            T vm[N], nm[N];
            own_rows(vm, nm);
            s_apply<N, COLLOC>(tab + TL.S, vm, r);
            put_row(FV, r);
            eo_apply<N, -1>(tab + TL.SG, vm, r);
            put_row(FT, r);
            s_apply<N, COLLOC>(tab + TL.S, nm, r);
            put_row(FN, r);
            if (interior) neighbour_rows(vp, np);
        }
        wave_sync();
        // ---- F1: own side along t2 at the face points (u, and du/dn, du/dt1
        // by S, du/dt2 by D after S), reduced to u- and the normal flux
        // g-.grad u-.  On a boundary face the mirror principle gives the
        // neighbour the same gradient and the same scaled normal, so its
        // normal flux equals the own one.
        T um[N], dsum[N];
        if (fact) {
            if constexpr (!EARLY) load_frec(dc, 1);
            // one derivative component at a time: u, du/dt2 = D u, du/dn, du/dt1
            T g[N];
            col(FV, um); s_apply<N, COLLOC>(tab + TL.S, um, um);
            eo_apply<N, -1>(tab + TL.D, um, g);
#pragma unroll
            for (int b = 0; b < N; ++b) dsum[b] = gmn(t2, b) * g[b];
            col(FN, g); s_apply<N, COLLOC>(tab + TL.S, g, g);
#pragma unroll
            for (int b = 0; b < N; ++b) dsum[b] = fma(gmn(D, b), g[b], dsum[b]);
            col(FT, g); s_apply<N, COLLOC>(tab + TL.S, g, g);
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const T dm = fma(gmn(t1, b), g[b], dsum[b]);
                dsum[b] = interior ? dm : dm + dm;
            }
        }
        wave_sync();
        // ---- G2: neighbour rows along t1
        if (fact) {
            if constexpr (!EARLY) load_frec(dc, 2);
            if (interior) {
                s_apply<N, COLLOC>(tab + TL.S, vp, r);
                put_row(FV, r);
                eo_apply<N, -1>(tab + TL.SG, vp, r);
                put_row(FT, r);
                s_apply<N, COLLOC>(tab + TL.S, np, r);
                put_row(FN, r);
            }
        }
        wave_sync();
        // ---- F2: neighbour side along t2, flux at the points, S^T / D^T
        // along t2
        if (fact) {
            const int a = rc;                  // this lane's column
            T up[N];
            if (interior) {
                T g[N];
                col(FV, up); s_apply<N, COLLOC>(tab + TL.S, up, up);
                eo_apply<N, -1>(tab + TL.D, up, g);
#pragma unroll
                for (int b = 0; b < N; ++b) dsum[b] = fma(gpn(t2, b), g[b], dsum[b]);
                col(FN, g); s_apply<N, COLLOC>(tab + TL.S, g, g);
#pragma unroll
                for (int b = 0; b < N; ++b) dsum[b] = fma(gpn(D, b), g[b], dsum[b]);
                col(FT, g); s_apply<N, COLLOC>(tab + TL.S, g, g);
#pragma unroll
                for (int b = 0; b < N; ++b) dsum[b] = fma(gpn(t1, b), g[b], dsum[b]);
            } else {
                // mirror principle: u+ = -u-
#pragma unroll
                for (int b = 0; b < N; ++b) up[b] = -um[b];
            }
            T vv[N], wd[N], w1[N], w2[N];
            const T hs = T(-0.5) * sg;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const T jump = um[b] - up[b];
                vv[b] = pen(b) * jump + hs * dsum[b];
                const T hj = hs * jump;
                wd[b] = hj * gmn(D, b);
                w1[b] = hj * gmn(t1, b);
                w2[b] = hj * gmn(t2, b);
                if constexpr (GEOM != GEOM_QPOINT) {
                    // per-cell records carry no point weights
                    const T jw = pick<N>(tab + TL.w, a) * tab[TL.w + b];
                    vv[b] *= jw; wd[b] *= jw; w1[b] *= jw; w2[b] *= jw;
                }
            }
            // integration, t2 part: a'' = S^T (v + D^T w_t2), c'' = S^T w_t1, b'' = S^T w_d
            T tmp[N];
            eo_apply<N, -1>(tab + TL.DT, w2, tmp);
#pragma unroll
            for (int b = 0; b < N; ++b) vv[b] += tmp[b];
            s_apply<N, COLLOC>(tab + TL.ST, vv, vv);
            s_apply<N, COLLOC>(tab + TL.ST, w1, w1);
            s_apply<N, COLLOC>(tab + TL.ST, wd, wd);
            T* s0 = fel(FV, D, c, s) + a;
            T* s1 = fel(FT, D, c, s) + a;
            T* s2 = fel(FN, D, c, s) + a;
#pragma unroll
            for (int b = 0; b < N; ++b) { s0[b * FR] = vv[b]; s1[b * FR] = w1[b]; s2[b * FR] = wd[b]; }
        }
        }   // per-point records
    });

    // Cell metric terms of this thread's z pencil (used in C5).
    // Cell steps: thread -> (cell c, pencil t).  Where a wavefront holds whole
    // cells (WAVE_CELLS), wavefront w owns cells w CPW ..., so the cell steps
    // only need wavefront-level syncs.
    constexpr int CPW = 64 / N2;
    constexpr bool WAVE_CELLS = 3 * CPW >= CPB;
    const int c = WAVE_CELLS ? wave * CPW + lane / N2 : tid / N2;   // cell of this thread in the cell steps
    const int t = WAVE_CELLS ? lane % N2 : tid % N2;                // pencil of this thread
    const int ta = t % N, tb = t / N;
    const bool act = (!WAVE_CELLS || lane < CPW * N2) && c < ncb;
    auto cell_sync = [&]() {
        if constexpr (WAVE_CELLS) wave_sync();
        else __syncthreads();
    };
    constexpr bool DIAGM = GEOM == GEOM_CELL_DIAG;   // diagonal per-cell metric: reference-coordinate cell term
    constexpr int NG = GEOM != GEOM_QPOINT ? 6 : 6 * N;
    T gpre[NG];
    auto load_gpre = [&]() {
        const int cell = cell0 + c;
        if constexpr (DIAGM) {
            // the diagonal G_00, G_11, G_22 of the stored 00,01,02,11,12,22
#pragma unroll
            for (int m = 0; m < 3; ++m) gpre[m] = p.cgeom[size_t(cell) * 8 + (m == 0 ? 0 : m == 1 ? 3 : 5)];
        } else if constexpr (GEOM == GEOM_CELL) {
#pragma unroll
            for (int m = 0; m < 6; ++m) gpre[m] = p.cgeom[size_t(cell) * 8 + m];
        } else {
            // chunks of points along z with 16-byte loads, then the
            // remaining points (layout of cell_metric_offset)
            const T* gq = p.cgeom + size_t(cell) * (6 * N3);
            const int tp = ta + N * tb;
            constexpr int CH = 16 / int(sizeof(T)), J = N / CH, R = N % CH;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
#pragma unroll
                for (int j = 0; j < J; ++j) load_run<CH>(gq + (m * J + j) * CH * N2 + CH * tp, gpre + m * N + j * CH);
                if constexpr (R > 0) load_run<R>(gq + 6 * J * CH * N2 + m * R * N2 + R * tp, gpre + m * N + J * CH);
            }
        }
    };
    if constexpr (EARLY) {
        if (act) load_gpre();
    }
    wave_sync();

    // ----------------------- I: along t1: S^T / D^T -> P (array FV), Q (array FT)
    // (affine face step: P and Q are complete already)
    if (!KRON && fact) {
        const int b = fab;
        T* s0 = fel(FV, wave, fc, fs) + b * FR;
        T* s1 = fel(FT, wave, fc, fs) + b * FR;
        const T* s2 = fel(FN, wave, fc, fs) + b * FR;
        T av[N], cv[N], bv[N];
#pragma unroll
        for (int a = 0; a < N; ++a) { av[a] = s0[a]; cv[a] = s1[a]; bv[a] = s2[a]; }
        eo_apply<N, -1>(tab + TL.DT, cv, cv);
#pragma unroll
        for (int a = 0; a < N; ++a) av[a] += cv[a];
        s_apply<N, COLLOC>(tab + TL.ST, av, av);
        s_apply<N, COLLOC>(tab + TL.ST, bv, bv);
#pragma unroll
        for (int a = 0; a < N; ++a) { s0[a] = av[a]; s1[a] = bv[a]; }
    }
    __syncthreads();

    // ================================================================ cell
    T* A = ldsX + (act ? c : 0) * CS;
    T* B = ldsF + 6 * Sh::FARR + (act ? c : 0) * CS;    // from the FN arrays on
    T* C = B + CPB * CS;
    T v[N];
    // Last step of either cell path: this thread's z pencil v (cell term in
    // nodal coefficients), plus e_layer (x) P + D_f (x) Q of the six faces,
    // written to y.
    auto add_faces_and_store = [&](T* v) {
        const int i1 = ta, i2 = tb;
        const auto df0 = tab + TL.df0;
        const auto df1 = tab + TL.df1;
        const T cx0 = pick<N>(df0, i1), cx1 = pick<N>(df1, i1);
        const T cy0 = pick<N>(df0, i2), cy1 = pick<N>(df1, i2);
        const bool hx0 = BASIS != 0 || i1 <= 1, hx1 = BASIS != 0 || i1 >= N - 2;
        const bool hy0 = BASIS != 0 || i2 <= 1, hy1 = BASIS != 0 || i2 >= N - 2;
        // value test rows: unit rows at the end layers, or dense (Gauss)
        const auto fv0 = tab + TL.FV0;
        const auto fv1 = tab + TL.FV1;
        const T vx0 = COLLOC ? pick<N>(fv0, i1) : T(i1 == 0), vx1 = COLLOC ? pick<N>(fv1, i1) : T(i1 == N - 1);
        const T vy0 = COLLOC ? pick<N>(fv0, i2) : T(i2 == 0), vy1 = COLLOC ? pick<N>(fv1, i2) : T(i2 == N - 1);
        const T* P0 = fel(0, 0, c, 0); const T* Q0 = fel(1, 0, c, 0);
        const T* P1 = fel(0, 0, c, 1); const T* Q1 = fel(1, 0, c, 1);
        const T* P2 = fel(0, 1, c, 0); const T* Q2 = fel(1, 1, c, 0);
        const T* P3 = fel(0, 1, c, 1); const T* Q3 = fel(1, 1, c, 1);
        const T* P4 = fel(0, 2, c, 0); const T* Q4 = fel(1, 2, c, 0);
        const T* P5 = fel(0, 2, c, 1); const T* Q5 = fel(1, 2, c, 1);
        T* __restrict__ yc = p.y + voff + size_t(cell0 + c) * N3 + i1 + N * i2;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T r = v[k];
            // x faces: tangential (t1, t2) = (i2, k), layer i1
            if constexpr (COLLOC) {
                r += vx0 * P0[k * FR + i2] + cx0 * Q0[k * FR + i2];
                r += vx1 * P1[k * FR + i2] + cx1 * Q1[k * FR + i2];
            } else {
                if (hx0) r += (i1 == 0 ? P0[k * FR + i2] : T(0)) + cx0 * Q0[k * FR + i2];
                if (hx1) r += (i1 == N - 1 ? P1[k * FR + i2] : T(0)) + cx1 * Q1[k * FR + i2];
            }
            // y faces: tangential (i1, k), layer i2
            if constexpr (COLLOC) {
                r += vy0 * P2[k * FR + i1] + cy0 * Q2[k * FR + i1];
                r += vy1 * P3[k * FR + i1] + cy1 * Q3[k * FR + i1];
            } else {
                if (hy0) r += (i2 == 0 ? P2[k * FR + i1] : T(0)) + cy0 * Q2[k * FR + i1];
                if (hy1) r += (i2 == N - 1 ? P3[k * FR + i1] : T(0)) + cy1 * Q3[k * FR + i1];
            }
            // z faces: tangential (i1, i2), layer k (compile time)
            if (BASIS != 0 || k <= 1) {
                if constexpr (COLLOC) r += fv0[k] * P4[i2 * FR + i1];
                else if (k == 0) r += P4[i2 * FR + i1];
                r += df0[k] * Q4[i2 * FR + i1];
            }
            if (BASIS != 0 || k >= N - 2) {
                if constexpr (COLLOC) r += fv1[k] * P5[i2 * FR + i1];
                else if (k == N - 1) r += P5[i2 * FR + i1];
                r += df1[k] * Q5[i2 * FR + i1];
            }
            if constexpr (EPI <= EPI_PJACOBI) yc[k * N2] = r;
            if constexpr (EPI != EPI_NONE) v[k] = r;
        }
    };
    // Chebyshev epilogues: this thread's z pencil of b, loaded before the
    // last cell step so that its latency overlaps that step
    const size_t coff = size_t(cell0 + c) * N3 + ta + N * tb;   // this thread's z pencil
    T eb[EPI >= EPI_CHEB_PJ ? N : 1];
    auto load_epi_b = [&]() {
        if constexpr (EPI >= EPI_CHEB_PJ) {
            if (act) {
#pragma unroll
                for (int k = 0; k < N; ++k) eb[k] = p.b[voff + coff + k * N2];
            }
        }
    };
    if constexpr (DIAGM) {
        // ---- Cell term with a diagonal metric (G_00, G_11, G_22 per cell)
        // in reference coordinates, with the 1D mass M = S^T W S and
        // stiffness L = S'^T W S' (exact with the n-point Gauss rule):
        //   y = G_00 (L x M x M) x + G_11 (M x L x M) x + G_22 (M x M x L) x
        // (x-direction factor first): three pencil steps instead of nine.
        // K1: x pencils (thread (i2, i3)): M and L along x
        if (act) {
            if constexpr (!EARLY) load_gpre();
            T l[N];
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(k, ta, tb)];
            eo_apply<N, +1>(tab + TL.LL, v, l);
            eo_apply<N, +1>(tab + TL.MM, v, v);
#pragma unroll
            for (int k = 0; k < N; ++k) { A[Sh::lds_idx(k, ta, tb)] = v[k]; B[Sh::lds_idx(k, ta, tb)] = l[k]; }
        }
        cell_sync();
        // K2: y pencils (thread (i1, i3)): M_y M_x x, and G_00 M_y L_x x + G_11 L_y M_x x
        if (act) {
            T l[N], t[N], q[N];
#pragma unroll
            for (int k = 0; k < N; ++k) { v[k] = A[Sh::lds_idx(ta, k, tb)]; l[k] = B[Sh::lds_idx(ta, k, tb)]; }
            eo_apply<N, +1>(tab + TL.MM, l, t);
            eo_apply<N, +1>(tab + TL.LL, v, q);
#pragma unroll
            for (int k = 0; k < N; ++k) t[k] = gpre[0] * t[k] + gpre[1] * q[k];
            eo_apply<N, +1>(tab + TL.MM, v, v);
#pragma unroll
            for (int k = 0; k < N; ++k) { A[Sh::lds_idx(ta, k, tb)] = v[k]; B[Sh::lds_idx(ta, k, tb)] = t[k]; }
        }
        cell_sync();
        // K3: z pencils (thread (i1, i2)): M_z t + G_22 L_z (M_y M_x x), faces, write
        load_epi_b();
        if (act) {
            T t[N], q[N];
#pragma unroll
            for (int k = 0; k < N; ++k) { v[k] = A[Sh::lds_idx(ta, tb, k)]; t[k] = B[Sh::lds_idx(ta, tb, k)]; }
            eo_apply<N, +1>(tab + TL.LL, v, q);
            eo_apply<N, +1>(tab + TL.MM, t, v);
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = fma(gpre[2], q[k], v[k]);
            add_faces_and_store(v);
        }
    } else {
    // C1: z pencils (thread (i1, i2)) : S along z
    if (act && !COLLOC) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, tb, k)];
        s_apply<N, COLLOC>(tab + TL.S, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, tb, k)] = v[k];
    }
    cell_sync();
    // C2: y pencils (thread (i1, q3)) : S along y
    if (act && !COLLOC) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
        s_apply<N, COLLOC>(tab + TL.S, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k];
    }
    cell_sync();
    // C3: x pencils (thread (q2, q3)) : S along x -> u; D along x -> du/dxi1
    if (act) {
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(k, ta, tb)];
        s_apply<N, COLLOC>(tab + TL.S, v, v);
        eo_apply<N, -1>(tab + TL.D, v, g);
#pragma unroll
        for (int k = 0; k < N; ++k) { A[Sh::lds_idx(k, ta, tb)] = v[k]; B[Sh::lds_idx(k, ta, tb)] = g[k]; }
    }
    cell_sync();
    // C4: y pencils : D along y -> du/dxi2
    if (act) {
        if constexpr (!EARLY) load_gpre();
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
        eo_apply<N, -1>(tab + TL.D, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) C[Sh::lds_idx(ta, k, tb)] = v[k];
    }
    cell_sync();
    // C5: z pencils (thread (q1, q2)) : D along z -> du/dxi3, metric, D^T along z
    if (act) {
        T g1[N], g2[N], g3[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            v[k] = A[Sh::lds_idx(ta, tb, k)];
            g1[k] = B[Sh::lds_idx(ta, tb, k)];
            g2[k] = C[Sh::lds_idx(ta, tb, k)];
        }
        eo_apply<N, -1>(tab + TL.D, v, g3);
        T w12 = T(1);
        if constexpr (GEOM == GEOM_CELL) w12 = pick<N>(tab + TL.w, ta) * pick<N>(tab + TL.w, tb);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T G[6];
            if constexpr (GEOM == GEOM_CELL) {
                const T w = w12 * tab[TL.w + k];
#pragma unroll
                for (int m = 0; m < 6; ++m) G[m] = gpre[m] * w;
            } else {
#pragma unroll
                for (int m = 0; m < 6; ++m) G[m] = gpre[m * N + k];
            }
            const T a1 = G[0] * g1[k] + G[1] * g2[k] + G[2] * g3[k];
            const T a2 = G[1] * g1[k] + G[3] * g2[k] + G[4] * g3[k];
            const T a3 = G[2] * g1[k] + G[4] * g2[k] + G[5] * g3[k];
            g1[k] = a1; g2[k] = a2; g3[k] = a3;
        }
        eo_apply<N, -1>(tab + TL.DT, g3, g3);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            A[Sh::lds_idx(ta, tb, k)] = g3[k];
            B[Sh::lds_idx(ta, tb, k)] = g1[k];
            C[Sh::lds_idx(ta, tb, k)] = g2[k];
        }
    }
    cell_sync();
    // C6: y pencils : r += D^T t2
    if (act) {
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) { v[k] = A[Sh::lds_idx(ta, k, tb)]; g[k] = C[Sh::lds_idx(ta, k, tb)]; }
        eo_apply<N, -1>(tab + TL.DT, g, g);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k] + g[k];
    }
    cell_sync();
    // C7: x pencils : r += D^T t1, then S^T along x
    if (act) {
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) { v[k] = A[Sh::lds_idx(k, ta, tb)]; g[k] = B[Sh::lds_idx(k, ta, tb)]; }
        eo_apply<N, -1>(tab + TL.DT, g, g);
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += g[k];
        s_apply<N, COLLOC>(tab + TL.ST, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(k, ta, tb)] = v[k];
    }
    cell_sync();
    // C8: y pencils : S^T along y
    if (act && !COLLOC) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
        s_apply<N, COLLOC>(tab + TL.ST, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k];
    }
    cell_sync();
    // C9: z pencils (thread (i1, i2)) : S^T along z, add face terms, write y
    load_epi_b();
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, tb, k)];
        s_apply<N, COLLOC>(tab + TL.ST, v, v);
        add_faces_and_store(v);
    }
    }   // quadrature cell term

    if constexpr (EPI != EPI_NONE) {
        // P^-1 on this cell, sweeps as in the stand-alone basis change: T
        // (or Z^T) along z, y, x, the diagonal, T^T (or Z) along x, y, z.
        // The thread holds its z pencil of y in v; A, which it last read at
        // the same places, is the work array (no other pencil touches them).
        constexpr bool FDM = EPI == EPI_CHEB_FDM;
        constexpr bool CHEB = EPI != EPI_PJACOBI;
        // operands of the later steps, loaded now: the diagonal (this
        // thread's x pencil) or the cell's four scalars, and u, u_old
        T d[N], cs[4], uu[CHEB ? N : 1], uold[CHEB ? N : 1];
        if (act) {
            if constexpr (FDM) {
#pragma unroll
                for (int m = 0; m < 4; ++m) cs[m] = p.dinv[size_t(cell0 + c) * 4 + m];
            } else {
                load_chunked_pencil<N>(p.dinv + size_t(cell0 + c) * N3, ta + N * tb, d);
            }
            if constexpr (CHEB) {
                const bool rd = T(p.sigma) != T(0);
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    uu[k] = p.x[voff + coff + k * N2];
                    uold[k] = rd ? p.uo[voff + coff + k * N2] : uu[k];
                }
                // the residual b - A u
#pragma unroll
                for (int k = 0; k < N; ++k) v[k] = eb[k] - v[k];
            }
        }
        auto fwd = [&](T* w) {
            if constexpr (FDM) fdm_fwd<N>(p.tab + TL.FZP, w);
            else eo_apply<N, +1>(tab + TL.T, w, w);
        };
        auto bwd = [&](T* w) {
            if constexpr (FDM) fdm_bwd<N>(p.tab + TL.FZP, w);
            else eo_apply<N, +1>(tab + TL.TT, w, w);
        };
        if (act) {
            fwd(v);
#pragma unroll
            for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, tb, k)] = v[k];
        }
        cell_sync();
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
            fwd(v);
#pragma unroll
            for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k];
        }
        cell_sync();
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(k, ta, tb)];
            fwd(v);
            if constexpr (FDM) {
                // 1 / (vol (lambda_i/h_1^2 + lambda_j/h_2^2 + lambda_k/h_3^2)) from the
                // cell's four scalars, by the hardware reciprocal refined with two
                // Newton steps (d > 0)
                const T c0 = cs[0], c3 = cs[3];
                const T* lam = p.tab + TL.FLAM;
                const T yz = pick<N>(lam, ta) * cs[1] + pick<N>(lam, tb) * cs[2];
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const T d = fma(lam[k], c0, yz);
                    T q;
                    if constexpr (sizeof(T) == 8) q = __builtin_amdgcn_rcp(d);
                    else q = __builtin_amdgcn_rcpf(d);
                    q = fma(q, fma(-d, q, T(1)), q);
                    q = fma(q, fma(-d, q, T(1)), q);
                    v[k] = v[k] * c3 * q;
                }
            } else {
#pragma unroll
                for (int k = 0; k < N; ++k) v[k] *= d[k];
            }
            bwd(v);
#pragma unroll
            for (int k = 0; k < N; ++k) A[Sh::lds_idx(k, ta, tb)] = v[k];
        }
        cell_sync();
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
            bwd(v);
#pragma unroll
            for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k];
        }
        cell_sync();
        if (act) {
#pragma unroll
            for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, tb, k)];
            bwd(v);
            if constexpr (EPI == EPI_PJACOBI) {
#pragma unroll
                for (int k = 0; k < N; ++k) p.z[voff + coff + k * N2] = v[k];
            } else {
                // uo <- u + sigma (u - uo) + theta P^-1 r  (sigma = 0: uo not read)
                const T sg = T(p.sigma), th = T(p.theta);
#pragma unroll
                for (int k = 0; k < N; ++k) p.uo[voff + coff + k * N2] = uu[k] + sg * (uu[k] - uold[k]) + th * v[k];
            }
        }
    }
}

// One operator: workgroup b handles cells b*CPB ... of it, in the
// z-interleaved XCD order (P = blocks per z-layer of cells, rounded).
template <int N, int BASIS, typename T, int GEOM>
__global__ void __launch_bounds__(Shape<N>::NT, (matvec_min_waves<N, BASIS, T, GEOM>()))
sipg_matvec_kernel(MatvecParams<T> p) {
    constexpr int CPB = cells_per_block(N);
    const int layer_blocks = (p.nx * p.ny + CPB / 2) / CPB;
    // blockIdx.y: one of gridDim.y right-hand sides stored one after another
    matvec_block<N, BASIS, T, GEOM>(p, xcd_block_zinterleaved(blockIdx.x, gridDim.x, layer_blocks),
                                    size_t(blockIdx.y) * size_t(p.ncells) * (N * N * N));
}

// The same product followed, cell by cell, by P^-1 of eq. (jacobi): y = A x
// and z = P^-1 y in one pass (p.dinv, p.z set).
template <int N, int BASIS, typename T, int GEOM>
__global__ void __launch_bounds__(Shape<N>::NT, (matvec_min_waves<N, BASIS, T, GEOM>()))
sipg_matvec_pjacobi_kernel(MatvecParams<T> p) {
    constexpr int CPB = cells_per_block(N);
    const int layer_blocks = (p.nx * p.ny + CPB / 2) / CPB;
    matvec_block<N, BASIS, T, GEOM, EPI_PJACOBI>(p, xcd_block_zinterleaved(blockIdx.x, gridDim.x, layer_blocks));
}

// One step of the Chebyshev smoother fused into the product (u = p.x; p.b,
// p.uo, p.dinv, p.sigma, p.theta set): uo <- u + sigma (u - uo) + theta P^-1
// (b - A u), P^-1 point Jacobi (EPI_CHEB_PJ) or block Jacobi (EPI_CHEB_FDM).
template <int N, int BASIS, typename T, int GEOM, int EPI>
__global__ void __launch_bounds__(Shape<N>::NT, (matvec_min_waves<N, BASIS, T, GEOM>()))
sipg_matvec_cheb_kernel(MatvecParams<T> p) {
    constexpr int CPB = cells_per_block(N);
    const int layer_blocks = (p.nx * p.ny + CPB / 2) / CPB;
    // blockIdx.y: one of gridDim.y right-hand sides stored one after another
    matvec_block<N, BASIS, T, GEOM, EPI>(p, xcd_block_zinterleaved(blockIdx.x, gridDim.x, layer_blocks),
                                         size_t(blockIdx.y) * size_t(p.ncells) * (N * N * N));
}

// Many independent operators of the same degree, basis, precision and
// geometry mode in one grid: the workgroups of operator o are the block
// indices blk_first[o] ... blk_first[o+1]-1 of the concatenated list, and
// blk_op[b] names the operator of block b.
template <int N, int BASIS, typename T, int GEOM>
__global__ void __launch_bounds__(Shape<N>::NT, (matvec_min_waves<N, BASIS, T, GEOM>()))
sipg_matvec_batched_kernel(const MatvecParams<T>* __restrict__ ops, const int* __restrict__ blk_op,
                           const int* __restrict__ blk_first) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int o = __builtin_amdgcn_readfirstlane(blk_op[b]);
    const MatvecParams<T> p = ops[o];
    matvec_block<N, BASIS, T, GEOM>(p, b - __builtin_amdgcn_readfirstlane(blk_first[o]));
}

}  // namespace sipg
