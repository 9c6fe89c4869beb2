// Element-wise matrix-free SIPG product y = A x on gfx950 (Section 3).
//
// One workgroup handles CPB consecutive cells.  Every phase below maps one
// thread to one n-long pencil of a cell (or of a face array) held in
// registers; the 1D contraction along the pencil is an even-odd
// multiply-add sweep with coefficients in scalar registers, and the change of
// pencil direction between sweeps goes through LDS.  Per cell:
//
//   gather  x of the cell (coalesced) into LDS; for each of the six faces the
//           own value/derivative layers (from LDS) and the neighbour's value
//           and derivative layers (from HBM: two layers for the Hermite-like
//           basis, all n for the nodal basis), combined with S_f and D_f
//           (eq. tensor_face) into face arrays
//   faces   2D interpolation to the face Gauss points (S along t1, then S and
//           D along t2), flux at the points, and the transposed sweeps back
//           to two coefficient arrays P (value test) and Q (normal-derivative
//           test) per face
//   cell    S along z, y, x, collocation D along x, y, z (eq. tensor_cell),
//           merged metric at the points (eq. integral_laplace), transposed
//           sweeps back
//   write   y_K = cell part + sum over faces of e_layer (x) P + D_f (x) Q,
//           one coalesced write per cell (element-wise face evaluation).
#pragma once

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
};

template <int N>
struct Shape {
    static constexpr int N2 = N * N, N3 = N * N * N;
    static constexpr int RS = (N % 2 == 0) ? N + 1 : N;   // LDS row stride (odd: no bank aliasing)
    static constexpr int CS = RS * N * N;                  // one cell array in LDS
    static constexpr int FA = RS * N;                      // one face array in LDS
    static constexpr int CPB = cells_per_block(N);
    static constexpr int NT = threads_per_block(N);
    static constexpr int WS = (24 * FA > 2 * CS) ? 24 * FA : 2 * CS;
    static constexpr int F1_ITEMS = (CPB * 6 * N2 + NT - 1) / NT;   // gather items per thread
    static constexpr int F3_ITEMS = (CPB * 6 * N + NT - 1) / NT;    // flux columns per thread
    static constexpr int PER_CELL = CS + 12 * FA + WS;     // words of T per cell
    __host__ __device__ static constexpr int lds_idx(int i1, int i2, int i3) { return i1 + RS * (i2 + N * i3); }
};

template <int N, typename T>
constexpr size_t matvec_lds_bytes() {
    using S = Shape<N>;
    constexpr size_t b = size_t(S::CPB) * S::PER_CELL * sizeof(T) + size_t(S::CPB) * 12 * sizeof(int);
    static_assert(b == matvec_lds_bytes_rt(N, sizeof(T)), "LDS size formula mismatch");
    static_assert(b <= 160 * 1024, "LDS budget of a gfx950 CU exceeded");
    static_assert(S::CPB * N * N <= S::NT && S::NT % 64 == 0 && S::NT <= 1024, "launch shape");
    return b;
}

// basis: 0 Hermite-like (derivative rows touch layers {0,1} / {n-2,n-1}),
//        1 nodal Gauss-Lobatto (derivative rows touch every layer).
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

template <int N, int BASIS>
struct Layers {
    static constexpr int NL = (BASIS == 0) ? 2 : N;
    // j-th layer of the derivative support at side s
    __host__ __device__ static constexpr int layer(int s, int j) { return BASIS == 0 ? (s ? N - 2 + j : j) : j; }
};

template <int N, int BASIS, typename T, int GEOM>
__global__ void __launch_bounds__(Shape<N>::NT)
sipg_matvec_kernel(MatvecParams<T> p) {
    using Sh = Shape<N>;
    using Ly = Layers<N, BASIS>;
    constexpr int N2 = Sh::N2, N3 = Sh::N3, RS = Sh::RS, CS = Sh::CS, FA = Sh::FA;
    constexpr int CPB = Sh::CPB, NT = Sh::NT;
    constexpr TableLayout TL(N);

    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    T* ldsX = lds;                                   // [CPB][CS]   x, later the cell work array A
    T* ldsPQ = lds + CPB * CS;                       // [CPB][6][2][FA]   face slots 0,1
    T* ldsW = ldsPQ + CPB * 12 * FA;                 // [CPB][WS]  face slots 2..5, later cell arrays B, C
    int* meta = reinterpret_cast<int*>(ldsW + CPB * Sh::WS);   // [CPB][12]: neighbour, face index

    const T* __restrict__ tab = p.tab;
    const int tid = threadIdx.x;
    // XCD-aware order: consecutive workgroups are dispatched round-robin over
    // the 8 XCDs, so give each XCD a contiguous range of cells (shared L2).
    const int nblk = gridDim.x;
    int blk = blockIdx.x;
    {
        const int per = (nblk + 7) / 8;
        const int xcd = blk % 8, slot = blk / 8;
        const int full = nblk % 8 == 0 ? 8 : nblk % 8;   // XCDs that get `per` blocks
        const int rem_per = per - 1;
        int start;
        if (xcd < full) start = xcd * per;
        else start = full * per + (xcd - full) * rem_per;
        blk = start + slot;
    }
    const int cell0 = blk * CPB;
    const int ncb = min(CPB, p.ncells - cell0);      // cells in this workgroup
    const int bx = cell0 % p.nx, by = (cell0 / p.nx) % p.ny, bz = cell0 / (p.nx * p.ny);
    auto topo = [&](int c, int f, int& nb, int& fi) {
        int ix, iy, iz;
        cell_coords(bx, by, bz, c, p.nx, p.ny, ix, iy, iz);
        face_topology(ix, iy, iz, f, p.nx, p.ny, p.nz, nb, fi);
    };

    // ---------------------------------------------------------------- meta
    for (int it = tid; it < ncb * 6; it += NT) {
        int nb, fi;
        topo(it / 6, it % 6, nb, fi);
        meta[(it / 6) * 12 + it % 6] = nb;
        meta[(it / 6) * 12 + 6 + it % 6] = fi;
    }

    // Prefetch into registers, before any LDS work and without waiting for
    // the metadata: the metric terms of this thread's first face-flux column
    // (used in F3) and the neighbour value/derivative layers of the gather (F1).
    constexpr int NREC = GEOM == GEOM_CELL ? 7 : 7 * N;
    T frec[NREC];
    if (tid < ncb * 6 * N) {
        const int a = tid % N, f = (tid / N) % 6, c = tid / (6 * N);
        const int d = f >> 1;
        int nb, fidx;
        topo(c, f, nb, fidx);
        const T* __restrict__ fg = d == 0 ? p.fgeom0 : d == 1 ? p.fgeom1 : p.fgeom2;
        if constexpr (GEOM == GEOM_CELL) {
#pragma unroll
            for (int k = 0; k < 7; ++k) frec[k] = fg[size_t(fidx) * 8 + k];
        } else {
#pragma unroll
            for (int k = 0; k < 7; ++k)
#pragma unroll
                for (int b = 0; b < N; ++b) frec[k * N + b] = fg[size_t(fidx) * (7 * N2) + k * N2 + a + N * b];
        }
    }
    const int c = tid / N2;                 // cell of this thread in the cell phases
    const int t = tid % N2;                 // pencil of this thread
    const int ta = t % N, tb = t / N;
    const bool act = c < ncb;
    T nbv[Sh::F1_ITEMS][Ly::NL];
#pragma unroll
    for (int r = 0; r < Sh::F1_ITEMS; ++r) {
        const int it = tid + r * NT;
        if (it < ncb * 6 * N2) {
            const int a = it % N, b = (it / N) % N, f = (it / N2) % 6, c = it / (6 * N2);
            const int d = f >> 1, s = f & 1;
            int nb, fi;
            topo(c, f, nb, fi);
            if (nb >= 0) {
                const T* __restrict__ xn = p.x + size_t(nb) * N3;
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) {
                    const int l = Ly::layer(1 - s, j);
                    const int g = d == 0 ? l + N * (a + N * b) : d == 1 ? a + N * (l + N * b) : a + N * (b + N * l);
                    nbv[r][j] = xn[g];
                }
            }
        }
    }
    // ---------------------------------------------------------------- load x
    {
        const T* __restrict__ xs = p.x + size_t(cell0) * N3;
        for (int e = tid; e < ncb * N3; e += NT) {
            const int c = e / N3, i = e % N3;
            const int i1 = i % N, i2 = (i / N) % N, i3 = i / N2;
            ldsX[c * CS + Sh::lds_idx(i1, i2, i3)] = xs[e];
        }
    }
    __syncthreads();

    auto slot = [&](int c, int f, int s) -> T* {
        return s < 2 ? ldsPQ + ((c * 6 + f) * 2 + s) * FA : ldsW + c * Sh::WS + (f * 4 + (s - 2)) * FA;
    };

    // ------------------------------------------------ F1: face layer gather
#pragma unroll
    for (int r = 0; r < Sh::F1_ITEMS; ++r) {
        const int it = tid + r * NT;
        if (it < ncb * 6 * N2) {
            const int a = it % N, b = (it / N) % N, f = (it / N2) % 6, c = it / (6 * N2);
            const int d = f >> 1, s = f & 1;
            const T* Xc = ldsX + c * CS;
            auto lidx = [&](int j) {
                return d == 0 ? Sh::lds_idx(j, a, b) : d == 1 ? Sh::lds_idx(a, j, b) : Sh::lds_idx(a, b, j);
            };
            const T* dfs = tab + (s ? TL.df1 : TL.df0);
            const T* dfn = tab + (s ? TL.df0 : TL.df1);
            const T vm = Xc[lidx(s ? N - 1 : 0)];
            T nm = T(0);
#pragma unroll
            for (int j = 0; j < Ly::NL; ++j) {
                const int l = Ly::layer(s, j);
                nm = fma(dfs[l], Xc[lidx(l)], nm);
            }
            const int row = b * RS + a;
            slot(c, f, 0)[row] = vm;
            slot(c, f, 1)[row] = nm;
            if (meta[c * 12 + f] >= 0) {
                // neighbour side: its value layer touches the face, its
                // derivative row combines the registers loaded above
                T vp = T(0), np = T(0);
#pragma unroll
                for (int j = 0; j < Ly::NL; ++j) {
                    const int l = Ly::layer(1 - s, j);
                    if (l == (s ? 0 : N - 1)) vp = nbv[r][j];
                    np = fma(dfn[l], nbv[r][j], np);
                }
                slot(c, f, 2)[row] = vp;
                slot(c, f, 3)[row] = np;
            }
        }
    }
    __syncthreads();

    // ------------------------------------ F2: S (and S') along t1 (rows)
    for (int it = tid; it < ncb * 6 * 4 * N; it += NT) {
        const int b = it % N, m = (it / N) % 4, f = (it / (4 * N)) % 6, c = it / (24 * N);
        if (m >= 2 && meta[c * 12 + f] < 0) continue;
        T* src = slot(c, f, m) + b * RS;
        T v[N], r[N];
#pragma unroll
        for (int a = 0; a < N; ++a) v[a] = src[a];
        eo_apply<N, +1>(tab + TL.S, v, r);
#pragma unroll
        for (int a = 0; a < N; ++a) src[a] = r[a];
        if (m == 0 || m == 2) {
            eo_apply<N, -1>(tab + TL.SG, v, r);
            T* dst = slot(c, f, 4 + (m >> 1)) + b * RS;
#pragma unroll
            for (int a = 0; a < N; ++a) dst[a] = r[a];
        }
    }
    __syncthreads();

    // ------------------- F3: S, D along t2 (columns), flux, transposed sweeps
    for (int it = tid; it < ncb * 6 * N; it += NT) {
        const int a = it % N, f = (it / N) % 6, c = it / (6 * N);
        const int d = f >> 1, s = f & 1;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const bool interior = meta[c * 12 + f] >= 0;
        const int fidx = meta[c * 12 + 6 + f];
        auto col = [&](int sl, T* v) {
            const T* src = slot(c, f, sl) + a;
#pragma unroll
            for (int b = 0; b < N; ++b) v[b] = src[b * RS];
        };
        T um[N], gdm[N], g1m[N], g2m[N];
        col(0, um);  eo_apply<N, +1>(tab + TL.S, um, um);
        col(1, gdm); eo_apply<N, +1>(tab + TL.S, gdm, gdm);
        col(4, g1m); eo_apply<N, +1>(tab + TL.S, g1m, g1m);
        eo_apply<N, -1>(tab + TL.D, um, g2m);
        T up[N], gdp[N], g1p[N], g2p[N];
        if (interior) {
            col(2, up);  eo_apply<N, +1>(tab + TL.S, up, up);
            col(3, gdp); eo_apply<N, +1>(tab + TL.S, gdp, gdp);
            col(5, g1p); eo_apply<N, +1>(tab + TL.S, g1p, g1p);
            eo_apply<N, -1>(tab + TL.D, up, g2p);
        } else {
            // mirror principle: u+ = -u-, grad u+ = grad u-
#pragma unroll
            for (int b = 0; b < N; ++b) { up[b] = -um[b]; gdp[b] = gdm[b]; g1p[b] = g1m[b]; g2p[b] = g2m[b]; }
        }
        const T* __restrict__ fg = d == 0 ? p.fgeom0 : d == 1 ? p.fgeom1 : p.fgeom2;
        if (it != tid) {   // later columns of this thread: load now
            if constexpr (GEOM == GEOM_CELL) {
#pragma unroll
                for (int k = 0; k < 7; ++k) frec[k] = fg[size_t(fidx) * 8 + k];
            } else {
#pragma unroll
                for (int k = 0; k < 7; ++k)
#pragma unroll
                    for (int b = 0; b < N; ++b) frec[k * N + b] = fg[size_t(fidx) * (7 * N2) + k * N2 + a + N * b];
            }
        }
        T wa = T(1);
        if constexpr (GEOM == GEOM_CELL) wa = pick<N>(tab + TL.w, a);
        T vv[N], wd[N], w1[N], w2[N];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            T rec[7];
            if constexpr (GEOM == GEOM_CELL) {
                const T jw = wa * tab[TL.w + b];
#pragma unroll
                for (int k = 0; k < 7; ++k) rec[k] = frec[k] * jw;
            } else {
#pragma unroll
                for (int k = 0; k < 7; ++k) rec[k] = frec[k * N + b];
            }
            // own-side (g-) and neighbour-side (g+) scaled normals in the
            // cell's reference coordinates; the stored record uses the normal
            // pointing from the lower to the upper cell of the face.
            T gm[3], gp[3];
            if (s == 1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) { gm[k] = rec[1 + k]; gp[k] = rec[4 + k]; }
            } else {
#pragma unroll
                for (int k = 0; k < 3; ++k) { gm[k] = -rec[4 + k]; gp[k] = -rec[1 + k]; }
            }
            const T jump = um[b] - up[b];
            const T dm = gm[d] * gdm[b] + gm[t1] * g1m[b] + gm[t2] * g2m[b];
            const T dp = gp[d] * gdp[b] + gp[t1] * g1p[b] + gp[t2] * g2p[b];
            vv[b] = rec[0] * jump - T(0.5) * (dm + dp);
            const T hj = T(-0.5) * jump;
            wd[b] = hj * gm[d];
            w1[b] = hj * gm[t1];
            w2[b] = hj * gm[t2];
        }
        // integration, t2 part: a'' = S^T (v + D^T w_t2), c'' = S^T w_t1, b'' = S^T w_d
        T tmp[N];
        eo_apply<N, -1>(tab + TL.DT, w2, tmp);
#pragma unroll
        for (int b = 0; b < N; ++b) vv[b] += tmp[b];
        eo_apply<N, +1>(tab + TL.ST, vv, vv);
        eo_apply<N, +1>(tab + TL.ST, w1, w1);
        eo_apply<N, +1>(tab + TL.ST, wd, wd);
        T* s0 = slot(c, f, 0) + a;
        T* s1 = slot(c, f, 1) + a;
        T* s2 = slot(c, f, 2) + a;
#pragma unroll
        for (int b = 0; b < N; ++b) { s0[b * RS] = vv[b]; s1[b * RS] = w1[b]; s2[b * RS] = wd[b]; }
    }
    __syncthreads();

    // Cell metric terms of this thread's z pencil (used in C5).
    constexpr int NG = GEOM == GEOM_CELL ? 6 : 6 * N;
    T gpre[NG];
    if (act) {
        const int cell = cell0 + c;
        if constexpr (GEOM == GEOM_CELL) {
#pragma unroll
            for (int m = 0; m < 6; ++m) gpre[m] = p.cgeom[size_t(cell) * 8 + m];
        } else {
            const T* gq = p.cgeom + size_t(cell) * (6 * N3) + ta + N * tb;
#pragma unroll
            for (int m = 0; m < 6; ++m)
#pragma unroll
                for (int k = 0; k < N; ++k) gpre[m * N + k] = __builtin_nontemporal_load(gq + m * N3 + N2 * k);
        }
    }

    // ----------------- F4: transposed sweeps along t1 -> P (slot 0), Q (slot 1)
    for (int it = tid; it < ncb * 6 * N; it += NT) {
        const int b = it % N, f = (it / N) % 6, c = it / (6 * N);
        T* s0 = slot(c, f, 0) + b * RS;
        T* s1 = slot(c, f, 1) + b * RS;
        const T* s2 = slot(c, f, 2) + b * RS;
        T av[N], cv[N], bv[N];
#pragma unroll
        for (int a = 0; a < N; ++a) { av[a] = s0[a]; cv[a] = s1[a]; bv[a] = s2[a]; }
        eo_apply<N, -1>(tab + TL.DT, cv, cv);
#pragma unroll
        for (int a = 0; a < N; ++a) av[a] += cv[a];
        eo_apply<N, +1>(tab + TL.ST, av, av);
        eo_apply<N, +1>(tab + TL.ST, bv, bv);
#pragma unroll
        for (int a = 0; a < N; ++a) { s0[a] = av[a]; s1[a] = bv[a]; }
    }
    __syncthreads();

    // ================================================================ cell
    T* A = ldsX + (act ? c : 0) * CS;
    T* B = ldsW + (act ? c : 0) * Sh::WS;
    T* C = B + CS;
    T v[N];
    // C1: z pencils (thread (i1, i2)) : S along z
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, tb, k)];
        eo_apply<N, +1>(tab + TL.S, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, tb, k)] = v[k];
    }
    __syncthreads();
    // C2: y pencils (thread (i1, q3)) : S along y
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
        eo_apply<N, +1>(tab + TL.S, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k];
    }
    __syncthreads();
    // C3: x pencils (thread (q2, q3)) : S along x -> u; D along x -> du/dxi1
    if (act) {
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(k, ta, tb)];
        eo_apply<N, +1>(tab + TL.S, v, v);
        eo_apply<N, -1>(tab + TL.D, v, g);
#pragma unroll
        for (int k = 0; k < N; ++k) { A[Sh::lds_idx(k, ta, tb)] = v[k]; B[Sh::lds_idx(k, ta, tb)] = g[k]; }
    }
    __syncthreads();
    // C4: y pencils : D along y -> du/dxi2
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
        eo_apply<N, -1>(tab + TL.D, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) C[Sh::lds_idx(ta, k, tb)] = v[k];
    }
    __syncthreads();
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
    __syncthreads();
    // C6: y pencils : r += D^T t2
    if (act) {
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) { v[k] = A[Sh::lds_idx(ta, k, tb)]; g[k] = C[Sh::lds_idx(ta, k, tb)]; }
        eo_apply<N, -1>(tab + TL.DT, g, g);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k] + g[k];
    }
    __syncthreads();
    // C7: x pencils : r += D^T t1, then S^T along x
    if (act) {
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) { v[k] = A[Sh::lds_idx(k, ta, tb)]; g[k] = B[Sh::lds_idx(k, ta, tb)]; }
        eo_apply<N, -1>(tab + TL.DT, g, g);
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] += g[k];
        eo_apply<N, +1>(tab + TL.ST, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(k, ta, tb)] = v[k];
    }
    __syncthreads();
    // C8: y pencils : S^T along y
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, k, tb)];
        eo_apply<N, +1>(tab + TL.ST, v, v);
#pragma unroll
        for (int k = 0; k < N; ++k) A[Sh::lds_idx(ta, k, tb)] = v[k];
    }
    __syncthreads();
    // C9: z pencils (thread (i1, i2)) : S^T along z, add face terms, write y
    if (act) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = A[Sh::lds_idx(ta, tb, k)];
        eo_apply<N, +1>(tab + TL.ST, v, v);
        const int i1 = ta, i2 = tb;
        const T* df0 = tab + TL.df0;
        const T* df1 = tab + TL.df1;
        const T cx0 = pick<N>(df0, i1), cx1 = pick<N>(df1, i1);
        const T cy0 = pick<N>(df0, i2), cy1 = pick<N>(df1, i2);
        const bool hx0 = BASIS != 0 || i1 <= 1, hx1 = BASIS != 0 || i1 >= N - 2;
        const bool hy0 = BASIS != 0 || i2 <= 1, hy1 = BASIS != 0 || i2 >= N - 2;
        const T* P0 = slot(c, 0, 0); const T* Q0 = slot(c, 0, 1);
        const T* P1 = slot(c, 1, 0); const T* Q1 = slot(c, 1, 1);
        const T* P2 = slot(c, 2, 0); const T* Q2 = slot(c, 2, 1);
        const T* P3 = slot(c, 3, 0); const T* Q3 = slot(c, 3, 1);
        const T* P4 = slot(c, 4, 0); const T* Q4 = slot(c, 4, 1);
        const T* P5 = slot(c, 5, 0); const T* Q5 = slot(c, 5, 1);
        T* __restrict__ yc = p.y + size_t(cell0 + c) * N3 + i1 + N * i2;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            T r = v[k];
            // x faces: tangential (t1, t2) = (i2, k), layer i1
            if (hx0) r += (i1 == 0 ? P0[k * RS + i2] : T(0)) + cx0 * Q0[k * RS + i2];
            if (hx1) r += (i1 == N - 1 ? P1[k * RS + i2] : T(0)) + cx1 * Q1[k * RS + i2];
            // y faces: tangential (i1, k), layer i2
            if (hy0) r += (i2 == 0 ? P2[k * RS + i1] : T(0)) + cy0 * Q2[k * RS + i1];
            if (hy1) r += (i2 == N - 1 ? P3[k * RS + i1] : T(0)) + cy1 * Q3[k * RS + i1];
            // z faces: tangential (i1, i2), layer k (compile time)
            if (BASIS != 0 || k <= 1) {
                if (k == 0) r += P4[i2 * RS + i1];
                r += df0[k] * Q4[i2 * RS + i1];
            }
            if (BASIS != 0 || k >= N - 2) {
                if (k == N - 1) r += P5[i2 * RS + i1];
                r += df1[k] * Q5[i2 * RS + i1];
            }
            yc[k * N2] = r;
        }
    }
}

}  // namespace sipg
