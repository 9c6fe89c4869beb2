// Instantiations of the matrix-free SIPG product for n = 4 (degree 3).
#include "matvec.hpp"
#include "setup.hpp"

namespace sipg {

template <int N, int BASIS, typename T, int GEOM>
static int launch_one(const sipg_op* op, const void* x, void* y, hipStream_t st) {
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
    constexpr int CPB = cells_per_block(N);
    constexpr int NT = threads_per_block(N);
    constexpr size_t lds = matvec_lds_bytes<N, T>();
    static bool attr = false;
    if (!attr) {
        SIPG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&sipg_matvec_kernel<N, BASIS, T, GEOM>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        attr = true;
    }
    const unsigned nblk = unsigned((op->ncells + CPB - 1) / CPB);
    sipg_matvec_kernel<N, BASIS, T, GEOM><<<nblk, NT, lds, st>>>(p);
    SIPG_HIP(hipGetLastError());
    return SIPG_OK;
}

template <>
int launch_matvec_n<4>(const sipg_op* op, const void* x, void* y, hipStream_t st) {
    const bool f64 = op->dtype == SIPG_F64;
    const bool hl = op->basis == SIPG_BASIS_HERMITE_LIKE;
    const bool cell = op->geom == GEOM_CELL;
    if (f64) {
        if (hl) return cell ? launch_one<4, 0, double, GEOM_CELL>(op, x, y, st) : launch_one<4, 0, double, GEOM_QPOINT>(op, x, y, st);
        return cell ? launch_one<4, 1, double, GEOM_CELL>(op, x, y, st) : launch_one<4, 1, double, GEOM_QPOINT>(op, x, y, st);
    }
    if (hl) return cell ? launch_one<4, 0, float, GEOM_CELL>(op, x, y, st) : launch_one<4, 0, float, GEOM_QPOINT>(op, x, y, st);
    return cell ? launch_one<4, 1, float, GEOM_CELL>(op, x, y, st) : launch_one<4, 1, float, GEOM_QPOINT>(op, x, y, st);
}

}  // namespace sipg
