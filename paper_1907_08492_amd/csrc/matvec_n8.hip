// Instantiations of the matrix-free SIPG product for n = 8 (degree 7).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(8)
