// Instantiations of the matrix-free SIPG product for n = 4 (degree 3).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(4)
