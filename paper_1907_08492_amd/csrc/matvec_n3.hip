// Instantiations of the matrix-free SIPG product for n = 3 (degree 2).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(3)
