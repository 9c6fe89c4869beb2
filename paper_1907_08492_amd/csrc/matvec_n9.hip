// Instantiations of the matrix-free SIPG product for n = 9 (degree 8).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(9)
