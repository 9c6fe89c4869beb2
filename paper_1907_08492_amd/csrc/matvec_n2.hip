// Instantiations of the matrix-free SIPG product for n = 2 (degree 1).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(2)
