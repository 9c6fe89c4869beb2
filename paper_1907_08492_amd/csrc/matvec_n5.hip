// Instantiations of the matrix-free SIPG product for n = 5 (degree 4).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(5)
