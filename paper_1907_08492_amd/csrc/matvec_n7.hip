// Instantiations of the matrix-free SIPG product for n = 7 (degree 6).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(7)
