// Instantiations of the matrix-free SIPG product for n = 6 (degree 5).
#include "matvec_launch.hpp"

SIPG_MATVEC_DEGREE(6)
