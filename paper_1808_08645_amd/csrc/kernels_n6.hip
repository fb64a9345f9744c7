// Stage and norm kernels for polynomial degree N = 6 (all c^2 degrees M <= min(N, 4)).
#include "stage_kernel.hpp"
BBW_DEGREE_UNIT(6)
