// double instances of the sweep and Q* kernels for m = 4..6.
#define REAL_T double
#define SUFFIX f64
#define PART _1
#define M_FIRST 4
#define M_LAST 6
#include "inst_template.hpp"
