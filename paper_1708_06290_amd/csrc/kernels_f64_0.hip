// double instances of the sweep and Q* kernels for m = 1..3.
#define REAL_T double
#define SUFFIX f64
#define PART _0
#define M_FIRST 1
#define M_LAST 3
#include "inst_template.hpp"
