// double instances of the sweep and Q* kernels for m = 10..12.
#define REAL_T double
#define SUFFIX f64
#define PART _3
#define M_FIRST 10
#define M_LAST 12
#include "inst_template.hpp"
