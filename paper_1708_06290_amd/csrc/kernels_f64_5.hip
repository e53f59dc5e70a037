// double instances of the sweep and Q* kernels for m = 15..16.
#define REAL_T double
#define SUFFIX f64
#define PART _5
#define M_FIRST 15
#define M_LAST 16
#include "inst_template.hpp"
