// double instances of the sweep and Q* kernels for m = 7..9.
#define REAL_T double
#define SUFFIX f64
#define PART _2
#define M_FIRST 7
#define M_LAST 9
#include "inst_template.hpp"
