// float instances of the sweep and Q* kernels for m = 4..6.
#define REAL_T float
#define SUFFIX f32
#define PART _1
#define M_FIRST 4
#define M_LAST 6
#include "inst_template.hpp"
