// float instances of the sweep and Q* kernels for m = 10..12.
#define REAL_T float
#define SUFFIX f32
#define PART _3
#define M_FIRST 10
#define M_LAST 12
#include "inst_template.hpp"
