// float instances of the sweep and Q* kernels for m = 13..14.
#define REAL_T float
#define SUFFIX f32
#define PART _4
#define M_FIRST 13
#define M_LAST 14
#include "inst_template.hpp"
