// Op-counting build of the oracle (see opcount.hpp) -- TEST INFRASTRUCTURE
// ONLY.  The same C ABI as liboracle, plus orc_opcount_reset / _get.
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

#include "opcount.hpp"

thread_local OpCounts orc_ops = {0, 0, 0, 0};

// the system headers above are already included, so only the oracle's own
// code takes C linkage (its exported names stay those of liboracle)
#define double cd
extern "C" {
#include "oracle.c"
}
#undef double

extern "C" void orc_opcount_reset(void) { orc_ops = OpCounts{0, 0, 0, 0}; }

// out[4] = {add/sub, mul, div, transcendental} since the last reset (calling thread)
extern "C" void orc_opcount_get(uint64_t *out) {
  out[0] = orc_ops.add;
  out[1] = orc_ops.mul;
  out[2] = orc_ops.div;
  out[3] = orc_ops.func;
}
