/* Complex-step build of the oracle (test infrastructure only): the same
 * source with real_t = double complex and exported names prefixed orc_. */
#define OR_COMPLEX 1
#include "hsgn_oracle.c"
