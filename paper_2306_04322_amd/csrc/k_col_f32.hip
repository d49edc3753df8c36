// Column-pass instantiations, single precision.
#define PF_T float
#include "k_col.inc"
