// Column-pass instantiations, double precision.
#define PF_T double
#include "k_col.inc"
