// Adjoint row-pass instantiations, double precision.
#define PF_T double
#include "k_adj.inc"
