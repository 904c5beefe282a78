/* oracle_int.h -- helpers private to the oracle.  TEST INFRASTRUCTURE ONLY. */
#ifndef SEIS_ORACLE_INT_H
#define SEIS_ORACLE_INT_H
#include "oracle.h"

extern const double OR_L8[5];
extern const double OR_D8[5];
extern const double OR_S4[2];

int or_layer_depth(int i, int n, int P);
void or_zeta_profile(const or_grid *g, int n, double *zeta);
int or_clampi(int v, int lo, int hi);
void or_cpml_at(const or_grid *g, int n, double x, double *a, double *b);

#endif
