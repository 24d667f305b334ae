// p2s_tables.h -- host table builders (Gauss rules, Legendre moment
// weights, linearization coefficients of eq. (3)).
#pragma once

namespace p2s {

// Gauss-Legendre rule with Q points on [-1,1], ascending.  0 or -1.
int gauss_rule(int Q, double *x, double *w);
// X_m1 Y_m2 = sum_k coef[k] L_k for families X, Y in {phi, phi', psi};
// coef has KPAD entries.  0 or -1.
int linearization(int xf, int m1, int yf, int m2, double *coef);
// Fill the whole table buffer (TAB_SIZE doubles, layout in p2s_internal.h).
void build_tables(double *tab);

}  // namespace p2s
