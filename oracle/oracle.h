/*
 * oracle.h -- plain FP64 CPU oracle for the hierarchical element-matrix
 * fill (direct full 3-D quadrature of eq. (2) of the paper).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  The product library never includes or
 * links it, and it shares no code with the product library.
 *
 * All pointers are host memory.  Layout conventions (the same meaning as the
 * product library's arguments, written out independently here):
 *  nodes   [E][27][3]  node (i,j,k) of the triquadratic map at i+3j+9k,
 *                      i along u; nominal position (i/2, j/2, k/2).
 *  mat     per element: SINCOSEXP {kappa}; ROTDIAG {R row-major (9), k (3)};
 *          PLANEWAVE {k (3), phase}; ALPHA_SAMPLED: coupling fields at the
 *          Gauss points, [F][Qu*Qv*Qw] with point (a*Qv+b)*Qw+c.
 *  orders  [E]         N per element (functions per direction).
 *  quad    [E][3]      Gauss points per axis (u, v, w).
 *  offsets [E+1]       start of each element's dense row-major block in out.
 *  status  [E]         bit 1: detJ <= 0 at a Gauss point; bit 2: non-finite.
 */
#ifndef P2S_ORACLE_H
#define P2S_ORACLE_H

#include <stdint.h>

#define ORACLE_MAX_Q 48
#define ORACLE_MAX_N 10

#define ORACLE_SCALAR 0
#define ORACLE_VECTOR 1

#define ORACLE_MAT_SINCOSEXP 0
#define ORACLE_MAT_ROTDIAG 1
#define ORACLE_MAT_PLANEWAVE 2
#define ORACLE_ALPHA_SAMPLED 3

#define ORACLE_STATUS_DETJ 1u
#define ORACLE_STATUS_NONFINITE 2u

#ifdef __cplusplus
extern "C" {
#endif

int oracle_gauss_legendre(int Q, double *x, double *w);
double oracle_phi(int m, double t);
double oracle_dphi(int m, double t);
double oracle_psi(int m, double t);
void oracle_map(const double *nodes, double u, double v, double w,
                double x[3], double J[3][3]);
void oracle_eps(int material, const double *p, const double x[3],
                double eps[3][3]);
int oracle_material_params(int material);
int oracle_num_fields(int problem);
int64_t oracle_num_dofs(int problem, int N);
double oracle_coupling(int problem, int material, const double *mp,
                       const double *nodes, int Qu, int Qv, int Qw,
                       double *out);
int oracle_fill(int problem, int material, int64_t E,
                const double *nodes, const double *mat,
                const int32_t *orders, const int32_t *quad,
                const int64_t *offsets, double sK, double sM,
                double *out, uint32_t *status, int nthreads);
int oracle_moments(int problem, int material, const double *mp,
                   const double *nodes, int Qu, int Qv, int Qw, int K,
                   double *out);

#ifdef __cplusplus
}
#endif

#endif
