/*
 * oracle.c -- plain FP64 CPU oracle for the hierarchical element-matrix fill.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes: the discrete Galerkin element matrix of eq. (2) of the
 * paper (Section II): every entry is obtained by a direct, full
 * three-dimensional tensor Gauss-Legendre quadrature of
 *     (test basis factor) x (coupling factor alpha_s) x (trial basis factor)
 * summed over the coupling terms s.  This is the "direct numerical
 * integration" the paper compares against (Section IV); no product-to-sum
 * identity (eq. 3) is used here.  Because eq. (3) is an exact polynomial
 * identity, the product-to-sum result equals this discrete value up to
 * rounding when both use the same Gauss rule (Section V: the method does not
 * change accuracy).
 *
 * Instance (the paper leaves the 3-D basis, geometry and material open):
 *  - reference cube (u,v,w) in [-1,1]^3 (the integration limits of eq. 2);
 *  - geometry: isoparametric triquadratic Lagrange map with 27 nodes on
 *    {-1,0,1}^3 (Section IV assumes isoparametric Lagrangian geometry);
 *  - basis (eq. 1): integrated Legendre, phi_0=(1-t)/2, phi_1=(1+t)/2,
 *    phi_m=(L_m-L_{m-2})/sqrt(2(2m-1)), m>=2; the curl-conforming vector
 *    basis takes psi_m=sqrt((2m+1)/2) L_m along the component's own axis
 *    and phi along the other two (3-D analogue of eq. 6);
 *  - scalar problem: anisotropic diffusion + mass,
 *      a(u,v) = s_K * int eps grad u . grad v + s_M * int eps u v;
 *  - vector problem: curl-curl + mass (3-D analogue of eqs. 5 and 7),
 *      a(E,F) = s_K * int (1/mu) curl E . curl F + s_M * int E . eps F,
 *    mu = 1, covariant Piola map E = J^{-T} E_hat.
 *
 * Parity status of each function is stated at the function.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* 1-D polynomial algebra                                              */
/* ------------------------------------------------------------------ */

/* Legendre L_0..L_n at t by the three-term (Bonnet) recurrence. */
static void legendre_upto(int n, double t, double *L)
{
    L[0] = 1.0;
    if (n >= 1) L[1] = t;
    for (int k = 1; k < n; ++k)
        L[k + 1] = ((2.0 * k + 1.0) * t * L[k] - k * L[k - 1]) / (k + 1.0);
}

/*
 * Gauss-Legendre rule with Q points on [-1,1]: Newton iteration on L_Q with
 * the derivative from (1-t^2) L_Q' = Q (L_{Q-1} - t L_Q); weights
 * w = 2 / ((1-t^2) L_Q'(t)^2).  Pinned against numpy's leggauss and against
 * polynomial exactness up to degree 2Q-1.
 */
int oracle_gauss_legendre(int Q, double *x, double *w)
{
    if (Q < 1 || Q > ORACLE_MAX_Q) return -1;
    const double pi = 3.14159265358979323846;
    double L[ORACLE_MAX_Q + 2];
    for (int i = 0; i < Q; ++i) {
        /* standard initial guess, roots ordered from +1 down to -1 */
        double t = cos(pi * (i + 0.75) / (Q + 0.5));
        for (int it = 0; it < 100; ++it) {
            legendre_upto(Q, t, L);
            double dp = Q * (L[Q - 1] - t * L[Q]) / (1.0 - t * t);
            double dt = L[Q] / dp;
            t -= dt;
            if (fabs(dt) < 1e-17) break;
        }
        legendre_upto(Q, t, L);
        double dp = Q * (L[Q - 1] - t * L[Q]) / (1.0 - t * t);
        /* store ascending */
        x[Q - 1 - i] = t;
        w[Q - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    return 0;
}

/* phi_m(t): integrated Legendre (hierarchical) shape function. */
double oracle_phi(int m, double t)
{
    if (m == 0) return 0.5 * (1.0 - t);
    if (m == 1) return 0.5 * (1.0 + t);
    double L[64];
    legendre_upto(m, t, L);
    return (L[m] - L[m - 2]) / sqrt(2.0 * (2.0 * m - 1.0));
}

/* phi_m'(t): derivative, using d/dt (L_m - L_{m-2}) = (2m-1) L_{m-1}. */
double oracle_dphi(int m, double t)
{
    if (m == 0) return -0.5;
    if (m == 1) return 0.5;
    double L[64];
    legendre_upto(m, t, L);
    return sqrt((2.0 * m - 1.0) / 2.0) * L[m - 1];
}

/* psi_m(t) = sqrt((2m+1)/2) L_m(t): orthonormal Legendre. */
double oracle_psi(int m, double t)
{
    double L[64];
    legendre_upto(m, t, L);
    return sqrt((2.0 * m + 1.0) / 2.0) * L[m];
}

/* ------------------------------------------------------------------ */
/* Geometry: triquadratic Lagrange map                                 */
/* ------------------------------------------------------------------ */

static void lagrange3(double t, double l[3], double dl[3])
{
    l[0] = 0.5 * t * (t - 1.0);
    l[1] = 1.0 - t * t;
    l[2] = 0.5 * t * (t + 1.0);
    dl[0] = t - 0.5;
    dl[1] = -2.0 * t;
    dl[2] = t + 0.5;
}

/* x(u,v,w) and J[r][c] = d x_r / d u_c for the 27-node element whose node
 * (i,j,k) (i along u) is stored at nodes[3*(i + 3j + 9k) + r]. */
void oracle_map(const double *nodes, double u, double v, double w,
                double x[3], double J[3][3])
{
    double lu[3], lv[3], lw[3], du[3], dv[3], dw[3];
    lagrange3(u, lu, du);
    lagrange3(v, lv, dv);
    lagrange3(w, lw, dw);
    for (int r = 0; r < 3; ++r) {
        x[r] = 0.0;
        J[r][0] = J[r][1] = J[r][2] = 0.0;
    }
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                const double *X = nodes + 3 * (i + 3 * j + 9 * k);
                double s = lu[i] * lv[j] * lw[k];
                double su = du[i] * lv[j] * lw[k];
                double sv = lu[i] * dv[j] * lw[k];
                double sw = lu[i] * lv[j] * dw[k];
                for (int r = 0; r < 3; ++r) {
                    x[r] += s * X[r];
                    J[r][0] += su * X[r];
                    J[r][1] += sv * X[r];
                    J[r][2] += sw * X[r];
                }
            }
}

static double det3(double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* inverse by adjugate / determinant */
static void inv3(double J[3][3], double d, double Ji[3][3])
{
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
}

/* ------------------------------------------------------------------ */
/* Materials                                                           */
/* ------------------------------------------------------------------ */

int oracle_material_params(int material)
{
    switch (material) {
    case ORACLE_MAT_SINCOSEXP: return 1;
    case ORACLE_MAT_ROTDIAG: return 12;
    case ORACLE_MAT_PLANEWAVE: return 4;
    default: return -1;
    }
}

/* Full 3x3 permittivity tensor eps(x) for the analytic materials. */
void oracle_eps(int material, const double *p, const double x[3],
                double eps[3][3])
{
    memset(eps, 0, 9 * sizeof(double));
    if (material == ORACLE_MAT_SINCOSEXP) {
        double k = p[0];
        double e = 1.0 + 0.5 * sin(k * x[0]) * cos(k * x[1]) * exp(-x[2]);
        eps[0][0] = eps[1][1] = eps[2][2] = e;
    } else if (material == ORACLE_MAT_PLANEWAVE) {
        double ph = p[0] * x[0] + p[1] * x[1] + p[2] * x[2] + p[3];
        double e = 1.0 + 0.8 * sin(ph);
        eps[0][0] = eps[1][1] = eps[2][2] = e;
    } else if (material == ORACLE_MAT_ROTDIAG) {
        /* eps = R^T diag(d) R with R row-major in p[0..8], k in p[9..11],
         * d_a = 1 + 0.5 sin(k.x + 2 pi a / 3). */
        const double *R = p;
        double kx = p[9] * x[0] + p[10] * x[1] + p[11] * x[2];
        const double two_pi_3 = 2.0 * 3.14159265358979323846 / 3.0;
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = 1.0 + 0.5 * sin(kx + two_pi_3 * a);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int a = 0; a < 3; ++a) s += R[3 * a + r] * d[a] * R[3 * a + c];
                eps[r][c] = s;
            }
    }
}

/* ------------------------------------------------------------------ */
/* Coupling factors at one point                                       */
/* ------------------------------------------------------------------ */

/*
 * Coupling factors of eq. (2) at one reference point.
 * Scalar problem: A = eps * detJ * J^{-1} J^{-T} (stiffness, 3x3) and
 *   am = eps * detJ (mass); eps must be isotropic (a multiple of I).
 * Vector problem: C = J^T J / (mu detJ) (curl-curl, mu = 1) and
 *   Mt = detJ * J^{-1} eps J^{-T} (mass).
 * Returns detJ.
 */
static double coupling_at(int problem, int material, const double *mp,
                          const double *nodes, double u, double v, double w,
                          double K[3][3], double Mt[3][3], double *am)
{
    double x[3], J[3][3], Ji[3][3], eps[3][3];
    oracle_map(nodes, u, v, w, x, J);
    double d = det3(J);
    inv3(J, d, Ji);
    oracle_eps(material, mp, x, eps);
    if (problem == ORACLE_SCALAR) {
        double e = eps[0][0];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int r = 0; r < 3; ++r) s += Ji[a][r] * Ji[b][r];
                K[a][b] = e * d * s;
            }
        *am = e * d;
    } else {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int r = 0; r < 3; ++r) s += J[r][a] * J[r][b];
                K[a][b] = s / d;
            }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) s += Ji[a][r] * eps[r][c] * Ji[b][c];
                Mt[a][b] = d * s;
            }
        *am = 0.0;
    }
    return d;
}

/* symmetric 3x3 from six stored values (00,11,22,01,02,12) */
static void sym_from6(const double *s6, double A[3][3])
{
    A[0][0] = s6[0]; A[1][1] = s6[1]; A[2][2] = s6[2];
    A[0][1] = A[1][0] = s6[3];
    A[0][2] = A[2][0] = s6[4];
    A[1][2] = A[2][1] = s6[5];
}

int oracle_num_fields(int problem)
{
    return problem == ORACLE_SCALAR ? 7 : 12;
}

int64_t oracle_num_dofs(int problem, int N)
{
    if (problem == ORACLE_SCALAR) return (int64_t)N * N * N;
    return 3 * (int64_t)(N - 1) * N * N;
}

/*
 * Coupling factors at all Qu*Qv*Qw Gauss points of one element, in the
 * packed field order used for sampled input:
 *   scalar: A00 A11 A22 A01 A02 A12 am         (7 fields)
 *   vector: C00 C11 C22 C01 C02 C12 M00 M11 M22 M01 M02 M12  (12 fields)
 * out[f * P + (a*Qv + b)*Qw + c], P = Qu*Qv*Qw, point (a,b,c) at
 * (xu[a], xv[b], xw[c]).  Unweighted.  Returns min detJ.
 */
double oracle_coupling(int problem, int material, const double *mp,
                       const double *nodes, int Qu, int Qv, int Qw,
                       double *out)
{
    double xu[ORACLE_MAX_Q], wu[ORACLE_MAX_Q], xv[ORACLE_MAX_Q], wv[ORACLE_MAX_Q];
    double xw[ORACLE_MAX_Q], ww[ORACLE_MAX_Q];
    oracle_gauss_legendre(Qu, xu, wu);
    oracle_gauss_legendre(Qv, xv, wv);
    oracle_gauss_legendre(Qw, xw, ww);
    int64_t P = (int64_t)Qu * Qv * Qw;
    double mind = INFINITY;
    for (int a = 0; a < Qu; ++a)
        for (int b = 0; b < Qv; ++b)
            for (int c = 0; c < Qw; ++c) {
                double K[3][3], Mt[3][3], am;
                double d = coupling_at(problem, material, mp, nodes, xu[a], xv[b], xw[c], K, Mt, &am);
                if (d < mind) mind = d;
                int64_t pt = ((int64_t)a * Qv + b) * Qw + c;
                double f[12];
                f[0] = K[0][0]; f[1] = K[1][1]; f[2] = K[2][2];
                f[3] = K[0][1]; f[4] = K[0][2]; f[5] = K[1][2];
                if (problem == ORACLE_SCALAR) {
                    f[6] = am;
                } else {
                    f[6] = Mt[0][0]; f[7] = Mt[1][1]; f[8] = Mt[2][2];
                    f[9] = Mt[0][1]; f[10] = Mt[0][2]; f[11] = Mt[1][2];
                }
                int F = oracle_num_fields(problem);
                for (int q = 0; q < F; ++q) out[q * P + pt] = f[q];
            }
    return mind;
}

/* ------------------------------------------------------------------ */
/* Basis values at one point                                           */
/* ------------------------------------------------------------------ */

/* scalar dof (m,n,p) -> value and reference gradient */
static void scalar_basis(int N, double u, double v, double w,
                         double *val, double (*grad)[3])
{
    double pu[16], pv[16], pw[16], du[16], dv[16], dw[16];
    for (int m = 0; m < N; ++m) {
        pu[m] = oracle_phi(m, u); du[m] = oracle_dphi(m, u);
        pv[m] = oracle_phi(m, v); dv[m] = oracle_dphi(m, v);
        pw[m] = oracle_phi(m, w); dw[m] = oracle_dphi(m, w);
    }
    int i = 0;
    for (int m = 0; m < N; ++m)
        for (int n = 0; n < N; ++n)
            for (int p = 0; p < N; ++p, ++i) {
                val[i] = pu[m] * pv[n] * pw[p];
                grad[i][0] = du[m] * pv[n] * pw[p];
                grad[i][1] = pu[m] * dv[n] * pw[p];
                grad[i][2] = pu[m] * pv[n] * dw[p];
            }
}

/*
 * vector dof of component g (0:u, 1:v, 2:w): E_hat = f e_g with
 * f = psi along axis g and phi along the other two axes.  Orders per
 * component: (N-1,N,N), (N,N-1,N), (N,N,N-1).  Writes E_hat and its
 * reference curl for every dof, blocks in component order, (m,n,p) with
 * p fastest inside a block.
 */
static void vector_basis(int N, double u, double v, double w,
                         double (*E)[3], double (*curl)[3])
{
    double t[3] = {u, v, w};
    double ph[3][16], dph[3][16], ps[3][16];
    for (int ax = 0; ax < 3; ++ax)
        for (int m = 0; m < N; ++m) {
            ph[ax][m] = oracle_phi(m, t[ax]);
            dph[ax][m] = oracle_dphi(m, t[ax]);
            ps[ax][m] = oracle_psi(m, t[ax]);
        }
    int i = 0;
    for (int g = 0; g < 3; ++g) {
        int dims[3] = {N, N, N};
        dims[g] = N - 1;
        for (int m = 0; m < dims[0]; ++m)
            for (int n = 0; n < dims[1]; ++n)
                for (int p = 0; p < dims[2]; ++p, ++i) {
                    int idx[3] = {m, n, p};
                    double val[3], der[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        if (ax == g) {
                            val[ax] = ps[ax][idx[ax]];
                            der[ax] = 0.0; /* never used: curl has no d/d(own axis) */
                        } else {
                            val[ax] = ph[ax][idx[ax]];
                            der[ax] = dph[ax][idx[ax]];
                        }
                    }
                    double f = val[0] * val[1] * val[2];
                    double fu = der[0] * val[1] * val[2];
                    double fv = val[0] * der[1] * val[2];
                    double fw = val[0] * val[1] * der[2];
                    E[i][0] = E[i][1] = E[i][2] = 0.0;
                    E[i][g] = f;
                    if (g == 0) { curl[i][0] = 0.0; curl[i][1] = fw;  curl[i][2] = -fv; }
                    if (g == 1) { curl[i][0] = -fw; curl[i][1] = 0.0; curl[i][2] = fu; }
                    if (g == 2) { curl[i][0] = fv;  curl[i][1] = -fu; curl[i][2] = 0.0; }
                }
    }
}

/* ------------------------------------------------------------------ */
/* The fill: direct full 3-D quadrature of eq. (2)                     */
/* ------------------------------------------------------------------ */

static int fill_one(int problem, int material, const double *mp,
                    const double *nodes, int N, int Qu, int Qv, int Qw,
                    double sK, double sM, double *M, uint32_t *st)
{
    int64_t nd = oracle_num_dofs(problem, N);
    double xu[ORACLE_MAX_Q], wu[ORACLE_MAX_Q], xv[ORACLE_MAX_Q], wv[ORACLE_MAX_Q];
    double xw[ORACLE_MAX_Q], ww[ORACLE_MAX_Q];
    oracle_gauss_legendre(Qu, xu, wu);
    oracle_gauss_legendre(Qv, xv, wv);
    oracle_gauss_legendre(Qw, xw, ww);

    double *val = NULL, (*g)[3] = NULL, (*E)[3] = NULL, (*C)[3] = NULL;
    if (problem == ORACLE_SCALAR) {
        val = (double *)malloc(sizeof(double) * nd);
        g = (double (*)[3])malloc(sizeof(double) * 3 * nd);
    } else {
        E = (double (*)[3])malloc(sizeof(double) * 3 * nd);
        C = (double (*)[3])malloc(sizeof(double) * 3 * nd);
    }
    memset(M, 0, sizeof(double) * nd * nd);
    uint32_t status = 0;
    int F = oracle_num_fields(problem);
    int64_t P = (int64_t)Qu * Qv * Qw;

    for (int a = 0; a < Qu; ++a)
        for (int b = 0; b < Qv; ++b)
            for (int c = 0; c < Qw; ++c) {
                double W = wu[a] * wv[b] * ww[c];
                double K[3][3], Mt[3][3], am = 0.0;
                if (material == ORACLE_ALPHA_SAMPLED) {
                    int64_t pt = ((int64_t)a * Qv + b) * Qw + c;
                    double f[12];
                    for (int q = 0; q < F; ++q) f[q] = mp[q * P + pt];
                    sym_from6(f, K);
                    if (problem == ORACLE_SCALAR) am = f[6];
                    else sym_from6(f + 6, Mt);
                } else {
                    double d = coupling_at(problem, material, mp, nodes,
                                           xu[a], xv[b], xw[c], K, Mt, &am);
                    if (!(d > 0.0)) status |= ORACLE_STATUS_DETJ;
                }
                if (problem == ORACLE_SCALAR) {
                    scalar_basis(N, xu[a], xv[b], xw[c], val, g);
                    for (int64_t i = 0; i < nd; ++i) {
                        double Kg[3];
                        for (int r = 0; r < 3; ++r)
                            Kg[r] = K[r][0] * g[i][0] + K[r][1] * g[i][1] + K[r][2] * g[i][2];
                        for (int64_t j = 0; j < nd; ++j) {
                            double stiff = Kg[0] * g[j][0] + Kg[1] * g[j][1] + Kg[2] * g[j][2];
                            double mass = am * val[i] * val[j];
                            M[i * nd + j] += W * (sK * stiff + sM * mass);
                        }
                    }
                } else {
                    vector_basis(N, xu[a], xv[b], xw[c], E, C);
                    for (int64_t i = 0; i < nd; ++i) {
                        double KC[3], ME[3];
                        for (int r = 0; r < 3; ++r) {
                            KC[r] = C[i][0] * K[0][r] + C[i][1] * K[1][r] + C[i][2] * K[2][r];
                            ME[r] = E[i][0] * Mt[0][r] + E[i][1] * Mt[1][r] + E[i][2] * Mt[2][r];
                        }
                        for (int64_t j = 0; j < nd; ++j) {
                            double stiff = KC[0] * C[j][0] + KC[1] * C[j][1] + KC[2] * C[j][2];
                            double mass = ME[0] * E[j][0] + ME[1] * E[j][1] + ME[2] * E[j][2];
                            M[i * nd + j] += W * (sK * stiff + sM * mass);
                        }
                    }
                }
            }
    for (int64_t i = 0; i < nd * nd; ++i)
        if (!isfinite(M[i])) { status |= ORACLE_STATUS_NONFINITE; break; }
    *st = status;
    free(val); free(g); free(E); free(C);
    return 0;
}

int oracle_fill(int problem, int material, int64_t E,
                const double *nodes, const double *mat,
                const int32_t *orders, const int32_t *quad,
                const int64_t *offsets, double sK, double sM,
                double *out, uint32_t *status, int nthreads)
{
    if (problem != ORACLE_SCALAR && problem != ORACLE_VECTOR) return -1;
    /* the scalar problem takes an isotropic permittivity only */
    if (problem == ORACLE_SCALAR && material == ORACLE_MAT_ROTDIAG) return -1;
    int P = oracle_material_params(material);
    if (material != ORACLE_ALPHA_SAMPLED && P < 0) return -1;
    for (int64_t e = 0; e < E; ++e) {
        int N = orders[e];
        if (N < 1 || N > ORACLE_MAX_N || (problem == ORACLE_VECTOR && N < 2)) return -2;
        for (int a = 0; a < 3; ++a)
            if (quad[3 * e + a] < 1 || quad[3 * e + a] > ORACLE_MAX_Q) return -3;
        int64_t nd = oracle_num_dofs(problem, N);
        if (offsets[e + 1] - offsets[e] != nd * nd) return -1;
    }
    /* per-element offset of the material/sampled data */
    int64_t *moff = (int64_t *)malloc(sizeof(int64_t) * (E + 1));
    moff[0] = 0;
    for (int64_t e = 0; e < E; ++e) {
        int64_t len = P;
        if (material == ORACLE_ALPHA_SAMPLED)
            len = (int64_t)oracle_num_fields(problem) * quad[3 * e] * quad[3 * e + 1] * quad[3 * e + 2];
        moff[e + 1] = moff[e] + len;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t e = 0; e < E; ++e) {
        fill_one(problem, material, mat + moff[e], nodes + 81 * e, orders[e],
                 quad[3 * e], quad[3 * e + 1], quad[3 * e + 2], sK, sM,
                 out + offsets[e], status + e);
    }
    free(moff);
    return 0;
}

/*
 * Moment tensor of eq. (4) by its plain definition, for tests of the
 * moment stage: I[f][k][l][q] = sum over all Gauss points of
 * w_a w_b w_c L_k(u_a) L_l(v_b) L_q(w_c) alpha_f(u_a,v_b,w_c),
 * for k,l,q < K and the packed coupling fields of oracle_coupling.
 */
int oracle_moments(int problem, int material, const double *mp,
                   const double *nodes, int Qu, int Qv, int Qw, int K,
                   double *out)
{
    if (K < 1 || K > 2 * ORACLE_MAX_N) return -1;
    int F = oracle_num_fields(problem);
    int64_t P = (int64_t)Qu * Qv * Qw;
    double *alpha = (double *)malloc(sizeof(double) * F * P);
    if (material == ORACLE_ALPHA_SAMPLED)
        memcpy(alpha, mp, sizeof(double) * F * P);
    else
        oracle_coupling(problem, material, mp, nodes, Qu, Qv, Qw, alpha);
    double xu[ORACLE_MAX_Q], wu[ORACLE_MAX_Q], xv[ORACLE_MAX_Q], wv[ORACLE_MAX_Q];
    double xw[ORACLE_MAX_Q], ww[ORACLE_MAX_Q];
    oracle_gauss_legendre(Qu, xu, wu);
    oracle_gauss_legendre(Qv, xv, wv);
    oracle_gauss_legendre(Qw, xw, ww);
    memset(out, 0, sizeof(double) * F * K * K * K);
    double Lu[2 * ORACLE_MAX_N + 2], Lv[2 * ORACLE_MAX_N + 2], Lw[2 * ORACLE_MAX_N + 2];
    for (int a = 0; a < Qu; ++a) {
        legendre_upto(K, xu[a], Lu);
        for (int b = 0; b < Qv; ++b) {
            legendre_upto(K, xv[b], Lv);
            for (int c = 0; c < Qw; ++c) {
                legendre_upto(K, xw[c], Lw);
                int64_t pt = ((int64_t)a * Qv + b) * Qw + c;
                double W = wu[a] * wv[b] * ww[c];
                for (int f = 0; f < F; ++f)
                    for (int k = 0; k < K; ++k)
                        for (int l = 0; l < K; ++l)
                            for (int q = 0; q < K; ++q)
                                out[(((int64_t)f * K + k) * K + l) * K + q] +=
                                    W * Lu[k] * Lv[l] * Lw[q] * alpha[f * P + pt];
            }
        }
    }
    free(alpha);
    return 0;
}
