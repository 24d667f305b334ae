// p2s_tables.cpp -- host construction of the FP64 tables used by the fill:
// Gauss-Legendre rules, Legendre moment weights and the product-to-sum
// (linearization) coefficients of eq. (3).  Built once per context.
#include <cmath>
#include <cstring>
#include <vector>

#include "p2s_internal.h"
#include "p2s_tables.h"

namespace p2s {

// Legendre values L_0..L_n at t (Bonnet recurrence).
static void legendre_values(int n, double t, double *L)
{
    L[0] = 1.0;
    if (n > 0) L[1] = t;
    for (int k = 2; k <= n; ++k)
        L[k] = ((2 * k - 1) * t * L[k - 1] - (k - 1) * L[k - 2]) / k;
}

int gauss_rule(int Q, double *x, double *w)
{
    if (Q < 1 || Q > MAXQ) return -1;
    const double pi = 3.141592653589793238462643383279502884;
    std::vector<double> L(Q + 1);
    // roots are symmetric: solve for the nonnegative half, mirror the rest
    for (int i = 0; i < (Q + 1) / 2; ++i) {
        // Tricomi-type initial guess for the (i+1)-th largest root
        double t = std::cos(pi * (4.0 * i + 3.0) / (4.0 * Q + 2.0));
        double dL = 0.0;
        for (int it = 0; it < 64; ++it) {
            legendre_values(Q, t, L.data());
            dL = Q * (t * L[Q] - L[Q - 1]) / (t * t - 1.0);
            double step = L[Q] / dL;
            t -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(t) + 1e-300) break;
        }
        legendre_values(Q, t, L.data());
        dL = Q * (t * L[Q] - L[Q - 1]) / (t * t - 1.0);
        double wt = 2.0 / ((1.0 - t * t) * dL * dL);
        x[Q - 1 - i] = t;
        w[Q - 1 - i] = wt;
        x[i] = -t;
        w[i] = wt;
    }
    if (Q % 2 == 1) x[Q / 2] = 0.0;  // exact centre root
    return 0;
}

// Legendre coefficients of family member m (length KPAD).
static void family_coefficients(int fam, int m, double *c)
{
    std::memset(c, 0, sizeof(double) * KPAD);
    if (fam == PHI) {
        if (m == 0) { c[0] = 0.5; c[1] = -0.5; return; }
        if (m == 1) { c[0] = 0.5; c[1] = 0.5; return; }
        double s = 1.0 / std::sqrt(2.0 * (2 * m - 1));
        c[m] = s;
        c[m - 2] = -s;
    } else if (fam == DPHI) {
        if (m == 0) { c[0] = -0.5; return; }
        if (m == 1) { c[0] = 0.5; return; }
        c[m - 1] = std::sqrt((2 * m - 1) / 2.0);
    } else {
        c[m] = std::sqrt((2 * m + 1) / 2.0);
    }
}

// Adams-Neumann linearization of a Legendre product:
// L_a L_b = sum_{r=0}^{min(a,b)} A_{a-r} A_r A_{b-r} / A_{a+b-r}
//           * (2a+2b-4r+1)/(2a+2b-2r+1) * L_{a+b-2r},
// with A_r = (2r-1)!!/r!  (A_0 = 1, A_r = A_{r-1} (2r-1)/r).
static void legendre_product(int a, int b, double *out /* KPAD + ... */)
{
    double A[2 * KPAD + 1];
    A[0] = 1.0;
    for (int r = 1; r <= 2 * KPAD; ++r) A[r] = A[r - 1] * (2.0 * r - 1.0) / r;
    int mn = a < b ? a : b;
    for (int r = 0; r <= mn; ++r) {
        int k = a + b - 2 * r;
        double c = A[a - r] * A[r] * A[b - r] / A[a + b - r] *
                   (2.0 * (a + b) - 4.0 * r + 1.0) / (2.0 * (a + b) - 2.0 * r + 1.0);
        out[k] += c;
    }
}

int linearization(int xf, int m1, int yf, int m2, double *coef)
{
    if (xf < 0 || xf >= NFAM || yf < 0 || yf >= NFAM) return -1;
    if (m1 < 0 || m2 < 0 || m1 >= MAXN || m2 >= MAXN) return -1;
    double cx[KPAD], cy[KPAD];
    family_coefficients(xf, m1, cx);
    family_coefficients(yf, m2, cy);
    double acc[4 * KPAD];
    std::memset(acc, 0, sizeof(acc));
    for (int a = 0; a < KPAD; ++a) {
        if (cx[a] == 0.0) continue;
        for (int b = 0; b < KPAD; ++b) {
            if (cy[b] == 0.0) continue;
            double tmp[4 * KPAD];
            std::memset(tmp, 0, sizeof(tmp));
            legendre_product(a, b, tmp);
            for (int k = 0; k < 4 * KPAD; ++k) acc[k] += cx[a] * cy[b] * tmp[k];
        }
    }
    // degrees beyond 2*MAXN-2 cannot occur for m1, m2 < MAXN
    uint32_t mask = prod_mask(xf, m1, yf, m2);
    for (int k = 0; k < KPAD; ++k) coef[k] = ((mask >> k) & 1u) ? acc[k] : 0.0;
    return 0;
}

void build_tables(double *tab)
{
    std::memset(tab, 0, sizeof(double) * TAB_SIZE);
    for (int xf = 0; xf < NFAM; ++xf)
        for (int yf = 0; yf < NFAM; ++yf)
            for (int m1 = 0; m1 < MAXN; ++m1)
                for (int m2 = 0; m2 < MAXN; ++m2)
                    linearization(xf, m1, yf, m2,
                                  tab + TAB_LIN + (3 * xf + yf) * LIN_STRIDE_T +
                                      m1 * LIN_STRIDE_M1 + m2 * KPAD);
    // packed copies in consumption order of the last contraction stage
    for (int N = 2; N <= MAXN; ++N)
        for (int X = 0; X < NFAM; ++X)
            for (int Y = 0; Y < NFAM; ++Y) {
                double *dst = tab + TAB_PACK + packed_offset(N, X, Y);
                const double *src = tab + TAB_LIN + (3 * X + Y) * LIN_STRIDE_T;
                int n = 0;
                for (int p1 = 0; p1 < fam_dim(X, N); ++p1)
                    for (int p2 = 0; p2 < fam_dim(Y, N); ++p2) {
                        const uint32_t m = prod_mask(X, p1, Y, p2);
                        for (int q = 0; q < KPAD; ++q)
                            if ((m >> q) & 1u) dst[n++] = src[p1 * LIN_STRIDE_M1 + p2 * KPAD + q];
                    }
            }
    double L[KPAD];
    for (int Q = 1; Q <= MAXQ; ++Q) {
        double *x = tab + TAB_GX + Q * MAXQ;
        double *w = tab + TAB_GW + Q * MAXQ;
        gauss_rule(Q, x, w);
        // basis values at the points from the Legendre expansions
        for (int a = 0; a < Q; ++a) {
            legendre_values(KPAD - 1, x[a], L);
            for (int fam = 0; fam < NFAM; ++fam)
                for (int m = 0; m < MAXN; ++m) {
                    double c[KPAD], v = 0.0;
                    family_coefficients(fam, m, c);
                    for (int k = 0; k < KPAD; ++k) v += c[k] * L[k];
                    tab[TAB_BASIS + Q * BASIS_STRIDE_Q + (fam * MAXN + m) * MAXQ + a] = v;
                }
        }
        for (int a = 0; a < Q; ++a) {
            legendre_values(KPAD - 1, x[a], L);
            for (int k = 0; k < KPAD; ++k)
                tab[TAB_LEGW + Q * LEGW_STRIDE_Q + k * MAXQ + a] = w[a] * L[k];
        }
        if (Q % 2 == 0 && Q / 2 >= 2 && Q / 2 <= MAXN) {
            const int N = Q / 2;
            const double *bas = tab + TAB_BASIS + Q * BASIS_STRIDE_Q;
            for (int X = 0; X < NFAM; ++X)
                for (int Y = 0; Y < NFAM; ++Y)
                    for (int m1 = 0; m1 < fam_dim(X, N); ++m1)
                        for (int m2 = 0; m2 < fam_dim(Y, N); ++m2)
                            for (int a = 0; a < Q; ++a)
                                tab[TAB_PT + N * PT_STRIDE_N + (3 * X + Y) * LIN_STRIDE_T + m1 * LIN_STRIDE_M1 +
                                    m2 * KPAD + a] = w[a] * bas[(X * MAXN + m1) * MAXQ + a] *
                                                     bas[(Y * MAXN + m2) * MAXQ + a];
        }
        double LL[MAXQ];
        for (int a = 0; a < Q; ++a) {
            legendre_values(Q - 1, x[a], LL);
            for (int j = 0; j < 4; ++j) {
                const int d = Q - 1 - j;
                tab[TAB_TAILW + Q * TAILW_STRIDE_Q + j * MAXQ + a] = d >= 0 ? 0.5 * (2 * d + 1) * w[a] * LL[d] : 0.0;
            }
        }
    }
}

}  // namespace p2s
