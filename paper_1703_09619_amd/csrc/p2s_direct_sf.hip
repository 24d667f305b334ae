// p2s_direct_sf.hip -- sum-factorized direct quadrature of eq. (2) on the
// GPU: the baseline against which the product-to-sum method's 3-D advantage
// is measured.  Every entry of a block is the Gauss sum
//   M = sign * sum_{a,b,c} Bu[m1][m2][a] Bv[n1][n2][b] Bw[p1][p2][c] alpha_s(a,b,c),
//   B[m1][m2][a] = w_a X_m1(x_a) Y_m2(x_a),
// taken one axis at a time (u, then v, then w) by the three stages of
// p2s_contract_impl.h with dense point tables in place of the sparse
// linearization tables and the coupling samples in place of the moments.
// The rule must have 2N points on every axis (the stages' extent).
#include "p2s_contract_impl.h"

namespace p2s {

int launch_contract_dsf(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                        const double *tab, const double *alpha, double *out, uint32_t *status, double sK, double sM,
                        hipStream_t st)
{
    if (count <= 0) return 0;
#define P2S_CASE(P, n)                                                                              \
    if (problem == P && N == n) {                                                                   \
        launch_contract_t<P, n, true>(desc, elist, e0, count, tab, alpha, out, status, sK, sM, st); \
        return 0;                                                                                   \
    }
    P2S_CASE(0, 2) P2S_CASE(0, 3) P2S_CASE(0, 4) P2S_CASE(0, 5) P2S_CASE(0, 6) P2S_CASE(0, 7) P2S_CASE(0, 8)
    P2S_CASE(1, 2) P2S_CASE(1, 3) P2S_CASE(1, 4) P2S_CASE(1, 5) P2S_CASE(1, 6) P2S_CASE(1, 7) P2S_CASE(1, 8)
#undef P2S_CASE
    return -1;
}

}  // namespace p2s
