// p2s_contract_packed.hip -- the product-to-sum contraction (eq. (4)) with
// packed symmetric output: each element matrix is stored as its upper
// triangle, row by row (row r holds columns c >= r), which halves the bytes
// written; the kernels are those of p2s_contract_impl.h without the mirrored
// stores.
#include "p2s_contract_impl.h"

namespace p2s {

int launch_contract_packed(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                           const double *tab, const double *mom, double *out, uint32_t *status, double sK, double sM,
                           hipStream_t st)
{
    if (count <= 0) return 0;
#define P2S_CASE(P, n)                                                                                     \
    if (problem == P && N == n) {                                                                          \
        launch_contract_t<P, n, false, true>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st); \
        return 0;                                                                                          \
    }
    P2S_CASE(0, 2) P2S_CASE(0, 3) P2S_CASE(0, 4) P2S_CASE(0, 5) P2S_CASE(0, 6) P2S_CASE(0, 7) P2S_CASE(0, 8)
    P2S_CASE(1, 2) P2S_CASE(1, 3) P2S_CASE(1, 4) P2S_CASE(1, 5) P2S_CASE(1, 6) P2S_CASE(1, 7) P2S_CASE(1, 8)
#undef P2S_CASE
    return -1;
}

}  // namespace p2s
