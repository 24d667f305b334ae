// p2s_contract.hip -- the contraction stage of the product-to-sum fill,
// eq. (4) of the paper, for gfx950 (wave64): per-block launches of the
// kernels in p2s_contract_impl.h over the moments, and a persistent
// schedule for batches of mixed orders.
#include "p2s_contract_impl.h"

namespace p2s {

// ---------------------------------------------------------------------------
// Persistent schedule for batches of mixed orders: one launch of a fixed
// grid; every workgroup takes the next work item (element, component, m1)
// from a list sorted by decreasing cost (longest-processing-time first)
// through an atomic counter, and leaves when the list is exhausted.

template <int PROB>
struct PersistentShape {
    static constexpr int threads()
    {
        int m = 0;
        m = cmax(m, CS<PROB, 2, 0>::THREADS); m = cmax(m, CS<PROB, 3, 0>::THREADS);
        m = cmax(m, CS<PROB, 4, 0>::THREADS); m = cmax(m, CS<PROB, 5, 0>::THREADS);
        m = cmax(m, CS<PROB, 6, 0>::THREADS); m = cmax(m, CS<PROB, 7, 0>::THREADS);
        m = cmax(m, CS<PROB, 8, 0>::THREADS);
        return m;
    }
    static constexpr int buf()
    {
        int m = 0;
        m = cmax(m, CS<PROB, 2, 0>::BUF); m = cmax(m, CS<PROB, 3, 0>::BUF);
        m = cmax(m, CS<PROB, 4, 0>::BUF); m = cmax(m, CS<PROB, 5, 0>::BUF);
        m = cmax(m, CS<PROB, 6, 0>::BUF); m = cmax(m, CS<PROB, 7, 0>::BUF);
        m = cmax(m, CS<PROB, 8, 0>::BUF);
        return m;
    }
    static constexpr int THREADS = threads();
    static constexpr int BUF = buf();
};

__global__ void k_reset_counter(int32_t *counter) { *counter = 0; }

__global__ __launch_bounds__(PersistentShape<0>::THREADS) void k_contract_persistent_scalar(
    const ElemDesc *__restrict__ desc, const WorkItem *__restrict__ items, int32_t nitems,
    int32_t *__restrict__ counter, const double *__restrict__ tab, const double *__restrict__ mom,
    double *__restrict__ out, uint32_t *__restrict__ status, double sK, double sM)
{
    __shared__ __attribute__((aligned(16))) double smem[PersistentShape<0>::BUF];
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = next;
        __syncthreads();  // every thread has read `next` before it is overwritten
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const ElemDesc d = desc[w.e];
        switch (d.N) {
        case 2: contract_item<0, 2, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        case 3: contract_item<0, 3, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        case 4: contract_item<0, 4, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        case 5: contract_item<0, 5, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        case 6: contract_item<0, 6, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        case 7: contract_item<0, 7, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        default: contract_item<0, 8, 0>(d, w.e, w.m1, tab, mom, out, status, sK, sM, smem, blockDim.x); break;
        }
    }
}

int launch_contract_persistent(int problem, const ElemDesc *desc, const WorkItem *items, int64_t nitems,
                               int32_t *counter, int grid, const double *tab, const double *mom, double *out,
                               uint32_t *status, double sK, double sM, hipStream_t st)
{
    if (problem != 0) return -1;
    if (nitems <= 0) return 0;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, counter);
    hipLaunchKernelGGL(k_contract_persistent_scalar, dim3(grid), dim3(PersistentShape<0>::THREADS), 0, st,
                       desc, items, (int32_t)nitems, counter, tab, mom, out, status, sK, sM);
    return 0;
}

int launch_contract(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0,
                    int64_t count, const double *tab, const double *mom, double *out, uint32_t *status,
                    double sK, double sM, hipStream_t st)
{
    if (count <= 0) return 0;
#define P2S_CASE(P, n)                                                                             \
    if (problem == P && N == n) {                                                                  \
        launch_contract_t<P, n>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);        \
        return 0;                                                                                  \
    }
    P2S_CASE(0, 2) P2S_CASE(0, 3) P2S_CASE(0, 4) P2S_CASE(0, 5) P2S_CASE(0, 6) P2S_CASE(0, 7) P2S_CASE(0, 8)
    P2S_CASE(1, 2) P2S_CASE(1, 3) P2S_CASE(1, 4) P2S_CASE(1, 5) P2S_CASE(1, 6) P2S_CASE(1, 7) P2S_CASE(1, 8)
#undef P2S_CASE
    return -1;
}

}  // namespace p2s

