// p2s_kernels.h -- host launchers of the HIP kernels (p2s_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "p2s_internal.h"

namespace p2s {

// Largest LDS a workgroup may use on gfx950.
constexpr size_t LDS_LIMIT = 160 * 1024;

int prepare_kernels();
size_t moments_smem_bytes(int maxN, int maxQu, int maxQuv);

void launch_coupling(int problem, const ElemDesc *desc, int64_t e0, int64_t count,
                     const double *nodes, const double *mat, int kind, int mat_stride,
                     const double *tab, double *alpha, uint32_t *status, hipStream_t st);
void launch_moments(int problem, int maxN, int maxQu, int maxQuv, const ElemDesc *desc, int64_t e0,
                    int64_t count, const double *alpha, const double *tab, double *mom, hipStream_t st);
int launch_contract(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0,
                    int64_t count, const double *tab, const double *mom, double *out, uint32_t *status,
                    double sK, double sM, hipStream_t st);

// One launch over a cost-sorted work list (scalar problem, mixed orders).
int launch_contract_persistent(int problem, const ElemDesc *desc, const WorkItem *items, int64_t nitems,
                               int32_t *counter, int grid, const double *tab, const double *mom, double *out,
                               uint32_t *status, double sK, double sM, hipStream_t st);

// Direct quadrature of eq. (2) (baseline method), from coupling samples.
void launch_direct(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count, const double *tab,
                   const double *alpha, double *out, double sK, double sM, hipStream_t st);

}  // namespace p2s
