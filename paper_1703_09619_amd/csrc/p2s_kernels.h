// p2s_kernels.h -- host launchers of the HIP kernels (p2s_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "p2s_internal.h"

namespace p2s {

// Largest LDS a workgroup may use on gfx950.
constexpr size_t LDS_LIMIT = 160 * 1024;

int prepare_kernels();
// Largest order and rule sizes of a plan, for the moment stage's LDS.
struct MomentShape {
    int maxN = 0, maxQ = 0;    // order; points on any axis
    int maxQu = 0, maxQuv = 0; // vector-unit form (rules of at most 16 points)
    int maxQw = 0, maxQvw = 0; // matrix-core form
};
size_t moments_smem_bytes(int maxN, int maxQw, int maxQvw, bool tail = false);
size_t moments_lds_bytes(const MomentShape &m);  // of the form launch_moments picks without tail records

// `only` (may be null): elements with only[e] == 0 are skipped; with it the
// coupling kernel ORs its status bits instead of overwriting them.
void launch_coupling(int problem, const ElemDesc *desc, int64_t e0, int64_t count,
                     const double *nodes, const double *mat, int kind, int mat_stride,
                     const double *tab, double *alpha, uint32_t *status, const int32_t *only, hipStream_t st);
// Moment stage: the matrix-core form with tail records when tailst is
// given, else the vector-unit form when every rule has at most 16 points,
// else the matrix-core form.  m bounds the shapes of the elements launched:
// elements e0..e0+count-1, or elist[e0..e0+count-1] when elist is given.
void launch_moments(int problem, const MomentShape &m, const ElemDesc *desc, int64_t e0, int64_t count,
                    const double *alpha, const double *tab, double *mom, const int32_t *only, double *tailst,
                    hipStream_t st, const int32_t *elist = nullptr);
int launch_contract(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0,
                    int64_t count, const double *tab, const double *mom, double *out, uint32_t *status,
                    double sK, double sM, hipStream_t st);

// The same contraction writing each element's upper triangle, packed row by
// row (p2s_contract_packed.hip).
int launch_contract_packed(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                           const double *tab, const double *mom, double *out, uint32_t *status, double sK, double sM,
                           hipStream_t st);

// Sum-factorized direct quadrature (p2s_direct_sf.hip): the contraction's
// three stages over the coupling samples alpha (rules of 2N points per axis).
int launch_contract_dsf(int problem, int N, const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                        const double *tab, const double *alpha, double *out, uint32_t *status, double sK, double sM,
                        hipStream_t st);

// One launch over a cost-sorted work list (scalar problem, mixed orders).
int launch_contract_persistent(int problem, const ElemDesc *desc, const WorkItem *items, int64_t nitems,
                               int32_t *counter, int grid, const double *tab, const double *mom, double *out,
                               uint32_t *status, double sK, double sM, hipStream_t st);

// Split-FP32 form of the moment stage and the contraction (p2s_split.hip):
// FP32 matrix-core products on exact operand slices, FP64 sums; FP64
// moments at mom + mom_off; uniform plans, Q <= 16.
// int8: the products on the INT8 matrix cores (seven-bit slices) instead of
// the FP32 ones.
void launch_moments_split(int problem, const ElemDesc *desc, int64_t e0, int64_t count, const double *alpha,
                          const double *tab, double *mom, bool int8, hipStream_t st);
void launch_contract_split(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count, const double *tab,
                           const double *mom, double *out, uint32_t *status, double sK, double sM, bool int8,
                           hipStream_t st);
int prepare_split_kernels();

// Direct quadrature of eq. (2) (baseline method), from coupling samples.
void launch_direct(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count, const double *tab,
                   const double *alpha, double *out, double sK, double sM, hipStream_t st);

// Learned quadrature order (p2s_learned.hip)
void launch_features(int64_t E, const double *nodes, const double *mat, int kind, int stride, float *X,
                     hipStream_t st);
void launch_mlp_forward(int64_t B, const float *params, const float *X, float *H1, float *H2, float *Z,
                        hipStream_t st);
void launch_mlp_backward(int64_t B, const float *params, const float *X, const float *H1, const float *H2,
                         const float *Z, const int32_t *labels, float *dZ, float *dH2, float *dH1, float *grad,
                         float *loss_b, float *loss, hipStream_t st);
void launch_adam(float *params, const float *grad, float *m, float *v, float lr, int step, hipStream_t st);
void launch_choose(int64_t E, const float *Z, float p_cover, int k_direct, int32_t *quad, ElemDesc *desc,
                   hipStream_t st);
void launch_tail_decide(ElemDesc *desc, int64_t e0, int64_t count, int F, const double *tailst, double theta,
                        int qfull, int32_t *redo, uint32_t *status, double *tau, hipStream_t st);
void launch_rel_error(int64_t E, int64_t len, const int64_t *off, const double *a, const double *b, double *err,
                      hipStream_t st);

}  // namespace p2s
