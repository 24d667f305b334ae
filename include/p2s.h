/*
 * p2s.h -- C ABI of the product-to-sum element-matrix fill for AMD Instinct
 * MI355X (gfx950).
 *
 * The library fills dense element matrices of a hierarchical finite-element
 * method on curved, inhomogeneous hexahedra (eq. (2) of Khodapanah, "A
 * Product to Sum Approach for Matrix Filling in a Hierarchical Finite-Element
 * Method", Section II) with the product-to-sum method:
 *   (a) moments:  I_s[k,l,q] = int int int L_k(u) L_l(v) L_q(w) alpha_s du dv dw
 *       by tensor Gauss quadrature of the sampled coupling factor alpha_s
 *       (the 3-D integrals of eq. (4));
 *   (b) tables:   every same-variable product of two 1-D basis/weighting
 *       functions is expanded in Legendre polynomials (eq. (3)), with
 *       coefficients tabulated once per context;
 *   (c) contraction: M = sum_s sum_{k,l,q} Cu Cv Cw I_s (eq. (4)), applied
 *       mode by mode.
 *
 * Instance of the paper's general form (Section II, eq. (1)):
 *   reference cube [-1,1]^3; triquadratic 27-node isoparametric map;
 *   integrated-Legendre basis phi_0=(1-t)/2, phi_1=(1+t)/2,
 *   phi_m=(L_m-L_{m-2})/sqrt(2(2m-1)); vector components use
 *   psi_m=sqrt((2m+1)/2) L_m along their own axis (orders (N-1,N,N),
 *   (N,N-1,N), (N,N,N-1), the 3-D analogue of eq. (6)).
 *
 *   P2S_SCALAR: stiff_scale * int eps grad(u).grad(v)
 *             + mass_scale  * int eps u v             (N^3 dofs)
 *   P2S_VECTOR: stiff_scale * int curl(E).curl(F)      (mu = 1)
 *             + mass_scale  * int E.eps F             (3 (N-1) N^2 dofs)
 *
 * Memory and ownership.  Pointers marked [device] are device memory on the
 * context's GPU, owned by the caller; [host] are host memory owned by the
 * caller.  The library owns its tables, plans and workspaces.  Calls that
 * take a stream enqueue work asynchronously on that HIP stream (NULL = the
 * default stream) and return after enqueueing; argument errors are detected
 * before anything is enqueued.  Execution calls allocate nothing.
 *
 * Errors.  Every int-returning call returns P2S_OK (0) or a negative
 * p2s_status; p2s_last_error() returns a message for the last failure on
 * that context.  Per-element numerical conditions are reported in the
 * status array, never in the return code.
 *
 * Thread safety.  A context may be used from one host thread at a time.
 */
#ifndef P2S_H
#define P2S_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p2s_ctx_s *p2s_ctx;
typedef struct p2s_plan_s *p2s_plan;

typedef enum {
    P2S_OK = 0,
    P2S_EINVAL = -1,   /* bad argument (null pointer, size, enum)          */
    P2S_EORDER = -2,   /* polynomial order outside [2, P2S_MAX_ORDER]       */
    P2S_EQUAD = -3,    /* Gauss points per axis outside [1, P2S_MAX_Q], or a
                          rule whose moment stage exceeds the 160 KiB of LDS
                          at the plan's largest order (order 8: up to 30
                          points per axis on a cubic rule; order 6 and
                          below: any allowed rule)                        */
    P2S_ENOMEM = -4,   /* device or host allocation failed (plan creation)  */
    P2S_EHIP = -5,     /* a HIP runtime call failed                         */
    P2S_ENODEV = -6,   /* no usable gfx950 device                           */
    P2S_ENOMODEL = -7  /* learned-order call without a loaded model         */
} p2s_status;

typedef enum { P2S_SCALAR = 0, P2S_VECTOR = 1 } p2s_problem;

/* Material models; material parameters per element, [E][P]:
 *  SINCOSEXP  P=1  eps = 1 + 0.5 sin(kappa x) cos(kappa y) exp(-z)  {kappa}
 *  ROTDIAG    P=12 eps = R^T diag(d) R, d_a = 1 + 0.5 sin(k.x + 2 pi a/3)
 *                  {R row-major (9), k (3)}                (vector only)
 *  PLANEWAVE  P=4  eps = 1 + 0.8 sin(k.x + phase)     {k (3), phase}
 *  ALPHA_SAMPLED   the coupling fields themselves at the Gauss points,
 *                  [E][F][Qu*Qv*Qw], point (a*Qv+b)*Qw+c (a along u),
 *                  F = 7 scalar (A00 A11 A22 A01 A02 A12 mass) or
 *                  12 vector (C00 C11 C22 C01 C02 C12 M00 M11 M22 M01 M02 M12);
 *                  all elements must share one rule; nodes are ignored.
 * Isotropic materials act as eps*I in the vector problem. */
typedef enum {
    P2S_MAT_SINCOSEXP = 0,
    P2S_MAT_ROTDIAG = 1,
    P2S_MAT_PLANEWAVE = 2,
    P2S_ALPHA_SAMPLED = 3
} p2s_material;

/* Arithmetic of stages (a) and (c).  FP64 throughout, or the split-FP32
 * form: every product of the moment and contraction GEMMs runs on the FP32
 * matrix cores on exact operand slices (per 16x16x4 step, each row and
 * column scaled by a power of two and split into four 10-bit integer
 * slices; the slice products of each order are summed exactly in FP32 and
 * added into FP64), with map/Jacobian/coupling/tables, intermediates and
 * every sum in FP64.  Relative error about 1e-11.  Uniform plans with at
 * most 16 Gauss points per axis (P2S_EQUAD otherwise). */
/* P2S_SPLIT_INT8: the same exact-slice products on the INT8 matrix cores
 * (v_mfma_i32_16x16x32_i8): per K-block of 16, six 7-bit slices per operand,
 * slice orders up to 5, exact int32 sums added into FP64; same limits. */
typedef enum { P2S_FP64 = 0, P2S_SPLIT_FP32 = 1, P2S_SPLIT_INT8 = 2 } p2s_precision;

/* Method: product-to-sum (the paper's method, Section II eqs. (3)-(4)),
 * or one of two GPU baselines computing the same discrete matrix of eq. (2):
 *  DIRECT     direct quadrature, every entry a full 3-D Gauss sum (the
 *             method the paper compares against, Section IV);
 *  DIRECT_SF  sum-factorized direct quadrature: the Gauss sum taken one
 *             axis at a time with dense tables of weighted basis products
 *             at the points.  Rules of exactly 2N points on every axis
 *             (P2S_EQUAD otherwise); FP64. */
typedef enum { P2S_METHOD_P2S = 0, P2S_METHOD_DIRECT = 1, P2S_METHOD_DIRECT_SF = 2 } p2s_method;

/* Output layout of each element's (symmetric) matrix: the dense row-major
 * block, or its upper triangle packed row by row (row r holds columns
 * c >= r: entry (r, c) at r*n - r*(r-1)/2 + (c - r), n = dofs), which
 * halves the bytes written.  The packed layout is available for the FP64
 * product-to-sum method with per-order-class launches (schedule mode 0). */
typedef enum { P2S_OUTPUT_DENSE = 0, P2S_OUTPUT_PACKED_UPPER = 1 } p2s_output;

typedef struct {
    int32_t problem;     /* p2s_problem                      */
    int32_t material;    /* p2s_material                     */
    int32_t precision;   /* p2s_precision                    */
    int32_t method;      /* p2s_method                       */
    double stiff_scale;  /* weight of the stiffness term (1) */
    double mass_scale;   /* weight of the mass term (1)      */
    int32_t output;      /* p2s_output (dense)               */
    int32_t reserved;    /* 0                                */
} p2s_terms;

#define P2S_MAX_ORDER 8
#define P2S_MAX_Q 32

/* per-element status bits */
#define P2S_STATUS_DETJ 1u      /* det J <= 0 at some Gauss point          */
#define P2S_STATUS_NONFINITE 2u /* non-finite value in the element matrix */
#define P2S_STATUS_FALLBACK 4u  /* learned order rejected, refilled at max */

/* Create a context on HIP device `device`: checks that it is gfx950,
 * builds the FP64 tables (Gauss rules up to P2S_MAX_Q points, Legendre
 * linearization of every basis-pair family up to P2S_MAX_ORDER) once on the
 * host and uploads them.  *out receives the handle. */
int p2s_create(p2s_ctx *out, int device);
void p2s_destroy(p2s_ctx ctx);
/* Message of the last failure on ctx (or of the last p2s_create failure
 * when ctx is NULL).  Valid until the next call on ctx. */
const char *p2s_last_error(p2s_ctx ctx);

/* Degrees of freedom of one element of order N (N^3 or 3 (N-1) N^2);
 * -1 for a bad problem or order. */
int64_t p2s_num_dofs(int problem, int N);

/* Output layout: offsets[e] is the start (in doubles) of element e's dense
 * row-major block, offsets[E] the total.  orders [host][E],
 * offsets [host][E+1]. */
int p2s_layout(int problem, int64_t E, const int32_t *orders, int64_t *offsets);
/* The same for an output layout (p2s_output): packed blocks hold
 * n (n + 1) / 2 doubles. */
int p2s_layout_output(int problem, int output, int64_t E, const int32_t *orders, int64_t *offsets);

/* Plan: the schedule, per-element descriptors and workspace for one batch
 * shape (E, orders [host][E], quad [host][E][3] Gauss points per axis).
 * Allocates device memory; execution then allocates nothing. */
int p2s_plan_create(p2s_ctx ctx, const p2s_terms *terms, int64_t E,
                    const int32_t *orders, const int32_t *quad, p2s_plan *out);
/* Enqueue the fill on `stream`:
 *  nodes    [device] [E][27][3]  node (i,j,k) at i+3j+9k, i along u
 *  material [device] per p2s_material
 *  out      [device] concatenated dense row-major FP64 blocks, p2s_layout
 *  status   [device] [E] per-element P2S_STATUS_* bits (overwritten)   */
int p2s_plan_execute(p2s_plan plan, const double *nodes, const double *material,
                     double *out, uint32_t *status, void *stream);
/* Bytes of device workspace held by the plan. */
int64_t p2s_plan_workspace_bytes(p2s_plan plan);
void p2s_plan_destroy(p2s_plan plan);

/* Stage timing.  With enable != 0, every later p2s_plan_execute records HIP
 * events on its stream around each stage launch (0 coupling, 1 moments,
 * 2 contraction, 3 other); p2s_plan_profile_read waits for those events and
 * returns, per stage, the summed milliseconds and the launch count since the
 * last read (then resets).  ms [host][4], launches [host][4]. */
int p2s_plan_profile(p2s_plan plan, int enable);
int p2s_plan_profile_read(p2s_plan plan, double *ms, int64_t *launches);

/* Schedule of the contraction stage.  mode 0: one launch per order class
 * (per component block J >= I for the vector problem), one workgroup per
 * row tile; mode 1 (scalar problem): one persistent launch of wgs_per_cu
 * workgroups per compute unit that take row tiles from a list sorted by
 * decreasing cost (longest first) through an atomic counter.  Every plan
 * starts in mode 0; p2s_plan_autotune chooses between them. */
int p2s_plan_set_schedule(p2s_plan plan, int mode, int wgs_per_cu);
int p2s_plan_get_schedule(p2s_plan plan, int *mode, int *wgs_per_cu);

/* Autotuner: times every candidate schedule on these buffers (one warm-up
 * and three timed executions each, HIP events on `stream`), keeps the
 * fastest, and records it in the JSON file cache_path [host] (keyed by
 * device, problem, order and rule histograms, E); a later call with the
 * same key reads the choice instead of timing.  cache_path may be NULL.
 * best_ms [host], may be NULL, receives the chosen schedule's time.
 * Synchronizes the stream. */
int p2s_plan_autotune(p2s_plan plan, const double *nodes, const double *material, double *out,
                      uint32_t *status, void *stream, const char *cache_path, double *best_ms);

/* Graph capture: records one execution with these buffers into a HIP
 * graph held by the plan (stream must not be the NULL stream);
 * p2s_plan_replay launches it on `stream`.  The graph keeps the buffer
 * addresses given at capture. */
int p2s_plan_capture(p2s_plan plan, const double *nodes, const double *material, double *out,
                     uint32_t *status, void *stream);
int p2s_plan_replay(p2s_plan plan, void *stream);

/* ------------------------------------------------------------------------
 * Learned quadrature order.  A network (FP32, 85 -> 128 -> 128 -> 57, ReLU)
 * maps an element's features to a distribution, per axis, over the Gauss
 * rule size K in {P2S_KMIN..P2S_KMAX} used to sample the coupling factor
 * for the moment stage.  Features [E][85] (FP32): the 81 node offsets from
 * the nominal unit cube divided by 0.3, then four material parameters
 * (plane wave: |k_x|, |k_y|, |k_z| / (16 pi), phase / (2 pi) - 1/2).  Logits [B][57]:
 * axis a's 19 classes at [a*19 .. a*19+18], class c <-> K = P2S_KMIN + c.
 * The parameters live in the context. */
#define P2S_MLP_IN 85
#define P2S_MLP_HIDDEN 128
#define P2S_MLP_OUT 57
#define P2S_MLP_PARAMS 34873
#define P2S_KMIN 6
#define P2S_KMAX 24

/* Initialise the parameters (He-normal weights from `seed`, zero biases),
 * reset Adam, and size the training scratch for batches up to max_batch. */
int p2s_mlp_init(p2s_ctx ctx, uint64_t seed, int64_t max_batch);
/* Parameters [host][P2S_MLP_PARAMS]: W1 [85][128], b1 [128], W2 [128][128],
 * b2 [128], W3 [128][57], b3 [57] (weights input-major). */
int p2s_mlp_set_params(p2s_ctx ctx, const float *params);
int p2s_mlp_get_params(p2s_ctx ctx, float *params);
/* Binary file: "P2SK", int32 version 1, int32 (85, 128, 57), float32 params. */
int p2s_mlp_save(p2s_ctx ctx, const char *path);
int p2s_mlp_load(p2s_ctx ctx, const char *path);
/* Features of E elements: nodes, material [device] as in p2s_plan_execute,
 * x [device][E][85]. */
int p2s_features(p2s_ctx ctx, int material, int64_t E, const double *nodes, const double *mat, float *x,
                 void *stream);
/* Forward pass, x [device][B][85] -> logits [device][B][57], B <= max_batch. */
int p2s_mlp_forward(p2s_ctx ctx, int64_t B, const float *x, float *logits, void *stream);
/* Mean-over-batch softmax cross-entropy (summed over the three axes) with
 * class labels [device][B][3]: loss [device] (one float, the batch SUM of
 * per-sample losses), gradient [device][P2S_MLP_PARAMS] of the mean loss
 * (grad may be NULL).  p2s_mlp_train_step does the same and applies one
 * Adam step (beta 0.9/0.999, eps 1e-8) with learning rate lr. */
int p2s_mlp_gradients(p2s_ctx ctx, int64_t B, const float *x, const int32_t *labels, float *grad, float *loss,
                      void *stream);
int p2s_mlp_train_step(p2s_ctx ctx, int64_t B, const float *x, const int32_t *labels, float lr, float *loss,
                       void *stream);
/* Per-axis rule: the smallest K whose predicted cumulative probability
 * reaches p_cover; quad [device][B][3]. */
int p2s_mlp_predict(p2s_ctx ctx, int64_t B, const float *x, float p_cover, int32_t *quad, void *stream);
/* Learned mode of a plan created with P2S_KMAX points on every axis (so its
 * workspace holds the full rule): each execution computes the features,
 * runs the network, chooses per axis the smallest K whose predicted
 * cumulative probability reaches p_cover (K >= k_direct: the full rule at
 * once; k_direct > P2S_KMAX disables that), samples the coupling factor with
 * the chosen rules and checks the tail.  For each axis x sampled below the
 * full rule and each field, the tail statistic takes the discrete Legendre
 * coefficients along x of the four highest degrees the rule resolves,
 * projected on the other two axes onto the moment degrees of eq. (4)
 * (T_x[j] below); their decay extrapolated to the first degree the moments
 * can alias, relative to the largest moment magnitude, is the axis value,
 * and its maximum over those axes the element's tail value.  Above theta
 * the element is sampled again with the full rule (status
 * P2S_STATUS_FALLBACK).  Axes already at the full rule take no statistic.
 * Orders up to 6 (P2S_EORDER otherwise).  Allocates its workspace here;
 * enable = 0 restores the plan's own rules. */
int p2s_plan_set_learned(p2s_plan plan, int enable, float p_cover, int k_direct, double theta);
/* Tail records of the moment stage at the plan's own rules (coupling and
 * moments only; no contraction): records [device][E][F][16], per field
 * env[axis][j] at axis*4+j, the largest magnitude of
 *   T_u[j][l][q] = sum t_j(a) W[l](b) W[q](c) alpha(a,b,c)   (axis 0),
 *   T_v[k][j][q], T_w[k][l][j]                                (axes 1, 2),
 * t_j(a) = (2d+1)/2 w_a L_d(x_a) for degree d = Q-1-j of that axis's rule,
 * W[l](b) = w_b L_l(x_b) for the moment degrees l < 2N-1; at 12+axis the
 * largest magnitude of the field's moment tensor; entry 15 is zero, and so
 * is every entry of an axis sampled with P2S_KMAX points or more.  The
 * statistic of p2s_plan_set_learned is computed from these.
 * Product-to-sum plans of orders up to 6 whose moment stage can hold the
 * tail rows (P2S_EQUAD otherwise); allocates its workspace on first use. */
int p2s_plan_tail_records(p2s_plan plan, const double *nodes, const double *material, double *records,
                          void *stream);
/* Rules used by the last execution: quad [host][E][3]. */
int p2s_plan_rules(p2s_plan plan, int32_t *quad);
/* Tail statistic of each element at its predicted rule in the last learned
 * execution: tau [host][E] (synchronizes the device). */
int p2s_plan_tail_values(p2s_plan plan, double *tau);
/* Per-element relative Frobenius difference ||a - b||_F / ||b||_F of blocks
 * [device] at offsets [device][E+1] (or of E blocks of len doubles when
 * offsets is NULL); err [device][E]. */
int p2s_rel_error(p2s_ctx ctx, int64_t E, int64_t len, const int64_t *offsets, const double *a, const double *b,
                  double *err, void *stream);

/* The fill of eq. (2) by the product-to-sum method of Section II (eqs.
 * (3)-(4)) in one call, arguments as for p2s_plan_create and
 * p2s_plan_execute: terms [host], orders [host][E], quad [host][E][3],
 * nodes/material/out/status [device] as in p2s_plan_execute, out laid out
 * by p2s_layout.  The context keeps the plans of the last 8 batch shapes
 * (terms, E, orders, quad compared exactly): the first call of a shape
 * creates its plan (allocates device memory and uploads descriptors, which
 * may block), every later call of that shape only enqueues the fill on
 * `stream` and returns, allocating nothing.  A ninth shape evicts the least
 * recently used plan (its memory is freed once the device has finished the
 * work queued on it).  Returns the plan-creation or launch error; numerical
 * conditions go to status. */
int p2s_fill_element_matrices(p2s_ctx ctx, const p2s_terms *terms, int64_t E,
                              const double *nodes, const double *material,
                              const int32_t *orders, const int32_t *quad,
                              double *out, uint32_t *status, void *stream);

/* Allocation-free fill, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same fill as p2s_fill_element_matrices (FP64
 * product-to-sum only) for E elements of one order N and one rule
 * (Qu, Qv, Qw); nodes, material, out, status [device] as in
 * p2s_plan_execute, out laid out as E blocks of p2s_num_dofs(N)^2 doubles.
 * Its workspace (descriptors, coupling samples, moments) is a fixed 64 MiB
 * device array that the library holds on each GPU for the life of the
 * process; the elements go through it in chunks, one chunk after another on
 * `stream`.  Nothing is allocated and nothing is copied from the host: the
 * call only enqueues kernels.  Every call on a GPU shares that GPU's array,
 * so calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialized by the caller.  Errors: P2S_EORDER,
 * P2S_EQUAD (points outside 1..P2S_MAX_Q or a rule the moment stage cannot
 * hold), P2S_EINVAL (other precision or method, bad enums, NULL buffers, or
 * an element whose workspace alone exceeds the 64 MiB). */
int p2s_fill_uniform_noalloc(p2s_ctx ctx, const p2s_terms *terms, int64_t E, int N,
                             int Qu, int Qv, int Qw, const double *nodes, const double *material,
                             double *out, uint32_t *status, void *stream);

/* ------------------------------------------------------------------------
 * The paper's own instance (Section III): 2-D curl-curl + mass element
 * matrices (eqs. (5), (7)) of curved quadrilaterals with the Chebyshev vector
 * basis of eq. (6), M = N:
 *   u-functions U_m(u) T_n(v), m < M, n <= M   (dof m (M+1) + n),
 *   v-functions T_m(u) U_n(v), m <= M, n < M   (dof M (M+1) + m M + n),
 * covariant components; entries of eqs. (8)-(15) with mu_r = 1, as
 * stiff_scale * S + mass_scale * M.  Geometry: fourth-order quadrilateral,
 * nodes [device][E][25][2], node (i,j) at i + 5 j on the reference points
 * (-1 + i/2, -1 + j/2).  Material [device][E][4]: eps_r = p0 exp(p1 x + p2 y
 * + p3) (the paper's 2 exp(x + y + 2) is (2, 1, 1, 2)).  Q x Q Gauss points.
 * method P2S_METHOD_P2S: the product-to-sum method of eqs. (16)-(19) (four
 * starting-point integral tables per element, every entry a gather-add of at
 * most eight of them); P2S_METHOD_DIRECT: direct 2-D quadrature of every
 * entry (the comparison of Table I).  out [device] E dense row-major blocks
 * of p2s_cheb2d_num_dofs(M)^2 doubles; status [device][E] (P2S_STATUS_DETJ,
 * and P2S_STATUS_NONFINITE for the product-to-sum form).
 * create: M in 1..18 (P2S_EORDER), Q in 1..P2S_MAX_Q (P2S_EQUAD); allocates
 * the workspace of E elements.  execute: enqueues on `stream`, allocates
 * nothing.  profile(enable, ms): ms [host][3] (may be NULL) receives the
 * mean milliseconds per execution of the geometry, moment (or nothing) and
 * contraction (or direct) kernels since the last call; while enabled,
 * execute waits for its own kernels. */
typedef struct p2s_cheb2d_s *p2s_cheb2d;
int64_t p2s_cheb2d_num_dofs(int M);
int p2s_cheb2d_create(p2s_ctx ctx, int64_t E, int M, int Q, p2s_cheb2d *out);
int p2s_cheb2d_execute(p2s_cheb2d plan, int method, const double *nodes, const double *material,
                       double stiff_scale, double mass_scale, double *out, uint32_t *status,
                       void *stream);
int p2s_cheb2d_profile(p2s_cheb2d plan, int enable, double *ms);
void p2s_cheb2d_destroy(p2s_cheb2d plan);
/* Device of a context (-1 for NULL). */
int p2s_context_device(p2s_ctx ctx);

/* Stage outputs, for verification of each step against its definition.
 * Coupling samples: alpha [device][E][F][Qu*Qv*Qw] (unweighted, packed
 * field order of P2S_ALPHA_SAMPLED).  Moments: [device][E][F][K][K][K],
 * K = 2N-1, the integrals of eq. (4).  Both need a plan of uniform shape. */
int p2s_plan_coupling(p2s_plan plan, const double *nodes, const double *material,
                      double *alpha, void *stream);
int p2s_plan_moments(p2s_plan plan, const double *nodes, const double *material,
                     double *moments, void *stream);

/* Host-side tables (no device needed).
 * Gauss-Legendre rule with Q points, ascending: x[Q], w[Q].
 * Linearization (eq. (3)): X_m1(t) Y_m2(t) = sum_k coef[k] L_k(t),
 * families 0 = phi, 1 = phi', 2 = psi; coef[2*P2S_MAX_ORDER]. */
int p2s_gauss_rule(int Q, double *x, double *w);
int p2s_linearization(int xfam, int m1, int yfam, int m2, double *coef);

#ifdef __cplusplus
}
#endif

#endif /* P2S_H */
