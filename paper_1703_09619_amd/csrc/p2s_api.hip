// p2s_api.hip -- C ABI and host runtime of the product-to-sum fill:
// contexts (tables built once), plans (descriptors, schedule, workspace),
// and the chunked execution of the three stages on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "p2s.h"
#include "p2s_internal.h"
#include "p2s_kernels.h"
#include "p2s_tables.h"

using namespace p2s;

struct p2s_ctx_s {
    int device = 0;
    double *d_tab = nullptr;
    std::string err;
    // learned quadrature order: network parameters, Adam state, training scratch
    bool mlp_ready = false;
    float *d_mlp = nullptr, *d_grad = nullptr, *d_adam_m = nullptr, *d_adam_v = nullptr;
    int adam_step = 0;
    int64_t mlp_bmax = 0;
    float *d_h1 = nullptr, *d_h2 = nullptr, *d_z = nullptr, *d_dz = nullptr, *d_dh2 = nullptr, *d_dh1 = nullptr,
          *d_lossb = nullptr;
    // plans of p2s_fill_element_matrices, least recently used first
    std::vector<p2s_plan> fill_cache;
    // device address of this GPU's `scratch` array
    double *scratch = nullptr;
};
constexpr size_t FILL_CACHE_PLANS = 8;

// Device scratch of p2s_fill_uniform_noalloc: descriptors, coupling samples
// and moment tensors of one chunk of elements.  Each GPU the library runs
// on holds its own copy for the life of the process.  Host code never uses
// the array's name as an address: p2s_create looks up the device address
// (hipGetSymbolAddress) and keeps it in the context.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

// Descriptors of `count` elements of one order and rule, element e's block
// at e * ndof2 of the chunk's output and its samples and moments at e times
// their per-element sizes in the scratch.
__global__ void k_uniform_desc(ElemDesc *__restrict__ desc, int64_t count, int N, int Qu, int Qv, int Qw,
                               int64_t ndof2, int64_t na, int64_t nm)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= count) return;
    ElemDesc d;
    d.N = N;
    d.Qu = Qu;
    d.Qv = Qv;
    d.Qw = Qw;
    d.out_off = e * ndof2;
    d.alpha_off = e * na;
    d.mom_off = e * nm;
    desc[e] = d;
}

struct Chunk {
    int64_t e0 = 0, count = 0;
    // per order class inside the chunk: (N, offset into elist, count), and
    // the largest rules of its elements (the moment stage's LDS shape)
    std::vector<std::array<int64_t, 3>> classes;
    std::vector<MomentShape> cshape;
    // persistent schedule: offset and count of this chunk's work items
    int64_t item0 = 0, nitem = 0;
};

struct p2s_plan_s {
    p2s_ctx ctx = nullptr;
    p2s_terms terms{};
    int64_t E = 0;
    bool uniform = true;
    int N = 0, Qu = 0, Qv = 0, Qw = 0;
    int maxN = 0;
    MomentShape mshape;  // largest order and rule sizes (moment-stage LDS)
    int mat_stride = 0;
    std::vector<int32_t> orders, quad;
    std::vector<int64_t> offsets;
    std::vector<Chunk> chunks;
    ElemDesc *d_desc = nullptr;
    int32_t *d_elist = nullptr;
    double *d_alpha = nullptr, *d_mom = nullptr;
    uint32_t *d_stage_status = nullptr;  // status sink of the stage-output calls
    int64_t alpha_cap = 0, mom_cap = 0;  // doubles
    int64_t bytes = 0;
    // schedule of the contraction: per-order-class launches (0) or one
    // persistent launch over a cost-sorted work list (1), with wpc
    // workgroups per compute unit
    int mode = 0, wpc = 1;
    WorkItem *d_items = nullptr;
    int32_t *d_counter = nullptr;
    int num_cu = 256;
    // learned quadrature order
    bool learned = false;
    float p_cover = 0.99f;
    int k_direct = MLP_KMAX + 1;
    double theta = 1e-9;
    float *d_lx = nullptr, *d_lh1 = nullptr, *d_lh2 = nullptr, *d_lz = nullptr;
    int32_t *d_redo = nullptr;
    double *d_tau = nullptr;     // tail statistic of the last learned execution
    double *d_tailst = nullptr;  // [E][F][TAIL_REC] records of the moment stage
    std::vector<ElemDesc> desc_host;
    // captured execution
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // stage timing (events recorded around each launch when enabled)
    bool profile = false;
    std::vector<std::array<hipEvent_t, 2>> ev[4];
    size_t ev_used[4] = {0, 0, 0, 0};
};

static void prof_begin(p2s_plan plan, int stage, hipStream_t st)
{
    if (!plan->profile) return;
    auto &v = plan->ev[stage];
    if (plan->ev_used[stage] == v.size()) {
        std::array<hipEvent_t, 2> e{};
        hipEventCreate(&e[0]);
        hipEventCreate(&e[1]);
        v.push_back(e);
    }
    hipEventRecord(v[plan->ev_used[stage]][0], st);
}

static void prof_end(p2s_plan plan, int stage, hipStream_t st)
{
    if (!plan->profile) return;
    hipEventRecord(plan->ev[stage][plan->ev_used[stage]][1], st);
    plan->ev_used[stage]++;
}

static thread_local std::string g_create_err;

static int fail(p2s_ctx ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_create_err = buf;
    return code;
}

#define HIP_TRY(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t _r = (call);                                                              \
        if (_r != hipSuccess)                                                                \
            return fail(ctx, P2S_EHIP, "%s failed: %s", #call, hipGetErrorString(_r));       \
    } while (0)

// ---------------------------------------------------------------------------

extern "C" {

const char *p2s_last_error(p2s_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int p2s_context_device(p2s_ctx ctx) { return ctx ? ctx->device : -1; }

int64_t p2s_num_dofs(int problem, int N)
{
    if ((problem != P2S_SCALAR && problem != P2S_VECTOR) || N < 2 || N > P2S_MAX_ORDER) return -1;
    return num_dofs(problem, N);
}

int p2s_layout(int problem, int64_t E, const int32_t *orders, int64_t *offsets)
{
    if (E < 0 || !offsets || (E > 0 && !orders)) return P2S_EINVAL;
    if (problem != P2S_SCALAR && problem != P2S_VECTOR) return P2S_EINVAL;
    offsets[0] = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int64_t nd = p2s_num_dofs(problem, orders[e]);
        if (nd < 0) return P2S_EORDER;
        offsets[e + 1] = offsets[e] + nd * nd;
    }
    return P2S_OK;
}

int p2s_layout_output(int problem, int output, int64_t E, const int32_t *orders, int64_t *offsets)
{
    if (output != P2S_OUTPUT_DENSE && output != P2S_OUTPUT_PACKED_UPPER) return P2S_EINVAL;
    if (E < 0 || !offsets || (E > 0 && !orders)) return P2S_EINVAL;
    if (problem != P2S_SCALAR && problem != P2S_VECTOR) return P2S_EINVAL;
    offsets[0] = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int64_t nd = p2s_num_dofs(problem, orders[e]);
        if (nd < 0) return P2S_EORDER;
        offsets[e + 1] = offsets[e] + (output == P2S_OUTPUT_DENSE ? nd * nd : nd * (nd + 1) / 2);
    }
    return P2S_OK;
}

int p2s_gauss_rule(int Q, double *x, double *w)
{
    if (!x || !w) return P2S_EINVAL;
    return gauss_rule(Q, x, w) == 0 ? P2S_OK : P2S_EQUAD;
}

int p2s_linearization(int xfam, int m1, int yfam, int m2, double *coef)
{
    if (!coef) return P2S_EINVAL;
    double c[KPAD];
    if (linearization(xfam, m1, yfam, m2, c) != 0) return P2S_EINVAL;
    for (int k = 0; k < 2 * P2S_MAX_ORDER; ++k) coef[k] = k < KPAD ? c[k] : 0.0;
    return P2S_OK;
}

int p2s_create(p2s_ctx *out, int device)
{
    if (!out) return fail(nullptr, P2S_EINVAL, "p2s_create: out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(nullptr, P2S_ENODEV, "p2s_create: no HIP device");
    if (device < 0 || device >= n) return fail(nullptr, P2S_ENODEV, "p2s_create: bad device %d", device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(nullptr, P2S_ENODEV, "p2s_create: cannot query device %d", device);
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, P2S_ENODEV, "p2s_create: device %d is %s, this library is built for gfx950",
                    device, prop.gcnArchName);
    p2s_ctx ctx = new p2s_ctx_s();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return fail(nullptr, P2S_EHIP, "p2s_create: hipSetDevice failed");
    }
    std::vector<double> tab(TAB_SIZE);
    build_tables(tab.data());
    if (hipMalloc(&ctx->d_tab, sizeof(double) * TAB_SIZE) != hipSuccess) {
        p2s_destroy(ctx);
        return fail(nullptr, P2S_ENOMEM, "p2s_create: table allocation failed");
    }
    {
        // with the context's device current: this GPU's copy of the scratch
        void *p = nullptr;
        const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess || !p) {
            p2s_destroy(ctx);
            return fail(nullptr, P2S_EHIP, "p2s_create: scratch symbol lookup failed: %s", hipGetErrorString(r));
        }
        ctx->scratch = static_cast<double *>(p);
    }
    if (hipMemcpy(ctx->d_tab, tab.data(), sizeof(double) * TAB_SIZE, hipMemcpyHostToDevice) != hipSuccess ||
        prepare_kernels() != 0 || prepare_split_kernels() != 0) {
        p2s_destroy(ctx);
        return fail(nullptr, P2S_EHIP, "p2s_create: table upload failed");
    }
    *out = ctx;
    return P2S_OK;
}

void p2s_destroy(p2s_ctx ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    for (p2s_plan p : ctx->fill_cache) p2s_plan_destroy(p);
    ctx->fill_cache.clear();
    if (ctx->d_tab) hipFree(ctx->d_tab);
    for (float *p : {ctx->d_mlp, ctx->d_grad, ctx->d_adam_m, ctx->d_adam_v, ctx->d_h1, ctx->d_h2, ctx->d_z,
                     ctx->d_dz, ctx->d_dh2, ctx->d_dh1, ctx->d_lossb})
        if (p) hipFree(p);
    delete ctx;
}

void p2s_plan_destroy(p2s_plan plan)
{
    if (!plan) return;
    hipSetDevice(plan->ctx->device);
    hipFree(plan->d_desc);
    hipFree(plan->d_elist);
    hipFree(plan->d_alpha);
    hipFree(plan->d_mom);
    hipFree(plan->d_stage_status);
    hipFree(plan->d_items);
    hipFree(plan->d_counter);
    hipFree(plan->d_lx);
    hipFree(plan->d_lh1);
    hipFree(plan->d_lh2);
    hipFree(plan->d_lz);
    hipFree(plan->d_redo);
    hipFree(plan->d_tau);
    hipFree(plan->d_tailst);
    if (plan->gexec) hipGraphExecDestroy(plan->gexec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    for (auto &v : plan->ev)
        for (auto &e : v) {
            hipEventDestroy(e[0]);
            hipEventDestroy(e[1]);
        }
    delete plan;
}

int64_t p2s_plan_workspace_bytes(p2s_plan plan) { return plan ? plan->bytes : -1; }

// Workspace budget per chunk (coupling samples + moments), in bytes.
static int64_t chunk_budget()
{
    static int64_t b = -1;
    if (b < 0) {
        const char *s = getenv("P2S_CHUNK_MB");
        b = (s ? atoll(s) : 4096) << 20;
    }
    return b;
}

int p2s_plan_create(p2s_ctx ctx, const p2s_terms *terms, int64_t E, const int32_t *orders,
                    const int32_t *quad, p2s_plan *out)
{
    if (!ctx) return P2S_EINVAL;
    if (!terms || !out) return fail(ctx, P2S_EINVAL, "plan: NULL argument");
    *out = nullptr;
    if (E < 0 || (E > 0 && (!orders || !quad))) return fail(ctx, P2S_EINVAL, "plan: bad E or NULL orders/quad");
    const int problem = terms->problem;
    if (problem != P2S_SCALAR && problem != P2S_VECTOR) return fail(ctx, P2S_EINVAL, "plan: bad problem %d", problem);
    const int kind = terms->material;
    int stride = 0;
    switch (kind) {
    case P2S_MAT_SINCOSEXP: stride = 1; break;
    case P2S_MAT_ROTDIAG: stride = 12; break;
    case P2S_MAT_PLANEWAVE: stride = 4; break;
    case P2S_ALPHA_SAMPLED: stride = 0; break;
    default: return fail(ctx, P2S_EINVAL, "plan: bad material %d", kind);
    }
    if (problem == P2S_SCALAR && kind == P2S_MAT_ROTDIAG)
        return fail(ctx, P2S_EINVAL, "plan: the scalar problem takes an isotropic material");
    if (terms->method != P2S_METHOD_P2S && terms->method != P2S_METHOD_DIRECT &&
        terms->method != P2S_METHOD_DIRECT_SF)
        return fail(ctx, P2S_EINVAL, "plan: bad method %d", terms->method);
    if (terms->method == P2S_METHOD_DIRECT_SF) {
        if (terms->precision != P2S_FP64)
            return fail(ctx, P2S_EINVAL, "plan: sum-factorized direct quadrature is FP64");
        for (int64_t e = 0; e < E; ++e)
            if (orders[e] >= 2 && orders[e] <= P2S_MAX_ORDER &&
                (quad[3 * e] != 2 * orders[e] || quad[3 * e + 1] != 2 * orders[e] || quad[3 * e + 2] != 2 * orders[e]))
                return fail(ctx, P2S_EQUAD, "plan: sum-factorized direct quadrature takes rules of 2N Gauss points "
                                            "per axis (element %lld: order %d)", (long long)e, orders[e]);
    }
    if (terms->precision != P2S_FP64 && terms->precision != P2S_SPLIT_FP32 && terms->precision != P2S_SPLIT_INT8)
        return fail(ctx, P2S_EINVAL, "plan: unsupported precision %d", terms->precision);
    if (terms->precision != P2S_FP64 && terms->method != P2S_METHOD_P2S)
        return fail(ctx, P2S_EINVAL, "plan: split-FP32 and split-INT8 precision are forms of the product-to-sum "
                                     "method");
    if (terms->output != P2S_OUTPUT_DENSE && terms->output != P2S_OUTPUT_PACKED_UPPER)
        return fail(ctx, P2S_EINVAL, "plan: bad output layout %d", terms->output);
    if (terms->output == P2S_OUTPUT_PACKED_UPPER &&
        (terms->method != P2S_METHOD_P2S || terms->precision != P2S_FP64))
        return fail(ctx, P2S_EINVAL, "plan: the packed output layout is written by the FP64 product-to-sum method");
    auto plan = new p2s_plan_s();
    plan->ctx = ctx;
    plan->terms = *terms;
    plan->E = E;
    plan->mat_stride = stride;
    plan->orders.assign(orders, orders + E);
    plan->quad.assign(quad, quad + 3 * E);
    plan->offsets.resize(E + 1);
    const int F = num_fields(problem);
    for (int64_t e = 0; e < E; ++e) {
        const int N = orders[e];
        if (N < 2 || N > P2S_MAX_ORDER) {
            delete plan;
            return fail(ctx, P2S_EORDER, "plan: element %lld has order %d (allowed 2..%d)", (long long)e, N,
                        P2S_MAX_ORDER);
        }
        for (int a = 0; a < 3; ++a)
            if (quad[3 * e + a] < 1 || quad[3 * e + a] > P2S_MAX_Q) {
                delete plan;
                return fail(ctx, P2S_EQUAD, "plan: element %lld has %d Gauss points on axis %d (allowed 1..%d)",
                            (long long)e, quad[3 * e + a], a, P2S_MAX_Q);
            }
        plan->maxN = std::max(plan->maxN, N);
        MomentShape &ms = plan->mshape;
        ms.maxN = plan->maxN;
        ms.maxQ = std::max({ms.maxQ, (int)quad[3 * e], (int)quad[3 * e + 1], (int)quad[3 * e + 2]});
        ms.maxQu = std::max(ms.maxQu, (int)quad[3 * e]);
        ms.maxQuv = std::max(ms.maxQuv, (int)(quad[3 * e] * quad[3 * e + 1]));
        ms.maxQw = std::max(ms.maxQw, (int)quad[3 * e + 2]);
        ms.maxQvw = std::max(ms.maxQvw, (int)(quad[3 * e + 1] * quad[3 * e + 2]));
        if (e > 0 && (N != orders[0] || quad[3 * e] != quad[0] || quad[3 * e + 1] != quad[1] ||
                      quad[3 * e + 2] != quad[2]))
            plan->uniform = false;
    }
    p2s_layout_output(problem, terms->output, E, orders, plan->offsets.data());
    if (E > 0) {
        plan->N = orders[0];
        plan->Qu = quad[0];
        plan->Qv = quad[1];
        plan->Qw = quad[2];
    }
    if (terms->method == P2S_METHOD_DIRECT && !plan->uniform) {
        delete plan;
        return fail(ctx, P2S_EINVAL, "plan: direct quadrature takes one order and rule for all elements");
    }
    if (kind == P2S_ALPHA_SAMPLED && !plan->uniform) {
        delete plan;
        return fail(ctx, P2S_EINVAL, "plan: sampled coupling input needs one order and rule for all elements");
    }
    if (terms->precision != P2S_FP64 && E > 0 &&
        (!plan->uniform || plan->Qu > SPLIT_MAXQ || plan->Qv > SPLIT_MAXQ || plan->Qw > SPLIT_MAXQ)) {
        delete plan;
        return fail(ctx, P2S_EQUAD, "plan: split-FP32 and split-INT8 precision take one order and one rule of at "
                                    "most %d points per axis for all elements", SPLIT_MAXQ);
    }
    if (E > 0 && (moments_lds_bytes(plan->mshape) > LDS_LIMIT ||
                  moments_smem_bytes(plan->maxN, plan->mshape.maxQw, plan->mshape.maxQvw) > LDS_LIMIT)) {
        delete plan;
        return fail(ctx, P2S_EQUAD, "plan: rule too large for the moment stage at order %d", plan->maxN);
    }
    // descriptors and chunks
    std::vector<ElemDesc> desc(E);
    const int64_t budget = chunk_budget();
    int64_t a_off = 0, m_off = 0;
    Chunk cur;
    auto close_chunk = [&](int64_t e_end) {
        cur.count = e_end - cur.e0;
        if (cur.count > 0) plan->chunks.push_back(cur);
        plan->alpha_cap = std::max(plan->alpha_cap, a_off);
        plan->mom_cap = std::max(plan->mom_cap, m_off);
        cur = Chunk();
        cur.e0 = e_end;
        a_off = m_off = 0;
    };
    for (int64_t e = 0; e < E; ++e) {
        const int N = orders[e], K = 2 * N - 1;
        const int64_t na = (int64_t)F * quad[3 * e] * quad[3 * e + 1] * quad[3 * e + 2];
        const int64_t nm = (int64_t)F * K * K * K;
        if (e > cur.e0 && (a_off + na + m_off + nm) * 8 > budget) close_chunk(e);
        desc[e].N = N;
        desc[e].Qu = quad[3 * e];
        desc[e].Qv = quad[3 * e + 1];
        desc[e].Qw = quad[3 * e + 2];
        desc[e].out_off = plan->offsets[e];
        desc[e].alpha_off = a_off;
        desc[e].mom_off = m_off;
        a_off += na;
        m_off += nm;
    }
    close_chunk(E);
    // order classes inside each chunk (element lists for the contraction)
    std::vector<int32_t> elist;
    if (!plan->uniform) {
        for (auto &c : plan->chunks) {
            for (int N = 2; N <= P2S_MAX_ORDER; ++N) {
                const int64_t start = (int64_t)elist.size();
                MomentShape cs;
                cs.maxN = N;
                for (int64_t e = c.e0; e < c.e0 + c.count; ++e)
                    if (orders[e] == N) {
                        elist.push_back((int32_t)e);
                        const int32_t *q = quad + 3 * e;
                        cs.maxQ = std::max({cs.maxQ, (int)q[0], (int)q[1], (int)q[2]});
                        cs.maxQu = std::max(cs.maxQu, (int)q[0]);
                        cs.maxQuv = std::max(cs.maxQuv, (int)(q[0] * q[1]));
                        cs.maxQw = std::max(cs.maxQw, (int)q[2]);
                        cs.maxQvw = std::max(cs.maxQvw, (int)(q[1] * q[2]));
                    }
                const int64_t cnt = (int64_t)elist.size() - start;
                if (cnt > 0) {
                    c.classes.push_back({N, start, cnt});
                    c.cshape.push_back(cs);
                }
            }
        }
    }
    // work list of the persistent schedule (scalar problem): items sorted by
    // decreasing cost inside each chunk, items of one element adjacent
    std::vector<WorkItem> items;
    if (problem == P2S_SCALAR) {
        for (auto &c : plan->chunks) {
            c.item0 = (int64_t)items.size();
            std::vector<std::pair<int64_t, WorkItem>> v;
            for (int64_t e = c.e0; e < c.e0 + c.count; ++e) {
                const int N = orders[e];
                for (int m1 = 0; m1 < N; ++m1) {
                    // output written by the item: its rows times the columns m2 >= m1
                    const int64_t cost = (int64_t)N * N * (N - m1) * N * N;
                    v.push_back({cost, WorkItem{(int32_t)e, 0, (int16_t)m1}});
                }
            }
            std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
            for (auto &x : v) items.push_back(x.second);
            c.nitem = (int64_t)items.size() - c.item0;
        }
    }
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) plan->num_cu = prop.multiProcessorCount;
    }
    hipSetDevice(ctx->device);
    bool ok = true;
    if (E > 0) {
        ok = ok && hipMalloc(&plan->d_desc, sizeof(ElemDesc) * E) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_alpha, sizeof(double) * std::max<int64_t>(plan->alpha_cap, 1)) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_mom, sizeof(double) * std::max<int64_t>(plan->mom_cap, 1)) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_stage_status, sizeof(uint32_t) * E) == hipSuccess;
        if (!elist.empty()) ok = ok && hipMalloc(&plan->d_elist, sizeof(int32_t) * elist.size()) == hipSuccess;
        if (!items.empty()) ok = ok && hipMalloc(&plan->d_items, sizeof(WorkItem) * items.size()) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_counter, sizeof(int32_t)) == hipSuccess;
    }
    if (!ok) {
        p2s_plan_destroy(plan);
        return fail(ctx, P2S_ENOMEM, "plan: workspace allocation failed");
    }
    plan->bytes = (int64_t)(sizeof(ElemDesc) * E + 8 * (plan->alpha_cap + plan->mom_cap) + 4 * elist.size() +
                            sizeof(WorkItem) * items.size());
    // every plan starts with the per-order-class launches: each order runs
    // its own kernel at that kernel's occupancy, while the persistent kernel
    // holds the bodies of all orders and runs one 512-lane workgroup per
    // compute unit (p2s_plan_autotune times both)
    plan->desc_host = desc;
    if (E > 0) {
        if (hipMemcpy(plan->d_desc, desc.data(), sizeof(ElemDesc) * E, hipMemcpyHostToDevice) != hipSuccess ||
            (!elist.empty() && hipMemcpy(plan->d_elist, elist.data(), sizeof(int32_t) * elist.size(),
                                         hipMemcpyHostToDevice) != hipSuccess) ||
            (!items.empty() && hipMemcpy(plan->d_items, items.data(), sizeof(WorkItem) * items.size(),
                                         hipMemcpyHostToDevice) != hipSuccess)) {
            p2s_plan_destroy(plan);
            return fail(ctx, P2S_EHIP, "plan: descriptor upload failed");
        }
    }
    *out = plan;
    return P2S_OK;
}

enum StageStop { STOP_COUPLING = 0, STOP_MOMENTS = 1, STOP_FULL = 2, STOP_TAILREC = 3 };

static int run_plan(p2s_plan plan, const double *nodes, const double *material, double *out,
                    uint32_t *status, hipStream_t st, int stop, double *stage_out)
{
    p2s_ctx ctx = plan->ctx;
    if (plan->E == 0) return P2S_OK;
    if (!material || !status || (stop == STOP_FULL && !out) || (stop != STOP_FULL && !stage_out))
        return fail(ctx, P2S_EINVAL, "execute: NULL buffer");
    if (!nodes && plan->terms.material != P2S_ALPHA_SAMPLED) return fail(ctx, P2S_EINVAL, "execute: NULL nodes");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int problem = plan->terms.problem;
    const int F = num_fields(problem);
    const bool learned = plan->learned && stop == STOP_FULL;
    if (learned) {
        if (!ctx->mlp_ready) return fail(ctx, P2S_ENOMODEL, "execute: learned order needs a loaded network");
        // features -> network -> per-axis rule, written into the descriptors
        prof_begin(plan, 3, st);
        launch_features(plan->E, nodes, material, plan->terms.material, plan->mat_stride, plan->d_lx, st);
        launch_mlp_forward(plan->E, ctx->d_mlp, plan->d_lx, plan->d_lh1, plan->d_lh2, plan->d_lz, st);
        launch_choose(plan->E, plan->d_lz, plan->p_cover, plan->k_direct, nullptr, plan->d_desc, st);
        prof_end(plan, 3, st);
    }
    for (const Chunk &c : plan->chunks) {
        prof_begin(plan, 0, st);
        launch_coupling(problem, plan->d_desc, c.e0, c.count, nodes, material, plan->terms.material,
                        plan->mat_stride, ctx->d_tab, plan->d_alpha, status, nullptr, st);
        prof_end(plan, 0, st);
        if (plan->terms.method == P2S_METHOD_DIRECT_SF && stop == STOP_FULL) {
            prof_begin(plan, 2, st);
            int r = 0;
            if (plan->uniform)
                r = launch_contract_dsf(problem, plan->N, plan->d_desc, nullptr, c.e0, c.count, ctx->d_tab,
                                        plan->d_alpha, out, status, plan->terms.stiff_scale, plan->terms.mass_scale, st);
            else
                for (const auto &cl : c.classes)
                    r |= launch_contract_dsf(problem, (int)cl[0], plan->d_desc, plan->d_elist, cl[1], cl[2],
                                             ctx->d_tab, plan->d_alpha, out, status, plan->terms.stiff_scale,
                                             plan->terms.mass_scale, st);
            prof_end(plan, 2, st);
            if (r != 0) return fail(ctx, P2S_EINVAL, "execute: no direct-quadrature kernel for this order");
            continue;
        }
        if (plan->terms.method == P2S_METHOD_DIRECT && stop == STOP_FULL) {
            prof_begin(plan, 3, st);
            launch_direct(problem, plan->N, plan->d_desc, c.e0, c.count, ctx->d_tab, plan->d_alpha, out,
                          plan->terms.stiff_scale, plan->terms.mass_scale, st);
            prof_end(plan, 3, st);
            continue;
        }
        if (stop == STOP_COUPLING) {
            const int64_t per = (int64_t)F * plan->Qu * plan->Qv * plan->Qw;
            HIP_TRY(ctx, hipMemcpyAsync(stage_out + c.e0 * per, plan->d_alpha, sizeof(double) * per * c.count,
                                        hipMemcpyDeviceToDevice, st));
            continue;
        }
        const bool split = plan->terms.precision != P2S_FP64;
        const bool int8 = plan->terms.precision == P2S_SPLIT_INT8;
        prof_begin(plan, 1, st);
        if (split && stop != STOP_TAILREC)
            launch_moments_split(problem, plan->d_desc, c.e0, c.count, plan->d_alpha, ctx->d_tab, plan->d_mom, int8,
                                 st);
        else if (!plan->uniform && !learned && stop != STOP_TAILREC)
            // mixed orders: one launch per order class, each with the LDS
            // shape of its own elements rather than of the largest order
            for (size_t k = 0; k < c.classes.size(); ++k)
                launch_moments(problem, c.cshape[k], plan->d_desc, c.classes[k][1], c.classes[k][2],
                               plan->d_alpha, ctx->d_tab, plan->d_mom, nullptr, nullptr, st, plan->d_elist);
        else
            launch_moments(problem, plan->mshape, plan->d_desc, c.e0, c.count,
                           plan->d_alpha, ctx->d_tab, plan->d_mom, nullptr,
                           (learned || stop == STOP_TAILREC) ? plan->d_tailst : nullptr, st);
        prof_end(plan, 1, st);
        if (stop == STOP_TAILREC) continue;
        if (learned) {
            // tail check; rejected elements are sampled again with the full rule
            prof_begin(plan, 3, st);
            launch_tail_decide(plan->d_desc, c.e0, c.count, F, plan->d_tailst, plan->theta, MLP_KMAX,
                               plan->d_redo, status, plan->d_tau, st);
            launch_coupling(problem, plan->d_desc, c.e0, c.count, nodes, material, plan->terms.material,
                            plan->mat_stride, ctx->d_tab, plan->d_alpha, status, plan->d_redo, st);
            launch_moments(problem, plan->mshape, plan->d_desc, c.e0, c.count,
                           plan->d_alpha, ctx->d_tab, plan->d_mom, plan->d_redo, nullptr, st);
            prof_end(plan, 3, st);
        }
        if (stop == STOP_MOMENTS) {
            const int K = 2 * plan->N - 1;
            const int64_t per = (int64_t)F * K * K * K;
            HIP_TRY(ctx, hipMemcpyAsync(stage_out + c.e0 * per, plan->d_mom, sizeof(double) * per * c.count,
                                        hipMemcpyDeviceToDevice, st));
            continue;
        }
        prof_begin(plan, 2, st);
        if (split) {
            launch_contract_split(problem, plan->N, plan->d_desc, c.e0, c.count, ctx->d_tab, plan->d_mom, out, status,
                                  plan->terms.stiff_scale, plan->terms.mass_scale, int8, st);
        } else if (plan->mode == 1) {
            launch_contract_persistent(problem, plan->d_desc, plan->d_items + c.item0, c.nitem, plan->d_counter,
                                       plan->num_cu * plan->wpc, ctx->d_tab, plan->d_mom, out, status,
                                       plan->terms.stiff_scale, plan->terms.mass_scale, st);
        } else {
            const auto contract = plan->terms.output == P2S_OUTPUT_PACKED_UPPER ? launch_contract_packed
                                                                                : launch_contract;
            if (plan->uniform)
                contract(problem, plan->N, plan->d_desc, nullptr, c.e0, c.count, ctx->d_tab, plan->d_mom, out,
                         status, plan->terms.stiff_scale, plan->terms.mass_scale, st);
            else
                for (const auto &cl : c.classes)
                    contract(problem, (int)cl[0], plan->d_desc, plan->d_elist, cl[1], cl[2], ctx->d_tab,
                             plan->d_mom, out, status, plan->terms.stiff_scale, plan->terms.mass_scale, st);
        }
        prof_end(plan, 2, st);
    }
    if (stop == STOP_TAILREC)
        HIP_TRY(ctx, hipMemcpyAsync(stage_out, plan->d_tailst, sizeof(double) * plan->E * F * TAIL_REC,
                                    hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

int p2s_plan_profile(p2s_plan plan, int enable)
{
    if (!plan) return P2S_EINVAL;
    plan->profile = enable != 0;
    for (auto &u : plan->ev_used) u = 0;
    return P2S_OK;
}

int p2s_plan_profile_read(p2s_plan plan, double *ms, int64_t *launches)
{
    if (!plan || !ms || !launches) return P2S_EINVAL;
    for (int s = 0; s < 4; ++s) {
        double tot = 0.0;
        for (size_t i = 0; i < plan->ev_used[s]; ++i) {
            HIP_TRY(plan->ctx, hipEventSynchronize(plan->ev[s][i][1]));
            float t = 0.f;
            HIP_TRY(plan->ctx, hipEventElapsedTime(&t, plan->ev[s][i][0], plan->ev[s][i][1]));
            tot += t;
        }
        ms[s] = tot;
        launches[s] = (int64_t)plan->ev_used[s];
        plan->ev_used[s] = 0;
    }
    return P2S_OK;
}

int p2s_plan_execute(p2s_plan plan, const double *nodes, const double *material, double *out,
                     uint32_t *status, void *stream)
{
    if (!plan) return P2S_EINVAL;
    return run_plan(plan, nodes, material, out, status, (hipStream_t)stream, STOP_FULL, nullptr);
}

int p2s_plan_coupling(p2s_plan plan, const double *nodes, const double *material, double *alpha, void *stream)
{
    if (!plan) return P2S_EINVAL;
    if (!plan->uniform) return fail(plan->ctx, P2S_EINVAL, "coupling output needs a uniform plan");
    return run_plan(plan, nodes, material, nullptr, plan->d_stage_status, (hipStream_t)stream, STOP_COUPLING,
                    alpha);
}

int p2s_plan_moments(p2s_plan plan, const double *nodes, const double *material, double *moments, void *stream)
{
    if (!plan) return P2S_EINVAL;
    if (!plan->uniform) return fail(plan->ctx, P2S_EINVAL, "moment output needs a uniform plan");
    return run_plan(plan, nodes, material, nullptr, plan->d_stage_status, (hipStream_t)stream, STOP_MOMENTS,
                    moments);
}

int p2s_plan_tail_records(p2s_plan plan, const double *nodes, const double *material, double *records,
                          void *stream)
{
    if (!plan) return P2S_EINVAL;
    p2s_ctx ctx = plan->ctx;
    if (plan->terms.method != P2S_METHOD_P2S) return fail(ctx, P2S_EINVAL, "tail records need the product-to-sum method");
    if (plan->maxN > TAIL_MAXN) return fail(ctx, P2S_EORDER, "tail records: orders up to %d", TAIL_MAXN);
    if (plan->E > 0 && moments_smem_bytes(plan->maxN, plan->mshape.maxQw, plan->mshape.maxQvw, true) > LDS_LIMIT)
        return fail(ctx, P2S_EQUAD, "tail records: rule too large for the moment stage with tail rows");
    if (plan->E > 0 && !plan->d_tailst) {
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        const int64_t n = plan->E * num_fields(plan->terms.problem) * TAIL_REC;
        if (hipMalloc(&plan->d_tailst, sizeof(double) * n) != hipSuccess)
            return fail(ctx, P2S_ENOMEM, "tail records: workspace allocation failed");
        plan->bytes += 8 * n;
    }
    return run_plan(plan, nodes, material, nullptr, plan->d_stage_status, (hipStream_t)stream, STOP_TAILREC,
                    records);
}

// Plans of the one-shot entry point, cached per batch shape in the context:
// the first call of a shape creates the plan (allocates, uploads its
// descriptors), later calls of the same shape reuse it and only enqueue.
static bool same_shape(p2s_plan p, const p2s_terms *t, int64_t E, const int32_t *orders, const int32_t *quad)
{
    const p2s_terms &a = p->terms;
    return a.problem == t->problem && a.material == t->material && a.precision == t->precision &&
           a.method == t->method && a.stiff_scale == t->stiff_scale && a.mass_scale == t->mass_scale &&
           a.output == t->output &&
           p->E == E && (E == 0 || (std::memcmp(p->orders.data(), orders, sizeof(int32_t) * E) == 0 &&
                                    std::memcmp(p->quad.data(), quad, sizeof(int32_t) * 3 * E) == 0));
}

int p2s_fill_element_matrices(p2s_ctx ctx, const p2s_terms *terms, int64_t E, const double *nodes,
                              const double *material, const int32_t *orders, const int32_t *quad,
                              double *out, uint32_t *status, void *stream)
{
    if (!ctx) return P2S_EINVAL;
    if (!terms) return fail(ctx, P2S_EINVAL, "fill: NULL terms");
    if (E < 0 || (E > 0 && (!orders || !quad))) return fail(ctx, P2S_EINVAL, "fill: bad E or NULL orders/quad");
    p2s_plan plan = nullptr;
    for (size_t i = 0; i < ctx->fill_cache.size(); ++i)
        if (same_shape(ctx->fill_cache[i], terms, E, orders, quad)) {
            plan = ctx->fill_cache[i];
            // most recently used last
            ctx->fill_cache.erase(ctx->fill_cache.begin() + i);
            ctx->fill_cache.push_back(plan);
            break;
        }
    if (!plan) {
        int r = p2s_plan_create(ctx, terms, E, orders, quad, &plan);
        if (r != P2S_OK) return r;
        if (ctx->fill_cache.size() >= FILL_CACHE_PLANS) {
            // the least recently used plan goes; hipFree inside waits for
            // the device, so work still queued on it completes first
            p2s_plan_destroy(ctx->fill_cache.front());
            ctx->fill_cache.erase(ctx->fill_cache.begin());
        }
        ctx->fill_cache.push_back(plan);
    }
    return p2s_plan_execute(plan, nodes, material, out, status, stream);
}

int p2s_fill_uniform_noalloc(p2s_ctx ctx, const p2s_terms *terms, int64_t E, int N, int Qu, int Qv, int Qw,
                             const double *nodes, const double *material, double *out, uint32_t *status,
                             void *stream)
{
    if (!ctx) return P2S_EINVAL;
    if (!terms) return fail(ctx, P2S_EINVAL, "noalloc: NULL terms");
    const int problem = terms->problem, kind = terms->material;
    if (problem != P2S_SCALAR && problem != P2S_VECTOR) return fail(ctx, P2S_EINVAL, "noalloc: bad problem %d", problem);
    int stride = 0;
    switch (kind) {
    case P2S_MAT_SINCOSEXP: stride = 1; break;
    case P2S_MAT_ROTDIAG: stride = 12; break;
    case P2S_MAT_PLANEWAVE: stride = 4; break;
    case P2S_ALPHA_SAMPLED: stride = 0; break;
    default: return fail(ctx, P2S_EINVAL, "noalloc: bad material %d", kind);
    }
    if (problem == P2S_SCALAR && kind == P2S_MAT_ROTDIAG)
        return fail(ctx, P2S_EINVAL, "noalloc: the scalar problem takes an isotropic material");
    if (terms->method != P2S_METHOD_P2S || terms->precision != P2S_FP64 || terms->output != P2S_OUTPUT_DENSE)
        return fail(ctx, P2S_EINVAL, "noalloc: FP64 product-to-sum with the dense layout only");
    if (E < 0) return fail(ctx, P2S_EINVAL, "noalloc: negative E");
    if (N < 2 || N > P2S_MAX_ORDER) return fail(ctx, P2S_EORDER, "noalloc: order %d (allowed 2..%d)", N, P2S_MAX_ORDER);
    if (Qu < 1 || Qu > P2S_MAX_Q || Qv < 1 || Qv > P2S_MAX_Q || Qw < 1 || Qw > P2S_MAX_Q)
        return fail(ctx, P2S_EQUAD, "noalloc: Gauss points per axis must be 1..%d", P2S_MAX_Q);
    MomentShape ms;
    ms.maxN = N;
    ms.maxQ = std::max({Qu, Qv, Qw});
    ms.maxQu = Qu;
    ms.maxQuv = Qu * Qv;
    ms.maxQw = Qw;
    ms.maxQvw = Qv * Qw;
    if (moments_lds_bytes(ms) > LDS_LIMIT || moments_smem_bytes(N, Qw, Qv * Qw) > LDS_LIMIT)
        return fail(ctx, P2S_EQUAD, "noalloc: rule too large for the moment stage at order %d", N);
    if (E == 0) return P2S_OK;
    if (!material || !out || !status || (!nodes && kind != P2S_ALPHA_SAMPLED))
        return fail(ctx, P2S_EINVAL, "noalloc: NULL buffer");
    if (!ctx->scratch) return fail(ctx, P2S_EHIP, "noalloc: no scratch on this device");
    const int F = num_fields(problem), K = 2 * N - 1;
    const int64_t P = (int64_t)Qu * Qv * Qw;
    const int64_t na = F * P, nm = (int64_t)F * K * K * K;
    const int64_t nd = num_dofs(problem, N), ndof2 = nd * nd;
    const int64_t mstride = kind == P2S_ALPHA_SAMPLED ? na : stride;
    // scratch layout of a chunk of c elements: descriptors (rounded up to
    // whole doubles), then c * na samples, then c * nm moments
    const int64_t cap = (int64_t)(NOALLOC_SCRATCH_BYTES / sizeof(double));
    const int64_t desc_d = (int64_t)((sizeof(ElemDesc) + sizeof(double) - 1) / sizeof(double));
    const int64_t per = desc_d + na + nm;
    const int64_t chunk = (cap - 64) / per;  // 64 doubles: alignment padding of two regions
    if (chunk < 1)
        return fail(ctx, P2S_EINVAL, "noalloc: one element needs %lld bytes of scratch, more than the %zu available",
                    (long long)(8 * per), NOALLOC_SCRATCH_BYTES);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    for (int64_t e0 = 0; e0 < E; e0 += chunk) {
        const int64_t c = std::min(chunk, E - e0);
        ElemDesc *desc = reinterpret_cast<ElemDesc *>(ctx->scratch);
        // regions start on 256-byte boundaries (32 doubles)
        double *alpha = ctx->scratch + (c * desc_d + 31) / 32 * 32;
        double *mom = alpha + (c * na + 31) / 32 * 32;
        hipLaunchKernelGGL(k_uniform_desc, dim3((unsigned)((c + 255) / 256)), dim3(256), 0, st, desc, c, N, Qu, Qv,
                           Qw, ndof2, na, nm);
        launch_coupling(problem, desc, 0, c, nodes ? nodes + e0 * 81 : nullptr, material + e0 * mstride, kind,
                        stride, ctx->d_tab, alpha, status + e0, nullptr, st);
        launch_moments(problem, ms, desc, 0, c, alpha, ctx->d_tab, mom, nullptr, nullptr, st);
        if (launch_contract(problem, N, desc, nullptr, 0, c, ctx->d_tab, mom, out + e0 * ndof2, status + e0,
                            terms->stiff_scale, terms->mass_scale, st) != 0)
            return fail(ctx, P2S_EINVAL, "noalloc: no contraction kernel for problem %d order %d", problem, N);
    }
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

int p2s_plan_set_schedule(p2s_plan plan, int mode, int wgs_per_cu)
{
    if (!plan) return P2S_EINVAL;
    if (mode != 0 && mode != 1) return fail(plan->ctx, P2S_EINVAL, "schedule: bad mode %d", mode);
    if (mode == 1 && plan->terms.problem != P2S_SCALAR)
        return fail(plan->ctx, P2S_EINVAL, "schedule: the persistent schedule is built for the scalar problem");
    if (mode == 1 && plan->terms.output != P2S_OUTPUT_DENSE)
        return fail(plan->ctx, P2S_EINVAL, "schedule: the persistent schedule writes the dense layout");
    if (mode == 1 && (wgs_per_cu < 1 || wgs_per_cu > 8))
        return fail(plan->ctx, P2S_EINVAL, "schedule: workgroups per CU must be 1..8");
    plan->mode = mode;
    plan->wpc = mode == 1 ? wgs_per_cu : 1;
    return P2S_OK;
}

int p2s_plan_get_schedule(p2s_plan plan, int *mode, int *wgs_per_cu)
{
    if (!plan || !mode || !wgs_per_cu) return P2S_EINVAL;
    *mode = plan->mode;
    *wgs_per_cu = plan->wpc;
    return P2S_OK;
}

// Cache key of a plan shape: problem, order histogram, rule histogram, E.
static std::string plan_key(p2s_plan plan)
{
    std::ostringstream k;
    k << "gfx950/p" << plan->terms.problem << "/o" << plan->terms.output << "/E" << plan->E << "/N";
    int hist[P2S_MAX_ORDER + 1] = {0};
    for (int n : plan->orders) hist[n]++;
    for (int n = 2; n <= P2S_MAX_ORDER; ++n)
        if (hist[n]) k << n << ":" << hist[n] << ",";
    std::map<int, int64_t> qh;
    for (int64_t e = 0; e < plan->E; ++e)
        qh[plan->quad[3 * e] * 10000 + plan->quad[3 * e + 1] * 100 + plan->quad[3 * e + 2]]++;
    k << "/Q";
    uint64_t h = 1469598103934665603ull;  // FNV-1a of the rule histogram
    for (auto &x : qh) {
        h = (h ^ (uint64_t)x.first) * 1099511628211ull;
        h = (h ^ (uint64_t)x.second) * 1099511628211ull;
    }
    k << std::hex << h;
    return k.str();
}

// Cache file: one JSON object, one entry per line:  "key": [mode, wpc, ms],
static std::map<std::string, std::array<double, 3>> read_cache(const char *path)
{
    std::map<std::string, std::array<double, 3>> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find('[', b);
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
        std::array<double, 3> v{};
        if (sscanf(line.c_str() + c, "[%lf, %lf, %lf]", &v[0], &v[1], &v[2]) == 3) m[line.substr(a + 1, b - a - 1)] = v;
    }
    return m;
}

static void write_cache(const char *path, const std::map<std::string, std::array<double, 3>> &m)
{
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        f.precision(17);
        f << "{\n";
        size_t i = 0;
        for (auto &x : m) {
            f << "  \"" << x.first << "\": [" << (int)x.second[0] << ", " << (int)x.second[1] << ", "
              << x.second[2] << "]" << (++i < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

int p2s_plan_autotune(p2s_plan plan, const double *nodes, const double *material, double *out,
                      uint32_t *status, void *stream, const char *cache_path, double *best_ms)
{
    if (!plan) return P2S_EINVAL;
    p2s_ctx ctx = plan->ctx;
    hipStream_t st = (hipStream_t)stream;
    const std::string key = plan_key(plan);
    if (cache_path) {
        auto m = read_cache(cache_path);
        auto it = m.find(key);
        if (it != m.end()) {
            int r = p2s_plan_set_schedule(plan, (int)it->second[0], (int)it->second[1]);
            if (r == P2S_OK) {
                if (best_ms) *best_ms = it->second[2];
                return P2S_OK;
            }
        }
    }
    std::vector<std::array<int, 2>> cand = {{0, 1}};
    if (plan->terms.problem == P2S_SCALAR && plan->terms.output == P2S_OUTPUT_DENSE) {
        cand.push_back({1, 1});
        cand.push_back({1, 2});
        cand.push_back({1, 4});
    }
    const bool prof = plan->profile;
    plan->profile = false;
    hipEvent_t t0, t1;
    HIP_TRY(ctx, hipEventCreate(&t0));
    HIP_TRY(ctx, hipEventCreate(&t1));
    double best = 1e300;
    std::array<int, 2> pick = {plan->mode, plan->wpc};
    int rc = P2S_OK;
    for (auto &c : cand) {
        plan->mode = c[0];
        plan->wpc = c[1];
        if ((rc = run_plan(plan, nodes, material, out, status, st, STOP_FULL, nullptr)) != P2S_OK) break;
        hipEventRecord(t0, st);
        const int reps = 3;
        for (int r = 0; r < reps && rc == P2S_OK; ++r) rc = run_plan(plan, nodes, material, out, status, st, STOP_FULL, nullptr);
        hipEventRecord(t1, st);
        if (rc != P2S_OK) break;
        hipEventSynchronize(t1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, t0, t1);
        if (ms / reps < best) {
            best = ms / reps;
            pick = c;
        }
    }
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    plan->profile = prof;
    plan->mode = pick[0];
    plan->wpc = pick[1];
    if (rc != P2S_OK) return rc;
    if (best_ms) *best_ms = best;
    if (cache_path) {
        auto m = read_cache(cache_path);
        m[key] = {(double)pick[0], (double)pick[1], best};
        write_cache(cache_path, m);
    }
    return P2S_OK;
}

int p2s_plan_capture(p2s_plan plan, const double *nodes, const double *material, double *out,
                     uint32_t *status, void *stream)
{
    if (!plan) return P2S_EINVAL;
    p2s_ctx ctx = plan->ctx;
    hipStream_t st = (hipStream_t)stream;
    if (!st) return fail(ctx, P2S_EINVAL, "capture: needs a non-default stream");
    if (plan->gexec) {
        hipGraphExecDestroy(plan->gexec);
        plan->gexec = nullptr;
    }
    if (plan->graph) {
        hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    const bool prof = plan->profile;
    plan->profile = false;  // no event records inside the graph
    HIP_TRY(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int r = run_plan(plan, nodes, material, out, status, st, STOP_FULL, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    plan->profile = prof;
    if (r != P2S_OK) {
        if (g) hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(ctx, P2S_EHIP, "capture: %s", hipGetErrorString(e));
    plan->graph = g;
    HIP_TRY(ctx, hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0));
    return P2S_OK;
}

int p2s_plan_replay(p2s_plan plan, void *stream)
{
    if (!plan) return P2S_EINVAL;
    if (!plan->gexec) return fail(plan->ctx, P2S_EINVAL, "replay: no captured execution");
    HIP_TRY(plan->ctx, hipGraphLaunch(plan->gexec, (hipStream_t)stream));
    return P2S_OK;
}

// ---------------------------------------------------------------------------
// Learned quadrature order

static int mlp_alloc(p2s_ctx ctx, int64_t bmax)
{
    if (!ctx->d_mlp) {
        for (float **p : {&ctx->d_mlp, &ctx->d_grad, &ctx->d_adam_m, &ctx->d_adam_v})
            if (hipMalloc(p, sizeof(float) * MLP_PARAMS) != hipSuccess)
                return fail(ctx, P2S_ENOMEM, "network: allocation failed");
        hipMemset(ctx->d_adam_m, 0, sizeof(float) * MLP_PARAMS);
        hipMemset(ctx->d_adam_v, 0, sizeof(float) * MLP_PARAMS);
    }
    if (bmax > ctx->mlp_bmax) {
        for (float *p : {ctx->d_h1, ctx->d_h2, ctx->d_z, ctx->d_dz, ctx->d_dh2, ctx->d_dh1, ctx->d_lossb})
            if (p) hipFree(p);
        bool ok = hipMalloc(&ctx->d_h1, sizeof(float) * bmax * MLP_H) == hipSuccess &&
                  hipMalloc(&ctx->d_h2, sizeof(float) * bmax * MLP_H) == hipSuccess &&
                  hipMalloc(&ctx->d_z, sizeof(float) * bmax * MLP_OUT) == hipSuccess &&
                  hipMalloc(&ctx->d_dz, sizeof(float) * bmax * MLP_OUT) == hipSuccess &&
                  hipMalloc(&ctx->d_dh2, sizeof(float) * bmax * MLP_H) == hipSuccess &&
                  hipMalloc(&ctx->d_dh1, sizeof(float) * bmax * MLP_H) == hipSuccess &&
                  hipMalloc(&ctx->d_lossb, sizeof(float) * bmax) == hipSuccess;
        if (!ok) return fail(ctx, P2S_ENOMEM, "network: scratch allocation failed");
        ctx->mlp_bmax = bmax;
    }
    return P2S_OK;
}

int p2s_mlp_init(p2s_ctx ctx, uint64_t seed, int64_t max_batch)
{
    if (!ctx) return P2S_EINVAL;
    if (max_batch < 1) return fail(ctx, P2S_EINVAL, "network: max_batch must be positive");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int r = mlp_alloc(ctx, max_batch);
    if (r != P2S_OK) return r;
    // He-normal weights from a splitmix64 stream (Box-Muller), zero biases
    std::vector<float> p(MLP_PARAMS, 0.f);
    uint64_t x = seed;
    auto next = [&]() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int fan_in, int n) {
        const double sd = std::sqrt(2.0 / fan_in);
        for (int i = 0; i < n; ++i) {
            const double u1 = next() + 1e-300, u2 = next();
            p[off + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    };
    fill(MLP_OFF_W1, MLP_IN, MLP_IN * MLP_H);
    fill(MLP_OFF_W2, MLP_H, MLP_H * MLP_H);
    fill(MLP_OFF_W3, MLP_H, MLP_H * MLP_OUT);
    HIP_TRY(ctx, hipMemcpy(ctx->d_mlp, p.data(), sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemset(ctx->d_adam_m, 0, sizeof(float) * MLP_PARAMS));
    HIP_TRY(ctx, hipMemset(ctx->d_adam_v, 0, sizeof(float) * MLP_PARAMS));
    ctx->adam_step = 0;
    ctx->mlp_ready = true;
    return P2S_OK;
}

int p2s_mlp_set_params(p2s_ctx ctx, const float *params)
{
    if (!ctx || !params) return P2S_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int r = mlp_alloc(ctx, std::max<int64_t>(ctx->mlp_bmax, 1));
    if (r != P2S_OK) return r;
    HIP_TRY(ctx, hipMemcpy(ctx->d_mlp, params, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice));
    ctx->mlp_ready = true;
    return P2S_OK;
}

int p2s_mlp_get_params(p2s_ctx ctx, float *params)
{
    if (!ctx || !params) return P2S_EINVAL;
    if (!ctx->mlp_ready) return fail(ctx, P2S_ENOMODEL, "network: no parameters");
    HIP_TRY(ctx, hipMemcpy(params, ctx->d_mlp, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost));
    return P2S_OK;
}

// File: "P2SK" magic, int32 version 1, int32 (in, hidden, out), float32 params.
int p2s_mlp_save(p2s_ctx ctx, const char *path)
{
    if (!ctx || !path) return P2S_EINVAL;
    std::vector<float> p(MLP_PARAMS);
    int r = p2s_mlp_get_params(ctx, p.data());
    if (r != P2S_OK) return r;
    FILE *f = fopen(path, "wb");
    if (!f) return fail(ctx, P2S_EINVAL, "network: cannot write %s", path);
    const int32_t hdr[4] = {1, MLP_IN, MLP_H, MLP_OUT};
    bool ok = fwrite("P2SK", 1, 4, f) == 4 && fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              fwrite(p.data(), sizeof(float), MLP_PARAMS, f) == (size_t)MLP_PARAMS;
    fclose(f);
    return ok ? P2S_OK : fail(ctx, P2S_EINVAL, "network: short write to %s", path);
}

int p2s_mlp_load(p2s_ctx ctx, const char *path)
{
    if (!ctx || !path) return P2S_EINVAL;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(ctx, P2S_EINVAL, "network: cannot read %s", path);
    char magic[4];
    int32_t hdr[4];
    std::vector<float> p(MLP_PARAMS);
    bool ok = fread(magic, 1, 4, f) == 4 && std::memcmp(magic, "P2SK", 4) == 0 && fread(hdr, sizeof(hdr), 1, f) == 1 &&
              hdr[0] == 1 && hdr[1] == MLP_IN && hdr[2] == MLP_H && hdr[3] == MLP_OUT &&
              fread(p.data(), sizeof(float), MLP_PARAMS, f) == (size_t)MLP_PARAMS;
    fclose(f);
    if (!ok) return fail(ctx, P2S_EINVAL, "network: %s is not a network file of this shape", path);
    return p2s_mlp_set_params(ctx, p.data());
}

int p2s_features(p2s_ctx ctx, int material, int64_t E, const double *nodes, const double *mat, float *x,
                 void *stream)
{
    if (!ctx || E < 0 || (E > 0 && (!nodes || !mat || !x))) return P2S_EINVAL;
    int stride = material == P2S_MAT_SINCOSEXP ? 1 : material == P2S_MAT_ROTDIAG ? 12
               : material == P2S_MAT_PLANEWAVE ? 4 : -1;
    if (stride < 0) return fail(ctx, P2S_EINVAL, "features: bad material %d", material);
    launch_features(E, nodes, mat, material, stride, x, (hipStream_t)stream);
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

static int mlp_check_batch(p2s_ctx ctx, int64_t B)
{
    if (!ctx->mlp_ready) return fail(ctx, P2S_ENOMODEL, "network: not initialised or loaded");
    if (B < 1 || B > ctx->mlp_bmax) return fail(ctx, P2S_EINVAL, "network: batch %lld outside 1..%lld",
                                                (long long)B, (long long)ctx->mlp_bmax);
    return P2S_OK;
}

int p2s_mlp_forward(p2s_ctx ctx, int64_t B, const float *x, float *logits, void *stream)
{
    if (!ctx || !x || !logits) return P2S_EINVAL;
    int r = mlp_check_batch(ctx, B);
    if (r != P2S_OK) return r;
    launch_mlp_forward(B, ctx->d_mlp, x, ctx->d_h1, ctx->d_h2, logits, (hipStream_t)stream);
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

int p2s_mlp_gradients(p2s_ctx ctx, int64_t B, const float *x, const int32_t *labels, float *grad, float *loss,
                      void *stream)
{
    if (!ctx || !x || !labels || !loss) return P2S_EINVAL;
    int r = mlp_check_batch(ctx, B);
    if (r != P2S_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    launch_mlp_forward(B, ctx->d_mlp, x, ctx->d_h1, ctx->d_h2, ctx->d_z, st);
    launch_mlp_backward(B, ctx->d_mlp, x, ctx->d_h1, ctx->d_h2, ctx->d_z, labels, ctx->d_dz, ctx->d_dh2,
                        ctx->d_dh1, ctx->d_grad, ctx->d_lossb, loss, st);
    if (grad)
        HIP_TRY(ctx, hipMemcpyAsync(grad, ctx->d_grad, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

int p2s_mlp_train_step(p2s_ctx ctx, int64_t B, const float *x, const int32_t *labels, float lr, float *loss,
                       void *stream)
{
    int r = p2s_mlp_gradients(ctx, B, x, labels, nullptr, loss, stream);
    if (r != P2S_OK) return r;
    launch_adam(ctx->d_mlp, ctx->d_grad, ctx->d_adam_m, ctx->d_adam_v, lr, ++ctx->adam_step, (hipStream_t)stream);
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

int p2s_mlp_predict(p2s_ctx ctx, int64_t B, const float *x, float p_cover, int32_t *quad, void *stream)
{
    if (!ctx || !x || !quad) return P2S_EINVAL;
    int r = mlp_check_batch(ctx, B);
    if (r != P2S_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    launch_mlp_forward(B, ctx->d_mlp, x, ctx->d_h1, ctx->d_h2, ctx->d_z, st);
    launch_choose(B, ctx->d_z, p_cover, MLP_KMAX + 1, quad, nullptr, st);
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

int p2s_plan_set_learned(p2s_plan plan, int enable, float p_cover, int k_direct, double theta)
{
    if (!plan) return P2S_EINVAL;
    p2s_ctx ctx = plan->ctx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (!enable) {
        plan->learned = false;
        if (plan->E > 0)
            HIP_TRY(ctx, hipMemcpy(plan->d_desc, plan->desc_host.data(), sizeof(ElemDesc) * plan->E,
                                   hipMemcpyHostToDevice));
        return P2S_OK;
    }
    if (plan->terms.material == P2S_ALPHA_SAMPLED || plan->terms.method != P2S_METHOD_P2S || !plan->uniform ||
        plan->Qu != MLP_KMAX || plan->Qv != MLP_KMAX || plan->Qw != MLP_KMAX)
        return fail(ctx, P2S_EINVAL, "learned order: needs a uniform product-to-sum plan created with %d points "
                                     "per axis", MLP_KMAX);
    if (plan->N > TAIL_MAXN) return fail(ctx, P2S_EORDER, "learned order: orders up to %d", TAIL_MAXN);
    if (moments_smem_bytes(plan->maxN, plan->mshape.maxQw, plan->mshape.maxQvw, true) > LDS_LIMIT)
        return fail(ctx, P2S_EQUAD, "learned order: rule too large for the moment stage with tail rows");
    if (!(p_cover > 0.f && p_cover <= 1.f) || !(theta > 0.0) || k_direct < MLP_KMIN)
        return fail(ctx, P2S_EINVAL, "learned order: bad p_cover / k_direct / theta");
    if (!plan->d_lx && plan->E > 0) {
        const int64_t E = plan->E;
        bool ok = hipMalloc(&plan->d_lx, sizeof(float) * E * MLP_IN) == hipSuccess &&
                  hipMalloc(&plan->d_lh1, sizeof(float) * E * MLP_H) == hipSuccess &&
                  hipMalloc(&plan->d_lh2, sizeof(float) * E * MLP_H) == hipSuccess &&
                  hipMalloc(&plan->d_lz, sizeof(float) * E * MLP_OUT) == hipSuccess &&
                  hipMalloc(&plan->d_redo, sizeof(int32_t) * E) == hipSuccess &&
                  hipMalloc(&plan->d_tau, sizeof(double) * E) == hipSuccess &&
                  (plan->d_tailst || hipMalloc(&plan->d_tailst, sizeof(double) * E *
                                                                    num_fields(plan->terms.problem) * TAIL_REC) ==
                                         hipSuccess);
        if (!ok) return fail(ctx, P2S_ENOMEM, "learned order: workspace allocation failed");
        plan->bytes += E * (int64_t)(4 * (MLP_IN + 2 * MLP_H + MLP_OUT) + 12 +
                                     8 * num_fields(plan->terms.problem) * TAIL_REC);
    }
    plan->learned = true;
    plan->p_cover = p_cover;
    plan->k_direct = k_direct;
    plan->theta = theta;
    return P2S_OK;
}

int p2s_plan_rules(p2s_plan plan, int32_t *quad)
{
    if (!plan || (!quad && plan->E > 0)) return P2S_EINVAL;
    std::vector<ElemDesc> d(plan->E);
    if (plan->E > 0)
        HIP_TRY(plan->ctx, hipMemcpy(d.data(), plan->d_desc, sizeof(ElemDesc) * plan->E, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < plan->E; ++e) {
        quad[3 * e] = d[e].Qu;
        quad[3 * e + 1] = d[e].Qv;
        quad[3 * e + 2] = d[e].Qw;
    }
    return P2S_OK;
}

int p2s_plan_tail_values(p2s_plan plan, double *tau)
{
    if (!plan || (!tau && plan->E > 0)) return P2S_EINVAL;
    if (!plan->d_tau) return fail(plan->ctx, P2S_EINVAL, "tail values: the plan has not run in learned mode");
    HIP_TRY(plan->ctx, hipMemcpy(tau, plan->d_tau, sizeof(double) * plan->E, hipMemcpyDeviceToHost));
    return P2S_OK;
}

int p2s_rel_error(p2s_ctx ctx, int64_t E, int64_t len, const int64_t *offsets, const double *a, const double *b,
                  double *err, void *stream)
{
    if (!ctx || E < 0 || (E > 0 && (!a || !b || !err)) || (!offsets && len < 1)) return P2S_EINVAL;
    launch_rel_error(E, len, offsets, a, b, err, (hipStream_t)stream);
    HIP_TRY(ctx, hipGetLastError());
    return P2S_OK;
}

}  // extern "C"
