// p2s_api.hip -- C ABI and host runtime of the product-to-sum fill:
// contexts (tables built once), plans (descriptors, schedule, workspace),
// and the chunked execution of the three stages on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
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
};

struct Chunk {
    int64_t e0 = 0, count = 0;
    // per order class inside the chunk: (N, offset into elist, count)
    std::vector<std::array<int64_t, 3>> classes;
};

struct p2s_plan_s {
    p2s_ctx ctx = nullptr;
    p2s_terms terms{};
    int64_t E = 0;
    bool uniform = true;
    int N = 0, Qu = 0, Qv = 0, Qw = 0;
    int maxN = 0, maxQu = 0, maxQuv = 0;
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
    if (hipMemcpy(ctx->d_tab, tab.data(), sizeof(double) * TAB_SIZE, hipMemcpyHostToDevice) != hipSuccess ||
        prepare_kernels() != 0) {
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
    if (ctx->d_tab) hipFree(ctx->d_tab);
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
        b = (s ? atoll(s) : 512) << 20;
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
    if (terms->precision != P2S_FP64 || terms->method != P2S_METHOD_P2S)
        return fail(ctx, P2S_EINVAL, "plan: unsupported precision/method combination");
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
        plan->maxQu = std::max(plan->maxQu, (int)quad[3 * e]);
        plan->maxQuv = std::max(plan->maxQuv, (int)(quad[3 * e] * quad[3 * e + 1]));
        if (e > 0 && (N != orders[0] || quad[3 * e] != quad[0] || quad[3 * e + 1] != quad[1] ||
                      quad[3 * e + 2] != quad[2]))
            plan->uniform = false;
    }
    p2s_layout(problem, E, orders, plan->offsets.data());
    if (E > 0) {
        plan->N = orders[0];
        plan->Qu = quad[0];
        plan->Qv = quad[1];
        plan->Qw = quad[2];
    }
    if (kind == P2S_ALPHA_SAMPLED && !plan->uniform) {
        delete plan;
        return fail(ctx, P2S_EINVAL, "plan: sampled coupling input needs one order and rule for all elements");
    }
    if (E > 0 && moments_smem_bytes(plan->maxN, plan->maxQu, plan->maxQuv) > LDS_LIMIT) {
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
                for (int64_t e = c.e0; e < c.e0 + c.count; ++e)
                    if (orders[e] == N) elist.push_back((int32_t)e);
                const int64_t cnt = (int64_t)elist.size() - start;
                if (cnt > 0) c.classes.push_back({N, start, cnt});
            }
        }
    }
    hipSetDevice(ctx->device);
    bool ok = true;
    if (E > 0) {
        ok = ok && hipMalloc(&plan->d_desc, sizeof(ElemDesc) * E) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_alpha, sizeof(double) * std::max<int64_t>(plan->alpha_cap, 1)) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_mom, sizeof(double) * std::max<int64_t>(plan->mom_cap, 1)) == hipSuccess;
        ok = ok && hipMalloc(&plan->d_stage_status, sizeof(uint32_t) * E) == hipSuccess;
        if (!elist.empty()) ok = ok && hipMalloc(&plan->d_elist, sizeof(int32_t) * elist.size()) == hipSuccess;
    }
    if (!ok) {
        p2s_plan_destroy(plan);
        return fail(ctx, P2S_ENOMEM, "plan: workspace allocation failed");
    }
    plan->bytes = (int64_t)(sizeof(ElemDesc) * E + 8 * (plan->alpha_cap + plan->mom_cap) + 4 * elist.size());
    if (E > 0) {
        if (hipMemcpy(plan->d_desc, desc.data(), sizeof(ElemDesc) * E, hipMemcpyHostToDevice) != hipSuccess ||
            (!elist.empty() && hipMemcpy(plan->d_elist, elist.data(), sizeof(int32_t) * elist.size(),
                                         hipMemcpyHostToDevice) != hipSuccess)) {
            p2s_plan_destroy(plan);
            return fail(ctx, P2S_EHIP, "plan: descriptor upload failed");
        }
    }
    *out = plan;
    return P2S_OK;
}

enum StageStop { STOP_COUPLING = 0, STOP_MOMENTS = 1, STOP_FULL = 2 };

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
    for (const Chunk &c : plan->chunks) {
        prof_begin(plan, 0, st);
        launch_coupling(problem, plan->d_desc, c.e0, c.count, nodes, material, plan->terms.material,
                        plan->mat_stride, ctx->d_tab, plan->d_alpha, status, st);
        prof_end(plan, 0, st);
        if (stop == STOP_COUPLING) {
            const int64_t per = (int64_t)F * plan->Qu * plan->Qv * plan->Qw;
            HIP_TRY(ctx, hipMemcpyAsync(stage_out + c.e0 * per, plan->d_alpha, sizeof(double) * per * c.count,
                                        hipMemcpyDeviceToDevice, st));
            continue;
        }
        prof_begin(plan, 1, st);
        launch_moments(problem, plan->maxN, plan->maxQu, plan->maxQuv, plan->d_desc, c.e0, c.count,
                       plan->d_alpha, ctx->d_tab, plan->d_mom, st);
        prof_end(plan, 1, st);
        if (stop == STOP_MOMENTS) {
            const int K = 2 * plan->N - 1;
            const int64_t per = (int64_t)F * K * K * K;
            HIP_TRY(ctx, hipMemcpyAsync(stage_out + c.e0 * per, plan->d_mom, sizeof(double) * per * c.count,
                                        hipMemcpyDeviceToDevice, st));
            continue;
        }
        prof_begin(plan, 2, st);
        if (plan->uniform) {
            launch_contract(problem, plan->N, plan->d_desc, nullptr, c.e0, c.count, ctx->d_tab,
                            plan->d_mom, out, status, plan->terms.stiff_scale, plan->terms.mass_scale, st);
        } else {
            for (const auto &cl : c.classes)
                launch_contract(problem, (int)cl[0], plan->d_desc, plan->d_elist, cl[1], cl[2], ctx->d_tab,
                                plan->d_mom, out, status, plan->terms.stiff_scale,
                                plan->terms.mass_scale, st);
        }
        prof_end(plan, 2, st);
    }
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

int p2s_fill_element_matrices(p2s_ctx ctx, const p2s_terms *terms, int64_t E, const double *nodes,
                              const double *material, const int32_t *orders, const int32_t *quad,
                              double *out, uint32_t *status, void *stream)
{
    p2s_plan plan = nullptr;
    int r = p2s_plan_create(ctx, terms, E, orders, quad, &plan);
    if (r != P2S_OK) return r;
    r = p2s_plan_execute(plan, nodes, material, out, status, stream);
    hipStreamSynchronize((hipStream_t)stream);
    p2s_plan_destroy(plan);
    return r;
}

}  // extern "C"
