// p2s_contract_impl.h -- device code of the contraction stage, eq. (4):
// M = sum_s sum_{k,l,q} Cu Cv Cw I_s, applied mode by mode, for gfx950
// (wave64).  Included by p2s_contract.hip (product-to-sum: moments and
// linearization coefficients) and p2s_direct_sf.hip (the same three stages
// as sum-factorized direct quadrature of eq. (2): coupling samples and
// weighted basis products at the Gauss points).
//
// One kernel per component block (I, J >= I) and one workgroup per (element,
// first-axis test index m1): it produces rows (m1, n1, p1) of component I
// against component J (the element matrix is symmetric; the part below the
// diagonal is stored as the mirror image).  Within a block the coupling
// terms are grouped: a group shares the (v, w) family pairs, a run shares
// the w pair.
//   stage A  A_g[m2][l][q] = sum_{s in g} sign_s sum_k Cu_s[m1][m2][k] I_s[k][l][q]
//            one thread per (group, l, q); each moment is loaded once and
//            reused for every m2                                     (LDS)
//   stage B  B[q] += sum_l Cv_g[n1][n2][l] A_g[m2][l][q]  over the groups
//            of a run; one lane per (m2, n1, n2)                   (registers)
//   stage C  acc[p1][p2] += sum_q Cw_run[p1][p2][q] B[q]           (registers)
// The term structure of every block is computed at compile time, so the
// family pairs, fields and signs are constants; stage C's sparsity is
// unrolled and its coefficients are scalar loads from a packed table.
// The finished tile goes through LDS so that every store instruction writes
// whole rows (1 KiB per wave instruction).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "p2s_internal.h"
#include "p2s_kernels.h"
#include "p2s_terms.h"

namespace p2s {

// ---------------------------------------------------------------------------
// Compile-time structure

struct MaskTableC {
    uint32_t m[NTYPE][MAXN][MAXN];
    constexpr MaskTableC() : m()
    {
        for (int t = 0; t < NTYPE; ++t)
            for (int a = 0; a < MAXN; ++a)
                for (int b = 0; b < MAXN; ++b) m[t][a][b] = prod_mask(t / 3, a, t % 3, b);
    }
};
static __constant__ MaskTableC c_cmasks = MaskTableC();

struct PackIndex {
    int16_t before[MAXN + 1][NTYPE][MAXN][MAXN];
    constexpr PackIndex() : before()
    {
        for (int n = 2; n <= MAXN; ++n)
            for (int t = 0; t < NTYPE; ++t) {
                int c = 0;
                for (int p1 = 0; p1 < fam_dim(t / 3, n); ++p1)
                    for (int p2 = 0; p2 < fam_dim(t % 3, n); ++p2) {
                        before[n][t][p1][p2] = (int16_t)c;
                        c += popcount32(prod_mask(t / 3, p1, t % 3, p2));
                    }
            }
    }
};
constexpr PackIndex kPackIndex = PackIndex();

struct PackOffsets {
    int off[MAXN + 1][NTYPE];
    constexpr PackOffsets() : off()
    {
        int o = 0;  // same running layout as packed_offset()
        for (int n = 2; n <= MAXN; ++n)
            for (int t = 0; t < NTYPE; ++t) {
                off[n][t] = o;
                o += (packed_count(t / 3, t % 3, n) + 1) & ~1;
            }
    }
};
constexpr PackOffsets kPackOffsets = PackOffsets();

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Compile-time shape of the work item of row component I against the column
// components JB <= J < JE: lane count, LDS batching and store tile.  PAIR
// (diagonal block only): the item holds the two row bands m1 and NM - 1 - m1,
// whose triangles m2 >= m1 together span NM + 1 column slabs.
template <int PROB, int N, int I, int JB = I, int JE = num_comp(PROB), bool DSF = false, bool PAIR = false>
struct CS {
    // contracted extent per axis: the 2N-1 Legendre degrees of the moments,
    // or (sum-factorized direct quadrature) the 2N Gauss points
    static constexpr int K = DSF ? 2 * N : 2 * N - 1;
    static constexpr int KS = DSF ? K : K + 1;  // LDS row stride (16-byte aligned rows)
    static constexpr int NC = num_comp(PROB);
    static constexpr int NDOF = num_dofs(PROB, N);
    static constexpr int NM_I = comp_dim(PROB, N, I, 0);
    static constexpr int NN_I = comp_dim(PROB, N, I, 1);
    static constexpr int NP_I = comp_dim(PROB, N, I, 2);
    static constexpr int max_over_j(int what)
    {
        int m = 0;
        for (int j = JB; j < JE; ++j) {
            int v = 0;
            if (what == 0)  // lane tasks
                v = (comp_dim(PROB, N, j, 0) + (PAIR ? 1 : 0)) * NN_I * comp_dim(PROB, N, j, 1);
            if (what == 1) v = make_block_c(PROB, I, j).ngroup;
            if (what == 2) v = comp_dim(PROB, N, j, 1);
            if (what == 3) v = comp_dim(PROB, N, j, 0) * comp_dim(PROB, N, j, 1) * comp_dim(PROB, N, j, 2);
            if (what == 4) v = comp_dim(PROB, N, j, 1) * comp_dim(PROB, N, j, 2);
            m = cmax(m, v);
        }
        return m;
    }
    // stage-B lanes in whole waves; from N = 7 on a CU holds a single
    // workgroup, so whole groups of four waves keep its four SIMDs evenly
    // loaded (and stage A's workers of two groups fit one pass)
    static constexpr int THREADS =
        N <= 6 ? ((max_over_j(0) + 63) / 64) * 64 : ((max_over_j(0) + 255) / 256) * 256;
    static constexpr int MAXG = max_over_j(1);
    static constexpr int A_ROWS = PAIR ? NM_I + 1 : N;              // column slabs held in LDS
    static constexpr int A_DOUBLES = A_ROWS * K * KS;               // stage-A result per group
    static constexpr int C_DOUBLES = NN_I * max_over_j(2) * KS;      // stage-B coefficients per group
    static constexpr int GROUP_DOUBLES = A_DOUBLES + C_DOUBLES;
    // groups per LDS batch: at most 40 KiB up to N = 6, so that four
    // three-wave workgroups share a CU (the 168-VGPR bound of k_contract
    // allows twelve waves per CU), ~62 KiB above; paired items, whose groups
    // are larger, at most 32 KiB: three groups per batch at N = 6, which
    // measured faster than four (the unrolled groups of a batch hold fewer
    // coefficients in scalar registers at once, so fewer spill).  The
    // point-table form (DSF) keeps four (52 KiB): two per batch, what 32 KiB
    // leaves of its larger groups, measured slower
    static constexpr int PAIR_BUDGET = DSF ? 6656 : 4096;
    static constexpr int G =
        cmax(1, cmin(MAXG, (N <= 6 ? (PAIR ? PAIR_BUDGET : 5120) : 7936) / GROUP_DOUBLES));
    static constexpr int TILE_MIN = NN_I * NP_I * (max_over_j(4) + 2);  // one m2 of the store tile
    static constexpr int BUF = cmax(G * GROUP_DOUBLES, TILE_MIN);
    static constexpr int SA = ((K * K + 63) / 64) * 64;              // stage-A workers per group
};

// constant address space: loads through it become scalar (SMEM) loads
typedef __attribute__((address_space(4))) const double cdouble;

// Output stores are streaming (each value is written once and not read
// again by the fill): non-temporal stores, which measured faster than plain
// ones for the element-matrix write pattern.
typedef double nt_double2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_out2(double *p, double a, double b)
{
    const nt_double2 v = {a, b};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_double2 *>(p));
}
__device__ __forceinline__ void store_out(double *p, double a) { __builtin_nontemporal_store(a, p); }
// Two values of a mirrored row segment [lo, hi).  The segments are short
// (NR values) and their ends fall inside 128-byte lines that the neighbouring
// bands' segments complete; a line wholly inside the segment is streamed like
// the rest of the output, while a shared line takes an ordinary store, which
// the L2 holds until the other piece arrives and then writes back whole.
// Streamed, the pieces reach HBM as partial-line writes.
__device__ __forceinline__ void store_mirror2(double *p, double a, double b, const double *lo, const double *hi)
{
    const uintptr_t line = reinterpret_cast<uintptr_t>(p) & ~uintptr_t(127);
    if (line >= reinterpret_cast<uintptr_t>(lo) && line + 128 <= reinterpret_cast<uintptr_t>(hi))
        store_out2(p, a, b);
    else
        *reinterpret_cast<double2 *>(p) = make_double2(a, b);
}

template <int N, int X, int Y, int P1, int P2>
__device__ __forceinline__ void stage_c_one(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                            cdouble *__restrict__ tb)
{
    if constexpr (P1 < fam_dim(X, N) && P2 < fam_dim(Y, N)) {
        constexpr uint32_t msk = prod_mask(X, P1, Y, P2);
        constexpr int base = kPackIndex.before[N][3 * X + Y][P1][P2];
#pragma unroll
        for (int q = 0; q < 2 * N - 1; ++q)
            if ((msk >> q) & 1u)
                acc[P1][P2] = fma(tb[base + popcount32(msk & ((1u << q) - 1u))], bv[q], acc[P1][P2]);
    }
}

// The coefficients of row p1 are loaded from a base that has passed
// through an empty asm taking every result of row p1 - 2 as input: their
// scalar loads cannot be issued before that row is done, so about two rows
// of coefficients are live at a time.  Issued early, the ~90 coefficients
// of a run (two scalar registers each) overflow the scalar register file
// and are spilled into vector-register lanes, at two lane reads per FMA.
template <int N>
__device__ __forceinline__ cdouble *after_row(cdouble *tb, const double (&r)[N])
{
    constexpr int A = 0, B = N > 1 ? 1 : 0, C = N > 2 ? 2 : 0, D = N > 3 ? 3 : 0, E = N > 4 ? 4 : 0,
                  F = N > 5 ? 5 : 0, G = N > 6 ? 6 : 0, H = N > 7 ? 7 : 0;
    asm volatile("" : "+s"(tb) : "v"(r[A]), "v"(r[B]), "v"(r[C]), "v"(r[D]), "v"(r[E]), "v"(r[F]), "v"(r[G]),
                 "v"(r[H]));
    return tb;
}

template <int N, int X, int Y, int P1, int... P2s>
__device__ __forceinline__ void stage_c_row(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                            cdouble *__restrict__ tb, std::integer_sequence<int, P2s...>)
{
    if constexpr (P1 >= 2)
        tb = after_row<N>(tb, acc[P1 - 2]);
    else
        asm volatile("" : "+s"(tb) : "v"(bv[0]));
    (stage_c_one<N, X, Y, P1, P2s>(acc, bv, tb), ...);
}

template <int N, int X, int Y, int... P1s>
__device__ __forceinline__ void stage_c_all(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                            cdouble *__restrict__ tb, std::integer_sequence<int, P1s...>)
{
    (stage_c_row<N, X, Y, P1s>(acc, bv, tb, std::make_integer_sequence<int, N>{}), ...);
}

template <int N, int T>
__device__ __forceinline__ void stage_c(double (&acc)[N][N], const double (&bv)[2 * N - 1],
                                        const double *__restrict__ pack)
{
    constexpr int X = T / 3, Y = T % 3;
    constexpr int off = kPackOffsets.off[N][T];
    static_assert(off == packed_offset(N, X, Y), "packed table layout");
    // every coefficient is a scalar load at an immediate offset from the base
    stage_c_all<N, X, Y>(acc, bv, (cdouble *)(pack + off), std::make_integer_sequence<int, N>{});
}

// Stage C of the sum-factorized direct quadrature: dense over the 2N Gauss
// points, coefficients w_c X_p1(x_c) Y_p2(x_c) from the point table (same
// [type][p1][p2][point] layout as the linearization table) as scalar loads.
template <int N, int T>
__device__ __forceinline__ void stage_c_points(double (&acc)[N][N], const double (&bv)[2 * N],
                                               const double *__restrict__ pt)
{
    constexpr int X = T / 3, Y = T % 3;
    cdouble *tb = (cdouble *)(pt + T * LIN_STRIDE_T);
#pragma unroll
    for (int p1 = 0; p1 < fam_dim(X, N); ++p1) {
        tb = after_row<N>(tb, acc[p1 >= 2 ? p1 - 2 : 0]);
#pragma unroll
        for (int p2 = 0; p2 < fam_dim(Y, N); ++p2)
#pragma unroll
            for (int q = 0; q < 2 * N; ++q)
                acc[p1][p2] = fma(tb[p1 * LIN_STRIDE_M1 + p2 * KPAD + q], bv[q], acc[p1][p2]);
    }
}

// Work-group id -> logical work item, so that consecutive items (the row
// tiles of one element, which share its moment tensors) run on the same XCD:
// the hardware deals work-group ids round-robin over the 8 XCDs.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t total_padded)
{
    const int64_t per = total_padded >> 3;
    return (w & 7) * per + (w >> 3);
}

// One work item: rows (m1, n1, p1) of component I of element e against the
// column components JB <= J < JE (JB >= I).  Called by all `nthreads` threads of a
// workgroup (nthreads >= THREADS; extra threads take part in the barriers
// and the cooperative loops only).  smem holds at least BUF doubles.
// DSF: the same three stages as sum-factorized direct quadrature of eq. (2):
// the moments are replaced by the coupling samples at the 2N-point rule
// (mom = the sample buffer) and the linearization coefficients by the
// weighted basis products w_a X_m1(x_a) Y_m2(x_a) at those points (dense).
// PAIR (diagonal block, JB = I, JE = I + 1): m1 is a pair index p and the
// item holds row bands p and NM - 1 - p (one band when they coincide); the
// lanes of the first band come first, and the stage-A rows of the two bands'
// triangles m2 >= m1 lie one after the other in LDS.  MERGE: the lines that
// a mirrored segment shares with its neighbours take ordinary stores (see
// store_mirror2); it pays only where the items that write the other pieces
// run alongside (the single-launch vector kernel with paired items).  SMEM:
// doubles of smem available to the store tile (0: the item's own BUF).
template <int PROB, int N, int I, int JB = I, int JE = num_comp(PROB), bool DSF = false, bool PACKED = false,
          bool PAIR = false, bool MERGE = false, int SMEM = 0>
__device__ __forceinline__ void contract_item(const ElemDesc &d, int64_t e, int m1,
                                              const double *__restrict__ tab, const double *__restrict__ mom,
                                              double *__restrict__ out, uint32_t *__restrict__ status,
                                              double sK, double sM, double *__restrict__ smem, int nthreads)
{
    using S = CS<PROB, N, I, JB, JE, DSF, PAIR>;
    static_assert(!PAIR || (JB == I && JE == I + 1), "paired items belong to a diagonal block");
    constexpr int K = S::K, KS = S::KS, NC = S::NC, NDOF = S::NDOF, G = S::G;
    constexpr int NM_I = S::NM_I, NN_I = S::NN_I, NP_I = S::NP_I, A_ROWS = S::A_ROWS;
    constexpr uint32_t FULL = (1u << K) - 1u;
    const double *lin = DSF ? tab + TAB_PT + N * PT_STRIDE_N : tab + TAB_LIN;
    const double *pack = tab + TAB_PACK;
    const double *I0 = mom + (DSF ? d.alpha_off : d.mom_off);
    double *obase = out + d.out_off;
    const int tid = threadIdx.x;
    // row bands: m1a = m1, and with PAIR the mirror band m1b when distinct
    const int m1a = m1;
    const int m1b = PAIR ? NM_I - 1 - m1 : m1;
    const bool two = PAIR && m1b > m1a;
    bool bad = false;

    static_for<JB, JE>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        constexpr BlockC BK = BlockOf<PROB, I, J>::B;
        constexpr int NM_J = comp_dim(PROB, N, J, 0), NN_J = comp_dim(PROB, N, J, 1),
                      NP_J = comp_dim(PROB, N, J, 2);
        constexpr int NBATCH = (BK.ngroup + G - 1) / G;
        // symmetric: inside the diagonal block only m2 >= m1
        const int nma = NM_J - ((J == I) ? m1a : 0);
        const int Ta = nma * NN_I * NN_J;
        const int nmb = two ? NM_J - m1b : 0;
        const bool bandb = tid >= Ta;   // lane of the second band
        const int lt = bandb ? tid - Ta : tid;
        const int m2lo = (J == I) ? (bandb ? m1b : m1a) : 0;
        const int nm = bandb ? nmb : nma;
        const bool active = bandb ? lt < nmb * NN_I * NN_J : true;
        const int n2 = lt % NN_J;
        const int m2 = active ? m2lo + (lt / NN_J) % nm : m2lo;
        const int n1 = active ? lt / (NN_J * nm) : 0;
        // stage-A row of this lane's m2: the absolute m2, or with PAIR the
        // compact rows of the first band's triangle, then the second's
        const int arow_m = PAIR ? (bandb ? nma + (m2 - m1b) : m2 - m1a) : m2;
        double acc[N][N];
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int b = 0; b < N; ++b) acc[a][b] = 0.0;
        double bsum[K];
#pragma unroll
        for (int q = 0; q < K; ++q) bsum[q] = 0.0;

        static_for<0, NBATCH>([&](auto Bc) {
            constexpr int g0 = decltype(Bc)::value * G;
            constexpr int ng = cmin(G, BK.ngroup - g0);
            double *Abuf = smem;                    // [ng][N][K][KS]
            double *Cbuf = smem + ng * S::A_DOUBLES;  // [ng][NN_I*NN_J][KS]
            // stage-B coefficient rows of this batch into LDS
            for (int x = tid; x < ng * NN_I * NN_J * K; x += nthreads) {
                const int gl = x / (NN_I * NN_J * K);
                const int r = x - gl * (NN_I * NN_J * K);
                const int nn = r / K, l = r - (r / K) * K;
                const int a1 = nn / NN_J, a2 = nn - (nn / NN_J) * NN_J;
                int tv = 0;
                static_for<0, ng>([&](auto gc) {
                    constexpr int g = decltype(gc)::value;
                    if (gl == g) tv = BK.t[BK.gstart[g0 + g]].tv;
                });
                Cbuf[gl * (NN_I * NN_J * KS) + nn * KS + l] =
                    lin[tv * LIN_STRIDE_T + a1 * LIN_STRIDE_M1 + a2 * KPAD + l];
            }
            // stage A: worker w -> (group gl, entry lq); gl is wave-uniform
            for (int w = tid; w < ng * S::SA; w += nthreads) {
                const int gl = w / S::SA;
                const int lq = w - gl * S::SA;
                if (lq < K * K) {
                    double a[A_ROWS];
#pragma unroll
                    for (int r = 0; r < A_ROWS; ++r) a[r] = 0.0;
                    static_for<0, ng>([&](auto gc) {
                        constexpr int g = decltype(gc)::value;
                        if (gl != g) return;
                        // m1 is wave-uniform: inside this dispatch it is a
                        // constant, so the degree masks of the k-sum and the
                        // coefficient offsets are constants and every
                        // coefficient is a scalar load
                        static_for<0, PAIR ? (NM_I + 1) / 2 : NM_I>([&](auto Mc) {
                            constexpr int M1 = decltype(Mc)::value;
                            if (m1 != M1) return;
                            // PAIR: the second band and its first row
                            constexpr int M1B = PAIR ? NM_I - 1 - M1 : M1;
                            constexpr int RB = NM_J - M1;
                            static_for<BK.gstart[g0 + g], BK.gstart[g0 + g + 1]>([&](auto sc_) {
                                constexpr TermC t = BK.t[decltype(sc_)::value];
                                const double sc = (t.scale ? sM : sK) * (double)t.sign;
                                const double *Ip = I0 + (int64_t)t.field * K * K * K + lq;
                                double v[K];
#pragma unroll
                                for (int k = 0; k < K; ++k) v[k] = Ip[k * K * K];
                                // the base passes through an empty asm here, inside
                                // the loop: the term's offset then folds into the
                                // loads' immediates instead of one hoisted 64-bit
                                // base per (m1, term) held in scalar registers
                                const double *lp = lin;
                                asm volatile("" : "+s"(lp));
                                cdouble *Cu = (cdouble *)(lp + t.tu * LIN_STRIDE_T + M1 * LIN_STRIDE_M1);
                                static_for<(J == I ? M1 : 0), NM_J>([&](auto mc) {
                                    constexpr int mm = decltype(mc)::value;
                                    constexpr uint32_t mk = DSF ? FULL : prod_mask(t.tu / 3, M1, t.tu % 3, mm);
                                    double xs = 0.0;
#pragma unroll
                                    for (int k = 0; k < K; ++k)
                                        if ((mk >> k) & 1u) xs = fma(Cu[mm * KPAD + k], v[k], xs);
                                    constexpr int r = PAIR ? mm - M1 : mm;
                                    a[r] = fma(sc, xs, a[r]);
                                });
                                if constexpr (PAIR && M1B > M1) {
                                    // the second band reuses the moment column v
                                    cdouble *Cb = (cdouble *)(lp + t.tu * LIN_STRIDE_T + M1B * LIN_STRIDE_M1);
                                    static_for<M1B, NM_J>([&](auto mc) {
                                        constexpr int mm = decltype(mc)::value;
                                        constexpr uint32_t mk = DSF ? FULL : prod_mask(t.tu / 3, M1B, t.tu % 3, mm);
                                        double xs = 0.0;
#pragma unroll
                                        for (int k = 0; k < K; ++k)
                                            if ((mk >> k) & 1u) xs = fma(Cb[mm * KPAD + k], v[k], xs);
                                        constexpr int r = RB + mm - M1B;
                                        a[r] = fma(sc, xs, a[r]);
                                    });
                                }
                            });
                        });
                    });
                    const int l = lq / K, q = lq - (lq / K) * K;
                    double *Ab = Abuf + gl * S::A_DOUBLES + l * KS + q;
                    if constexpr (PAIR) {
                        const int nrow = nma + nmb;
#pragma unroll
                        for (int r = 0; r < A_ROWS; ++r)
                            if (r < nrow) Ab[r * K * KS] = a[r];
                    } else {
                        const int mlo = (J == I) ? m1a : 0;
#pragma unroll
                        for (int mm = 0; mm < NM_J; ++mm)
                            if (mm >= mlo) Ab[mm * K * KS] = a[mm];
                    }
                }
            }
            __syncthreads();
            if (active) {
                static_for<0, ng>([&](auto gc) {
                    constexpr int g = decltype(gc)::value;
                    constexpr int tv = BK.t[BK.gstart[g0 + g]].tv;
                    constexpr int tw = BK.t[BK.gstart[g0 + g]].tw;
                    // stage B: two set bits of the degree mask per step
                    uint32_t ml = DSF ? FULL : c_cmasks.m[tv][n1][n2];
                    const double *crow = Cbuf + g * (NN_I * NN_J * KS) + (n1 * NN_J + n2) * KS;
                    const double *arow = Abuf + g * S::A_DOUBLES + arow_m * K * KS;
                    while (ml) {
                        const int l0 = __ffs(ml) - 1;
                        ml &= ml - 1u;
                        const bool two = ml != 0u;
                        const int l1 = two ? __ffs(ml) - 1 : l0;
                        ml &= two ? ml - 1u : ml;
                        const double c0 = crow[l0];
                        const double c1 = two ? crow[l1] : 0.0;
                        const double2 *r0 = reinterpret_cast<const double2 *>(arow + l0 * KS);
                        const double2 *r1 = reinterpret_cast<const double2 *>(arow + l1 * KS);
#pragma unroll
                        for (int h = 0; h < KS / 2; ++h) {
                            const double2 x0 = r0[h], x1 = r1[h];
                            bsum[2 * h] = fma(c1, x1.x, fma(c0, x0.x, bsum[2 * h]));
                            if (2 * h + 1 < K) bsum[2 * h + 1] = fma(c1, x1.y, fma(c0, x0.y, bsum[2 * h + 1]));
                        }
                    }
                    if constexpr (BK.cflag[g0 + g] != 0) {
                        if constexpr (DSF)
                            stage_c_points<N, tw>(acc, bsum, lin);
                        else
                            stage_c<N, tw>(acc, bsum, pack);
#pragma unroll
                        for (int q = 0; q < K; ++q) bsum[q] = 0.0;
                    }
                });
            }
            __syncthreads();
        });

        // coalesced stores through LDS: the tile holds all rows (n1, p1) of
        // a row band and the columns (m2, n2, p2) of a chunk of the band's
        // m2, so that every mirrored row segment (the band's NR values) is
        // written whole by one workgroup in one pass; one band after the other
        for (int band = 0; band < (two ? 2 : 1); ++band) {
            const int m1s = band ? m1b : m1a;
            const int mlo = (J == I) ? m1s : 0;  // first column slab of the band
            const int rowbase = comp_offset(PROB, N, I) + m1s * NN_I * NP_I;
            const bool mine = active && bandb == (band != 0);
            constexpr int NR = NN_I * NP_I;      // tile rows
            constexpr int CW = NN_J * NP_J;      // tile columns per m2
            constexpr int TB = SMEM > 0 ? SMEM : S::BUF;
            constexpr int CM = cmax(1, (TB / NR - 1) / CW);  // m2 per chunk
            static_assert(NR * ((CM * CW) | 1) <= TB, "store tile exceeds the LDS buffer");
            for (int ma = mlo; ma < NM_J; ma += CM) {
                const int mb = ma + CM < NM_J ? ma + CM : NM_J;
                const int W = (mb - ma) * CW;    // tile width
                // odd row stride: the transposed (mirror) reads below step two
                // rows per lane, which an odd stride spreads over distinct banks
                const int WS = W | 1;
                if (mine && m2 >= ma && m2 < mb) {
                    double *tl = smem + n1 * NP_I * WS + ((m2 - ma) * NN_J + n2) * NP_J;
#pragma unroll
                    for (int p1 = 0; p1 < NP_I; ++p1)
#pragma unroll
                        for (int p2 = 0; p2 < NP_J; ++p2) {
                            bad |= !isfinite(acc[p1][p2]);
                            tl[p1 * WS + p2] = acc[p1][p2];
                        }
                }
                __syncthreads();
                const int colj = comp_offset(PROB, N, J) + ma * CW;
                if constexpr (PACKED) {
                    // packed upper triangle: row rg holds columns cg >= rg at
                    // rg NDOF - rg (rg - 1) / 2 + (cg - rg); no mirror
                    const int dr = nthreads / W, dc = nthreads - dr * W;
                    int r = tid / W, c = tid - r * W;
                    while (r < NR) {
                        const int64_t rg = rowbase + r, cg = colj + c;
                        if (cg >= rg) store_out(obase + (rg * NDOF - rg * (rg - 1) / 2 + (cg - rg)), smem[r * WS + c]);
                        r += dr;
                        c += dc;
                        if (c >= W) {
                            c -= W;
                            ++r;
                        }
                    }
                    __syncthreads();
                    continue;
                }
                // mirrored rows start after the diagonal slab m2 == m1 of block (I,I)
                const int cmir = (J == I && ma == mlo) ? CW : 0;
                double *drow = obase + (int64_t)rowbase * NDOF + colj;
                const bool d16 = (NDOF % 2 == 0) && (W % 2 == 0) &&
                                 ((reinterpret_cast<uintptr_t>(drow) & 15u) == 0);
                // the element index x = tid + i*nthreads of an (r, c) grid of
                // width wd is walked incrementally: one division per thread
                // and phase instead of one per stored element
                if (d16) {
                    const int hw = W / 2, dr = nthreads / hw, dc = nthreads - dr * hw;
                    int r = tid / hw, h = tid - r * hw;
                    while (r < NR) {
                        const int c = 2 * h;
                        // two 8-byte LDS reads (rows are only 8-byte aligned)
                        store_out2(drow + (int64_t)r * NDOF + c, smem[r * WS + c], smem[r * WS + c + 1]);
                        r += dr;
                        h += dc;
                        if (h >= hw) {
                            h -= hw;
                            ++r;
                        }
                    }
                } else {
                    const int dr = nthreads / W, dc = nthreads - dr * W;
                    int r = tid / W, c = tid - r * W;
                    while (r < NR) {
                        store_out(drow + (int64_t)r * NDOF + c, smem[r * WS + c]);
                        r += dr;
                        c += dc;
                        if (c >= W) {
                            c -= W;
                            ++r;
                        }
                    }
                }
                // mirror: tile column c is output row colj + c, holding the NR
                // contiguous values of columns rowbase + r
                double *mrow = obase + (int64_t)colj * NDOF + rowbase;
                const int nc = W - cmir;
                const bool m16 = (NDOF % 2 == 0) && (NR % 2 == 0) &&
                                 ((reinterpret_cast<uintptr_t>(mrow) & 15u) == 0);
                if (m16) {
                    const int hr = NR / 2, dq = nthreads / hr, dh = nthreads - dq * hr;
                    int q = tid / hr, h = tid - q * hr;  // tile column cmir + q, row pair h
                    while (q < nc) {
                        const int c = cmir + q, r = 2 * h;
                        double *seg = mrow + (int64_t)c * NDOF;
                        if constexpr (MERGE)
                            store_mirror2(seg + r, smem[r * WS + c], smem[(r + 1) * WS + c], seg, seg + NR);
                        else
                            store_out2(seg + r, smem[r * WS + c], smem[(r + 1) * WS + c]);
                        q += dq;
                        h += dh;
                        if (h >= hr) {
                            h -= hr;
                            ++q;
                        }
                    }
                } else {
                    const int dq = nthreads / NR, dh = nthreads - dq * NR;
                    int q = tid / NR, r = tid - q * NR;
                    while (q < nc) {
                        const int c = cmir + q;
                        store_out(mrow + (int64_t)c * NDOF + r, smem[r * WS + c]);
                        q += dq;
                        r += dh;
                        if (r >= NR) {
                            r -= NR;
                            ++q;
                        }
                    }
                }
                __syncthreads();
            }
        }
    });
    if (__syncthreads_or(bad) && tid == 0) atomicOr(status + e, P2S_STATUS_NONFINITE_BIT);
}

// One launch per column block (I, J >= I), each kernel holding the code of
// a single block: the scalar problem, and the vector problem above order 6.
// The scalar problem's block is diagonal: up to order 7 its items are
// paired like those of the single-launch vector kernel (a whole pair fills
// NM + 1 slabs' worth of lanes where an unpaired item fills on average half
// of its workgroup; the scalar N = 6 contraction measured 23 % faster, the
// mixed-order batch 3 % more with order 7 paired too).  Order 8 stays
// unpaired: a pair needs 576 lanes, more than the unpaired workgroup's 512.
template <int PROB, int N, int I, int J, bool DSF>
struct BlockItems {
    static constexpr bool PAIR = PROB == 0 && N <= 7;
    using S = CS<PROB, N, I, J, J + 1, DSF, PAIR>;
    static constexpr int ITEMS = PAIR ? (S::NM_I + 1) / 2 : S::NM_I;
};

template <int PROB, int N, int I, int J, bool DSF = false, bool PACKED = false>
__global__ __launch_bounds__((BlockItems<PROB, N, I, J, DSF>::S::THREADS), (N <= 6 ? 3 : 2)) void k_contract(
    const ElemDesc *__restrict__ desc, const int32_t *__restrict__ elist, int64_t e0, int64_t nitems,
    int64_t padded, const double *__restrict__ tab, const double *__restrict__ mom,
    double *__restrict__ out, uint32_t *__restrict__ status, double sK, double sM)
{
    using B = BlockItems<PROB, N, I, J, DSF>;
    using S = typename B::S;
    const int64_t item = xcd_remap(blockIdx.x, padded);
    if (item >= nitems) return;
    const int64_t eidx = e0 + item / B::ITEMS;
    const int64_t e = elist ? (int64_t)elist[eidx] : eidx;
    const int m1 = (int)(item % B::ITEMS);
    const ElemDesc d = desc[e];
    __shared__ __attribute__((aligned(16))) double smem[S::BUF];
    contract_item<PROB, N, I, J, J + 1, DSF, PACKED, B::PAIR>(d, e, m1, tab, mom, out, status, sK, sM, smem,
                                                              S::THREADS);
}

template <int PROB, int N, int I, int J, bool DSF = false, bool PACKED = false>
static void launch_contract_i(const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                              const double *tab, const double *mom, double *out, uint32_t *status,
                              double sK, double sM, hipStream_t st)
{
    using B = BlockItems<PROB, N, I, J, DSF>;
    using S = typename B::S;
    const int64_t nitems = count * B::ITEMS;
    const int64_t padded = (nitems + 7) / 8 * 8;
    hipLaunchKernelGGL((k_contract<PROB, N, I, J, DSF, PACKED>), dim3((unsigned)padded), dim3(S::THREADS), 0, st, desc,
                       elist, e0, nitems, padded, tab, mom, out, status, sK, sM);
}

// All six blocks of the vector problem in one launch (orders up to 6), work
// items in element order: the items of an element (block by block, m1 by
// m1; 25 at N = 6) are consecutive, so after the remap below they run
// together on one XCD.  The element matrix's rows are 4320 bytes at N = 6 and the mirrored
// row segments 288 bytes, so about a quarter of the 128-byte lines of the
// output are written in pieces by two work items, and a fourteenth by two
// blocks.  Written by workgroups of one XCD at about the same time, the
// pieces merge in that XCD's L2 before the line goes to HBM; written by
// separate launches, they reach HBM as partial-line writes, at about half
// the rate of whole lines.  Each workgroup runs one block's body; the
// instruction footprint of six bodies costs less than those partial writes.
constexpr int kBlockI[6] = {0, 0, 0, 1, 1, 2};
constexpr int kBlockJ[6] = {0, 1, 2, 1, 2, 2};

// The diagonal blocks' items are paired (row bands m1 and NM - 1 - m1): an
// unpaired item of a diagonal block fills only the lanes of its triangle
// m2 >= m1, on average half of them, and its length varies with m1; a pair
// spans NM + 1 slabs whatever m1, close to an off-diagonal item's NM, and its
// two bands share the moment loads of stage A.  Items of about equal length
// finish, and store, at about the same time, which is what lets the L2 merge
// the pieces of the lines they share (MERGE).
template <int N, bool DSF>
struct VectorBlocks {
    template <int b>
    using S = CS<1, N, kBlockI[b], kBlockJ[b], kBlockJ[b] + 1, DSF, kBlockI[b] == kBlockJ[b]>;
    static constexpr int THREADS = cmax(cmax(cmax(S<0>::THREADS, S<1>::THREADS), cmax(S<2>::THREADS, S<3>::THREADS)),
                                        cmax(S<4>::THREADS, S<5>::THREADS));
    // at N = 6 the store tile takes all the LDS a workgroup gets when the CU
    // holds twelve waves (three per SIMD, what the registers allow): fewer,
    // longer chunks per row, so fewer row segments split between chunks
    // (52 KiB against the batches' 38 KiB measured 3 % faster).  The share
    // is rounded down to a multiple of 2560 bytes, less 512 bytes for the
    // kernel's other shared variables: at N = 6 a workgroup of 53,504 bytes
    // ran three to a CU, one of 53,840 bytes (a third of 160 KiB less 1 KiB)
    // measured 20 % slower, as with two, which fits LDS allocated in blocks
    // of 1280 or 2560 bytes.  Lower orders need fewer registers and may hold
    // more waves, which a larger tile would cap.
    static constexpr int WGS_PER_CU = cmax(1, 12 / (THREADS / 64));
    static constexpr int LDS_FIT = N == 6 ? ((160 * 1024 / WGS_PER_CU) / 2560 * 2560 - 512) / 8 : 0;
    static constexpr int BUF = cmax(
        LDS_FIT, cmax(cmax(cmax(S<0>::BUF, S<1>::BUF), cmax(S<2>::BUF, S<3>::BUF)), cmax(S<4>::BUF, S<5>::BUF)));
    // items of block b, first item of block b within an element, and items
    // per element
    static constexpr int items(int b)
    {
        const int nm = comp_dim(1, N, kBlockI[b], 0);
        return kBlockI[b] == kBlockJ[b] ? (nm + 1) / 2 : nm;
    }
    static constexpr int first(int b)
    {
        int o = 0;
        for (int x = 0; x < b; ++x) o += items(x);
        return o;
    }
    static constexpr int ITEMS = first(6);
};

template <int N, bool DSF = false, bool PACKED = false>
__global__ __launch_bounds__((VectorBlocks<N, DSF>::THREADS), 3) void k_contract_vector(
    const ElemDesc *__restrict__ desc, const int32_t *__restrict__ elist, int64_t e0, int64_t nitems,
    int64_t padded, const double *__restrict__ tab, const double *__restrict__ mom,
    double *__restrict__ out, uint32_t *__restrict__ status, double sK, double sM)
{
    using V = VectorBlocks<N, DSF>;
    const int64_t item = xcd_remap(blockIdx.x, padded);
    if (item >= nitems) return;
    const int64_t eidx = e0 + item / V::ITEMS;
    const int r = (int)(item % V::ITEMS);
    const int64_t e = elist ? (int64_t)elist[eidx] : eidx;
    const ElemDesc d = desc[e];
    __shared__ __attribute__((aligned(16))) double smem[V::BUF];
    static_for<0, 6>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int I = kBlockI[b], J = kBlockJ[b];
        constexpr int lo = V::first(b), n = V::items(b);
        if (r >= lo && r < lo + n)
            contract_item<1, N, I, J, J + 1, DSF, PACKED, I == J, true, V::BUF>(d, e, r - lo, tab, mom, out,
                                                                                status, sK, sM, smem, V::THREADS);
    });
}

// The blocks (I, J >= I) of one problem and order: the scalar problem's
// single block, the vector problem's six in one launch up to order 6 and
// one launch each above (from order 7 on a CU holds a single workgroup).
template <int PROB, int N, bool DSF = false, bool PACKED = false>
static void launch_contract_t(const ElemDesc *desc, const int32_t *elist, int64_t e0, int64_t count,
                              const double *tab, const double *mom, double *out, uint32_t *status,
                              double sK, double sM, hipStream_t st)
{
    if constexpr (PROB == 1 && N <= 6) {
        using V = VectorBlocks<N, DSF>;
        const int64_t nitems = count * V::ITEMS;
        const int64_t padded = (nitems + 7) / 8 * 8;
        hipLaunchKernelGGL((k_contract_vector<N, DSF, PACKED>), dim3((unsigned)padded), dim3(V::THREADS), 0, st,
                           desc, elist, e0, nitems, padded, tab, mom, out, status, sK, sM);
        return;
    }
    launch_contract_i<PROB, N, 0, 0, DSF, PACKED>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);
    if constexpr (PROB == 1) {
        launch_contract_i<PROB, N, 0, 1, DSF, PACKED>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);
        launch_contract_i<PROB, N, 0, 2, DSF, PACKED>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);
        launch_contract_i<PROB, N, 1, 1, DSF, PACKED>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);
        launch_contract_i<PROB, N, 1, 2, DSF, PACKED>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);
        launch_contract_i<PROB, N, 2, 2, DSF, PACKED>(desc, elist, e0, count, tab, mom, out, status, sK, sM, st);
    }
}

}  // namespace p2s
