// p2s_split.hip -- split-FP32 form of the moment stage (eq. (4)) and of the
// contraction, on the FP32 matrix cores of gfx950 (v_mfma_f32_16x16x4f32),
// with results exact to about 2^-40 per product.
//
// Every 16x16x4 matrix step D += A B (A 16x4, B 4x16, FP64 operands) is
// taken on exact slices.  Per step, each row of A and each column of B is
// scaled by a power of two 2^e (e from the largest magnitude of its four
// values) into (-1, 1) and split into four signed integer slices of 10
// bits, x 2^-e = sum_p s_p 2^(-10 (p+1)), |s_0| <= 1024, |s_p| <= 512.  The
// slice products s_p t_q are integers below 2^20, and the ten products with
// p + q <= 3 are summed by level p + q on the FP32 matrix cores: a level
// holds at most 16 such products, below 2^24, so every FP32 sum is exact.
// The four level sums are then scaled back and added into FP64
// accumulators.  The dropped levels (p + q >= 4) and the last slice's
// rounding are below 2^-40 of the row and column scales.  The coupling
// samples, tables, intermediates between the GEMM steps and every sum stay
// FP64; only the products run on the FP32 matrix cores.  (Splitting each
// operand into just two FP32 parts, hi = fl32(x) and lo = fl32(x - hi),
// leaves the FP32 accumulation itself inexact: about 1e-7 relative.)
//
// MFMA 16x16x4 lane layout (wave64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; result register i of lane l is D[4(l/16)+i][l%16].
#include <hip/hip_runtime.h>

#include "p2s_internal.h"
#include "p2s_kernels.h"
#include "p2s_terms.h"

namespace p2s {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// x in (-1, 1): four signed 10-bit integer slices, x ~ sum_p s[p] 2^(-10 (p+1)).
__device__ __forceinline__ void slices4(double x, float (&s)[4])
{
    double t = x * 1024.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const double a = rint(t);
        s[p] = (float)a;
        t = (t - a) * 1024.0;
    }
}

// One exact 16x16x4 step: this lane supplies a = A[r16][k4] and
// b = B[k4][r16] (FP64) and receives acc[i] += D[4 k4 + i][r16].
__device__ __forceinline__ void exact_step(double a, double b, double (&acc)[4])
{
    const int k4 = (threadIdx.x & 63) >> 4;
    // row r16 of A and column r16 of B live in the lanes r16 + 16 j
    double ma = fabs(a), mb = fabs(b);
    ma = fmax(ma, __shfl_xor(ma, 16, 64));
    ma = fmax(ma, __shfl_xor(ma, 32, 64));
    mb = fmax(mb, __shfl_xor(mb, 16, 64));
    mb = fmax(mb, __shfl_xor(mb, 32, 64));
    int ea = 0, eb = 0;
    (void)frexp(ma, &ea);  // ma = m 2^ea, m in [1/2, 1) (ea = 0 for 0)
    (void)frexp(mb, &eb);
    float sa[4], sb[4];
    slices4(ldexp(a, -ea), sa);
    slices4(ldexp(b, -eb), sb);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    const f4 L0 = mfma(sa[0], sb[0], z);
    const f4 L1 = mfma(sa[1], sb[0], mfma(sa[0], sb[1], z));
    const f4 L2 = mfma(sa[2], sb[0], mfma(sa[1], sb[1], mfma(sa[0], sb[2], z)));
    const f4 L3 = mfma(sa[3], sb[0], mfma(sa[2], sb[1], mfma(sa[1], sb[2], mfma(sa[0], sb[3], z))));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int er = __shfl(ea, 4 * k4 + i, 64);  // exponent of result row 4 k4 + i
        const double lv = ((double)L0[i] + ldexp((double)L1[i], -10)) +
                          (ldexp((double)L2[i], -20) + ldexp((double)L3[i], -30));
        acc[i] += ldexp(lv, er + eb - 20);
    }
}

// The same product on the INT8 matrix cores (v_mfma_i32_16x16x32_i8) for a
// whole K-block of 16: this lane holds a[j] = A[r16][4j + k4] and
// b[j] = B[4j + k4][r16], j = 0..3.  Rows of A and columns of B take one
// power-of-two scale over the block and six signed 7-bit slices,
// x 2^-e = 2^-6 sum_p s_p 2^(-7p), |s_p| <= 64.  Level l = p + q collects
// the products s_p t_q; one 16x16x32 instruction holds two slice pairs
// (p, q) for the 16 values of k (each lane supplies its own four k for both
// pairs, so no operand crosses lanes), and its int32 sum of at most 32
// products below 2^12 is exact.  Levels 0..5 take 12 instructions; the
// dropped levels are below 2^-42 of the row and column scales.
typedef int i4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ i4 mfma_i8(long a, long b, i4 c)
{
    return __builtin_amdgcn_mfma_i32_16x16x32_i8(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void slices6(double x, int (&s)[6])
{
    double t = x * 64.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const double a = rint(t);
        s[p] = (int)a;
        t = (t - a) * 128.0;
    }
}

__device__ __forceinline__ long pack8(int b0, int b1, int b2, int b3, int b4, int b5, int b6, int b7)
{
    const unsigned lo = (unsigned)(b0 & 255) | ((unsigned)(b1 & 255) << 8) | ((unsigned)(b2 & 255) << 16) |
                        ((unsigned)(b3 & 255) << 24);
    const unsigned hi = (unsigned)(b4 & 255) | ((unsigned)(b5 & 255) << 8) | ((unsigned)(b6 & 255) << 16) |
                        ((unsigned)(b7 & 255) << 24);
    return (long)(((unsigned long)hi << 32) | lo);
}

__device__ __forceinline__ void exact_block_i8(const double (&a)[4], const double (&b)[4], double (&acc)[4])
{
    const int k4 = (threadIdx.x & 63) >> 4;
    double ma = fmax(fmax(fabs(a[0]), fabs(a[1])), fmax(fabs(a[2]), fabs(a[3])));
    double mb = fmax(fmax(fabs(b[0]), fabs(b[1])), fmax(fabs(b[2]), fabs(b[3])));
    ma = fmax(ma, __shfl_xor(ma, 16, 64));
    ma = fmax(ma, __shfl_xor(ma, 32, 64));
    mb = fmax(mb, __shfl_xor(mb, 16, 64));
    mb = fmax(mb, __shfl_xor(mb, 32, 64));
    int ea = 0, eb = 0;
    (void)frexp(ma, &ea);
    (void)frexp(mb, &eb);
    int sa[4][6], sb[4][6];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        slices6(ldexp(a[j], -ea), sa[j]);
        slices6(ldexp(b[j], -eb), sb[j]);
    }
    int er[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) er[i] = __shfl(ea, 4 * k4 + i, 64);  // exponent of result row 4 k4 + i
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        i4 c = {0, 0, 0, 0};
#pragma unroll
        for (int p = 0; p <= l; p += 2) {
            // bytes 0..3: pair (p, l-p); bytes 4..7: pair (p+1, l-p-1) (zero past l)
            const bool two = p + 1 <= l;
            const long pa = pack8(sa[0][p], sa[1][p], sa[2][p], sa[3][p], two ? sa[0][p + 1] : 0,
                                  two ? sa[1][p + 1] : 0, two ? sa[2][p + 1] : 0, two ? sa[3][p + 1] : 0);
            const long pb = pack8(sb[0][l - p], sb[1][l - p], sb[2][l - p], sb[3][l - p], two ? sb[0][l - p - 1] : 0,
                                  two ? sb[1][l - p - 1] : 0, two ? sb[2][l - p - 1] : 0,
                                  two ? sb[3][l - p - 1] : 0);
            c = mfma_i8(pa, pb, c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += ldexp((double)c[i], er[i] + eb - 12 - 7 * l);
    }
}

// One K-block of 16 of D += A B: a[j] = A[r16][4j + k4], b[j] = B[4j + k4][r16].
template <bool I8>
__device__ __forceinline__ void exact_block(const double (&a)[4], const double (&b)[4], double (&acc)[4])
{
    if constexpr (I8) {
        exact_block_i8(a, b, acc);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) exact_step(a[j], b[j], acc);
    }
}

// ---------------------------------------------------------------------------
// Moments: one workgroup (4 waves) per (element, field); Q <= 16 per axis,
// K = 2N-1 <= 15.  Three GEMM passes, each one K-block of 16 (four steps):
//   P1[ab][q] = sum_c alpha[ab][c] Ww[q][c]
//   P2[a][l][q] = sum_b Wv[l][b] P1[ab][q]
//   I[k][l][q] = sum_a Wu[k][a] P2[a][l][q]
// with W[k][a] = w_a L_k(x_a); FP64 intermediates in LDS, FP64 output.

constexpr int PS = 17;  // LDS row stride of the pass results (doubles)
constexpr size_t MOMENTS_SPLIT_LDS = sizeof(double) * 2 * 256 * PS;

template <bool I8>
__global__ __launch_bounds__(256) void k_moments_split(const ElemDesc *__restrict__ desc, int64_t e0,
                                                       const double *__restrict__ alpha,
                                                       const double *__restrict__ tab, double *__restrict__ mom)
{
    extern __shared__ double sms[];
    double *P1 = sms, *P2 = sms + 256 * PS;
    const int64_t e = e0 + blockIdx.x;
    const int f = blockIdx.y;
    const ElemDesc d = desc[e];
    const int Qu = d.Qu, Qv = d.Qv, Qw = d.Qw, K = 2 * d.N - 1;
    const int P = Qu * Qv * Qw;
    const double *A = alpha + d.alpha_off + (int64_t)f * P;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    // W[k][a] rows k < 16 (Legendre weights), zero for a >= Q
    const double *Wu = tab + TAB_LEGW + Qu * LEGW_STRIDE_Q, *Wv = tab + TAB_LEGW + Qv * LEGW_STRIDE_Q,
                 *Ww = tab + TAB_LEGW + Qw * LEGW_STRIDE_Q;

    // pass 1: M = ab (Qu*Qv <= 256 rows), K = c, N = q
    const int nab = Qu * Qv;
    for (int mt = wave; mt < 16; mt += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int ab = mt * 16 + r16;
        double xa[4], xb[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int cc = ks * 4 + k4;
            xa[ks] = (ab < nab && cc < Qw) ? A[(int64_t)ab * Qw + cc] : 0.0;
            xb[ks] = Ww[r16 * MAXQ + cc];
        }
        exact_block<I8>(xa, xb, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) P1[(mt * 16 + 4 * k4 + i) * PS + r16] = acc[i];
    }
    __syncthreads();
    // pass 2: per a, M = l, K = b, N = q
    for (int a = wave; a < Qu; a += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        double xa[4], xb[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int b = ks * 4 + k4;
            xa[ks] = Wv[r16 * MAXQ + b];
            xb[ks] = b < Qv ? P1[(a * Qv + b) * PS + r16] : 0.0;
        }
        exact_block<I8>(xa, xb, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) P2[(a * 16 + 4 * k4 + i) * PS + r16] = acc[i];
    }
    __syncthreads();
    // pass 3: M = k, K = a, N = (l,q) in 16 tiles of 16 (tile nt has l = nt)
    double *I = mom + d.mom_off + (int64_t)f * K * K * K;
    for (int nt = wave; nt < 16; nt += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        double xa[4], xb[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int a = ks * 4 + k4;
            xa[ks] = Wu[r16 * MAXQ + a];
            xb[ks] = a < Qu ? P2[(a * 16 + nt) * PS + r16] : 0.0;
        }
        exact_block<I8>(xa, xb, acc);
        const int l = nt, q = r16;
        if (l < K && q < K)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 4 * k4 + i;
                if (k < K) I[(k * K + l) * K + q] = acc[i];
            }
    }
}

// ---------------------------------------------------------------------------
// Contraction: one workgroup (4 waves) per (element, row component I, m1)
// for the block (I,J); all per-axis index ranges are padded to 8 (MAXN),
// so (n1,n2) and (p1,p2) are 64-wide.  The block's terms come grouped by
// (v,w) family pair, runs of groups share the w pair (p2s_terms.h).
//   stage A  Ag[m2][l][q] = sum_{s in g} sc_s sum_k Cu_s[m1][m2][k] I_s[k][l][q]
//            M = m2 (16, 8 used), K = k, N = (l,q) 256; once per m1
//   stage B  Bsum[n1n2][q] = sum_{g in run} sum_l Cv_g[n1n2][l] Ag[m2][l][q]
//            M = n1n2 (wave w owns rows 16w..16w+15), K = l, N = q
//   stage C  acc[n1n2][p1p2] += sum_q Bsum[n1n2][q] Cw_run[p1p2][q]
//            M = n1n2, K = q, N = p1p2 (4 tiles)
// Every step is exact_step; Ag, Bsum and acc are FP64.  Blocks of at most
// five groups (the vector problem) stage each m2's tile through LDS for
// row-wise stores; the scalar problem (nine groups) needs that LDS for Ag
// and stores straight from the accumulators.

constexpr int SPLIT_TILE_STRIDE = 65;  // doubles per LDS tile row
constexpr int SPLIT_TILED_MAXG = 5;

template <int NG>
constexpr size_t contract_split_lds()
{
    return sizeof(double) * ((size_t)NG * 8 * 256 + 4 * 16 * PS +
                             (NG <= SPLIT_TILED_MAXG ? 64 * SPLIT_TILE_STRIDE : 0));
}

template <int PROB, int I, int J, bool I8>
__global__ __launch_bounds__(256) void k_contract_split(const ElemDesc *__restrict__ desc, int64_t e0, int64_t count,
                                                        int64_t total_padded, const double *__restrict__ tab,
                                                        const double *__restrict__ mom, double *__restrict__ out,
                                                        uint32_t *__restrict__ status, double sK, double sM)
{
    constexpr BlockC BK = BlockOf<PROB, I, J>::B;
    constexpr int NG = BK.ngroup;
    constexpr bool TILED = NG <= SPLIT_TILED_MAXG;
    extern __shared__ double smc[];
    double *Ag = smc;                       // [NG][8][256]
    double *Bt = Ag + NG * 8 * 256;         // [4][16][PS]
    double *tile = Bt + 4 * 16 * PS;        // [64][SPLIT_TILE_STRIDE] (TILED)

    // work item: consecutive items (the m1 rows of one element) on one XCD
    const int64_t w = blockIdx.x;
    const int64_t per = total_padded >> 3;
    const int64_t item = (w & 7) * per + (w >> 3);
    const ElemDesc d0 = desc[e0];
    const int N = d0.N;
    const int NM_I = comp_dim(PROB, N, I, 0), NN_I = comp_dim(PROB, N, I, 1), NP_I = comp_dim(PROB, N, I, 2);
    const int NM_J = comp_dim(PROB, N, J, 0), NN_J = comp_dim(PROB, N, J, 1), NP_J = comp_dim(PROB, N, J, 2);
    if (item >= count * NM_I) return;
    const int64_t e = e0 + item / NM_I;
    const int m1 = (int)(item % NM_I);
    const ElemDesc d = desc[e];
    const int K = 2 * N - 1, NDOF = num_dofs(PROB, N);
    const double *Im = mom + d.mom_off;
    double *obase = out + d.out_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const double *LIN = tab + TAB_LIN;

    // stage A
    static_for<0, NG>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        for (int nt = wave; nt < 16; nt += 4) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            static_for<BK.gstart[g], BK.gstart[g + 1]>([&](auto sc_) {
                constexpr TermC t = BK.t[decltype(sc_)::value];
                const double sc = (t.scale ? sM : sK) * (double)t.sign;
                const double *Is = Im + (int64_t)t.field * K * K * K;
                double xa[4], xb[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k = ks * 4 + k4;
                    const int m2 = r16 < MAXN ? r16 : MAXN - 1;  // rows 8..15 are padding
                    xa[ks] = r16 < MAXN ? sc * LIN[t.tu * LIN_STRIDE_T + m1 * LIN_STRIDE_M1 + m2 * KPAD + k] : 0.0;
                    xb[ks] = (k < K && nt < K && r16 < K) ? Is[(k * K + nt) * K + r16] : 0.0;
                }
                exact_block<I8>(xa, xb, acc);
            });
            if (k4 < 2)
#pragma unroll
                for (int i = 0; i < 4; ++i) Ag[(g * 8 + 4 * k4 + i) * 256 + nt * 16 + r16] = acc[i];
        }
    });
    __syncthreads();

    const int m2lo = (J == I) ? m1 : 0;
    const int rowbase = comp_offset(PROB, N, I) + m1 * NN_I * NP_I;
    bool bad = false;
    // stage B/C rows of this wave: n1n2 = 16 wave + r16 (A operand of B)
    const int bn1 = (16 * wave + r16) >> 3, bn2 = (16 * wave + r16) & 7;
    for (int m2 = m2lo; m2 < NM_J; ++m2) {
        double acc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0;
        double cb[4] = {0.0, 0.0, 0.0, 0.0};
        static_for<0, NG>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            constexpr int tv = BK.t[BK.gstart[g]].tv;
            constexpr int tw = BK.t[BK.gstart[g]].tw;
            // stage B for group g, accumulated over the run
            {
                double xa[4], xb[4];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int l = ks * 4 + k4;
                    xa[ks] = LIN[tv * LIN_STRIDE_T + bn1 * LIN_STRIDE_M1 + bn2 * KPAD + l];
                    xb[ks] = Ag[(g * 8 + m2) * 256 + l * 16 + r16];
                }
                exact_block<I8>(xa, xb, cb);
            }
            if constexpr (BK.cflag[g] != 0) {
                // transpose the wave's Bsum tile for use as the A operand
                double *bt = Bt + wave * 16 * PS;
#pragma unroll
                for (int i = 0; i < 4; ++i) bt[(4 * k4 + i) * PS + r16] = cb[i];
                __syncthreads();
                // stage C for this run, 4 column tiles of (p1,p2)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int pp = nt * 16 + r16;
                    const int p1 = pp >> 3, p2 = pp & 7;
                    double cc[4] = {0.0, 0.0, 0.0, 0.0};
                    double xa[4], xb[4];
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int q = ks * 4 + k4;
                        xa[ks] = bt[r16 * PS + q];
                        xb[ks] = LIN[tw * LIN_STRIDE_T + p1 * LIN_STRIDE_M1 + p2 * KPAD + q];
                    }
                    exact_block<I8>(xa, xb, cc);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[nt * 4 + i] += cc[i];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < 4; ++i) cb[i] = 0.0;
            }
        });
        const int colbase = comp_offset(PROB, N, J) + m2 * NN_J * NP_J;
        if constexpr (TILED) {
            // tile[n1n2][p1p2] in FP64
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    tile[(16 * wave + 4 * k4 + i) * SPLIT_TILE_STRIDE + nt * 16 + r16] = acc[nt * 4 + i];
            __syncthreads();
            // rows (n1,p1) of m1 against columns (n2,p2) of m2.  Threads take a
            // padded 8x8 grid: the low six bits of the thread id give the
            // contiguous pair of a row, the high bits the row (four per pass).
            const int t = threadIdx.x & 63, ta = t >> 3, tb = t & 7;  // (n2,p2) / (n1,p1) of the thread
            for (int rr = threadIdx.x >> 6; rr < 64; rr += blockDim.x >> 6) {
                const int ra = rr >> 3, rb = rr & 7;                  // (n1,p1) / (n2,p2) of the row
                if (ra < NN_I && rb < NP_I && ta < NN_J && tb < NP_J) {
                    const double v = tile[(ra * 8 + ta) * SPLIT_TILE_STRIDE + rb * 8 + tb];
                    bad |= !isfinite(v);
                    obase[(int64_t)(rowbase + ra * NP_I + rb) * NDOF + colbase + ta * NP_J + tb] = v;
                }
                if ((J != I || m2 != m1) && ra < NN_J && rb < NP_J && ta < NN_I && tb < NP_I)
                    obase[(int64_t)(colbase + ra * NP_J + rb) * NDOF + rowbase + ta * NP_I + tb] =
                        tile[(ta * 8 + ra) * SPLIT_TILE_STRIDE + tb * 8 + rb];
            }
            __syncthreads();
        } else {
            // straight from the accumulators: lane holds (n1,n2) rows 4 k4 + i
            // of its wave's 16 and (p1,p2) = 16 nt + r16
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int nn = 16 * wave + 4 * k4 + i, pp = nt * 16 + r16;
                    const int n1 = nn >> 3, n2 = nn & 7, p1 = pp >> 3, p2 = pp & 7;
                    if (n1 < NN_I && n2 < NN_J && p1 < NP_I && p2 < NP_J) {
                        const double v = acc[nt * 4 + i];
                        bad |= !isfinite(v);
                        const int r = rowbase + n1 * NP_I + p1, c = colbase + n2 * NP_J + p2;
                        obase[(int64_t)r * NDOF + c] = v;
                        if (J != I || m2 != m1) obase[(int64_t)c * NDOF + r] = v;
                    }
                }
        }
    }
    bad = __syncthreads_or(bad);
    if (bad && threadIdx.x == 0) atomicOr(status + e, P2S_STATUS_NONFINITE_BIT);
}

// ---------------------------------------------------------------------------

void launch_moments_split(int problem, const ElemDesc *desc, int64_t e0, int64_t count, const double *alpha,
                          const double *tab, double *mom, bool int8, hipStream_t st)
{
    if (count <= 0) return;
    if (int8)
        hipLaunchKernelGGL(k_moments_split<true>, dim3((unsigned)count, num_fields(problem)), dim3(256),
                           MOMENTS_SPLIT_LDS, st, desc, e0, alpha, tab, mom);
    else
        hipLaunchKernelGGL(k_moments_split<false>, dim3((unsigned)count, num_fields(problem)), dim3(256),
                           MOMENTS_SPLIT_LDS, st, desc, e0, alpha, tab, mom);
}

template <int PROB, int I, int J, bool I8>
static void launch_block(int N, const ElemDesc *desc, int64_t e0, int64_t count, const double *tab,
                         const double *mom, double *out, uint32_t *status, double sK, double sM, hipStream_t st)
{
    const int64_t items = count * comp_dim(PROB, N, I, 0);
    const int64_t padded = (items + 7) & ~int64_t(7);
    constexpr size_t lds = contract_split_lds<BlockOf<PROB, I, J>::B.ngroup>();
    hipLaunchKernelGGL((k_contract_split<PROB, I, J, I8>), dim3((unsigned)padded), dim3(256), lds, st, desc, e0,
                       count, padded, tab, mom, out, status, sK, sM);
}

template <bool I8>
static void launch_split_blocks(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count,
                                const double *tab, const double *mom, double *out, uint32_t *status, double sK,
                                double sM, hipStream_t st)
{
    if (problem == 0) {
        launch_block<0, 0, 0, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
        return;
    }
    launch_block<1, 0, 0, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
    launch_block<1, 0, 1, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
    launch_block<1, 0, 2, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
    launch_block<1, 1, 1, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
    launch_block<1, 1, 2, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
    launch_block<1, 2, 2, I8>(N, desc, e0, count, tab, mom, out, status, sK, sM, st);
}

void launch_contract_split(int problem, int N, const ElemDesc *desc, int64_t e0, int64_t count, const double *tab,
                           const double *mom, double *out, uint32_t *status, double sK, double sM, bool int8,
                           hipStream_t st)
{
    if (count <= 0) return;
    if (int8)
        launch_split_blocks<true>(problem, N, desc, e0, count, tab, mom, out, status, sK, sM, st);
    else
        launch_split_blocks<false>(problem, N, desc, e0, count, tab, mom, out, status, sK, sM, st);
}

template <int PROB, int I, int J, bool I8>
static int allow_lds()
{
    constexpr size_t lds = contract_split_lds<BlockOf<PROB, I, J>::B.ngroup>();
    static_assert(lds <= 160 * 1024, "split contraction exceeds the LDS of a CU");
    return hipFuncSetAttribute((const void *)k_contract_split<PROB, I, J, I8>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess ? 0 : -1;
}

template <bool I8>
static int allow_all()
{
    int r = hipFuncSetAttribute((const void *)k_moments_split<I8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)MOMENTS_SPLIT_LDS) == hipSuccess ? 0 : -1;
    r |= allow_lds<0, 0, 0, I8>();
    r |= allow_lds<1, 0, 0, I8>();
    r |= allow_lds<1, 0, 1, I8>();
    r |= allow_lds<1, 0, 2, I8>();
    r |= allow_lds<1, 1, 1, I8>();
    r |= allow_lds<1, 1, 2, I8>();
    r |= allow_lds<1, 2, 2, I8>();
    return r;
}

int prepare_split_kernels() { return allow_all<false>() | allow_all<true>(); }

}  // namespace p2s
