// p2s_terms.h -- compile-time coupling-term structure of each component
// block (I,J) of the element matrix, eq. (2) expanded with eq. (3): which
// coupling field, sign and scale, and which 1-D basis-pair family per axis.
#pragma once

#include <type_traits>

#include "p2s_internal.h"

namespace p2s {

constexpr int MAX_TERMS = 10;  // scalar: 9 stiffness + 1 mass; vector: 5 per block

struct TermC {
    int field, sign, scale, tu, tv, tw;
};

struct BlockC {
    int nterm = 0, ngroup = 0;
    int gstart[MAX_TERMS + 1] = {};
    int cflag[MAX_TERMS] = {};
    TermC t[MAX_TERMS] = {};
};

constexpr int sym_c(int a, int b)
{
    return a == b ? a : ((a < b ? a : b) == 0 ? ((a > b ? a : b) == 1 ? 3 : 4) : 5);
}

constexpr int levi_c(int a, int b, int c)
{
    return (a == b || b == c || a == c) ? 0
         : (((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) ? 1 : -1);
}

// Coupling terms of block (i,j) of eq. (2), sorted by (tw, tv) and grouped.
// Scalar: 9 stiffness terms (a,b) with field eps detJ (J^-1 J^-T)_ab,
//   derivative on axis a (test) and b (trial), plus the mass term.
// Vector: E_i = f e_i, f = psi along axis i, phi elsewhere; the reference
//   curl (curl f e_i)_c = eps_{c e i} d_e f (e = 3-c-i) gives 4 curl terms
//   (c != i, d != j) with field (J^T J/detJ)_cd and sign eps_{cei} eps_{dfj},
//   plus the mass term with field (detJ J^-1 eps J^-T)_ij.
constexpr BlockC make_block_c(int prob, int i, int j)
{
    BlockC b{};
    TermC t[MAX_TERMS] = {};
    int n = 0;
    if (prob == 0) {
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                t[n].field = sym_c(a, c);
                t[n].sign = 1;
                t[n].scale = 0;
                t[n].tu = 3 * (a == 0 ? DPHI : PHI) + (c == 0 ? DPHI : PHI);
                t[n].tv = 3 * (a == 1 ? DPHI : PHI) + (c == 1 ? DPHI : PHI);
                t[n].tw = 3 * (a == 2 ? DPHI : PHI) + (c == 2 ? DPHI : PHI);
                ++n;
            }
        t[n].field = 6;
        t[n].sign = 1;
        t[n].scale = 1;
        t[n].tu = t[n].tv = t[n].tw = 3 * PHI + PHI;
        ++n;
    } else {
        for (int c = 0; c < 3; ++c) {
            if (c == i) continue;
            for (int d = 0; d < 3; ++d) {
                if (d == j) continue;
                const int e = 3 - c - i, f = 3 - d - j;
                int ty[3] = {0, 0, 0};
                for (int ax = 0; ax < 3; ++ax) {
                    const int X = ax == i ? PSI : (ax == e ? DPHI : PHI);
                    const int Y = ax == j ? PSI : (ax == f ? DPHI : PHI);
                    ty[ax] = 3 * X + Y;
                }
                t[n].field = sym_c(c, d);
                t[n].sign = levi_c(c, e, i) * levi_c(d, f, j);
                t[n].scale = 0;
                t[n].tu = ty[0];
                t[n].tv = ty[1];
                t[n].tw = ty[2];
                ++n;
            }
        }
        int ty[3] = {0, 0, 0};
        for (int ax = 0; ax < 3; ++ax) ty[ax] = 3 * (ax == i ? PSI : PHI) + (ax == j ? PSI : PHI);
        t[n].field = 6 + sym_c(i, j);
        t[n].sign = 1;
        t[n].scale = 1;
        t[n].tu = ty[0];
        t[n].tv = ty[1];
        t[n].tw = ty[2];
        ++n;
    }
    // stable insertion sort by (tw, tv)
    for (int a = 1; a < n; ++a) {
        TermC x = t[a];
        int p = a - 1;
        while (p >= 0 && (t[p].tw > x.tw || (t[p].tw == x.tw && t[p].tv > x.tv))) {
            t[p + 1] = t[p];
            --p;
        }
        t[p + 1] = x;
    }
    b.nterm = n;
    int g = 0;
    for (int s = 0; s < n; ++s) {
        b.t[s] = t[s];
        if (s == 0 || t[s].tw != t[s - 1].tw || t[s].tv != t[s - 1].tv) b.gstart[g++] = s;
    }
    b.gstart[g] = n;
    b.ngroup = g;
    for (int k = 0; k < g; ++k)
        b.cflag[k] = (k + 1 == g || t[b.gstart[k + 1]].tw != t[b.gstart[k]].tw) ? 1 : 0;
    return b;
}

template <int PROB, int I, int J>
struct BlockOf {
    static constexpr BlockC B = make_block_c(PROB, I, J);
};

// compile-time loop: f(integral_constant<int, i>) for i in [B, E)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

}  // namespace p2s
