// Spin projection in the chiral basis: (1 -/+ gamma_mu) has rank two, so a
// four-spinor p maps to a half spinor (h0, h1) and the two lower components
// of the result follow from h0, h1 by a sign or a factor of +/- i.
//   gamma_1 p = (-i p3, -i p2,  i p1,  i p0)
//   gamma_2 p = (  -p3,    p2,    p1,  -p0)
//   gamma_3 p = (-i p2,  i p3,  i p0, -i p1)
//   gamma_4 p = (   p2,    p3,    p0,    p1)
#pragma once

#include "ov_device.h"

namespace ov {

// Half-spinor projection of (1 + SGN gamma_MU) p; SGN = -1 for forward hops.
template <int MU, int SGN, class R>
__device__ __forceinline__ void project(const cx<R> (&p)[4][3], cx<R> (&h)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (MU == 0) {   // gamma_1 p = (-i p3, -i p2, i p1, i p0)
            if (SGN < 0) { h[0][c] = cadd(p[0][c], cimul(p[3][c])); h[1][c] = cadd(p[1][c], cimul(p[2][c])); }
            else         { h[0][c] = csub(p[0][c], cimul(p[3][c])); h[1][c] = csub(p[1][c], cimul(p[2][c])); }
        } else if (MU == 1) {   // gamma_2 p = (-p3, p2, p1, -p0)
            if (SGN < 0) { h[0][c] = cadd(p[0][c], p[3][c]); h[1][c] = csub(p[1][c], p[2][c]); }
            else         { h[0][c] = csub(p[0][c], p[3][c]); h[1][c] = cadd(p[1][c], p[2][c]); }
        } else if (MU == 2) {   // gamma_3 p = (-i p2, i p3, i p0, -i p1)
            if (SGN < 0) { h[0][c] = cadd(p[0][c], cimul(p[2][c])); h[1][c] = csub(p[1][c], cimul(p[3][c])); }
            else         { h[0][c] = csub(p[0][c], cimul(p[2][c])); h[1][c] = cadd(p[1][c], cimul(p[3][c])); }
        } else {                // gamma_4 p = (p2, p3, p0, p1)
            if (SGN < 0) { h[0][c] = csub(p[0][c], p[2][c]); h[1][c] = csub(p[1][c], p[3][c]); }
            else         { h[0][c] = cadd(p[0][c], p[2][c]); h[1][c] = cadd(p[1][c], p[3][c]); }
        }
    }
}

// acc += (1 + SGN gamma_MU) expansion of the multiplied half spinor g.
template <int MU, int SGN, class R>
__device__ __forceinline__ void expand_add(cx<R> (&acc)[4][3], const cx<R> (&g)[2][3])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[0][c] = cadd(acc[0][c], g[0][c]);
        acc[1][c] = cadd(acc[1][c], g[1][c]);
        if (MU == 0) {
            if (SGN < 0) { acc[2][c] = cadd(acc[2][c], cnimul(g[1][c])); acc[3][c] = cadd(acc[3][c], cnimul(g[0][c])); }
            else         { acc[2][c] = cadd(acc[2][c], cimul(g[1][c]));  acc[3][c] = cadd(acc[3][c], cimul(g[0][c])); }
        } else if (MU == 1) {
            if (SGN < 0) { acc[2][c] = csub(acc[2][c], g[1][c]); acc[3][c] = cadd(acc[3][c], g[0][c]); }
            else         { acc[2][c] = cadd(acc[2][c], g[1][c]); acc[3][c] = csub(acc[3][c], g[0][c]); }
        } else if (MU == 2) {
            if (SGN < 0) { acc[2][c] = cadd(acc[2][c], cnimul(g[0][c])); acc[3][c] = cadd(acc[3][c], cimul(g[1][c])); }
            else         { acc[2][c] = cadd(acc[2][c], cimul(g[0][c]));  acc[3][c] = cadd(acc[3][c], cnimul(g[1][c])); }
        } else {
            if (SGN < 0) { acc[2][c] = csub(acc[2][c], g[0][c]); acc[3][c] = csub(acc[3][c], g[1][c]); }
            else         { acc[2][c] = cadd(acc[2][c], g[0][c]); acc[3][c] = cadd(acc[3][c], g[1][c]); }
        }
    }
}

}  // namespace ov
