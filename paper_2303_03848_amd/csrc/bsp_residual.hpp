// Pieces of the PINN loss gradient (eqs. (11)-(14)) shared by the
// multi-launch float32 pass and the fused bfloat16 step: parameter layout,
// the three point sets, the derivative streams rebuilt from a layer cache,
// the first layer and the head (output layer, loss terms, output adjoints).
#pragma once

#include "bsp_common.hpp"
#include "bsp_net.hpp"

namespace bsp {

// Offsets of the parameters in the flat float32 vector (torch nn.Linear
// order: W1[w][n_in], b1[w], W2[w][w], b2[w], ..., wo[w], bo).
struct NetLayout {
    int n_in, depth, W;
    long offW[17], offb[17];  // layer l = 1..depth
    long off_wo, off_bo, total;
};

inline NetLayout net_layout(const pinn_net& n) {
    NetLayout L{};
    L.n_in = n.n_in;
    L.depth = n.depth;
    L.W = n.width;
    long o = 0;
    int fan = n.n_in;
    for (int l = 1; l <= n.depth; ++l) {
        L.offW[l] = o;
        o += (long)n.width * fan;
        L.offb[l] = o;
        o += n.width;
        fan = n.width;
    }
    L.off_wo = o;
    o += n.width;
    L.off_bo = o;
    o += 1;
    L.total = o;
    return L;
}

// The interior (f), terminal (e) and boundary (b) points, in that order.
struct Points {
    const float *Xf, *Xe, *Xb;
    int nf, ne, nb, n_in;
    float sigma, r;   // used when n_in == 2
    int is_put;
    const float *ye, *yb;  // value targets of the terminal / boundary sets, or null
};

__device__ __forceinline__ const float* point_row(const Points& P, long i) {
    if (i < P.nf) return P.Xf + i * P.n_in;
    if (i < P.nf + P.ne) return P.Xe + (i - P.nf) * P.n_in;
    return P.Xb + (i - P.nf - P.ne) * P.n_in;
}

// Input streams of the layer after `c` (cache of the previous layer).
__device__ __forceinline__ void streams_from_cache(const float* c, long plane, long idx,
                                                   float& a, float& at, float& ax, float& axx) {
    const float av = c[idx], zt = c[plane + idx], zx = c[2 * plane + idx],
                zxx = c[3 * plane + idx];
    const float s = 1.0f - av * av;
    a = av;
    at = s * zt;
    ax = s * zx;
    axx = s * zxx - 2.0f * av * s * zx * zx;
}

// The same from the four cache values of one (point, unit).
__device__ __forceinline__ void streams_of_values(float av, float zt, float zx, float zxx,
                                                  float& a, float& at, float& ax, float& axx) {
    const float s = 1.0f - av * av;
    a = av;
    at = s * zt;
    ax = s * zx;
    axx = s * zxx - 2.0f * av * s * zx * zx;
}

// Adjoints of z and its derivative streams through a = tanh(z), given the
// adjoints (A, At, Ax, Axx) of (a, a_t, a_x, a_xx) and the cache values.
__device__ __forceinline__ void tanh_adjoint(float A, float At, float Ax, float Axx, float a,
                                             float zt, float zx, float zxx, float& zb,
                                             float& zb_t, float& zb_x, float& zb_xx) {
    const float s = 1.0f - a * a;
    zb_t = s * At;
    zb_x = s * Ax - 4.0f * a * s * zx * Axx;
    zb_xx = s * Axx;
    zb = s * (A - 2.0f * a * (zt * At + zx * Ax + zxx * Axx) -
              2.0f * zx * zx * (1.0f - 3.0f * a * a) * Axx);
}

// Head of one point i < n with inputs x and value target y (used by terminal
// and boundary points when the caller gives targets): given v (bias
// included) and its derivative streams, the output adjoints g0..g3 of
// (v, v_t, v_x, v_xx) and the point's squared loss term lc.
__device__ __forceinline__ void head_point_x(const Points& P, long i, const float* x, float ytgt,
                                             float v, float vt, float vx, float vxx, float& g0,
                                             float& g1, float& g2, float& g3, float& lc) {
    const float sig = P.n_in == 4 ? x[2] : P.sigma;
    const float rr = P.n_in == 4 ? x[3] : P.r;
    g0 = g1 = g2 = g3 = 0.f;
    if (i < P.nf) {
        const float xx = x[1];
        const float f = vt - 0.5f * sig * sig * xx * xx * vxx - rr * xx * vx + rr * v;
        lc = f * f;
        const float df = 2.0f * f / (float)P.nf;
        g0 = rr * df;
        g1 = df;
        g2 = -rr * xx * df;
        g3 = -0.5f * sig * sig * xx * xx * df;
    } else if (i < P.nf + P.ne) {
        const float xx = x[1];
        const float y = P.ye ? ytgt
                             : (P.is_put ? fmaxf(1.0f - xx, 0.0f) : fmaxf(xx - 1.0f, 0.0f));
        lc = (v - y) * (v - y);
        g0 = 2.0f * (v - y) / (float)P.ne;
    } else {
        const float tau = x[0], xx = x[1];
        const float disc = expf(-rr * tau);
        const bool lower = xx == 0.0f;
        const float y = P.yb ? ytgt
                             : (P.is_put ? (lower ? disc : 0.0f) : (lower ? 0.0f : xx - disc));
        lc = (v - y) * (v - y);
        g0 = 2.0f * (v - y) / (float)P.nb;
    }
}

// The value target of point i (its terminal or boundary target when given, else 0).
__device__ __forceinline__ float point_target(const Points& P, long i) {
    if (i >= P.nf && i < P.nf + P.ne) return P.ye ? P.ye[i - P.nf] : 0.f;
    if (i >= P.nf + P.ne) return P.yb ? P.yb[i - P.nf - P.ne] : 0.f;
    return 0.f;
}

__device__ __forceinline__ void head_point(const Points& P, long i, float v, float vt, float vx,
                                           float vxx, float& g0, float& g1, float& g2,
                                           float& g3, float& lc) {
    head_point_x(P, i, point_row(P, i), point_target(P, i), v, vt, vx, vxx, g0, g1, g2, g3, lc);
}

}  // namespace bsp
