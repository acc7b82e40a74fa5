// Block-level solver for the tridiagonal systems of the theta-method
//   (I - theta dt L) V^{m+1} = (I + (1 - theta) dt L) V^m + boundary terms,
// one system per thread block, the state kept in registers for all steps.
//
// The matrix is the same at every step (the coefficients of the
// Black-Scholes operator do not depend on time), so everything but the
// right-hand side is factored once in `setup`.
//
// Partition: thread p owns the MC consecutive unknowns i0 = p*MC .. i0+MC-1.
// Its last unknown z_p is an interface unknown; the MC-1 interior unknowns
// depend on the two neighbouring interface unknowns only:
//     x_int = y + z_{p-1} v + z_p w,
// where y solves the interior block with the actual right-hand side and v, w
// are its (constant) responses to unit coupling at the two ends.  Substituting
// into the interface rows gives a tridiagonal system of T unknowns
//     A_p z_{p-1} + B_p z_p + C_p z_{p+1} = D_p,
// solved by parallel cyclic reduction (PCR).  The reduction multipliers are
// constant and kept per thread.
//
// Truncated PCR: the interface system is strictly diagonally dominant and each
// PCR stage squares the relative size of the off-diagonal couplings
// (|A'|/|B'| ~ (|A|/|B|)^2).  Setup runs stages until every remaining coupling
// is below 2^-60 of its diagonal and records that stage count; the steps then
// run only those stages.  The neglected terms are below the rounding error of
// the result, so the solve stays exact to working precision.
//
// Interior rows use a scaled LU: with pivots u_q, the forward sweep works on
// d_q / u_q (the right-hand-side coefficients are pre-divided by u_q), so one
// step costs per node 3 operations for the right-hand side, 1 forward, 1
// backward and 2 for the interface correction.
//
// Exchanges between threads: with T = 64 the block is one wavefront; unit
// shifts use DPP lane moves and longer strides ds_bpermute, with no LDS and no
// barrier.  With T > 64 exchanges go through LDS with block barriers.
// Nodes beyond M are padding rows of the identity, decoupled from the rest.
#pragma once

#include "bsp_common.hpp"

namespace bsp {

// Value of `v` held by lane `src` of this wavefront (src taken modulo 64).
__device__ __forceinline__ double lane_fetch(double v, int src) {
    const int addr = src << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// DPP wavefront shifts by one lane: lane i receives lane i-1 (from_prev) or
// lane i+1 (from_next); the lane without a source receives 0.
__device__ __forceinline__ double dpp_from_prev(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_from_next(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

constexpr double kPcrTruncation = 8.673617379884035e-19;  // 2^-60

template <int T, int MC>
struct BlockTri {
    static_assert(MC >= 2, "at least one interior row per chunk");
    static constexpr int LOGT = ilog2(T);
    static constexpr int NI = MC - 1;
    static constexpr bool WAVE = (T == 64);

    double ea[MC], eb[MC], ec[MC];  // explicit part (I + (1-theta) dt L), interior rows / u_q
    double m[NI], cu[NI];           // scaled interior LU: a_q/u_q, c_q/u_q
    double v[NI], w[NI];            // interior responses to z_{p-1}, z_p
    double aq, cq;                  // interface row: implicit sub/super diagonal
    double vF, wF;                  // v[0], w[0] of the next chunk
    double k1[LOGT > 0 ? LOGT : 1], k2[LOGT > 0 ? LOGT : 1], invB;
    double blo, bhi;                // boundary-forcing coefficients (scaled like their row)
    int p, r_hi, nst;
    bool own_lo, own_hi;

    // --- exchanges: value held by thread p - s (up) / p + s (down), 0 outside [0, T)
    __device__ __forceinline__ double wave_up(double x, int s) const {
        if (s == 1) return dpp_from_prev(x);
        const double y = lane_fetch(x, p - s);
        return (p - s >= 0) ? y : 0.0;
    }
    __device__ __forceinline__ double wave_down(double x, int s) const {
        if (s == 1) return dpp_from_next(x);
        const double y = lane_fetch(x, p + s);
        return (p + s < T) ? y : 0.0;
    }

    // Forward/backward sweep of the scaled interior LU on a right-hand side
    // already divided by the pivots.
    __device__ __forceinline__ void interior_solve(double (&t)[MC]) const {
#pragma unroll
        for (int q = 1; q < NI; ++q) t[q] = fma(-m[q], t[q - 1], t[q]);
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) t[q] = fma(-cu[q], t[q + 1], t[q]);
    }

    // h = theta*dt (implicit weight), e = (1-theta)*dt (explicit weight).
    // lds: at least 3*T doubles (unused when T == 64).  Contains block barriers.
    __device__ void setup(double s2, double r, double h, double e, int M, double* lds) {
        p = threadIdx.x;
        const int i0 = p * MC;
        double a[MC], b[MC], c[MC];
#pragma unroll
        for (int q = 0; q < MC; ++q) {
            const int g = i0 + q;
            double al, be, ga;
            op_row(s2, r, (double)(g + 1), al, be, ga);
            const bool pad = g >= M;
            a[q] = (pad || g == 0) ? 0.0 : -h * al;
            b[q] = pad ? 1.0 : 1.0 - h * be;
            c[q] = (g >= M - 1) ? 0.0 : -h * ga;
            ea[q] = (pad || g == 0) ? 0.0 : e * al;
            eb[q] = pad ? 0.0 : 1.0 + e * be;
            ec[q] = (g >= M - 1) ? 0.0 : e * ga;
        }
        double bnd_lo, bnd_hi;
        {
            double al, be, ga;
            op_row(s2, r, 1.0, al, be, ga);
            bnd_lo = al;
            op_row(s2, r, (double)M, al, be, ga);
            bnd_hi = ga;
        }
        own_lo = (p == 0);
        own_hi = (p == (M - 1) / MC);
        r_hi = (M - 1) % MC;

        // scaled LU of the interior block
        double iu[NI];
        double u = b[0];
        iu[0] = 1.0 / u;
        m[0] = 0.0;
        cu[0] = c[0] * iu[0];
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            u = b[q] - (a[q] * iu[q - 1]) * c[q - 1];
            iu[q] = 1.0 / u;
            m[q] = a[q] * iu[q];
            cu[q] = c[q] * iu[q];
        }
        {
            double t[MC];
#pragma unroll
            for (int q = 0; q < MC; ++q) t[q] = 0.0;
            t[0] = -a[0] * iu[0];
            interior_solve(t);
#pragma unroll
            for (int q = 0; q < NI; ++q) v[q] = t[q];
#pragma unroll
            for (int q = 0; q < MC; ++q) t[q] = 0.0;
            t[NI - 1] = -c[NI - 1] * iu[NI - 1];
            interior_solve(t);
#pragma unroll
            for (int q = 0; q < NI; ++q) w[q] = t[q];
        }
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            ea[q] *= iu[q];
            eb[q] *= iu[q];
            ec[q] *= iu[q];
        }
        blo = bnd_lo * iu[0];
        bhi = bnd_hi;
#pragma unroll
        for (int q = 0; q < NI; ++q)
            if (q == r_hi) bhi = bnd_hi * iu[q];
        aq = a[MC - 1];
        cq = c[MC - 1];
        const double bq = b[MC - 1];

        if constexpr (WAVE) {
            vF = wave_down(v[0], 1);
            wF = wave_down(w[0], 1);
        } else {
            lds[p] = v[0];
            lds[T + p] = w[0];
            __syncthreads();
            vF = (p + 1 < T) ? lds[p + 1] : 0.0;
            wF = (p + 1 < T) ? lds[T + p + 1] : 0.0;
            __syncthreads();
        }

        double A = aq * v[NI - 1];
        double B = bq + aq * w[NI - 1] + cq * vF;
        double C = cq * wF;
        nst = LOGT;
        bool done = false;
#pragma unroll
        for (int k = 0; k < LOGT; ++k) {
            k1[k] = 0.0;
            k2[k] = 0.0;
            if (!done) {
                // stop once every coupling is negligible (uniform decision over the block)
                const double rel = (fabs(A) + fabs(C)) / fabs(B);
                if (block_all_below(rel, lds)) {
                    nst = k;
                    done = true;
                }
            }
            if (!done) {
                const int s = 1 << k;
                double Am, Bm, Cm, Ap, Bp, Cp;
                if constexpr (WAVE) {
                    Am = wave_up(A, s);
                    Bm = wave_up(B, s);
                    Cm = wave_up(C, s);
                    Ap = wave_down(A, s);
                    Bp = wave_down(B, s);
                    Cp = wave_down(C, s);
                    if (p - s < 0) Bm = 1.0;
                    if (p + s >= T) Bp = 1.0;
                } else {
                    lds[p] = A;
                    lds[T + p] = B;
                    lds[2 * T + p] = C;
                    __syncthreads();
                    Am = 0.0, Bm = 1.0, Cm = 0.0, Ap = 0.0, Bp = 1.0, Cp = 0.0;
                    if (p - s >= 0) {
                        Am = lds[p - s];
                        Bm = lds[T + p - s];
                        Cm = lds[2 * T + p - s];
                    }
                    if (p + s < T) {
                        Ap = lds[p + s];
                        Bp = lds[T + p + s];
                        Cp = lds[2 * T + p + s];
                    }
                    __syncthreads();
                }
                const double m1 = (p - s >= 0) ? A / Bm : 0.0;
                const double m2 = (p + s < T) ? C / Bp : 0.0;
                k1[k] = m1;
                k2[k] = m2;
                const double An = -m1 * Am;
                const double Cn = -m2 * Cp;
                const double Bn = B - m1 * Cm - m2 * Ap;
                A = An;
                B = Bn;
                C = Cn;
            }
        }
        invB = 1.0 / B;
    }

    // True on every thread iff x <= kPcrTruncation on every thread of the block.
    __device__ __forceinline__ bool block_all_below(double x, double* lds) const {
        const bool mine = x <= kPcrTruncation;
        if constexpr (WAVE) {
            return __all(mine);
        } else {
            __syncthreads();
            const int ok = __syncthreads_and(mine ? 1 : 0);
            (void)lds;
            return ok != 0;
        }
    }

    // Initial halo: left = last node of chunk p-1, right = first node of chunk p+1.
    __device__ __forceinline__ void halo(const double (&V)[MC], double& hl, double& hr,
                                         double* lds) const {
        if constexpr (WAVE) {
            hl = wave_up(V[MC - 1], 1);
            hr = wave_down(V[0], 1);
        } else {
            lds[p] = V[0];
            lds[T + p] = V[MC - 1];
            __syncthreads();
            hl = (p > 0) ? lds[T + p - 1] : 0.0;
            hr = (p + 1 < T) ? lds[p + 1] : 0.0;
            __syncthreads();
        }
    }

    // One step.  V: this chunk (in/out); hl, hr: halo values (in/out, kept
    // current for the next step).  flo, fhi: boundary forcing, i.e.
    // (1-theta) dt g(tau_old) + theta dt g(tau_new) at S = 0 and S = S_max.
    // lds: at least 4*T doubles (unused when T == 64).
    __device__ __forceinline__ void step(double (&V)[MC], double& hl, double& hr, double flo,
                                         double fhi, double* lds) const {
        double d[MC];
#pragma unroll
        for (int q = 0; q < MC; ++q) {
            const double left = (q == 0) ? hl : V[q - 1];
            const double right = (q == MC - 1) ? hr : V[q + 1];
            d[q] = fma(ea[q], left, fma(eb[q], V[q], ec[q] * right));
        }
        if (own_lo) d[0] = fma(blo, flo, d[0]);
        if (own_hi) {
#pragma unroll
            for (int q = 0; q < MC; ++q)
                if (q == r_hi) d[q] = fma(bhi, fhi, d[q]);
        }
        interior_solve(d);

        double yF, z, zl, zr;
        if constexpr (WAVE) {
            yF = wave_down(d[0], 1);
            double D = fma(-aq, d[NI - 1], fma(-cq, yF, d[MC - 1]));
#pragma unroll
            for (int k = 0; k < LOGT; ++k) {
                if (k < nst) {
                    const int s = 1 << k;
                    const double Dm = wave_up(D, s);
                    const double Dp = wave_down(D, s);
                    D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
                }
            }
            z = D * invB;
            zl = wave_up(z, 1);
            zr = wave_down(z, 1);
        } else {
            double* ybuf = lds;
            double* pb0 = lds + T;
            double* pb1 = lds + 2 * T;
            double* zbuf = lds + 3 * T;
            ybuf[p] = d[0];
            __syncthreads();
            yF = (p + 1 < T) ? ybuf[p + 1] : 0.0;
            double D = fma(-aq, d[NI - 1], fma(-cq, yF, d[MC - 1]));
#pragma unroll
            for (int k = 0; k < LOGT; ++k) {
                if (k < nst) {
                    const int s = 1 << k;
                    double* buf = (k & 1) ? pb1 : pb0;
                    buf[p] = D;
                    __syncthreads();
                    const double Dm = (p - s >= 0) ? buf[p - s] : 0.0;
                    const double Dp = (p + s < T) ? buf[p + s] : 0.0;
                    D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
                }
            }
            z = D * invB;
            zbuf[p] = z;
            __syncthreads();
            zl = (p > 0) ? zbuf[p - 1] : 0.0;
            zr = (p + 1 < T) ? zbuf[p + 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NI; ++q) V[q] = fma(zl, v[q], fma(z, w[q], d[q]));
        V[MC - 1] = z;
        hl = zl;
        hr = fma(z, vF, fma(zr, wF, yF));
    }
};

}  // namespace bsp
