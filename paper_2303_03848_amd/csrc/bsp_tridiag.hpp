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
// solved by parallel cyclic reduction over the block through LDS; the
// reduction multipliers are constant and kept per thread, so one step costs
// one interior forward/backward sweep per thread and log2(T) exchange rounds.
// Nodes beyond M are padding rows of the identity, decoupled from the rest.
#pragma once

#include "bsp_common.hpp"

namespace bsp {

template <int T, int MC>
struct BlockTri {
    static_assert(MC >= 2, "at least one interior row per chunk");
    static constexpr int LOGT = ilog2(T);
    static constexpr int NI = MC - 1;

    double ea[MC], eb[MC], ec[MC];  // explicit part (I + (1-theta) dt L)
    double l[NI], iu[NI], cu[NI];   // interior LU: l (sub-diagonal multipliers), 1/u, c/u
    double v[NI], w[NI];            // interior responses to z_{p-1}, z_p
    double aq, cq;                  // interface row: implicit sub/super diagonal
    double vF, wF;                  // v[0], w[0] of the next chunk
    double k1[LOGT > 0 ? LOGT : 1], k2[LOGT > 0 ? LOGT : 1], invB;
    double bnd_lo, bnd_hi;          // operator coefficients coupling to the boundary values
    int p, r_hi;
    bool own_lo, own_hi;

    __device__ __forceinline__ void interior_solve(double (&t)[MC]) const {
#pragma unroll
        for (int q = 1; q < NI; ++q) t[q] = fma(-l[q], t[q - 1], t[q]);
        t[NI - 1] *= iu[NI - 1];
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) t[q] = fma(-cu[q], t[q + 1], t[q] * iu[q]);
    }

    // h = theta*dt (implicit weight), e = (1-theta)*dt (explicit weight).
    // lds: at least 3*T doubles.  Contains block barriers.
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

        double u = b[0];
        iu[0] = 1.0 / u;
        cu[0] = c[0] * iu[0];
        l[0] = 0.0;
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            l[q] = a[q] * iu[q - 1];
            u = b[q] - l[q] * c[q - 1];
            iu[q] = 1.0 / u;
            cu[q] = c[q] * iu[q];
        }
        {
            double t[MC];
#pragma unroll
            for (int q = 0; q < MC; ++q) t[q] = 0.0;
            t[0] = -a[0];
            interior_solve(t);
#pragma unroll
            for (int q = 0; q < NI; ++q) v[q] = t[q];
#pragma unroll
            for (int q = 0; q < MC; ++q) t[q] = 0.0;
            t[NI - 1] = -c[NI - 1];
            interior_solve(t);
#pragma unroll
            for (int q = 0; q < NI; ++q) w[q] = t[q];
        }
        aq = a[MC - 1];
        cq = c[MC - 1];
        const double bq = b[MC - 1];

        lds[p] = v[0];
        lds[T + p] = w[0];
        __syncthreads();
        vF = (p + 1 < T) ? lds[p + 1] : 0.0;
        wF = (p + 1 < T) ? lds[T + p + 1] : 0.0;
        __syncthreads();

        double A = aq * v[NI - 1];
        double B = bq + aq * w[NI - 1] + cq * vF;
        double C = cq * wF;
#pragma unroll
        for (int k = 0; k < LOGT; ++k) {
            const int s = 1 << k;
            lds[p] = A;
            lds[T + p] = B;
            lds[2 * T + p] = C;
            __syncthreads();
            double Am = 0.0, Bm = 1.0, Cm = 0.0, Ap = 0.0, Bp = 1.0, Cp = 0.0;
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
        invB = 1.0 / B;
    }

    // Initial halo: left = last node of chunk p-1, right = first node of chunk p+1.
    __device__ __forceinline__ void halo(const double (&V)[MC], double& hl, double& hr,
                                         double* lds) const {
        lds[p] = V[0];
        lds[T + p] = V[MC - 1];
        __syncthreads();
        hl = (p > 0) ? lds[T + p - 1] : 0.0;
        hr = (p + 1 < T) ? lds[p + 1] : 0.0;
        __syncthreads();
    }

    // One step.  V: this chunk (in/out); hl, hr: halo values (in/out, kept
    // current for the next step).  flo, fhi: boundary forcing, i.e.
    // (1-theta) dt g(tau_old) + theta dt g(tau_new) at S = 0 and S = S_max.
    // lds: at least 4*T doubles.  Contains LOGT + 2 block barriers.
    __device__ __forceinline__ void step(double (&V)[MC], double& hl, double& hr, double flo,
                                         double fhi, double* lds) const {
        double d[MC];
#pragma unroll
        for (int q = 0; q < MC; ++q) {
            const double left = (q == 0) ? hl : V[q - 1];
            const double right = (q == MC - 1) ? hr : V[q + 1];
            d[q] = fma(ea[q], left, fma(eb[q], V[q], ec[q] * right));
        }
        if (own_lo) d[0] = fma(bnd_lo, flo, d[0]);
        if (own_hi) {
#pragma unroll
            for (int q = 0; q < MC; ++q)
                if (q == r_hi) d[q] = fma(bnd_hi, fhi, d[q]);
        }
        interior_solve(d);

        double* ybuf = lds;
        double* pb0 = lds + T;
        double* pb1 = lds + 2 * T;
        double* zbuf = lds + 3 * T;
        ybuf[p] = d[0];
        __syncthreads();
        const double yF = (p + 1 < T) ? ybuf[p + 1] : 0.0;
        double D = fma(-aq, d[NI - 1], fma(-cq, yF, d[MC - 1]));
#pragma unroll
        for (int k = 0; k < LOGT; ++k) {
            const int s = 1 << k;
            double* buf = (k & 1) ? pb1 : pb0;
            buf[p] = D;
            __syncthreads();
            const double Dm = (p - s >= 0) ? buf[p - s] : 0.0;
            const double Dp = (p + s < T) ? buf[p + s] : 0.0;
            D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
        }
        const double z = D * invB;
        zbuf[p] = z;
        __syncthreads();
        const double zl = (p > 0) ? zbuf[p - 1] : 0.0;
        const double zr = (p + 1 < T) ? zbuf[p + 1] : 0.0;
#pragma unroll
        for (int q = 0; q < NI; ++q) V[q] = fma(zl, v[q], fma(z, w[q], d[q]));
        V[MC - 1] = z;
        hl = zl;
        hr = fma(z, vF, fma(zr, wF, yF));
    }
};

}  // namespace bsp
