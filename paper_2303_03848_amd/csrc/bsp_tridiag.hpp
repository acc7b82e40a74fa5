// One-wavefront solver for the tridiagonal systems of the theta-method
//   (I - h L) V^{m+1} = (I + e L) V^m + f,   h = theta dt,  e = (1 - theta) dt,
// one system per thread block, the state kept in registers for all steps.
//
// Implicit form of a step.  With A = I - h L, the explicit operator is
//   I + e L = kappa I - mu A,   kappa = 1 + e/h,  mu = e/h,
// so a step is V^{m+1} = A^{-1} (kappa V^m + f) - mu V^m: one solve with A and
// no product with the explicit stencil (Crank-Nicolson: kappa = 2, mu = 1;
// implicit Euler: kappa = 1, mu = 0).  This is the same linear map as the
// textbook evaluation, with less work per node and no neighbour values.
//
// The matrix is the same at every step (the coefficients of the
// Black-Scholes operator do not depend on time), so everything but the
// right-hand side is factored once in `setup`.
//
// Partition: lane p owns the MC consecutive unknowns i0 = p*MC .. i0+MC-1.
// Its last unknown z_p is an interface unknown; the MC-1 interior unknowns
// depend on the two neighbouring interface unknowns only:
//     x_int = d + z_{p-1} v + z_p w,
// where d solves the interior block with the actual right-hand side and v, w
// are its (constant) responses to unit coupling at the two ends.  Substituting
// into the interface rows gives a tridiagonal system of 64 unknowns
//     A_p z_{p-1} + B_p z_p + C_p z_{p+1} = D_p,
// solved by parallel cyclic reduction (PCR) across the lanes.  The reduction
// multipliers are constant and kept per lane.
//
// Truncated PCR: the interface system is strictly diagonally dominant and each
// PCR stage squares the relative size of the off-diagonal couplings
// (|A'|/|B'| ~ (|A|/|B|)^2).  Setup runs stages until every remaining coupling
// is below 2^-60 of its diagonal and records that stage count; the steps then
// run only those stages.  The neglected terms are below the rounding error of
// the result, so the solve stays exact to working precision.
//
// Interior rows use the LU factors l_q = a_q / u_{q-1} (unit lower) and
// u_q (upper, super-diagonal c_q), with kappa folded into the backward sweep:
// per node a step costs 1 forward, 2 backward and 3 update operations.
//
// Exchanges: strides 1, 2, 4 use (chained) DPP lane moves, longer strides
// ds_bpermute, with no LDS and no barrier.  Lanes whose partner lies outside the
// wavefront carry a zero PCR multiplier, so the (wrapped, finite) value they
// fetch does not contribute.  Nodes beyond M are identity rows, decoupled
// from the rest, and keep their value (kappa - mu = 1).
#pragma once

#include "bsp_common.hpp"

namespace bsp {

// Value of `v` held by lane `src` of this wavefront, src taken modulo 64.
// The wrap is explicit: a byte address outside the wavefront (including one
// the compiler forms with the instruction's offset field) does not wrap in
// hardware and returns undefined data.
__device__ __forceinline__ double lane_fetch(double v, int src) {
    const int addr = (src & 63) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// DPP wavefront shifts by one lane: lane i receives lane i-1 (from_prev) or
// lane i+1 (from_next); the lane without a source receives 0 (bound control).
// Shifts by 2 and 4 chain these moves: a few cycles each, against a round
// trip through the LDS crossbar for ds_bpermute.
__device__ __forceinline__ double dpp_from_prev(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_from_next(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int S>
__device__ __forceinline__ double dpp_prev_n(double v) {
#pragma unroll
    for (int i = 0; i < S; ++i) v = dpp_from_prev(v);
    return v;
}
template <int S>
__device__ __forceinline__ double dpp_next_n(double v) {
#pragma unroll
    for (int i = 0; i < S; ++i) v = dpp_from_next(v);
    return v;
}

// Wavefront-uniform copy of an int (lives in a scalar register).
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

constexpr double kPcrTruncation = 8.673617379884035e-19;  // 2^-60

// Interior block of one chunk: LU factors, kappa-scaled backward sweep, and
// the responses v, w.  Shared by the one- and multi-wavefront solvers.
template <int MC>
struct ChunkLU {
    static constexpr int NI = MC - 1;
    double l[NI], ku[NI], cu[NI];  // l_q = a_q/u_{q-1}, ku_q = kappa/u_q, cu_q = c_q/u_q
    double v[NI], w[NI];           // interior responses to z_{p-1}, z_p

    // Factor the interior rows a, b, c (first NI entries used).
    __device__ __forceinline__ void factor(const double (&a)[MC], const double (&b)[MC],
                                           const double (&c)[MC], double kappa) {
        double iu[NI];
        double u = b[0];
        iu[0] = 1.0 / u;
        l[0] = 0.0;
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            l[q] = a[q] * iu[q - 1];
            u = b[q] - l[q] * c[q - 1];
            iu[q] = 1.0 / u;
        }
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            ku[q] = kappa * iu[q];
            cu[q] = c[q] * iu[q];
        }
        // v = A_int^{-1} (-a_0 e_0),  w = A_int^{-1} (-c_{NI-1} e_{NI-1})
        double t[NI];
        t[0] = -a[0];
#pragma unroll
        for (int q = 1; q < NI; ++q) t[q] = -l[q] * t[q - 1];
        t[NI - 1] *= iu[NI - 1];
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) t[q] = fma(-cu[q], t[q + 1], t[q] * iu[q]);
#pragma unroll
        for (int q = 0; q < NI; ++q) v[q] = t[q];
        w[NI - 1] = -c[NI - 1] * iu[NI - 1];
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) w[q] = -cu[q] * w[q + 1];
    }

    // d <- kappa A_int^{-1} d  (forward, then kappa-scaled backward sweep).
    __device__ __forceinline__ void solve(double (&d)[MC]) const {
#pragma unroll
        for (int q = 1; q < NI; ++q) d[q] = fma(-l[q], d[q - 1], d[q]);
        d[NI - 1] *= ku[NI - 1];
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) d[q] = fma(-cu[q], d[q + 1], ku[q] * d[q]);
    }
};

// Matrix rows of chunk p (global rows p*MC ..), implicit weight h.  Rows at or
// beyond M are identity rows.  Also the boundary coefficients alpha_1
// (S = dS row, coupling to S = 0) and gamma_M (coupling to S = S_max).
template <int MC>
__device__ __forceinline__ void chunk_rows(double s2, double r, double h, int M, int p,
                                           double (&a)[MC], double (&b)[MC], double (&c)[MC],
                                           double& alpha1, double& gammaM) {
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        const int g = p * MC + q;
        double al, be, ga;
        op_row(s2, r, (double)(g + 1), al, be, ga);
        const bool pad = g >= M;
        a[q] = (pad || g == 0) ? 0.0 : -h * al;
        b[q] = pad ? 1.0 : 1.0 - h * be;
        c[q] = (g >= M - 1) ? 0.0 : -h * ga;
    }
    double al, be, ga;
    op_row(s2, r, 1.0, al, be, ga);
    alpha1 = al;
    op_row(s2, r, (double)M, al, be, ga);
    gammaM = ga;
}

// Boundary forcing of chunk p.  Row 0 is interior row 0 of chunk 0:
// r_0 += blo * flo.  Row M-1 is either the interface row of its chunk
// (D += bhiD * fhi, no per-node work) or an interior row (hi_in, r_{r_hi} +=
// bhi * fhi).  Coefficients are zero on the chunks they do not concern.
struct Forcing {
    double blo, bhiD, bhi;
    int r_hi;
    bool hi_in;
    __device__ __forceinline__ void init(int p, int MC, int M, double alpha1, double gammaM,
                                         double kappa) {
        blo = (p == 0) ? alpha1 / kappa : 0.0;
        const bool owner = p == (M - 1) / MC;
        r_hi = (M - 1) % MC;
        hi_in = owner && r_hi < MC - 1;
        bhiD = (owner && r_hi == MC - 1) ? gammaM : 0.0;
        bhi = gammaM / kappa;
    }
    // Right-hand side of the interior rows: V (+ forcing / kappa).  HI false:
    // the grid is a multiple of the chunk, so row M-1 is an interface row
    // and no interior row takes forcing (hi_in is false; saying so at compile
    // time drops the per-step select over the rows).
    template <int MC, bool HI = true>
    __device__ __forceinline__ void rhs(const double (&V)[MC], double flo, double fhi,
                                        double (&d)[MC]) const {
#pragma unroll
        for (int q = 0; q < MC; ++q) d[q] = V[q];
        d[0] = fma(blo, flo, d[0]);
        if (HI && hi_in) {
#pragma unroll
            for (int q = 0; q < MC - 1; ++q)
                if (q == r_hi) d[q] = fma(bhi, fhi, d[q]);
        }
    }
};

template <int T, int MC>
struct BlockTri {
    static_assert(T == 64, "one wavefront (several: BlockTriH)");
    static_assert(MC >= 2, "at least one interior row per chunk");
    static constexpr int LOGT = 6;
    static constexpr int NI = MC - 1;
    static constexpr int kThreads = 64;

    ChunkLU<MC> lu;
    Forcing fc;
    double aq, cq, kap, mu;         // interface row: sub/super diagonal; step constants
    double k1[LOGT], k2[LOGT], invB;
    // pipelined steps: L~^{-1} v, L~^{-1} w; the sweep multipliers in the
    // scaled variables xi_q = x_q / ku_q; ku-scaled interface couplings and
    // forcing coefficients
    double al[NI], be[NI], lh[NI], ch[NI];
    double aqk, cqk, blok, bhik;
    int p, nst;

    __device__ __forceinline__ int stages() const { return nst; }

    __device__ __forceinline__ double up(double x, int s) const {
        if (s == 1) return dpp_from_prev(x);
        if (s == 2) return dpp_prev_n<2>(x);
        if (s == 4) return dpp_prev_n<4>(x);
        return lane_fetch(x, p - s);
    }
    __device__ __forceinline__ double down(double x, int s) const {
        if (s == 1) return dpp_from_next(x);
        if (s == 2) return dpp_next_n<2>(x);
        if (s == 4) return dpp_next_n<4>(x);
        return lane_fetch(x, p + s);
    }

    // h = theta*dt > 0 (implicit weight), e = (1-theta)*dt (explicit weight).
    // lds is not used (kept for a common interface).
    __device__ __forceinline__ void setup(double s2, double r, double h, double e, int M,
                                          double* lds) {
        (void)lds;
        p = threadIdx.x & 63;  // lane: the block may hold several independent wavefronts
        kap = 1.0 + e / h;
        mu = e / h;
        double a[MC], b[MC], c[MC], alpha1, gammaM;
        chunk_rows<MC>(s2, r, h, M, p, a, b, c, alpha1, gammaM);
        lu.factor(a, b, c, kap);
        fc.init(p, MC, M, alpha1, gammaM, kap);
        aq = a[MC - 1];
        cq = c[MC - 1];
        const double vF = dpp_from_next(lu.v[0]);
        const double wF = dpp_from_next(lu.w[0]);
        double A = aq * lu.v[NI - 1];
        double B = b[MC - 1] + aq * lu.w[NI - 1] + cq * vF;
        double C = cq * wF;
        nst = LOGT;
        bool done = false;
#pragma unroll
        for (int k = 0; k < LOGT; ++k) {
            k1[k] = 0.0;
            k2[k] = 0.0;
            if (!done && __all(((fabs(A) + fabs(C)) / fabs(B)) <= kPcrTruncation)) {
                nst = k;
                done = true;
            }
            if (!done) {
                const int s = 1 << k;
                // exchanges first, on every lane (a DPP or bpermute under a
                // partial exec mask reads nothing from the disabled lanes)
                const bool lo = p - s >= 0, hi = p + s < T;
                const double Au = up(A, s), Bu = up(B, s), Cu = up(C, s);
                const double Ad = down(A, s), Bd = down(B, s), Cd = down(C, s);
                const double Am = lo ? Au : 0.0, Bm = lo ? Bu : 1.0, Cm = lo ? Cu : 0.0;
                const double Ap = hi ? Ad : 0.0, Bp = hi ? Bd : 1.0, Cp = hi ? Cd : 0.0;
                const double m1 = lo ? A / Bm : 0.0;
                const double m2 = hi ? C / Bp : 0.0;
                k1[k] = m1;
                k2[k] = m2;
                const double An = -m1 * Am, Cn = -m2 * Cp, Bn = B - m1 * Cm - m2 * Ap;
                A = An;
                B = Bn;
                C = Cn;
            }
        }
        invB = 1.0 / B;
        nst = wave_uniform(nst);
        // forward-swept interface responses for the pipelined steps
        al[0] = lu.v[0];
        be[0] = lu.w[0];
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            al[q] = fma(-lu.l[q], al[q - 1], lu.v[q]);
            be[q] = fma(-lu.l[q], be[q - 1], lu.w[q]);
        }
        // x_q = ku_q xi_q turns the backward sweep x_q = ku_q y_q - cu_q x_{q+1}
        // into xi_q = y_q - ch_q xi_{q+1} and the forward sweep of x,
        // F_q = x_q - l_q F_{q-1} with F_q = ku_q phi_q, into
        // phi_q = xi_q - lh_q phi_{q-1}: one FMA per node each.
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            lh[q] = (q > 0) ? lu.l[q] * lu.ku[q - 1] / lu.ku[q] : 0.0;
            ch[q] = (q < NI - 1) ? lu.cu[q] * lu.ku[q + 1] / lu.ku[q] : 0.0;
        }
        aqk = aq * lu.ku[NI - 1];
        cqk = cq * dpp_from_next(lu.ku[0]);  // cq = 0 on the last lane
        blok = fc.blo / lu.ku[0];
        double kr = 1.0;
#pragma unroll
        for (int q = 0; q < NI; ++q)
            if (q == fc.r_hi) kr = lu.ku[q];
        bhik = fc.bhi / kr;
    }

    // ---------------------------------------------------------------------
    // Pipelined steps (Crank-Nicolson, mu = 1, and implicit Euler, mu = 0).
    // With L~ the unit lower factor of the interior block, the forward sweep
    // of step m+1 is
    //   y = L~^{-1} (V^m + f^{m+1}/kappa) = yP + z_{p-1} al + z_p be,
    //   yP = L~^{-1} (P^m + f^{m+1}/kappa),  al = L~^{-1} v,  be = L~^{-1} w,
    // where P^m is step m's interior value before its interface correction
    // (V^m = P^m + z_{p-1} v + z_p w).  yP depends only on P^m, so its
    // sweep runs while step m's interface reduction waits on lane exchanges;
    // once z is known, y is two independent FMAs per node.  The interior
    // state itself is never formed between steps.  With x = kappa-scaled
    // solve of step m+1 (before its interface correction),
    //   P^{m+1} = x - mu V^m   and   V^m = L~ y - f^{m+1}/kappa,
    // so the next step's sweep is
    //   yP' = L~^{-1} (x + (mu f^{m+1} + f^{m+2})/kappa) - mu y,
    // whose forcing enters only the rows that carry it (row 0, row M-1) at the
    // start of the recursion.  In the scaled variables xi, phi the step costs
    // five operations per interior node: two for y, one backward, one forward,
    // one for yP'.
    struct Pipe {
        double A[MC];     // yP of the coming step (interior entries)
        double z, zl;     // interface values of the last step (own, left)
        double Vi;        // the interface node's value
    };

    // Starts a run from state V; flo, fhi: forcing of the first step.
    __device__ __forceinline__ void pipe_begin(const double (&V)[MC], double flo, double fhi,
                                               Pipe& P) const {
        double B[MC];
#pragma unroll
        for (int q = 0; q < MC; ++q) B[q] = V[q];
        const double tt = fc.hi_in ? fc.bhi * fhi : 0.0;
#pragma unroll
        for (int q = 0; q < NI; ++q) B[q] += (q == fc.r_hi) ? tt : 0.0;
        P.A[0] = fma(fc.blo, flo, B[0]);
#pragma unroll
        for (int q = 1; q < NI; ++q) P.A[q] = fma(-lu.l[q], P.A[q - 1], B[q]);
        P.z = 0.0;
        P.zl = 0.0;
        P.Vi = V[MC - 1];
    }

    // One step: flo, fhi its forcing; flo_n, fhi_n the next step's (zero
    // after the last step).  EX: mu = 1 (Crank-Nicolson), else mu = 0.
    // NST: reduction stages (>= 0 compile-time, no branches; -1: nst at run
    // time).  HI: row M-1 is an interior row of some chunk (a grid that is
    // not a multiple of MC); its forcing is then added by selects on every
    // lane, so the step body stays free of branches.
    template <bool EX, int NST, bool HI>
    __device__ __forceinline__ void pipe_step(Pipe& P, double flo, double fhi, double flo_n,
                                              double fhi_n, double* /*lds: unused*/ = nullptr) const {
        double y[NI], xi[NI];
        // y just ahead of the backward chain that consumes it, so that each
        // link of the chain has independent work beside it
        y[NI - 1] = fma(P.zl, al[NI - 1], fma(P.z, be[NI - 1], P.A[NI - 1]));
        if (NI >= 2) y[NI - 2] = fma(P.zl, al[NI - 2], fma(P.z, be[NI - 2], P.A[NI - 2]));
        xi[NI - 1] = y[NI - 1];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) {
            if (q >= 1) y[q - 1] = fma(P.zl, al[q - 1], fma(P.z, be[q - 1], P.A[q - 1]));
            xi[q] = fma(-ch[q], xi[q + 1], y[q]);
            __builtin_amdgcn_sched_barrier(0);
        }
        const double xF = dpp_from_next(xi[0]);  // xi_0 of the next chunk
        double D = fma(kap, P.Vi, fma(fc.bhiD, fhi, fma(-aqk, xi[NI - 1], -cqk * xF)));
        // interface reduction
        if constexpr (NST >= 0) {
#pragma unroll
            for (int k = 0; k < NST; ++k) {
                const int s = 1 << k;
                const double Dm = up(D, s);
                const double Dp = down(D, s);
                D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
            }
        } else {
#pragma unroll
            for (int k = 0; k < LOGT; ++k) {
                if (k < nst) {
                    const int s = 1 << k;
                    const double Dm = up(D, s);
                    const double Dp = down(D, s);
                    D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
                }
            }
        }
        // next step's forward sweep: independent of the reduction above
        double tt = 0.0;
        if constexpr (HI) tt = fc.hi_in ? bhik * (EX ? fhi + fhi_n : fhi_n) : 0.0;
        double ph = fma(blok, EX ? flo + flo_n : flo_n, xi[0]);
        if constexpr (HI) ph += (fc.r_hi == 0) ? tt : 0.0;
        P.A[0] = EX ? fma(lu.ku[0], ph, -y[0]) : lu.ku[0] * ph;
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            double xq = xi[q];
            if constexpr (HI) xq += (q == fc.r_hi) ? tt : 0.0;
            ph = fma(-lh[q], ph, xq);
            P.A[q] = EX ? fma(lu.ku[q], ph, -y[q]) : lu.ku[q] * ph;
        }
        const double z = D * invB;
        P.zl = dpp_from_prev(z);
        P.z = z;
        P.Vi = EX ? z - P.Vi : z;
    }

    // Ends a run (the last pipe_step had zero next-step forcing): V = state.
    __device__ __forceinline__ void pipe_end(const Pipe& P, double (&V)[MC]) const {
        double y[MC];
#pragma unroll
        for (int q = 0; q < NI; ++q) y[q] = fma(P.zl, al[q], fma(P.z, be[q], P.A[q]));
        V[0] = y[0];
#pragma unroll
        for (int q = 1; q < NI; ++q) V[q] = fma(lu.l[q], y[q - 1], y[q]);
        V[MC - 1] = P.Vi;
    }

    // One step.  V: this chunk (in/out).  flo, fhi: boundary forcing
    // e g(tau_old) + h g(tau_new) at S = 0 and S = S_max.  EX: the step has
    // an explicit part (mu != 0); without it V is dead once the solve starts.
    template <bool EX>
    __device__ __forceinline__ void step(double (&V)[MC], double flo, double fhi,
                                         double* lds) const {
        (void)lds;
        double d[MC];
        fc.rhs(V, flo, fhi, d);
        lu.solve(d);
        const double yF = dpp_from_next(d[0]);
        double D = fma(kap, V[MC - 1], fma(fc.bhiD, fhi, fma(-aq, d[NI - 1], -cq * yF)));
        // explicit remainder -mu V, off the critical path of the reduction
        double rz = 0.0;
        if constexpr (EX) {
#pragma unroll
            for (int q = 0; q < NI; ++q) d[q] = fma(-mu, V[q], d[q]);
            rz = -mu * V[MC - 1];
        }
#pragma unroll
        for (int k = 0; k < LOGT; ++k) {
            if (k < nst) {
                const int s = 1 << k;
                const double Dm = up(D, s);
                const double Dp = down(D, s);
                D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
            }
        }
        const double z = D * invB;
        const double zl = dpp_from_prev(z);
#pragma unroll
        for (int q = 0; q < NI; ++q) V[q] = fma(zl, lu.v[q], fma(z, lu.w[q], d[q]));
        V[MC - 1] = z + rz;
    }
};

}  // namespace bsp
