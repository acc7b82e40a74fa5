// Tridiagonal block solver for large grids (M up to 16384), where the
// per-node factorisation does not fit in registers or LDS of one compute unit.
//
// Same partition, implicit step form and truncated parallel cyclic reduction
// as BlockTri, with two differences:
//  * the interior LU factors and responses (l, kappa/u, c/u, v, w) of every
//    node live in a global table computed once per launch by k_large_setup
//    and are streamed every step (coalesced: table[f][q][thread]); all
//    systems of a launch share one table, so it stays in the L2 / infinity
//    cache;
//  * the interface system of the T threads is reduced through LDS with one
//    barrier per PCR stage.
// Per-thread interface data (PCR multipliers, interface row, stage count) is
// a second table ptab[field][thread].
#pragma once

#include "bsp_common.hpp"
#include "bsp_tridiag.hpp"

namespace bsp {

constexpr double kPcrTruncationLarge = 8.673617379884035e-19;  // 2^-60

enum { kLgL = 0, kLgKU, kLgCU, kLgV, kLgW, kLgFields };
// per-thread fields of ptab: aq, cq, invB, nst, (4 spare), k1[16], k2[16]
constexpr int kLgP = 8 + 32;

template <int T, int MC>
struct BlockTriG {
    static constexpr int LOGT = ilog2(T);
    static constexpr int NI = MC - 1;
    static_assert(LOGT <= 16, "stage table");

    const double* tab;
    const double* ptab;
    const double* kst;  // LDS copy of this block's stage multipliers [2][LOGT][T]
    Forcing fc;
    double aq, cq, invB, kap, mu;
    int p, nst;

    // Table reads are raw buffer loads: one descriptor over this shape's
    // table, the lane offset p*8 in one register and the row offset
    // (f*MC + q)*T*8 as a scalar, so no per-lane address arithmetic; they are
    // not flat loads either, whose completion every LDS wait would also have
    // to await.  Reads past the table's size return zero.
    static constexpr int kTabBytes = kLgFields * MC * T * 8;
    using Rsrc = __amdgpu_buffer_rsrc_t;

    __device__ __forceinline__ double coef(Rsrc rs, int f, int q) const {
        return __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(rs, p * 8, (f * MC + q) * T * 8, 0));
    }

    // h = theta*dt > 0, e = (1-theta)*dt; tables built by k_large_setup for
    // the same (s2, r, h, e, M).
    // kst_lds: 2 * LOGT * T doubles of LDS for the stage multipliers (each
    // thread reads only its own, so no barrier is needed after the copy).
    __device__ __forceinline__ void load(const double* tab_, const double* ptab_, double s2,
                                         double r, double h, double e, int M, double* kst_lds) {
        tab = tab_;
        ptab = ptab_;
        p = threadIdx.x;
#pragma unroll
        for (int k = 0; k < LOGT; ++k) {
            kst_lds[k * T + p] = ptab[(8 + k) * T + p];
            kst_lds[(LOGT + k) * T + p] = ptab[(24 + k) * T + p];
        }
        kst = kst_lds;
        kap = 1.0 + e / h;
        mu = e / h;
        aq = ptab[0 * T + p];
        cq = ptab[1 * T + p];
        invB = ptab[2 * T + p];
        nst = wave_uniform((int)ptab[3 * T + p]);
        double al, be, ga, gammaM;
        op_row(s2, r, 1.0, al, be, ga);
        const double alpha1 = al;
        op_row(s2, r, (double)M, al, be, ga);
        gammaM = ga;
        fc.init(p, MC, M, alpha1, gammaM, kap);
    }

    // Coefficient stream of one step, in the order the step consumes it:
    // forward elimination l_1 .. l_{NI-1}; back substitution kappa/u_{NI-1},
    // then (c/u_q, kappa/u_q) for q = NI-2 .. 0; responses (v_q, w_q) for
    // q = 0 .. NI-1.  Each load is issued kPD positions ahead of its use (a
    // ring of kPD registers), so the chains wait on L2 latency once per step
    // instead of once per node; the last prefetches are in flight across the
    // interface reduction.
    static constexpr int kNF = NI - 1, kNB = 1 + 2 * (NI - 1), kNS = kNF + kNB + 2 * NI;
    // loads ahead (fewer for 32-node chunks, whose state and right-hand side
    // already take 128 registers); nodes per scheduling group
    static constexpr int kPD = MC >= 32 ? 8 : 16, kG = 4;
    static constexpr int sfield(int s) {
        return s < kNF ? kLgL
               : s < kNF + kNB ? ((s == kNF || ((s - kNF - 1) & 1)) ? kLgKU : kLgCU)
                               : (((s - kNF - kNB) & 1) ? kLgW : kLgV);
    }
    static constexpr int sq(int s) {
        return s < kNF ? s + 1
               : s < kNF + kNB ? (s == kNF ? NI - 1 : NI - 2 - (s - kNF - 1) / 2)
                               : (s - kNF - kNB) / 2;
    }

    // One step (see BlockTri::step).  lds: 4*T doubles; the stage multipliers
    // are read from their LDS copy (a global read after each stage's barrier
    // would put its latency on the critical path).
    template <bool EX>
    __device__ __forceinline__ void step(double (&V)[MC], double flo, double fhi,
                                         double* lds) const {
        // Opaque per step: the compiler must not hoist the table loads out of
        // the step loop (that is the register footprint this solver avoids).
        const double* tb0 = tab;
        asm volatile("" : "+s"(tb0));
        // dword 3: the raw-buffer format word of gfx9-family descriptors
        const Rsrc tb = __builtin_amdgcn_make_buffer_rsrc((void*)tb0, (short)0, kTabBytes,
                                                          0x00020000);
        double ring[kPD];
#pragma unroll
        for (int s = 0; s < kPD; ++s) ring[s] = coef(tb, sfield(s), sq(s));
        double d[MC];
        fc.rhs(V, flo, fhi, d);
        // forward elimination, kG nodes per group: take the group's
        // coefficients, issue the loads kPD positions on, then compute
#pragma unroll
        for (int q0 = 1; q0 < NI; q0 += kG) {
            double c[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int s = q0 - 1 + j;
                if (q0 + j < NI) {
                    c[j] = ring[s % kPD];
                    if (s + kPD < kNS) ring[s % kPD] = coef(tb, sfield(s + kPD), sq(s + kPD));
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < kG; ++j)
                if (q0 + j < NI) d[q0 + j] = fma(-c[j], d[q0 + j - 1], d[q0 + j]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // back substitution: kappa/u_{NI-1} alone, then (c/u_q, kappa/u_q)
        {
            const int s = kNF;
            const double ku = ring[s % kPD];
            if (s + kPD < kNS) ring[s % kPD] = coef(tb, sfield(s + kPD), sq(s + kPD));
            d[NI - 1] *= ku;
        }
#pragma unroll
        for (int e0 = 0; e0 < NI - 1; e0 += kG) {  // e: q = NI-2-e
            double cu[kG], ku[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int s = kNF + 1 + 2 * (e0 + j);
                if (e0 + j < NI - 1) {
                    cu[j] = ring[s % kPD];
                    if (s + kPD < kNS) ring[s % kPD] = coef(tb, sfield(s + kPD), sq(s + kPD));
                    ku[j] = ring[(s + 1) % kPD];
                    if (s + 1 + kPD < kNS)
                        ring[(s + 1) % kPD] = coef(tb, sfield(s + 1 + kPD), sq(s + 1 + kPD));
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int q = NI - 2 - (e0 + j);
                if (e0 + j < NI - 1) d[q] = fma(-cu[j], d[q + 1], d[q] * ku[j]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }

        double* ybuf = lds;
        double* pb0 = lds + T;
        double* pb1 = lds + 2 * T;
        double* zbuf = lds + 3 * T;
        ybuf[p] = d[0];
        __syncthreads();
        const double yF = (p + 1 < T) ? ybuf[p + 1] : 0.0;
        double D = fma(kap, V[MC - 1], fma(fc.bhiD, fhi, fma(-aq, d[NI - 1], -cq * yF)));
        // explicit remainder -mu V; V is dead from here on
        double rz = 0.0;
        if constexpr (EX) {
#pragma unroll
            for (int q = 0; q < NI; ++q) d[q] = fma(-mu, V[q], d[q]);
            rz = -mu * V[MC - 1];
        }
        for (int k = 0; k < nst; ++k) {
            const int s = 1 << k;
            double* buf = (k & 1) ? pb1 : pb0;
            buf[p] = D;
            __syncthreads();
            const double Dm = (p - s >= 0) ? buf[p - s] : 0.0;
            const double Dp = (p + s < T) ? buf[p + s] : 0.0;
            D = fma(-kst[k * T + p], Dm, fma(-kst[(LOGT + k) * T + p], Dp, D));
        }
        const double z = D * invB;
        zbuf[p] = z;
        __syncthreads();
        const double zl = (p > 0) ? zbuf[p - 1] : 0.0;
        // interior values from the responses (v_q, w_q)
#pragma unroll
        for (int q0 = 0; q0 < NI; q0 += kG) {
            double vv[kG], ww[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int s = kNF + kNB + 2 * (q0 + j);
                if (q0 + j < NI) {
                    vv[j] = ring[s % kPD];
                    if (s + kPD < kNS) ring[s % kPD] = coef(tb, sfield(s + kPD), sq(s + kPD));
                    ww[j] = ring[(s + 1) % kPD];
                    if (s + 1 + kPD < kNS)
                        ring[(s + 1) % kPD] = coef(tb, sfield(s + 1 + kPD), sq(s + 1 + kPD));
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < kG; ++j)
                if (q0 + j < NI) V[q0 + j] = fma(zl, vv[j], fma(z, ww[j], d[q0 + j]));
            __builtin_amdgcn_sched_barrier(0);
        }
        V[MC - 1] = z + rz;
    }
};

// Builds the tables of BlockTriG<T, MC> for one (option, theta, dt): one
// block of T threads; each thread walks its chunk sequentially in global
// memory, then the interface system is reduced through LDS.
template <int T, int MC>
__global__ __launch_bounds__(T) void k_large_setup(double s2, double r, double h, double e,
                                                   int M, double* __restrict__ tab,
                                                   double* __restrict__ ptab) {
    constexpr int LOGT = ilog2(T), NI = MC - 1;
    __shared__ double lds[3 * T];
    const int p = threadIdx.x, i0 = p * MC;
    const double kappa = 1.0 + e / h;
    auto A = [&](int g) {
        double al, be, ga;
        op_row(s2, r, (double)(g + 1), al, be, ga);
        return (g >= M || g == 0) ? 0.0 : -h * al;
    };
    auto B = [&](int g) {
        double al, be, ga;
        op_row(s2, r, (double)(g + 1), al, be, ga);
        return g >= M ? 1.0 : 1.0 - h * be;
    };
    auto C = [&](int g) {
        double al, be, ga;
        op_row(s2, r, (double)(g + 1), al, be, ga);
        return g >= M - 1 ? 0.0 : -h * ga;
    };
    auto at = [&](int f, int q) -> double& { return tab[((long)f * MC + q) * T + p]; };
    // LU of the interior rows 0..NI-1: l_q = a_q/u_{q-1}; KU holds 1/u_q until
    // the responses are done, then kappa/u_q
    double u = B(i0);
    at(kLgL, 0) = 0.0;
    at(kLgKU, 0) = 1.0 / u;
    at(kLgCU, 0) = C(i0) / u;
    for (int q = 1; q < NI; ++q) {
        const double l = A(i0 + q) / u;
        u = B(i0 + q) - l * C(i0 + q - 1);
        at(kLgL, q) = l;
        at(kLgKU, q) = 1.0 / u;
        at(kLgCU, q) = C(i0 + q) / u;
    }
    // responses: v to -a_0 e_0, w to -c_{NI-1} e_{NI-1}
    double t = -A(i0);
    at(kLgV, 0) = t;
    for (int q = 1; q < NI; ++q) {
        t = -at(kLgL, q) * t;
        at(kLgV, q) = t;
    }
    at(kLgV, NI - 1) *= at(kLgKU, NI - 1);
    for (int q = NI - 2; q >= 0; --q)
        at(kLgV, q) = fma(-at(kLgCU, q), at(kLgV, q + 1), at(kLgV, q) * at(kLgKU, q));
    at(kLgW, NI - 1) = -C(i0 + NI - 1) * at(kLgKU, NI - 1);
    for (int q = NI - 2; q >= 0; --q) at(kLgW, q) = -at(kLgCU, q) * at(kLgW, q + 1);
    for (int q = 0; q < NI; ++q) at(kLgKU, q) *= kappa;

    const double aq = A(i0 + MC - 1), cq = C(i0 + MC - 1), bq = B(i0 + MC - 1);
    lds[p] = at(kLgV, 0);
    lds[T + p] = at(kLgW, 0);
    __syncthreads();
    const double vF = (p + 1 < T) ? lds[p + 1] : 0.0;
    const double wF = (p + 1 < T) ? lds[T + p + 1] : 0.0;
    __syncthreads();
    double Aq = aq * at(kLgV, NI - 1);
    double Bq = bq + aq * at(kLgW, NI - 1) + cq * vF;
    double Cq = cq * wF;
    int nst = LOGT;
    bool done = false;
    for (int k = 0; k < 16; ++k) {
        ptab[(8 + k) * T + p] = 0.0;
        ptab[(24 + k) * T + p] = 0.0;
    }
    for (int k = 0; k < LOGT; ++k) {
        const int mine = ((fabs(Aq) + fabs(Cq)) / fabs(Bq)) <= kPcrTruncationLarge;
        const int all = __syncthreads_and(mine);
        if (!done && all) {
            nst = k;
            done = true;
        }
        if (done) break;
        const int s = 1 << k;
        lds[p] = Aq;
        lds[T + p] = Bq;
        lds[2 * T + p] = Cq;
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
        const double m1 = (p - s >= 0) ? Aq / Bm : 0.0;
        const double m2 = (p + s < T) ? Cq / Bp : 0.0;
        ptab[(8 + k) * T + p] = m1;
        ptab[(24 + k) * T + p] = m2;
        const double An = -m1 * Am, Cn = -m2 * Cp, Bn = Bq - m1 * Cm - m2 * Ap;
        Aq = An;
        Bq = Bn;
        Cq = Cn;
    }
    ptab[0 * T + p] = aq;
    ptab[1 * T + p] = cq;
    ptab[2 * T + p] = 1.0 / Bq;
    ptab[3 * T + p] = (double)nst;
    for (int f = 4; f < 8; ++f) ptab[f * T + p] = 0.0;
}

}  // namespace bsp
