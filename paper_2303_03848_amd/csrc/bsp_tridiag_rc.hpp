// Tridiagonal block solver for large grids (up to 16384 nodes on 512 threads)
// that keeps one coefficient field per node on chip and recomputes the rest.
//
// Same partition and implicit step form as BlockTriG (each thread owns MC
// consecutive rows: MC-1 interior rows eliminated locally and one interface
// row; the interface system is reduced by truncated parallel cyclic
// reduction through LDS), but nothing is read from global memory after the
// set-up:
//  * kappa/u_q, the scaled reciprocal pivot of interior row q, is the one
//    field kept per node, in LDS (NI x T doubles, read twice per step);
//  * the row coefficients are closed forms in the grid index j (centred
//    differences of eq. (1)): with A' = A/kappa, C' = C/kappa,
//        A'(j) = j (c2 j + c1),  C'(j) = j (c2 j - c1),
//        c2 = -h sigma^2 / (2 kappa),  c1 = h r / (2 kappa),
//    so the multipliers l_q = A'_q kappa/u_{q-1} and c_q/u_q = C'_q kappa/u_q
//    cost a few FMAs;
//  * the interface responses are not stored: once the interface values are
//    known, a second forward and backward sweep solves the interior rows for
//    the correction they cause (the two couplings as the right-hand side) and
//    adds it to the state, so only the state and one work array live in
//    registers;
//  * the interface reduction's multipliers of the first kRcRegStages stages
//    stay in registers; further stages (stiff steps only) carry the reduced
//    coefficients through LDS and recompute their multipliers each step.
// Each block builds all of this itself, so launches share no table.  The step
// is bound by FP64 arithmetic and LDS instead of L2 bandwidth.
//
// Rows outside the grid: chunks wholly past row M-1 are identity rows (no
// couplings, state zero); the tail of the chunk holding row M-1 keeps its
// natural closed-form coefficients, and since the coupling C of row M-1 to
// row M is zero the real rows never see them (that padding is driven one
// way only).  Row 0 has no left coupling (A = 0).  HI: row M-1 is an
// interior row of its chunk (M not a multiple of MC), whose C' is zeroed by
// a select.
#pragma once

#include "bsp_common.hpp"
#include "bsp_tridiag.hpp"

namespace bsp {

constexpr int kRcRegStages = 4;  // interface-reduction stages with multipliers in registers
constexpr double kPcrTruncationRc = 8.673617379884035e-19;  // 2^-60

// Scaled closed-form row coefficients of thread p's chunk (grid index
// j = J + q of row q, J = p MC + 1): A'(j) = j (c2 j + c1), C'(j) = j (c2 j - c1).
// The sweeps walk j up or down by one (exact: j is an integer), so a
// coefficient costs an add, an FMA and a multiply.
struct RcRows {
    double c2, c1, J;
    // pad: a chunk wholly outside the grid (identity rows: no couplings)
    __device__ __forceinline__ void init(double s2, double r, double h, double kap, int p, int MC,
                                         bool pad) {
        c2 = pad ? 0.0 : -h * s2 / (2.0 * kap);
        c1 = pad ? 0.0 : h * r / (2.0 * kap);
        J = (double)(p * MC + 1);
    }
    __device__ __forceinline__ double A(double j) const { return j * fma(c2, j, c1); }
    __device__ __forceinline__ double C(double j) const { return j * fma(c2, j, -c1); }
    __device__ __forceinline__ double Aq(int q) const { return A(J + (double)q); }
    __device__ __forceinline__ double Cq(int q) const { return C(J + (double)q); }
};

template <int T, int MC, bool HI>
struct BlockTriR {
    static constexpr int LOGT = ilog2(T);
    static constexpr int NI = MC - 1;
    static_assert(MC >= 4, "chunks of at least four rows");

    const double* ku;  // LDS [NI][T]: kappa / u_q
    Forcing fc;
    RcRows rows;
    double aq, cq, invB, kap, mu, a0s, cNI;
    double k1[kRcRegStages], k2[kRcRegStages];
    double Ar, Br, Cr;  // reduced interface row after kRcRegStages stages
    int p, nst, zq;

    __device__ __forceinline__ double Cz(const RcRows& rw, double j, int q) const {
        const double c = rw.C(j);
        return (HI && q == zq) ? 0.0 : c;
    }

    // Factorisation, responses and interface reduction for one (option,
    // theta, dt); h = theta*dt > 0, e = (1-theta)*dt.  Whole block.
    // ku_lds: NI*T doubles (each thread writes and reads only its own column);
    // lds: 3T doubles of scratch.
    __device__ __forceinline__ void setup(double s2, double r, double h, double e, int M,
                                          double* ku_lds, double* lds) {
        p = threadIdx.x;
        kap = 1.0 + e / h;
        mu = e / h;
        const int i0 = p * MC;
        const bool pad = i0 >= M;
        rows.init(s2, r, h, kap, p, MC, pad);
        const bool owner = p == (M - 1) / MC;
        zq = (HI && owner) ? (M - 1) % MC : -1;
        auto Cs = [&](int q) { return (i0 + q == M - 1) ? 0.0 : rows.Cq(q); };
        auto Bs = [&](int q) {
            const double j = (double)(i0 + q + 1);
            return (pad ? 1.0 : fma(h, fma(s2 * j, j, r), 1.0)) / kap;
        };
        // LU of the interior rows with the step's own multipliers
        double* kuc = ku_lds + p;
        double kp = 1.0 / Bs(0);
        kuc[0] = kp;
        for (int q = 1; q < NI; ++q) {
            const double l = rows.Aq(q) * kp;
            kp = 1.0 / fma(-l, Cs(q - 1), Bs(q));
            kuc[q * T] = kp;
        }
        ku = ku_lds;
        // end values of the responses v (to the left interface value) and w
        // (to the right one), by the step's correction sweeps
        a0s = (i0 == 0) ? 0.0 : rows.Aq(0);
        cNI = Cs(NI - 1);
        double vlast, wlast, vfirst, wfirst;
        {
            double g[NI];
            g[0] = -a0s;
            for (int q = 1; q < NI; ++q) g[q] = -(rows.Aq(q) * kuc[(q - 1) * T]) * g[q - 1];
            double vv = kuc[(NI - 1) * T] * g[NI - 1];
            double ww = kuc[(NI - 1) * T] * -cNI;
            vlast = vv;
            wlast = ww;
            for (int q = NI - 2; q >= 0; --q) {
                vv = kuc[q * T] * fma(-Cs(q), vv, g[q]);
                ww = kuc[q * T] * (-Cs(q) * ww);
            }
            vfirst = vv;
            wfirst = ww;
        }

        // interface row i = i0 + MC - 1 (unscaled coefficients)
        const int i = i0 + MC - 1;
        aq = kap * rows.Aq(MC - 1);
        const double bq = kap * Bs(MC - 1);
        cq = (i == M - 1) ? 0.0 : kap * rows.Cq(MC - 1);
        lds[p] = vfirst;
        lds[T + p] = wfirst;
        __syncthreads();
        const double vF = (p + 1 < T) ? lds[p + 1] : 0.0;
        const double wF = (p + 1 < T) ? lds[T + p + 1] : 0.0;
        __syncthreads();
        double A_ = aq * vlast;
        double B_ = bq + aq * wlast + cq * vF;
        double C_ = cq * wF;
        nst = LOGT;
        bool done = false;
#pragma unroll
        for (int k = 0; k < kRcRegStages; ++k) k1[k] = k2[k] = 0.0;
        Ar = A_;
        Br = B_;
        Cr = C_;
        for (int k = 0; k < LOGT; ++k) {
            if (k == kRcRegStages) {
                Ar = A_;
                Br = B_;
                Cr = C_;
            }
            const int mine = ((fabs(A_) + fabs(C_)) / fabs(B_)) <= kPcrTruncationRc;
            if (__syncthreads_and(mine)) {
                nst = k;
                done = true;
            }
            if (done) break;
            const int s = 1 << k;
            lds[p] = A_;
            lds[T + p] = B_;
            lds[2 * T + p] = C_;
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
            const double m1 = (p - s >= 0) ? A_ / Bm : 0.0;
            const double m2 = (p + s < T) ? C_ / Bp : 0.0;
#pragma unroll
            for (int kk = 0; kk < kRcRegStages; ++kk)
                if (kk == k) {
                    k1[kk] = m1;
                    k2[kk] = m2;
                }
            const double An = -m1 * Am, Cn = -m2 * Cp, Bn = B_ - m1 * Cm - m2 * Ap;
            A_ = An;
            B_ = Bn;
            C_ = Cn;
        }
        nst = wave_uniform(nst);
        invB = 1.0 / B_;
        double al, be, ga, gammaM;
        op_row(s2, r, 1.0, al, be, ga);
        const double alpha1 = al;
        op_row(s2, r, (double)M, al, be, ga);
        gammaM = ga;
        fc.init(p, MC, M, alpha1, gammaM, kap);
        __syncthreads();  // lds is scratch of the steps from here on
    }

    // One step V <- A^{-1}(kappa V + f) - mu V (see BlockTri::step).  Pass 1:
    // forward and backward sweep of the interior rows with zero interface
    // values (y), interface reduction; pass 2: forward and backward sweep of
    // the correction caused by the interface values (zl on row 0, z on row
    // NI-1), added to the state.  lds: 4T doubles.
    template <bool EX>
    __device__ __forceinline__ void step(double (&V)[MC], double flo, double fhi,
                                         double* lds) const {
        // Opaque per step: the row coefficients and the pivot reads are the
        // same every step, and hoisting them out of the step loop would take
        // 2 x 31 doubles of registers per thread (the footprint this solver
        // avoids); recomputing and rereading them is what it is built for.
        RcRows rw = rows;
        int col = p;
        asm volatile("" : "+v"(rw.c2), "+v"(rw.c1), "+v"(rw.J), "+v"(col));
        const double* kuc = ku + col;
        double d[MC];
        fc.rhs(V, flo, fhi, d);
        double kum = kuc[0];
        double j = rw.J;
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            j += 1.0;
            const double l = rw.A(j) * kum;
            kum = kuc[q * T];
            d[q] = fma(-l, d[q - 1], d[q]);
        }
        double y = d[NI - 1] * kum;
        const double yl = y;
        V[NI - 1] = EX ? fma(-mu, V[NI - 1], y) : y;
        // the backward sweep reads the pivots again (not kept from the forward one)
        int colb = p;
        asm volatile("" : "+v"(colb));
        const double* kucb = ku + colb;
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) {
            j -= 1.0;
            y = kucb[q * T] * fma(-Cz(rw, j, q), y, d[q]);
            V[q] = EX ? fma(-mu, V[q], y) : y;
        }
        // interface rows: y_0 of the next chunk, then the reduced system
        double* ybuf = lds;
        double* pb0 = lds + T;
        double* pb1 = lds + 2 * T;
        double* zbuf = lds + 3 * T;
        ybuf[p] = y;
        __syncthreads();
        const double yF = (p + 1 < T) ? ybuf[p + 1] : 0.0;
        double D = fma(kap, V[MC - 1], fma(fc.bhiD, fhi, fma(-aq, yl, -cq * yF)));
        const double rz = EX ? -mu * V[MC - 1] : 0.0;
#pragma unroll
        for (int k = 0; k < kRcRegStages; ++k) {
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
        if (nst > kRcRegStages) {
            // stiff steps: the reduced coefficients travel with D and the
            // multipliers are recomputed (the set-up's operations exactly)
            double A_ = Ar, B_ = Br, C_ = Cr;
            for (int k = kRcRegStages; k < nst; ++k) {
                const int s = 1 << k;
                __syncthreads();  // ybuf and zbuf are free (read above / written below)
                ybuf[p] = A_;
                pb0[p] = B_;
                zbuf[p] = C_;
                pb1[p] = D;
                __syncthreads();
                double Am = 0.0, Bm = 1.0, Cm = 0.0, Dm = 0.0;
                double Ap = 0.0, Bp = 1.0, Cp = 0.0, Dp = 0.0;
                if (p - s >= 0) {
                    Am = ybuf[p - s];
                    Bm = pb0[p - s];
                    Cm = zbuf[p - s];
                    Dm = pb1[p - s];
                }
                if (p + s < T) {
                    Ap = ybuf[p + s];
                    Bp = pb0[p + s];
                    Cp = zbuf[p + s];
                    Dp = pb1[p + s];
                }
                const double m1 = (p - s >= 0) ? A_ / Bm : 0.0;
                const double m2 = (p + s < T) ? C_ / Bp : 0.0;
                D = fma(-m1, Dm, fma(-m2, Dp, D));
                const double An = -m1 * Am, Cn = -m2 * Cp, Bn = B_ - m1 * Cm - m2 * Ap;
                A_ = An;
                B_ = Bn;
                C_ = Cn;
            }
            __syncthreads();  // before zbuf is written
        }
        const double z = D * invB;
        zbuf[p] = z;
        __syncthreads();
        const double zl = (p > 0) ? zbuf[p - 1] : 0.0;
        // pass 2: the interior rows' correction for the interface values
        RcRows r2 = rows;
        int col2 = p;
        asm volatile("" : "+v"(r2.c2), "+v"(r2.c1), "+v"(r2.J), "+v"(col2));
        const double* kub = ku + col2;
        double t = -a0s * zl;
        d[0] = t;
        kum = kub[0];
        j = r2.J;
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            j += 1.0;
            const double l = r2.A(j) * kum;
            kum = kub[q * T];
            t = -l * t;
            d[q] = t;
        }
        t = kum * fma(-cNI, z, d[NI - 1]);
        V[NI - 1] += t;
        int col2b = p;
        asm volatile("" : "+v"(col2b));
        const double* kubb = ku + col2b;
#pragma unroll
        for (int q = NI - 2; q >= 0; --q) {
            j -= 1.0;
            t = kubb[q * T] * fma(-Cz(r2, j, q), t, d[q]);
            V[q] += t;
        }
        V[MC - 1] = z + rz;
    }
};

}  // namespace bsp
