// Tridiagonal block solver for large grids (up to 16384 nodes on 512 threads)
// that keeps one coefficient field per node on chip and recomputes the rest.
//
// Same partition and implicit step form as BlockTri (each thread owns MC
// consecutive rows: MC-1 interior rows eliminated locally and one interface
// row; the interface system is reduced by truncated parallel cyclic
// reduction, here through LDS with one barrier per stage), but with 512
// threads of 16 or 32 rows nothing per row fits in registers beside the
// state, and nothing is read from global memory after the set-up:
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
// A sweep walks them by their differences (second differences are the
// constant 2 c2): up the chunk from A'_0, A'_1 - A'_0, down it from
// C'_{NI-1}, C'_{NI-1} - C'_{NI-2}, two adds per row.  The set-up takes the
// same walks, so the pivots and the steps see bitwise the same coefficients.
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
    // A'_0 and A'_1 - A'_0; next row: a += da, da += 2 c2
    __device__ __forceinline__ void startA(double& a, double& da) const {
        a = A(J);
        da = fma(c2, fma(2.0, J, 1.0), c1);
    }
    __device__ __forceinline__ void upA(double& a, double& da) const {
        a += da;
        da = fma(2.0, c2, da);
    }
    // C'_{n} and C'_{n} - C'_{n-1} for row n; next row down: c -= dc, dc -= 2 c2
    __device__ __forceinline__ void startC(int n, double& c, double& dc) const {
        const double jt = J + (double)n;
        c = C(jt);
        dc = fma(c2, fma(2.0, jt, -1.0), -c1);
    }
    __device__ __forceinline__ void downC(double& c, double& dc) const {
        c -= dc;
        dc = fma(-2.0, c2, dc);
    }
};

// Factorisation and interface data of one block (set-up); the steps are in
// BlockTriR below.
template <int T, int MC, bool HI>
struct RcFact {
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
        // the sweeps' coefficients: A'_q up the chunk, C'_q down it
        double Aw[NI], Cw[NI];
        {
            double a, da, c, dc;
            rows.startA(a, da);
            Aw[0] = a;
            for (int q = 1; q < NI; ++q) {
                rows.upA(a, da);
                Aw[q] = a;
            }
            rows.startC(NI - 1, c, dc);
            Cw[NI - 1] = c;
            for (int q = NI - 2; q >= 0; --q) {
                rows.downC(c, dc);
                Cw[q] = c;
            }
        }
        auto Cs = [&](int q) { return (i0 + q == M - 1) ? 0.0 : Cw[q]; };
        auto Bs = [&](int q) {
            const double j = (double)(i0 + q + 1);
            return (pad ? 1.0 : fma(h, fma(s2 * j, j, r), 1.0)) / kap;
        };
        // LU of the interior rows with the step's own multipliers
        double* kuc = ku_lds + p;
        double kp = 1.0 / Bs(0);
        kuc[0] = kp;
        for (int q = 1; q < NI; ++q) {
            const double l = Aw[q] * kp;
            kp = 1.0 / fma(-l, Cs(q - 1), Bs(q));
            kuc[q * T] = kp;
        }
        ku = ku_lds;
        // end values of the responses v (to the left interface value) and w
        // (to the right one), by the step's correction sweeps
        a0s = (i0 == 0) ? 0.0 : Aw[0];
        cNI = Cs(NI - 1);
        double vlast, wlast, vfirst, wfirst;
        {
            double g[NI];
            g[0] = -a0s;
            for (int q = 1; q < NI; ++q) g[q] = -(Aw[q] * kuc[(q - 1) * T]) * g[q - 1];
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
        aq = kap * rows.A(rows.J + (double)(MC - 1));
        const double bq = kap * Bs(MC - 1);
        cq = (i == M - 1) ? 0.0 : kap * rows.C(rows.J + (double)(MC - 1));
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

};

// The steps.  CN: Crank-Nicolson (kappa = 2, mu = 1 as constants).  SLOW:
// the interface reduction needs more than kRcRegStages stages (the kernel
// picks this instance when the set-up found so).
template <int T, int MC, bool HI, bool CN, bool SLOW>
struct BlockTriR : RcFact<T, MC, HI> {
    using F = RcFact<T, MC, HI>;
    using F::NI;
    using F::ku;
    using F::fc;
    using F::rows;
    using F::aq;
    using F::cq;
    using F::invB;
    using F::kap;
    using F::mu;
    using F::a0s;
    using F::cNI;
    using F::k1;
    using F::k2;
    using F::Ar;
    using F::Br;
    using F::Cr;
    using F::p;
    using F::nst;
    using F::zq;
    __device__ __forceinline__ explicit BlockTriR(const F& f) : F(f) {}

    // Pivot reads kPD rows ahead of their use (a ring of registers), so the
    // sweeps wait on LDS latency once per sweep instead of once per row pair.
    // Reads go in pairs of adjacent rows (one two-address LDS read each, whose
    // offsets reach every row without address arithmetic).
    static constexpr int kPD = NI >= 8 ? 8 : (NI & ~1);
    static_assert(NI >= 3, "paired pivot reads");

    // Forward sweep over rows 1..NI-1 with l_q = A'_q kappa/u_{q-1}:
    // body(q, l).  Returns kappa/u_{NI-1}.
    // Pivot of row q from two column bases (rows 0..15 and 16.. of this
    // thread's column), so every read's LDS offset fits the instruction.
    struct Col {
        const double* lo;
        const double* hi;
        __device__ __forceinline__ double operator[](int q) const {
            return q < 16 ? lo[q * T] : hi[(q - 16) * T];
        }
    };
    __device__ __forceinline__ Col col() const {
        int a = p, b = p + 16 * T;
        asm volatile("" : "+v"(a), "+v"(b));  // opaque: see step()
        return Col{ku + a, ku + b};
    }

    template <class Body>
    __device__ __forceinline__ double forward(const RcRows& rw, const Col& kuc,
                                              Body&& body) const {
        double kr[kPD];
#pragma unroll
        for (int i = 0; i < kPD; ++i) kr[i] = kuc[i];
        double a, da;
        rw.startA(a, da);
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            const double kprev = kr[(q - 1) % kPD];
            if ((q - 1) & 1) {  // rows q-2, q-1 consumed: their slots take rows q-2+kPD, q-1+kPD
                if (q - 2 + kPD < NI) kr[(q - 2) % kPD] = kuc[q - 2 + kPD];
                if (q - 1 + kPD < NI) kr[(q - 1) % kPD] = kuc[q - 1 + kPD];
            }
            rw.upA(a, da);
            body(q, a * kprev);
        }
        return kr[(NI - 1) % kPD];
    }

    // Backward sweep over rows NI-2..0: body(q, C'_q, kappa/u_q).
    template <class Body>
    __device__ __forceinline__ void backward(const RcRows& rw, const Col& kuc,
                                             Body&& body) const {
        constexpr int PB = NI - 1 >= kPD ? kPD : ((NI - 1) & ~1);
        static_assert(PB >= 2, "paired pivot reads");
        double kr[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) kr[i] = kuc[NI - 2 - i];
        double c, dc;
        rw.startC(NI - 1, c, dc);
#pragma unroll
        for (int e = 0; e < NI - 1; ++e) {  // q = NI-2-e
            const int q = NI - 2 - e;
            const double kq = kr[e % PB];
            if (e & 1) {  // rows of e-1, e consumed: their slots take the rows PB further down
                if (e - 1 + PB < NI - 1) kr[(e - 1) % PB] = kuc[q + 1 - PB];
                if (e + PB < NI - 1) kr[e % PB] = kuc[q - PB];
            }
            rw.downC(c, dc);
            body(q, (HI && q == zq) ? 0.0 : c, kq);
        }
    }

    // One step V <- A^{-1}(kappa V + f) - mu V (see BlockTri::step).  Pass 1:
    // forward and backward sweep of the interior rows with zero interface
    // values (y), interface reduction; pass 2: forward and backward sweep of
    // the correction caused by the interface values (zl on row 0, z on row
    // NI-1), added to the state.  lds: 4T doubles.
    template <bool EX>
    __device__ __forceinline__ void step(double (&V)[MC], double flo, double fhi,
                                         double* lds) const {
        // Opaque per sweep: the row coefficients and the pivot reads are the
        // same every step; hoisting them out of the step loop, or keeping
        // them from one sweep to the next, would take 2 x 31 doubles of
        // registers per thread (the footprint this solver avoids).
        // Recomputing and rereading them is what it is built for.
        const double kap_ = CN ? 2.0 : kap, mu_ = CN ? 1.0 : mu;
        RcRows rw = rows;
        asm volatile("" : "+v"(rw.c2), "+v"(rw.c1), "+v"(rw.J));
        double d[MC];
        fc.template rhs<MC, HI>(V, flo, fhi, d);
        const double kum = forward(rw, col(), [&](int q, double l) {
            d[q] = fma(-l, d[q - 1], d[q]);
        });
        double y = d[NI - 1] * kum;
        const double yl = y;
        V[NI - 1] = EX ? fma(-mu_, V[NI - 1], y) : y;
        backward(rw, col(), [&](int q, double c, double kq) {
            y = kq * fma(-c, y, d[q]);
            V[q] = EX ? fma(-mu_, V[q], y) : y;
        });
        // interface rows: y_0 of the next chunk, then the reduced system
        double* ybuf = lds;
        double* pb0 = lds + T;
        double* pb1 = lds + 2 * T;
        double* zbuf = lds + 3 * T;
        ybuf[p] = y;
        __syncthreads();
        const double yF = (p + 1 < T) ? ybuf[p + 1] : 0.0;
        double D = fma(kap_, V[MC - 1], fma(fc.bhiD, fhi, fma(-aq, yl, -cq * yF)));
        const double rz = EX ? -mu_ * V[MC - 1] : 0.0;
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
        if constexpr (SLOW) {
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
        asm volatile("" : "+v"(r2.c2), "+v"(r2.c1), "+v"(r2.J));
        double t = -a0s * zl;
        d[0] = t;
        const double kum2 = forward(r2, col(), [&](int q, double l) {
            t = -l * t;
            d[q] = t;
        });
        t = kum2 * fma(-cNI, z, d[NI - 1]);
        V[NI - 1] += t;
        backward(r2, col(), [&](int q, double c, double kq) {
            t = kq * fma(-c, t, d[q]);
            V[q] += t;
        });
        V[MC - 1] = z + rz;
    }
};

}  // namespace bsp
