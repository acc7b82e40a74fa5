// Three-level tridiagonal block solver for blocks of W wavefronts (T = 64 W
// threads), the multi-wavefront counterpart of BlockTri's one-wavefront path.
//
// Level 1 (thread): as in BlockTri, thread c owns MC consecutive nodes whose
//   interior is eliminated locally; what remains is one interface unknown
//   z_c per thread with rows  A_c z_{c-1} + B_c z_c + C_c z_{c+1} = D_c.
// Level 2 (wavefront): within wavefront w, lanes 0..62 are "interior" again
//   and lane 63 is the wavefront's interface unknown Z_w.  The interior rows
//   are solved by truncated parallel cyclic reduction across the lanes (DPP
//   and ds_bpermute only, no LDS, no barrier):  z = yt + Z_{w-1} vt + Z_w wt,
//   with constant responses vt, wt to the two neighbouring interface unknowns.
// Level 3 (block): the W rows of the interface unknowns,
//   alpha_w Z_{w-1} + beta_w Z_w + gamma_w Z_{w+1} = rho_w,
//   are assembled from three values per wavefront exchanged through LDS
//   (one block barrier per step) and solved redundantly by every lane with
//   precomputed Thomas factors.
// Per step: one barrier, against log2(T) + 2 for a flat reduction over LDS.
#pragma once

#include "bsp_common.hpp"
#include "bsp_tridiag.hpp"

namespace bsp {

template <int W, int MC>
struct BlockTriH {
    static_assert(W >= 2, "use BlockTri for one wavefront");
    static_assert(MC >= 2, "at least one interior row per chunk");
    static constexpr int T = 64 * W;
    static constexpr int NI = MC - 1;
    static constexpr int NS = 6;  // intra-wavefront reduction stages (strides 1..32)

    static constexpr int kThreads = T;

    ChunkLU<MC> lu;
    Forcing fc;
    double aq, cq, kap, mu;
    double k1[NS], k2[NS], invB2, vt, wt;  // level 2
    double A63;                            // lane 63: its own row's A
    // pipelined steps: level 1 as in BlockTri (forward-swept responses,
    // kappa-scaled sweep multipliers and couplings, forcing coefficients)
    double al[NI], be[NI], lh[NI], ch[NI];
    double aqk, cqk, blok, bhik;
    int p, lane, wave, nst2;
    mutable int par;  // step parity: double-buffered exchange slots

    __device__ __forceinline__ int stages() const { return nst2; }

    __device__ __forceinline__ double up(double x, int s) const {
        if (s == 1) return dpp_from_prev(x);
        if (s == 2) return dpp_prev_n<2>(x);
        if (s == 4) return dpp_prev_n<4>(x);
        return lane_fetch(x, lane - s);
    }
    __device__ __forceinline__ double down(double x, int s) const {
        if (s == 1) return dpp_from_next(x);
        if (s == 2) return dpp_next_n<2>(x);
        if (s == 4) return dpp_next_n<4>(x);
        return lane_fetch(x, lane + s);
    }

    // Level-2 reduction of one right-hand side (zero at lane 63).  Lanes whose
    // partner lies outside the wavefront have zero multipliers.
    __device__ __forceinline__ double wave_reduce(double D) const {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (k < nst2) {
                const int s = 1 << k;
                const double Dm = up(D, s);
                const double Dp = down(D, s);
                D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
            }
        }
        return D;
    }

    // LDS regions (doubles): setup scratch [0, 2T); exchange slots
    // [2T, 2T + 6W); level-3 constants [3T, 3T + 5W).  The last two persist
    // between steps.
    __device__ __forceinline__ void setup(double s2, double r, double h, double e, int M,
                                          double* lds) {
        p = threadIdx.x;
        lane = p & 63;
        wave = wave_uniform(p >> 6);
        par = 0;
        kap = 1.0 + e / h;
        mu = e / h;
        double a[MC], b[MC], c[MC], alpha1, gammaM;
        chunk_rows<MC>(s2, r, h, M, p, a, b, c, alpha1, gammaM);
        lu.factor(a, b, c, kap);
        fc.init(p, MC, M, alpha1, gammaM, kap);
        aq = a[MC - 1];
        cq = c[MC - 1];
        const double bq = b[MC - 1];

        // level-1 row of chunk p (needs the next chunk's v[0], w[0])
        lds[p] = lu.v[0];
        lds[T + p] = lu.w[0];
        lds[2 * T + p] = lu.ku[0];
        __syncthreads();
        const double vF = (p + 1 < T) ? lds[p + 1] : 0.0;
        const double wF = (p + 1 < T) ? lds[T + p + 1] : 0.0;
        const double kuF = (p + 1 < T) ? lds[2 * T + p + 1] : 0.0;
        __syncthreads();
        // level-1 tables of the pipelined steps (see BlockTri::setup)
        al[0] = lu.v[0];
        be[0] = lu.w[0];
#pragma unroll
        for (int q = 1; q < NI; ++q) {
            al[q] = fma(-lu.l[q], al[q - 1], lu.v[q]);
            be[q] = fma(-lu.l[q], be[q - 1], lu.w[q]);
        }
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            lh[q] = (q > 0) ? lu.l[q] * lu.ku[q - 1] / lu.ku[q] : 0.0;
            ch[q] = (q < NI - 1) ? lu.cu[q] * lu.ku[q + 1] / lu.ku[q] : 0.0;
        }
        aqk = aq * lu.ku[NI - 1];
        cqk = cq * kuF;
        blok = fc.blo / lu.ku[0];
        double kr = 1.0;
#pragma unroll
        for (int q = 0; q < NI; ++q)
            if (q == fc.r_hi) kr = lu.ku[q];
        bhik = fc.bhi / kr;
        const double A = aq * lu.v[NI - 1];
        const double B = bq + aq * lu.w[NI - 1] + cq * vF;
        const double C = cq * wF;

        // level 2: lanes 0..62 without their couplings outside the wavefront;
        // lane 63 is an identity row
        double A2 = (lane == 0) ? 0.0 : A;
        double B2 = B;
        double C2 = (lane == 62) ? 0.0 : C;
        if (lane == 63) {
            A2 = 0.0;
            B2 = 1.0;
            C2 = 0.0;
        }
        nst2 = NS;
        bool done = false;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            k1[k] = 0.0;
            k2[k] = 0.0;
            if (!done && __all(((fabs(A2) + fabs(C2)) / fabs(B2)) <= kPcrTruncation)) {
                nst2 = k;
                done = true;
            }
            if (!done) {
                const int s = 1 << k;
                // exchanges first, on every lane (a DPP or bpermute under a
                // partial exec mask reads nothing from the disabled lanes)
                const bool lo = lane - s >= 0, hi = lane + s < 64;
                const double Au = up(A2, s), Bu = up(B2, s), Cu = up(C2, s);
                const double Ad = down(A2, s), Bd = down(B2, s), Cd = down(C2, s);
                const double Am = lo ? Au : 0.0, Bm = lo ? Bu : 1.0, Cm = lo ? Cu : 0.0;
                const double Ap = hi ? Ad : 0.0, Bp = hi ? Bd : 1.0, Cp = hi ? Cd : 0.0;
                const double m1 = lo ? A2 / Bm : 0.0;
                const double m2 = hi ? C2 / Bp : 0.0;
                k1[k] = m1;
                k2[k] = m2;
                const double An = -m1 * Am, Cn = -m2 * Cp, Bn = B2 - m1 * Cm - m2 * Ap;
                A2 = An;
                B2 = Bn;
                C2 = Cn;
            }
        }
        nst2 = wave_uniform(nst2);
        invB2 = 1.0 / B2;
        vt = wave_reduce(lane == 0 ? -A : 0.0) * invB2;
        wt = wave_reduce(lane == 62 ? -C : 0.0) * invB2;
        if (lane == 63) {
            vt = 0.0;
            wt = 0.0;
        }

        // level 3: the interface rows of the wavefronts
        const double vt62 = dpp_from_prev(vt), wt62 = dpp_from_prev(wt);
        if (lane == 0) {
            lds[2 * wave] = vt;
            lds[2 * wave + 1] = wt;
        }
        __syncthreads();
        A63 = A;
        const double vt0n = (wave + 1 < W) ? lds[2 * (wave + 1)] : 0.0;
        const double wt0n = (wave + 1 < W) ? lds[2 * (wave + 1) + 1] : 0.0;
        __syncthreads();
        double* pub = lds + 2 * T;  // alpha, beta, gamma, cq63, C63 per wavefront
        if (lane == 63) {
            pub[wave] = A * vt62;
            pub[W + wave] = B + A * wt62 + C * vt0n;
            pub[2 * W + wave] = C * wt0n;
            pub[3 * W + wave] = cq;
            pub[4 * W + wave] = C;
        }
        __syncthreads();
        if (p == 0) {
            double* L3 = lds + 3 * T;  // l3, iu3, g3, cq63, C63
            double uu = pub[W];
            L3[0] = 0.0;
            L3[W] = 1.0 / uu;
            for (int q = 1; q < W; ++q) {
                const double l = pub[q] / uu;
                uu = pub[W + q] - l * pub[2 * W + q - 1];
                L3[q] = l;
                L3[W + q] = 1.0 / uu;
            }
            for (int q = 0; q < W; ++q) {
                L3[2 * W + q] = pub[2 * W + q];
                L3[3 * W + q] = pub[3 * W + q];
                L3[4 * W + q] = pub[4 * W + q];
            }
        }
        __syncthreads();
    }

    // ---------------------------------------------------------------------
    // Pipelined steps (Crank-Nicolson, mu = 1, and implicit Euler, mu = 0):
    // level 1 exactly as BlockTri::pipe_step (forward sweep of the next step
    // during the interface solve, sweeps in kappa-scaled variables); the
    // interface values come from levels 2 and 3 as in step(), and the next
    // step's forward sweep runs between the publication of the wavefront
    // interface rows and the block barrier.
    struct Pipe {
        double A[MC];
        double z, zl;
        double Vi;
    };

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

    // Level-2 reduction with a compile-time stage count (NST >= 0) or nst2.
    template <int NST>
    __device__ __forceinline__ double wave_reduce_n(double D) const {
        if constexpr (NST >= 0) {
#pragma unroll
            for (int k = 0; k < NST; ++k) {
                const int s = 1 << k;
                const double Dm = up(D, s);
                const double Dp = down(D, s);
                D = fma(-k1[k], Dm, fma(-k2[k], Dp, D));
            }
            return D;
        } else {
            return wave_reduce(D);
        }
    }

    template <bool EX, int NST, bool HI>
    __device__ __forceinline__ void pipe_step(Pipe& P, double flo, double fhi, double flo_n,
                                              double fhi_n, double* lds) const {
        double y[NI], xi[NI];
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
        // level 1 -> 2 (lane 63: the next chunk's term enters at level 3)
        const double xF = dpp_from_next(xi[0]);
        const double D = fma(kap, P.Vi, fma(fc.bhiD, fhi, fma(-aqk, xi[NI - 1], -cqk * xF)));
        const double yt = wave_reduce_n<NST>(lane == 63 ? 0.0 : D) * invB2;
        const double yt62 = dpp_from_prev(yt);
        // level 3: publish this wavefront's interface row terms
        double* slot = lds + 2 * T + par * 3 * W;
        par ^= 1;
        if (lane == 63) slot[wave] = fma(-A63, yt62, D);
        if (lane == 0) {
            slot[W + wave] = lu.ku[0] * xi[0];
            slot[2 * W + wave] = yt;
        }
        // next step's forward sweep, independent of the interface values
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
        __syncthreads();
        double Zm, Z0;
        level3(slot, lds, Zm, Z0);
        const double z = (lane == 63) ? Z0 : fma(Zm, vt, fma(Z0, wt, yt));
        double zl = dpp_from_prev(z);
        if (lane == 0) zl = Zm;
        P.z = z;
        P.zl = zl;
        P.Vi = EX ? z - P.Vi : z;
    }

    __device__ __forceinline__ void pipe_end(const Pipe& P, double (&V)[MC]) const {
        double y[MC];
#pragma unroll
        for (int q = 0; q < NI; ++q) y[q] = fma(P.zl, al[q], fma(P.z, be[q], P.A[q]));
        V[0] = y[0];
#pragma unroll
        for (int q = 1; q < NI; ++q) V[q] = fma(lu.l[q], y[q - 1], y[q]);
        V[MC - 1] = P.Vi;
    }

    // Level 3 from a filled exchange slot: the wavefront interface values
    // Z_{w-1} (Zm) and Z_w (Z0) of this wavefront (every lane solves the W
    // rows with the precomputed Thomas factors).
    __device__ __forceinline__ void level3(const double* slot, const double* lds, double& Zm,
                                           double& Z0) const {
        const double* L3 = lds + 3 * T;
        double Z[W];
        double rp = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            double rho = slot[q];
            if (q + 1 < W) rho = fma(-L3[3 * W + q], slot[W + q + 1],
                                     fma(-L3[4 * W + q], slot[2 * W + q + 1], rho));
            rp = (q == 0) ? rho : fma(-L3[q], rp, rho);
            Z[q] = rp;
        }
        Z[W - 1] *= L3[W + W - 1];
#pragma unroll
        for (int q = W - 2; q >= 0; --q) Z[q] = (Z[q] - L3[2 * W + q] * Z[q + 1]) * L3[W + q];
        Zm = 0.0;
        Z0 = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (q == wave - 1) Zm = Z[q];
            if (q == wave) Z0 = Z[q];
        }
    }

    // One step (see BlockTri::step).  Contains one block barrier.
    template <bool EX>
    __device__ __forceinline__ void step(double (&V)[MC], double flo, double fhi,
                                         double* lds) const {
        double d[MC];
        fc.rhs(V, flo, fhi, d);
        lu.solve(d);

        // level 1 -> level 2
        const double yF = dpp_from_next(d[0]);  // lane 63: 0, its term enters at level 3
        const double D = fma(kap, V[MC - 1], fma(fc.bhiD, fhi, fma(-aq, d[NI - 1], -cq * yF)));
        const double yt = wave_reduce(lane == 63 ? 0.0 : D) * invB2;
        const double yt62 = dpp_from_prev(yt);

        // level 3: publish, one barrier, solve
        double* slot = lds + 2 * T + par * 3 * W;
        par ^= 1;
        if (lane == 63) slot[wave] = fma(-A63, yt62, D);
        if (lane == 0) {
            slot[W + wave] = d[0];
            slot[2 * W + wave] = yt;
        }
        double rz = 0.0;
        if constexpr (EX) {
#pragma unroll
            for (int q = 0; q < NI; ++q) d[q] = fma(-mu, V[q], d[q]);
            rz = -mu * V[MC - 1];
        }
        __syncthreads();
        double Zm, Z0;
        level3(slot, lds, Zm, Z0);

        // back-substitution
        const double z = (lane == 63) ? Z0 : fma(Zm, vt, fma(Z0, wt, yt));
        double zl = dpp_from_prev(z);
        if (lane == 0) zl = Zm;
#pragma unroll
        for (int q = 0; q < NI; ++q) V[q] = fma(zl, lu.v[q], fma(z, lu.w[q], d[q]));
        V[MC - 1] = z + rz;
    }
};

}  // namespace bsp
