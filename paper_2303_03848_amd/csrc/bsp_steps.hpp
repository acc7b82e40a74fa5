// Device building blocks shared by the single-option and batched kernels:
// chunk loads/stores, a run of theta-steps, and the serial Parareal sweep.
#pragma once

#include <type_traits>

#include "bsp_common.hpp"
#include "bsp_tridiag.hpp"
#include "bsp_tridiag_hier.hpp"

namespace bsp {

// Solver of a block shape: one wavefront -> BlockTri (lane exchanges only);
// several wavefronts -> BlockTriH (one block barrier per step).
template <int T, int MC>
struct SolverSel {
    using type = BlockTriH<T / 64, MC>;
};
template <int MC>
struct SolverSel<64, MC> {
    using type = BlockTri<64, MC>;
};
template <int T, int MC>
using Solver = typename SolverSel<T, MC>::type;

// Block shapes (threads, nodes per thread) the tridiagonal kernels are built for.
#define BSP_TRI_SHAPES(X) \
    X(64, 2) X(64, 4) X(64, 8) X(64, 16) X(128, 4) X(128, 8) X(128, 16) X(256, 4) X(256, 8) \
        X(256, 16) X(512, 8)

template <int T, int MC>
__device__ __forceinline__ void load_chunk(const double* __restrict__ src, int M, double (&V)[MC]) {
    const int i0 = threadIdx.x * MC;
#pragma unroll
    for (int q = 0; q < MC; ++q) V[q] = (i0 + q < M) ? src[i0 + q] : 0.0;
}

template <int T, int MC>
__device__ __forceinline__ void store_chunk(double* __restrict__ dst, int M, const double (&V)[MC]) {
    const int i0 = threadIdx.x * MC;
#pragma unroll
    for (int q = 0; q < MC; ++q)
        if (i0 + q < M) dst[i0 + q] = V[q];
}

// Chunk-major layout of a level of T * MC nodes (the overlapped solve on
// large grids keeps its internal copies of U, Fv, Gold and Vt this way):
// node p*MC + q sits at q*T + p, so that thread p's chunk is read and
// written by whole-wavefront accesses of 64 consecutive doubles; entries past
// the grid hold zero (written by the conversion, never stored to again).
template <int T, int MC>
__device__ __forceinline__ void load_cm(const double* __restrict__ src, double (&V)[MC]) {
#pragma unroll
    for (int q = 0; q < MC; ++q) V[q] = src[q * T + threadIdx.x];
}

template <int T, int MC>
__device__ __forceinline__ void store_cm(double* __restrict__ dst, int M, const double (&V)[MC]) {
    const int i0 = threadIdx.x * MC;
#pragma unroll
    for (int q = 0; q < MC; ++q)
        if (i0 + q < M) dst[q * T + threadIdx.x] = V[q];
}

// Steps per boundary-forcing table (two tables of this many doubles in LDS).
constexpr int kForceChunk = 1024;

// Shared memory of a tridiagonal kernel: the solver's 4T doubles followed by
// the two forcing tables.  Loads and stores of a whole system are staged
// through it so that consecutive lanes touch consecutive doubles (whole
// 128-byte lines per wavefront access) instead of MC-strided chunks; it is
// at least T * MC doubles for that.
template <int T, int MC>
constexpr int smem_doubles() {
    return 4 * T + 2 * kForceChunk > T * MC ? 4 * T + 2 * kForceChunk : T * MC;
}

// Barrier of the threads working on one system: the block, or (WAVE) one
// wavefront that works on its own system.
template <bool WAVE>
__device__ __forceinline__ void system_sync() {
    if constexpr (WAVE)
        wave_lds_sync();
    else
        __syncthreads();
}

// Whole-system load through shared memory (T * MC doubles of smem).  Uses
// all of smem: call it before the solver's setup.  WAVE: T = 64 and the
// system belongs to the calling wavefront alone.
template <int T, int MC, bool WAVE = false>
__device__ __forceinline__ void load_system(const double* __restrict__ src, int M, double (&V)[MC],
                                            double* smem) {
    static_assert(T * MC <= smem_doubles<T, MC>(), "staging area too small");
    static_assert(!WAVE || T == 64, "one wavefront");
    const int p = WAVE ? (threadIdx.x & 63) : threadIdx.x;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const int i = k * T + p;
        smem[i] = (i < M) ? src[i] : 0.0;
    }
    system_sync<WAVE>();
#pragma unroll
    for (int q = 0; q < MC; ++q) V[q] = smem[p * MC + q];
    system_sync<WAVE>();
}

// Whole-system store through shared memory, once the solver is done with it.
template <int T, int MC, bool WAVE = false>
__device__ __forceinline__ void store_system(double* __restrict__ dst, int M, const double (&V)[MC],
                                             double* smem) {
    static_assert(!WAVE || T == 64, "one wavefront");
    const int p = WAVE ? (threadIdx.x & 63) : threadIdx.x;
    system_sync<WAVE>();
#pragma unroll
    for (int q = 0; q < MC; ++q) smem[p * MC + q] = V[q];
    system_sync<WAVE>();
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const int i = k * T + p;
        if (i < M) dst[i] = smem[i];
    }
}

// `steps` theta-steps of size dt from tau0 on the state V (this block's system).
// EX: theta < 1 (the step has an explicit part); false for implicit Euler.
// The boundary forcing of each step, (1-theta) dt g(tau_m) + theta dt g(tau_{m+1})
// at S = 0 and S = S_max, is tabulated in LDS for a chunk of steps by all
// threads in parallel, so the sequential step loop evaluates no exponential.
// ftab: 2 * kForceChunk doubles of LDS.
template <class S>
struct IsWaveSolver : std::false_type {};
template <int MC>
struct IsWaveSolver<BlockTri<64, MC>> : std::true_type {};
// Solvers with the pipelined step interface (pipe_begin / pipe_step / pipe_end).
template <class S>
struct HasPipe : std::false_type {};
template <int MC>
struct HasPipe<BlockTri<64, MC>> : std::true_type {};
template <int W, int MC>
struct HasPipe<BlockTriH<W, MC>> : std::true_type {};

// One-wavefront blocks: the pipelined steps of BlockTri (pipe_begin /
// pipe_step / pipe_end), with the reduction stage count as a compile-time
// constant so that the reduction and the next forward sweep share one
// straight-line block.  The forcing tables here hold steps m0+1 .. m0+n+1
// (each step also needs the next step's forcing); entries past the last
// step are zero.
// POLL: the run checks *stop every kPollSteps steps (the flag is loaded one
// period before it is tested, so the load is never waited for) and returns
// false when it is set; the state is then left half-propagated.
constexpr int kPollSteps = 64;
// The plain step loop (large grids) runs kRunSteps steps between checks: the
// compiler spills part of the state around each check point (scratch
// traffic), so the runs are longer there (a check costs at most kRunSteps
// steps of latency once the flag is set).
constexpr int kRunSteps = 256;

// Forcing table of the pipelined steps for steps m0+1 .. m0+n+1 (entries
// past the last step are zero), built by the block's T threads.
template <int T, bool WAVE = false>
__device__ __forceinline__ void fill_piped_table(const OptionDev& o, double tau0, double dt,
                                                 int steps, double theta, int m0, int n,
                                                 double* ftab) {
    const double h = theta * dt, e = (1.0 - theta) * dt;
    system_sync<WAVE>();
    for (int i = WAVE ? (threadIdx.x & 63) : threadIdx.x; i <= n; i += T) {
        const int m = m0 + 1 + i;
        double lo = 0.0, hi = 0.0;
        if (m <= steps) {
            double lo0, hi0, lo1, hi1;
            dirichlet(o, exp(-o.r * (tau0 + (double)(m - 1) * dt)), lo0, hi0);
            dirichlet(o, exp(-o.r * (tau0 + (double)m * dt)), lo1, hi1);
            lo = fma(e, lo0, h * lo1);
            hi = fma(e, hi0, h * hi1);
        }
        ftab[i] = lo;
        ftab[kForceChunk + i] = hi;
    }
    system_sync<WAVE>();
}

// prefilled: the first table (m0 = 0) is already in ftab.
template <class S_t, int MC, bool EX, int NST, bool HI, bool POLL, bool WAVE>
__device__ __forceinline__ bool piped_run(const S_t& S, const OptionDev& o, double (&V)[MC],
                                          double tau0, double dt, int steps, double theta,
                                          bool homog, double* lds, double* ftab,
                                          const int* stop, bool prefilled) {
    constexpr int T = S_t::kThreads, CH = kForceChunk - 1;
    auto fill = [&](int m0, int n) {  // entries i = 0..n: step m0 + 1 + i
        fill_piped_table<T, WAVE>(o, tau0, dt, steps, theta, m0, n, ftab);
    };
    typename S_t::Pipe P;
    int n = min(CH, steps);
    if (!homog && !prefilled) fill(0, n);
    S.pipe_begin(V, homog ? 0.0 : ftab[0], homog ? 0.0 : ftab[kForceChunk], P);
    int sv = 0;
    for (int m0 = 0; m0 < steps;) {
        double lo = homog ? 0.0 : ftab[0], hi = homog ? 0.0 : ftab[kForceChunk];
        auto run = [&](int i0, int i1) {
            for (int i = i0; i < i1; ++i) {
                const double lo_n = homog ? 0.0 : ftab[i + 1];
                const double hi_n = homog ? 0.0 : ftab[kForceChunk + i + 1];
                S.template pipe_step<EX, NST, HI>(P, lo, hi, lo_n, hi_n, lds);
                lo = lo_n;
                hi = hi_n;
            }
        };
        if constexpr (POLL) {
            for (int i0 = 0; i0 < n; i0 += kPollSteps) {
                if (sv) return false;
                if constexpr (T == 64)
                    sv = pipe_load(stop);  // one wavefront: the loaded value is uniform
                else
                    sv = __syncthreads_or(pipe_load(stop) != 0);  // the same decision in every wavefront
                run(i0, min(n, i0 + kPollSteps));
            }
        } else {
            run(0, n);
        }
        m0 += n;
        if (m0 < steps) {
            n = min(CH, steps - m0);
            if (!homog) fill(m0, n);
        }
    }
    S.pipe_end(P, V);
    return true;
}

// On several wavefronts the pipelined steps pay off over a run of steps; a
// single step (the coarse propagator) takes the plain step there.
constexpr int kPipeMinSteps = 2;

// True when theta_steps takes the pipelined path.  A block-level run on one
// wavefront takes it for any step count (the form that generates the best
// code for the standalone fine kernel); a wavefront working alone (WAVE)
// and several wavefronts need kPipeMinSteps.
template <bool EX, bool WAVE = false, class Solver>
__device__ __forceinline__ bool piped_path(const Solver& S, int steps) {
    if constexpr (IsWaveSolver<Solver>::value && !WAVE) {
        (void)steps;
        return !EX || S.mu == 1.0;
    } else if constexpr (HasPipe<Solver>::value) {
        return (!EX || S.mu == 1.0) && steps >= kPipeMinSteps;
    }
    return false;
}

// Runs `steps` theta-steps on V.  POLL: check *stop every kPollSteps steps
// and return false once it is set (the same decision in every thread).  prefilled: on the pipelined path the
// first forcing table is already in ftab (fill_piped_table with m0 = 0).
// WAVE: the calling wavefront works on this system alone (one-wavefront
// solver, Crank-Nicolson or implicit Euler).
template <int T, int MC, bool EX, class Solver, bool POLL = false, bool WAVE = false>
__device__ __forceinline__ bool theta_steps(const Solver& S, const OptionDev& o,
                                            double (&V)[MC], double tau0, double dt, int steps,
                                            double theta, bool homog, double* lds, double* ftab,
                                            const int* stop = nullptr, bool prefilled = false) {
    static_assert(!WAVE || IsWaveSolver<Solver>::value, "wavefront-level runs need BlockTri");
    // The pipelined steps cover mu = 1 (Crank-Nicolson) and mu = 0 (implicit
    // Euler) (on several wavefronts: runs of kPipeMinSteps or more); the rest
    // takes the plain step loop.
    if constexpr (HasPipe<Solver>::value) if (piped_path<EX, WAVE>(S, steps)) {
        // HI: row M-1 lies inside a chunk (grid not a multiple of MC) and
        // carries forcing; homogeneous runs have none.
        const bool hi = !homog && S.fc.r_hi != MC - 1;
#define BSP_RUN(NST_, HI_)                                                                  \
    return piped_run<Solver, MC, EX, NST_, HI_, POLL, WAVE>(S, o, V, tau0, dt, steps, theta, \
                                                            homog, lds, ftab, stop, prefilled)
        if (hi) {
            switch (S.stages()) {
                case 0: BSP_RUN(0, true);
                case 1: BSP_RUN(1, true);
                case 2: BSP_RUN(2, true);
                case 3: BSP_RUN(3, true);
                default: BSP_RUN(-1, true);
            }
        } else {
            switch (S.stages()) {
                case 0: BSP_RUN(0, false);
                case 1: BSP_RUN(1, false);
                case 2: BSP_RUN(2, false);
                case 3: BSP_RUN(3, false);
                default: BSP_RUN(-1, false);
            }
        }
#undef BSP_RUN
    }
    const double h = theta * dt, e = (1.0 - theta) * dt;
    int sv = 0;
    for (int m0 = 0; m0 < steps; m0 += kForceChunk) {
        const int nch = min(kForceChunk, steps - m0);
        if (!homog) {
            system_sync<WAVE>();  // the previous chunk's table has been consumed
            for (int i = WAVE ? (threadIdx.x & 63) : threadIdx.x; i < nch; i += T) {
                const int mm = m0 + i;
                double lo0, hi0, lo1, hi1;
                dirichlet(o, exp(-o.r * (tau0 + (double)mm * dt)), lo0, hi0);
                dirichlet(o, exp(-o.r * (tau0 + (double)(mm + 1) * dt)), lo1, hi1);
                ftab[i] = fma(e, lo0, h * lo1);
                ftab[kForceChunk + i] = fma(e, hi0, h * hi1);
            }
            system_sync<WAVE>();
        }
        double flo_n = homog ? 0.0 : ftab[0];
        double fhi_n = homog ? 0.0 : ftab[kForceChunk];
        // POLL: runs of kRunSteps steps with the check between them, so the
        // step loop itself carries no test
        for (int i0 = 0; i0 < nch; i0 += kRunSteps) {
            if constexpr (POLL) {  // the same decision in every thread of the system
                if (sv) return false;
                if constexpr (WAVE || T == 64)
                    sv = __builtin_amdgcn_readfirstlane(pipe_load(stop));
                else
                    sv = __syncthreads_or(pipe_load(stop) != 0);
            }
            const int i1 = min(nch, i0 + kRunSteps);
            for (int i = i0; i < i1; ++i) {
                const double flo = flo_n, fhi = fhi_n;
                if (!homog && i + 1 < nch) {
                    flo_n = ftab[i + 1];
                    fhi_n = ftab[kForceChunk + i + 1];
                }
                S.template step<EX>(V, flo, fhi, lds);
            }
        }
    }
    return true;
}

// Staged correction of one slice (chunks of MC >= 8 nodes per thread, where
// a chunk-order access puts a whole wavefront on 64 different cache lines).
// The coarse values g, in chunk order (thread p holds nodes p*MC ..
// p*MC + MC-1), go through shared memory in rows of MC + 1 doubles (the pad
// keeps both access orders free of bank conflicts); consecutive threads then
// read and write consecutive nodes of Fv, Gold and U; the new values come
// back to chunk order in g (zero past the grid); uo1 holds the old values of
// U[n+1], un1 receives the new ones.  predict: U[n+1] = Gold[n] = g and g is
// left as it is.  A pass covers the chunks of
// staged_chunks<T, MC>() threads (at most 4096 nodes), so the staging area is
// staged_doubles<T, MC>() doubles of `stage`, which the forcing tables may
// share (they are refilled by every run of steps; barriers separate the two).
template <int T, int MC>
constexpr int staged_chunks() {
    return T * MC <= 4096 ? T : 4096 / MC;
}
template <int T, int MC>
constexpr int staged_doubles() {
    return staged_chunks<T, MC>() * (MC + 1);
}
// Shared memory of a sweep kernel: the solver's 4T doubles (which hold
// factors kept from the setup: the staging area stays clear of them), then
// the forcing tables with the staging area of the correction over them.
template <int T, int MC>
constexpr int sweep_smem_doubles() {
    return 4 * T +
           (2 * kForceChunk > staged_doubles<T, MC>() ? 2 * kForceChunk : staged_doubles<T, MC>());
}

// The coarse value of slice n at node i, by coarse kind:
//   kCoarseSolve:  G = g (the solve's result);
//   kCoarseNet:    G = Vt_{n+1} (the network alone; g is not used);
//   kCoarseNetDev: G = Vt_{n+1} + g (g: the solved deviation from the network),
//                  and the state carried to the next slice is the new
//                  iterate's deviation U[n+1] - Vt_{n+1}.
enum { kCoarseSolve = 0, kCoarseNet = 1, kCoarseNetDev = 2 };

template <int T, int MC, int MODE = kCoarseSolve>
__device__ __forceinline__ void correct_staged(double (&g)[MC], int M, bool predict,
                                               const double* __restrict__ fv,
                                               double* __restrict__ go, const double* uo1,
                                               double* un1, const double* __restrict__ vt1,
                                               double* stage, double& dmax, int& bad) {
    constexpr int CH = staged_chunks<T, MC>();
    constexpr int J = CH * MC / T;  // nodes per thread and pass
    static_assert(CH * MC % T == 0 && T % CH == 0, "whole passes");
    const int p = threadIdx.x;
#pragma unroll 1
    for (int c0 = 0; c0 < T; c0 += CH) {
        const int pl = p - c0;
        const bool mine = pl >= 0 && pl < CH;
        __syncthreads();  // earlier readers of this shared memory are done
        if (mine && MODE != kCoarseNet) {
#pragma unroll
            for (int q = 0; q < MC; ++q) stage[pl * (MC + 1) + q] = g[q];
        }
        __syncthreads();
        const int base = c0 * MC;
        if (predict) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int t = j * T + p, i = base + t;
                if (i < M) {
                    const double v = MODE != kCoarseSolve ? vt1[i] : 0.0;
                    const double gg = MODE == kCoarseSolve ? stage[t + t / MC]
                                      : MODE == kCoarseNet ? v
                                                           : v + stage[t + t / MC];
                    un1[i] = gg;
                    go[i] = gg;
                    if (MODE == kCoarseNetDev) stage[t + t / MC] = gg - v;
                }
            }
            if (MODE != kCoarseNetDev) continue;
        } else {
            // the loads of the whole pass are issued together: one memory
            // round trip per pass (the stores of a group may alias the next
            // group's loads as far as the compiler knows, which would
            // serialise groups)
            constexpr int G = J;
            static_assert(J % G == 0, "whole groups");
#pragma unroll
            for (int j0 = 0; j0 < J; j0 += G) {
                double f[G], gl[G], uo[G], v[G];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int i = base + (j0 + j) * T + p;
                    f[j] = (i < M) ? fv[i] : 0.0;
                    gl[j] = (i < M) ? go[i] : 0.0;
                    uo[j] = (i < M) ? uo1[i] : 0.0;
                    v[j] = (MODE != kCoarseSolve && i < M) ? vt1[i] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int t = (j0 + j) * T + p, i = base + t;
                    if (i < M) {
                        const double gg = MODE == kCoarseSolve ? stage[t + t / MC]
                                          : MODE == kCoarseNet ? v[j]
                                                               : v[j] + stage[t + t / MC];
                        const double unew = f[j] + (gg - gl[j]);
                        go[i] = gg;
                        un1[i] = unew;
                        dmax = fmax(dmax, fabs(unew - uo[j]));
                        bad |= !isfinite(unew);
                        stage[t + t / MC] = MODE == kCoarseNetDev ? unew - v[j] : unew;
                    }
                }
            }
        }
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int q = 0; q < MC; ++q)
                g[q] = (p * MC + q < M) ? stage[pl * (MC + 1) + q] : 0.0;
        }
    }
    __syncthreads();  // the next coarse solve may overwrite the staging area
}

// g[q] = op(g[q], src[p*MC + q]) for this thread's chunk (0 past the grid),
// with src read in node order through the staging area (passes as in
// correct_staged; chunks of 8 or more nodes per thread).
template <int T, int MC, class Op>
__device__ __forceinline__ void combine_staged(const double* __restrict__ src, int M,
                                               double (&g)[MC], double* stage, Op op) {
    constexpr int CH = staged_chunks<T, MC>();
    constexpr int J = CH * MC / T;
    static_assert(CH * MC % T == 0 && T % CH == 0, "whole passes");
    const int p = threadIdx.x;
#pragma unroll 1
    for (int c0 = 0; c0 < T; c0 += CH) {
        const int base = c0 * MC;
        __syncthreads();  // earlier readers of this shared memory are done
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int t = j * T + p, i = base + t;
            stage[t + t / MC] = (i < M) ? src[i] : 0.0;
        }
        __syncthreads();
        const int pl = p - c0;
        if (pl >= 0 && pl < CH) {
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = op(g[q], stage[pl * (MC + 1) + q]);
        }
    }
    __syncthreads();  // the coarse solve may overwrite the staging area
}

// The correction of correct_staged on chunk-major levels (no staging: every
// access is coalesced in chunk order).  Same operations per node, so the
// same results.  uo1 and un1 may be the same level (each entry is read
// before it is written); rows are taken in groups of G, a group's loads
// issued together (a second buffer to overlap the next group's loads made
// the sweep block spill).  predict: U[n+1] = Gold[n] = the coarse value.
template <int T, int MC, int MODE>
__device__ __forceinline__ void correct_cm(double (&g)[MC], int M, bool predict,
                                           const double* __restrict__ fv,
                                           double* __restrict__ go, const double* uo1,
                                           double* un1, const double* __restrict__ vt1,
                                           double& dmax, int& bad) {
    constexpr int G = 8;
    static_assert(MC % G == 0, "whole groups");
    const int p = threadIdx.x, i0 = p * MC;
    if (predict) {
#pragma unroll
        for (int q = 0; q < MC; ++q) {
            const int c = q * T + p;
            if (i0 + q < M) {
                const double v = MODE != kCoarseSolve ? vt1[c] : 0.0;
                const double gg = MODE == kCoarseSolve ? g[q]
                                  : MODE == kCoarseNet ? v
                                                       : v + g[q];
                un1[c] = gg;
                go[c] = gg;
                g[q] = MODE == kCoarseNetDev ? gg - v : gg;
            } else {
                g[q] = 0.0;
            }
        }
        return;
    }
    double f[G], gl[G], uo[G], v[G];
    auto load = [&](int q0) {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int c = (q0 + j) * T + p;
            f[j] = fv[c];
            gl[j] = go[c];
            uo[j] = uo1[c];
            v[j] = MODE != kCoarseSolve ? vt1[c] : 0.0;
        }
    };
#pragma unroll
    for (int q0 = 0; q0 < MC; q0 += G) {
        load(q0);
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int q = q0 + j, c = q * T + p;
            if (i0 + q < M) {
                const double gg = MODE == kCoarseSolve ? g[q]
                                  : MODE == kCoarseNet ? v[j]
                                                       : v[j] + g[q];
                const double unew = f[j] + (gg - gl[j]);
                go[c] = gg;
                un1[c] = unew;
                dmax = fmax(dmax, fabs(unew - uo[j]));
                bad |= !isfinite(unew);
                g[q] = MODE == kCoarseNetDev ? unew - v[j] : unew;
            } else {
                g[q] = 0.0;
            }
        }
    }
}

// One option's serial Parareal sweep over slices n = n0..N-1 in one block:
//   g = G(U[n])                       (state carried in registers)
//   predict: U[n+1] = g, Gold[n] = g
//   else:    U[n+1] = Fv[n] + (g - Gold[n]), Gold[n] = g,
//            dmax = max |U_new[n+1] - U_old[n+1]|, bad |= non-finite.
// S (BlockTri, BlockTriH or BlockTriR) must be set up for implicit Euler with
// dt = dT / coarse_steps.  For MC >= 8, lds must hold sweep_smem_doubles<T,
// MC>() doubles with ftab = lds + 4T (the staged correction uses the space
// after the solver's 4T doubles).
// pipe (overlapped solve; ps its counters): the slice's fine result is
// waited for after the coarse solve, U[n+1] is overwritten only once the
// fine launch of iteration k - taken_lag has read it, and each finished
// slice is published.  Returns false if the block must stop (see PipeSync).
// Uin / Uout: the previous iterate (the sweep's first state and the old
// values of the defect) and the buffer the new iterate goes to; the same
// array except in the one-launch solve, which alternates two buffers by
// iteration parity (there the first state is also copied to Uout, so that
// Uout holds a whole iterate, and taken_lag is 1: Uout held iterate k-2).
template <int T, int MC, class Solver, bool CM = false>
__device__ __forceinline__ bool sweep_slices(const Solver& S, const OptionDev& o, int M,
                                             int N, int n0, int coarse_steps, int kind, bool predict,
                                             double dT, const double* Uin, double* Uout,
                                             const double* __restrict__ Fv,
                                             double* __restrict__ Gold,
                                             const double* __restrict__ Vt, double* lds,
                                             double* ftab, double& dmax, int& bad,
                                             const PipeSync& ps = PipeSync{}, bool pipe = false,
                                             const int* stop = nullptr, int* pslot = nullptr,
                                             int taken_lag = 0, int pbatch = 1) {
    const double dtc = dT / (double)coarse_steps;
    const int i0 = threadIdx.x * MC;
    const bool net = kind != BS_COARSE_IE;
    if (pipe && predict && n0 == 0) pipe_signal(ps.ready, 1);  // U[0], written before the launch
    // Loads that do not depend on the coarse solve go first, so their latency
    // overlaps it (when registers allow: small chunks); larger chunks move
    // the slice's global traffic through the staged, node-order correction.
    constexpr bool kPrefetch = MC <= 4;
    static_assert(!CM || !kPrefetch, "chunk-major levels are for chunks of 8 or more nodes");
    // CM: the levels of Uin, Uout, Fv, Gold and Vt are chunk-major, T * MC
    // doubles apart
    const long ld = CM ? (long)T * MC : (long)M;
    double V[MC];
    if constexpr (CM)
        load_cm<T, MC>(Uin + n0 * ld, V);
    else
        load_chunk<T, MC>(Uin + (long)n0 * M, M, V);
    if (Uout != Uin) {
        // Uout[n0] still holds the iterate the fine launch of iteration
        // k - taken_lag reads
        if (pipe && !pipe_wait<false>(ps, ps.taken + n0, ps.k - taken_lag, stop, pslot))
            return false;
        if constexpr (CM)
            store_cm<T, MC>(Uout + n0 * ld, M, V);
        else
            store_chunk<T, MC>(Uout + (long)n0 * M, M, V);
    }
    if (!kPrefetch && kind == BS_COARSE_PINN_IE) {
        // staged path: the state carried from slice to slice is the
        // deviation from the network, U[n] - Vt_n
        if constexpr (CM) {
            double v0[MC];
            load_cm<T, MC>(Vt + n0 * ld, v0);
#pragma unroll
            for (int q = 0; q < MC; ++q) V[q] = V[q] - v0[q];
        } else {
            combine_staged<T, MC>(Vt + (long)n0 * M, M, V, lds + 4 * T,
                                  [](double a, double v) { return a - v; });
        }
    }
    for (int n = n0; n < N; ++n) {
        const double* uo1 = Uin + (n + 1) * ld;
        double* un1 = Uout + (n + 1) * ld;
        double* go = Gold + n * ld;
        double fv[MC], gold[MC], uold[MC], vt0[MC], vt1[MC];
        if constexpr (kPrefetch) {
            if (!predict && !pipe) {
                load_chunk<T, MC>(Fv + (long)n * M, M, fv);
                load_chunk<T, MC>(go, M, gold);
                load_chunk<T, MC>(uo1, M, uold);
            }
            if (net) {
                load_chunk<T, MC>(Vt + (long)(n + 1) * M, M, vt1);
                if (kind == BS_COARSE_PINN_IE) load_chunk<T, MC>(Vt + (long)n * M, M, vt0);
            }
        }
        double g[MC];
        if (kind == BS_COARSE_IE) {
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = V[q];
            theta_steps<T, MC, false>(S, o, g, (double)n * dT, dtc, coarse_steps, 1.0, false, lds,
                                      ftab);
        } else if (kind == BS_COARSE_PINN) {
            if constexpr (kPrefetch) {
#pragma unroll
                for (int q = 0; q < MC; ++q) g[q] = vt1[q];
            } else {
#pragma unroll
                for (int q = 0; q < MC; ++q) g[q] = 0.0;  // the correction takes Vt_{n+1}
            }
        } else {
            // G = Vt_{n+1} + E(U[n] - Vt_n); the staged path carries the
            // deviation in V and adds Vt_{n+1} in the correction
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = kPrefetch ? V[q] - vt0[q] : V[q];
            theta_steps<T, MC, false>(S, o, g, (double)n * dT, dtc, coarse_steps, 1.0, true, lds,
                                      ftab);
            if constexpr (kPrefetch) {
#pragma unroll
                for (int q = 0; q < MC; ++q) g[q] = vt1[q] + g[q];
            }
        }
        if (pipe && !predict && pbatch == 1) {
            // this iteration's fine result of slice n, then U[n+1] free to overwrite
            if (!pipe_wait(ps, ps.fdone + n, ps.k, stop, pslot)) return false;
            // Fv[n], and (written by the previous iteration's sweep, which has
            // passed slice n once Fv[n] is written) Gold[n] and U[n+1]
            if constexpr (kPrefetch) {
                load_chunk<T, MC>(Fv + (long)n * M, M, fv);
                load_chunk<T, MC>(go, M, gold);
                load_chunk<T, MC>(uo1, M, uold);
            }
            if (n + 1 < N &&
                !pipe_wait<false>(ps, ps.taken + n + 1, ps.k - taken_lag, stop, pslot))
                return false;
        } else if (pipe && !predict && (n - n0) % pbatch == 0) {
            // batched hand-offs: the fine results of slices n .. n+pbatch-1,
            // then one acquire for all of them (each acquire also drops this
            // compute unit's cached lines, among them the solver's tables)
            const int nb = min(n + pbatch, N);
            for (int m = n; m < nb; ++m)
                if (!pipe_wait<false>(ps, ps.fdone + m, ps.k, stop, pslot)) return false;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (int m = n; m < nb && m + 1 < N; ++m)
                if (!pipe_wait<false>(ps, ps.taken + m + 1, ps.k - taken_lag, stop, pslot))
                    return false;
        }
        if constexpr (CM) {
            const double* vn1 = net ? Vt + (n + 1) * ld : nullptr;
            if (kind == BS_COARSE_IE)
                correct_cm<T, MC, kCoarseSolve>(g, M, predict, Fv + n * ld, go, uo1, un1, vn1,
                                                dmax, bad);
            else if (kind == BS_COARSE_PINN)
                correct_cm<T, MC, kCoarseNet>(g, M, predict, Fv + n * ld, go, uo1, un1, vn1,
                                              dmax, bad);
            else
                correct_cm<T, MC, kCoarseNetDev>(g, M, predict, Fv + n * ld, go, uo1, un1, vn1,
                                                 dmax, bad);
#pragma unroll
            for (int q = 0; q < MC; ++q) V[q] = g[q];
        } else if constexpr (!kPrefetch) {
            // chunks of 8 or more nodes: the slice's global traffic goes
            // through the staged, node-order correction
            const double* vn1 = net ? Vt + (long)(n + 1) * M : nullptr;
            if (kind == BS_COARSE_IE)
                correct_staged<T, MC, kCoarseSolve>(g, M, predict, Fv + (long)n * M, go, uo1,
                                                    un1, vn1, lds + 4 * T, dmax, bad);
            else if (kind == BS_COARSE_PINN)
                correct_staged<T, MC, kCoarseNet>(g, M, predict, Fv + (long)n * M, go, uo1, un1,
                                                  vn1, lds + 4 * T, dmax, bad);
            else
                correct_staged<T, MC, kCoarseNetDev>(g, M, predict, Fv + (long)n * M, go, uo1,
                                                     un1, vn1, lds + 4 * T, dmax, bad);
#pragma unroll
            for (int q = 0; q < MC; ++q) V[q] = g[q];
        } else if (predict) {
            store_chunk<T, MC>(un1, M, g);
            store_chunk<T, MC>(go, M, g);
#pragma unroll
            for (int q = 0; q < MC; ++q) V[q] = g[q];
        } else {
            const double* fvn = Fv + (long)n * M;
#pragma unroll
            for (int q = 0; q < MC; ++q) {
                if (i0 + q < M) {
                    const double f = kPrefetch ? fv[q] : fvn[i0 + q];
                    const double gl = kPrefetch ? gold[q] : go[i0 + q];
                    const double uo = kPrefetch ? uold[q] : uo1[i0 + q];
                    const double unew = f + (g[q] - gl);
                    go[i0 + q] = g[q];
                    un1[i0 + q] = unew;
                    dmax = fmax(dmax, fabs(unew - uo));
                    bad |= !isfinite(unew);
                    V[q] = unew;
                } else {
                    V[q] = 0.0;
                }
            }
        }
        if (pipe && (predict || pbatch == 1)) {
            pipe_signal(ps.ready + n + 1, predict ? 1 : ps.k + 1);
        } else if (pipe && ((n - n0) % pbatch == pbatch - 1 || n == N - 1)) {
            // one release for the batch's new iterates
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0)
                for (int m = n - (n - n0) % pbatch; m <= n; ++m)
                    __hip_atomic_store(ps.ready + m + 1, ps.k + 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    return true;
}

// Block max of dmax and OR of bad; the result is valid in thread 0.
template <int T>
__device__ __forceinline__ void block_defect(double& dmax, int& bad, double* lds) {
    __syncthreads();
    lds[threadIdx.x] = dmax;
    lds[T + threadIdx.x] = bad ? 1.0 : 0.0;
    __syncthreads();
    for (int s = T / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + s]);
            lds[T + threadIdx.x] = fmax(lds[T + threadIdx.x], lds[T + threadIdx.x + s]);
        }
        __syncthreads();
    }
    dmax = lds[0];
    bad = lds[T] != 0.0;
}

}  // namespace bsp
