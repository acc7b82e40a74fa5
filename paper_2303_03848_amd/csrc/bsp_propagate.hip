// Propagator kernels: expiry payoff, the batched theta-method (Crank-Nicolson
// fine F, implicit-Euler coarse G) and the serial Parareal correction sweep.
#include <mutex>
#include <shared_mutex>

#include "bsp_common.hpp"
#include "bsp_steps.hpp"
#include "bsp_tridiag_large.hpp"
#include "bsp_tridiag_rc.hpp"

namespace bsp {

// ------------------------------------------------------------- payoff

// Expiry condition (eq. (2) and its put analogue) at S_j = (i+1) dS, sampled
// (mode 0) or averaged over the cell [S_j - dS/2, S_j + dS/2] (mode 1).
__global__ void k_initial(OptionDev o, int M, int mode, double* __restrict__ u0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double S = (double)(i + 1) * o.dS;
    const double K = o.K;
    double v;
    if (mode == 0) {
        v = o.is_put ? fmax(K - S, 0.0) : fmax(S - K, 0.0);
    } else {
        const double lo = S - 0.5 * o.dS, hi = S + 0.5 * o.dS;
        if (!o.is_put) {
            v = (hi <= K) ? 0.0 : (lo >= K) ? 0.5 * (lo + hi) - K : (hi - K) * (hi - K) / (2.0 * o.dS);
        } else {
            v = (lo >= K) ? 0.0 : (hi <= K) ? K - 0.5 * (lo + hi) : (K - lo) * (K - lo) / (2.0 * o.dS);
        }
    }
    u0[i] = v;
}

int launch_initial(const OptionDev& o, int M, int payoff_mode, double* u0, hipStream_t stream) {
    hipLaunchKernelGGL(k_initial, dim3((M + 255) / 256), dim3(256), 0, stream, o, M, payoff_mode,
                       u0);
    BSP_LAUNCHED();
    return BS_OK;
}

// ------------------------------------------------ batched theta-method

struct ThetaArgs {
    OptionDev o;
    int M, steps, sys_offset;
    const double* tau0;
    double tau_start, tau_stride, dt, theta;
    const double* u_in;
    long ld_in;
    double* u_out;
    long ld_out;
    const int* stop;  // when non-null and set, the launch does nothing
    PipeSync ps;      // overlapped solve (k_theta_pipe only)
};

__device__ __forceinline__ bool stopped(const int* stop) {
    return stop && *(volatile const int*)stop;
}

__global__ void k_set_int(int* p, int v) { *p = v; }

__global__ void k_fill_int(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int launch_fill_int(int* p, int n, int v, hipStream_t stream) {
    if (n <= 0) return BS_OK;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
    BSP_LAUNCHED();
    return BS_OK;
}

__global__ void k_fill_double(double* p, int n, double v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int launch_fill_double(double* p, int n, double v, hipStream_t stream) {
    if (n <= 0) return BS_OK;
    hipLaunchKernelGGL(k_fill_double, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
    BSP_LAUNCHED();
    return BS_OK;
}

int launch_set_int(int* p, int v, hipStream_t stream) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, p, v);
    BSP_LAUNCHED();
    return BS_OK;
}

// Status of iteration k with defect dmax: 1 non-finite, 2 diverged (k >= 2
// and the defect above growth x first, the defect of iteration 1), else 0.
__device__ __forceinline__ int sweep_status(int k, double dmax, int bad, double first,
                                            double growth) {
    if (bad) return 1;
    return (k >= 2 && dmax > growth * first) ? 2 : 0;
}

// Iteration record of the asynchronous solve (thread 0, after block_defect).
// result[2] holds the defect of iteration 1 (written by that iteration's
// sweep, which has completed when k >= 2).  Returns the status.
__device__ __forceinline__ int sweep_record(const SweepArgs& a, double dmax, int bad) {
    if (a.k == 1) a.result[2] = dmax;
    const int status = sweep_status(a.k, dmax, bad, a.result[2], a.growth);
    a.result[0] = dmax;
    a.result[1] = (double)status;
    if (a.hist) {  // host memory: visible to the host once the launch completes
        a.hist[2 * a.k] = dmax;
        a.hist[2 * a.k + 1] = (double)status;
        __threadfence_system();
    }
    if (a.stop && (status || dmax <= a.tol)) *a.stop = 1;
    return status;
}

// One block per system.  PIPE (overlapped Parareal solve): system sys is
// slice n = sys + sys_offset of iteration ps.k.  Everything that does not
// depend on the state (factors, the first forcing table) is built first;
// then it waits until U[n] holds iterate k-1, reports having read it, polls
// the stop flag while stepping, and writes Fv[n] only after the sweep of
// iteration k-1 has consumed the previous one (U[n+1] holds iterate k-1).
// smem: the solver's LDS, the forcing tables, and (PIPE) the staging area
// of the state, kept apart from the tables built before the load.
template <int T, int MC, bool PIPE>
__device__ __forceinline__ void theta_body(const ThetaArgs& a, double* smem, int* pslot) {
    double* lds = smem;
    double* ftab = smem + 4 * T;
    double* stage = PIPE ? smem + smem_doubles<T, MC>() : smem;
    if (stopped(a.stop)) return;
    const int sys = blockIdx.x;
    const int n = sys + a.sys_offset;
    const double tau0 = a.tau0 ? a.tau0[sys] : a.tau_start + (double)n * a.tau_stride;
    using S_t = Solver<T, MC>;
    S_t S;
    double V[MC];
    bool prefilled = false;
    if constexpr (PIPE) {
        S.setup(a.o.s2, a.o.r, a.theta * a.dt, (1.0 - a.theta) * a.dt, a.M, lds);
        const bool ex = a.theta != 1.0;
        if (ex ? piped_path<true>(S, a.steps) : piped_path<false>(S, a.steps)) {
            fill_piped_table<T>(a.o, tau0, a.dt, a.steps, a.theta, 0,
                                min(kForceChunk - 1, a.steps), ftab);
            prefilled = true;
        }
        if (!pipe_wait(a.ps, a.ps.ready + n, a.ps.k, a.stop, pslot)) return;
        load_system<T, MC>(a.u_in + (long)sys * a.ld_in, a.M, V, stage);
        pipe_mark(a.ps.taken + n, a.ps.k);
    } else {
        load_system<T, MC>(a.u_in + (long)sys * a.ld_in, a.M, V, stage);
        S.setup(a.o.s2, a.o.r, a.theta * a.dt, (1.0 - a.theta) * a.dt, a.M, lds);
    }
    const bool ok =
        (a.theta == 1.0)
            ? theta_steps<T, MC, false, S_t, PIPE>(S, a.o, V, tau0, a.dt, a.steps, 1.0,
                                                   false, lds, ftab, a.stop, prefilled)
            : theta_steps<T, MC, true, S_t, PIPE>(S, a.o, V, tau0, a.dt, a.steps, a.theta,
                                                  false, lds, ftab, a.stop, prefilled);
    if (!ok) return;
    if constexpr (PIPE)
        if (!pipe_wait<false>(a.ps, a.ps.ready + n + 1, a.ps.k, a.stop, pslot)) return;
    store_system<T, MC>(a.u_out + (long)sys * a.ld_out, a.M, V, stage);
    if constexpr (PIPE) pipe_signal(a.ps.fdone + n, a.ps.k);
}

template <int T, int MC>
__global__ __launch_bounds__(T) void k_theta_batch(ThetaArgs a) {
    __shared__ double smem[smem_doubles<T, MC>()];
    theta_body<T, MC, false>(a, smem, nullptr);
}

// One block per compute unit is the intended occupancy of the large-chunk
// shapes: the compiler may use the whole register file (no scratch spills).
template <int T, int MC>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_theta_pipe(
    ThetaArgs a) {
    __shared__ double smem[smem_doubles<T, MC>() + T * MC];
    __shared__ int pslot;
    theta_body<T, MC, true>(a, smem, &pslot);
}

// ---------------------------------------------------- Parareal sweep

template <int T, int MC>
__global__ __launch_bounds__(T) void k_sweep(SweepArgs a) {
    __shared__ double smem[sweep_smem_doubles<T, MC>()];
    double* lds = smem;
    double* ftab = smem + 4 * T;
    __shared__ int pslot;
    if (stopped(a.stop)) return;
    Solver<T, MC> S;
    S.setup(a.o.s2, a.o.r, a.dT / (double)a.coarse_steps, 0.0, a.M, lds);
    double dmax = 0.0;
    int bad = 0;
    const PipeSync ps = a.ps;
    if (!sweep_slices<T, MC>(S, a.o, a.M, a.N, a.n0, a.coarse_steps, a.kind, a.predict != 0, a.dT,
                             a.U, a.U, a.Fv, a.Gold, a.Vt, lds, ftab, dmax, bad, ps,
                             ps.ready != nullptr, a.stop, &pslot))
        return;
    if (!a.predict) {
        block_defect<T>(dmax, bad, lds);
        if (threadIdx.x == 0) sweep_record(a, dmax, bad);
    }
}

// ------------------------------------------------------ persistent solve

// A whole Parareal solve in one launch, for grids whose fine kernel is one
// wavefront per system and whose sweep runs on 256 threads.  Blocks
// 0 .. nfb-1 hold four fine wavefronts each: wavefront w of block b owns
// slice n = 4b + w for every iteration, building its factors and forcing
// table once; per iteration it waits until U[n] holds the previous iterate,
// propagates it, and publishes Fv[n].  The remaining nsb blocks sweep: block
// j runs iterations k = j, j + nsb, ... (k = 0 is the coarse prediction), so
// the sweep of iteration k+1 follows the sweep of iteration k slice by slice
// instead of waiting for it to end.  Every hand-off goes through the
// progress counters of PipeSync; the iterates are those of the
// launch-after-launch iteration with the same block shapes.
//
// Two state buffers: iterate k is written to U (k even) or U2 (k odd), so the
// sweep of iteration k+1, which runs while iteration k's defect is still
// being reduced, never touches iterate k.  The sweep of iteration k writes
// over iterate k-2, and first waits until iteration k-2 has been decided (if
// the solve stopped there or earlier it returns without writing).  The last
// block to finish copies the final iterate to U when it lies in U2.
template <int MCF>
constexpr int persist_fine_lds() {  // doubles per fine wavefront
    return 2 * kForceChunk + 64 * MCF;
}

__device__ __forceinline__ double* persist_buf(const PersistArgs& a, int k) {
    return (k & 1) ? a.U2 : a.U;
}

template <int MCF>
__device__ __forceinline__ void persist_fine(const PersistArgs& a, double* smem) {
    const int w = threadIdx.x >> 6;
    const int n = 4 * (int)blockIdx.x + w;
    if (n >= a.N) return;  // the role has no block-wide barrier
    double* ftab = smem + w * persist_fine_lds<MCF>();
    double* stage = ftab + 2 * kForceChunk;
    const double dt = a.dT / (double)a.fine_steps;
    const double tau0 = (double)n * a.dT;
    BlockTri<64, MCF> S;
    S.setup(a.o.s2, a.o.r, 0.5 * dt, 0.5 * dt, a.M, nullptr);
    // one table serves every iteration
    const bool pre = a.fine_steps <= kForceChunk - 1 && piped_path<true, true>(S, a.fine_steps);
    if (pre) fill_piped_table<64, true>(a.o, tau0, dt, a.fine_steps, 0.5, 0, a.fine_steps, ftab);
    const int klast = min(a.kmax, n + 1);  // iteration k propagates slices n >= k-1
    for (int k = 1; k <= klast; ++k) {
        if (!pipe_wait_wave(a.ps, a.ps.ready + n, k, a.stop)) return;
        double V[MCF];
        load_system<64, MCF, true>(persist_buf(a, k - 1) + (long)n * a.M, a.M, V, stage);
        if ((threadIdx.x & 63) == 0)
            __hip_atomic_store(a.ps.taken + n, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!theta_steps<64, MCF, true, BlockTri<64, MCF>, true, true>(
                S, a.o, V, tau0, dt, a.fine_steps, 0.5, false, nullptr, ftab, a.stop, pre))
            return;
        if (!pipe_wait_wave<false>(a.ps, a.ps.ready + n + 1, k, a.stop)) return;
        store_system<64, MCF, true>(a.Fv + (long)n * a.M, a.M, V, stage);
        pipe_signal_wave(a.ps.fdone + n, k);
    }
}

template <int MCS>
__device__ __forceinline__ void persist_sweep(const PersistArgs& a, int j, double* smem,
                                              int* pslot) {
    constexpr int T = 256;
    double* lds = smem;
    double* ftab = smem + 4 * T;
    Solver<T, MCS> S;
    S.setup(a.o.s2, a.o.r, a.dT / (double)a.coarse_steps, 0.0, a.M, lds);
    for (int k = j; k <= a.kmax; k += a.nsb) {
        const bool predict = k == 0;
        const int n0 = predict ? 0 : min(k - 1, a.N - 1);
        PipeSync ps = a.ps;
        ps.k = k;
        if (k >= 2) {
            // Uout holds iterate k-2: keep it until iteration k-2 is decided
            if (!pipe_wait(ps, a.decided + k - 2, 1, a.stop, pslot)) return;
            // the solve may have stopped at k-2 or earlier: the same decision
            // in every thread
            if (__syncthreads_or(pipe_load(a.stop) != 0)) return;
        }
        // the sweep's first state U[n0] (iterate k; for k >= 1 written by the
        // sweep of iteration k-1)
        if (!predict && !pipe_wait(ps, ps.ready + n0, k, a.stop, pslot)) return;
        double dmax = 0.0;
        int bad = 0;
        const double* Uin = persist_buf(a, predict ? 0 : k - 1);
        double* Uout = persist_buf(a, k);
        if (!sweep_slices<T, MCS>(S, a.o, a.M, a.N, n0, a.coarse_steps, a.kind, predict, a.dT,
                                  Uin, Uout, a.Fv, a.Gold, a.Vt, lds, ftab, dmax, bad, ps, true,
                                  a.stop, pslot, predict ? 0 : 1))
            return;
        if (!predict) {
            block_defect<T>(dmax, bad, lds);
            // the guard compares with iteration 1's defect: recorded by then
            if (k >= 2 && !pipe_wait(ps, a.decided + 1, 1, a.stop, pslot)) return;
            if (threadIdx.x == 0) {
                SweepArgs sa{};
                sa.result = a.result;
                sa.stop = a.stop;
                sa.hist = a.hist;
                sa.tol = a.tol;
                sa.k = k;
                sa.growth = a.growth;
                const double first = k == 1 ? dmax : a.result[2];
                if (sweep_status(k, dmax, bad, first, a.growth) || dmax <= a.tol)
                    atomicMax(a.stop_rank, a.kmax + 1 - k);  // before the stop flag
                sweep_record(sa, dmax, bad);
            }
        }
        pipe_signal(a.decided + k, 1);  // the prediction too: the sweep of k = 2 waits for it
    }
}

template <int MCF, int MCS>
__global__ __launch_bounds__(256) void k_parareal_persist(PersistArgs a) {
    static_assert(4 * persist_fine_lds<MCF>() >= 4 * 256 + 2 * kForceChunk, "sweep LDS");
    __shared__ double smem[4 * persist_fine_lds<MCF>()];
    __shared__ int pslot;
    if ((int)blockIdx.x < a.nfb)
        persist_fine<MCF>(a, smem);
    else
        persist_sweep<MCS>(a, (int)blockIdx.x - a.nfb, smem, &pslot);
    // every role has returned; the last block to get here moves the final
    // iterate to U if it lies in U2 (no block writes either buffer any more)
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int before = __hip_atomic_fetch_add(a.exited, 1, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        pslot = before == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!pslot) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int rank = pipe_load(a.stop_rank);
    const int kfinal = rank ? a.kmax + 1 - rank : a.kmax;
    if (!(kfinal & 1)) return;
    const long total = (long)(a.N + 1) * a.M;
    for (long i = threadIdx.x; i < total; i += blockDim.x) a.U[i] = a.U2[i];
}

bool persist_capable(int M, int N) {
    const TriShape f = shape_for(0, M), w = shape_for(1, M);
    return persist_possible(M, N) && f.T == 64 &&
           (f.MC == 2 || f.MC == 4 || f.MC == 8 || f.MC == 16) && w.T == 256 && w.MC == 4;
}

// Resident-block capacity of one kernel on the current device (blocks per
// compute unit x compute units), queried once per device.
static int resident_blocks(const void* fn, int threads, int slot) {
    static int cache[16][8] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
    if (cache[dev][slot]) return cache[dev][slot];
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    cache[dev][slot] = per_cu * cus;
    return cache[dev][slot];
}

int launch_parareal_persist(const PersistArgs& in, hipStream_t stream) {
    PersistArgs a = in;
    if (!persist_capable(a.M, a.N)) {
        set_error("no persistent solve for M = %d, N = %d with the current block shapes", a.M, a.N);
        return BS_ERR_ARG;
    }
    a.nfb = (a.N + 3) / 4;
    a.nsb = min(3, a.kmax + 1);
    const dim3 grid(a.nfb + a.nsb), block(256);
    const TriShape f = shape_for(0, a.M);
    const void* fn = nullptr;
    int slot = 0;
    switch (f.MC) {
        case 2: fn = (const void*)k_parareal_persist<2, 4>; slot = 0; break;
        case 4: fn = (const void*)k_parareal_persist<4, 4>; slot = 1; break;
        case 8: fn = (const void*)k_parareal_persist<8, 4>; slot = 2; break;
        default: fn = (const void*)k_parareal_persist<16, 4>; slot = 3; break;
    }
    // The blocks wait on each other, so all of them must be resident at once:
    // an ordinary launch whose grid fits the device's resident capacity (one
    // block per compute unit here).  Waits that do not end (another kernel
    // holding the compute units) end at the time limit with an error.
    const int cap = resident_blocks(fn, 256, slot);
    if ((int)grid.x > cap) {
        set_error("one-launch solve needs %u resident blocks, the device holds %d", grid.x, cap);
        return BS_ERR_HIP;
    }
    switch (f.MC) {
        case 2: hipLaunchKernelGGL((k_parareal_persist<2, 4>), grid, block, 0, stream, a); break;
        case 4: hipLaunchKernelGGL((k_parareal_persist<4, 4>), grid, block, 0, stream, a); break;
        case 8: hipLaunchKernelGGL((k_parareal_persist<8, 4>), grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL((k_parareal_persist<16, 4>), grid, block, 0, stream, a); break;
    }
    BSP_LAUNCHED();
    return BS_OK;
}

// ------------------------------------------------------- large grids

// 512-thread shapes with 16 or 32 nodes per thread (grids beyond 4096 nodes)
// use the streamed-coefficient solver.
static bool is_large(TriShape sh) { return sh.T == 512 && sh.MC >= 16; }

// Never set: the stop flag of launches that have none.
static __device__ int g_no_stop = 0;

// F / G on large grids: one block per system and compute unit; each block
// builds its own factorisation (BlockTriR keeps the pivots in LDS and
// recomputes everything else), so concurrent launches share nothing.

template <int T, int MC, bool HI>
__global__ __launch_bounds__(T) void k_rc_theta(ThetaArgs a) {
    __shared__ double lds[4 * T];
    __shared__ double ftab[2 * kForceChunk];
    __shared__ double kus[(MC - 1) * T];
    if (stopped(a.stop)) return;
    const int sys = blockIdx.x;
    RcFact<T, MC, HI> Fa;
    Fa.setup(a.o.s2, a.o.r, a.theta * a.dt, (1.0 - a.theta) * a.dt, a.M, kus, lds);
    const double tau0 =
        a.tau0 ? a.tau0[sys] : a.tau_start + (double)(sys + a.sys_offset) * a.tau_stride;
    double V[MC];
    load_chunk<T, MC>(a.u_in + (long)sys * a.ld_in, a.M, V);
    const bool slow = Fa.nst > kRcRegStages;  // the same in every thread of the block
    // The steps run in polled runs (the stop flag is checked between runs of
    // kRunSteps steps): besides ending a cancelled launch early, the check
    // points let the register allocator keep the step loop free of spills
    // (measured: 40 scratch accesses per step without them, none with them).
    const int* stop = a.stop ? a.stop : &g_no_stop;
#define BSP_RC_RUN(CN_, SLOW_, EX_, TH_)                                                    \
    theta_steps<T, MC, EX_, BlockTriR<T, MC, HI, CN_, SLOW_>, true>(                      \
        BlockTriR<T, MC, HI, CN_, SLOW_>(Fa), a.o, V, tau0, a.dt, a.steps, TH_, false, lds, \
        ftab, stop)
    bool ok;
    if (a.theta == 0.5)
        ok = slow ? BSP_RC_RUN(true, true, true, 0.5) : BSP_RC_RUN(true, false, true, 0.5);
    else if (a.theta == 1.0)
        ok = slow ? BSP_RC_RUN(false, true, false, 1.0) : BSP_RC_RUN(false, false, false, 1.0);
    else
        ok = BSP_RC_RUN(false, true, true, a.theta);
#undef BSP_RC_RUN
    if (!ok) return;
    store_chunk<T, MC>(a.u_out + (long)sys * a.ld_out, a.M, V);
}

// The serial sweep on large grids: one block; the implicit-Euler solves
// stream their factors from the tables a.tab / a.ptab (built by
// k_large_setup in the caller's workspace), which keeps LDS free for the
// staged correction's 4096-node passes.
template <int T, int MC>
__global__ __launch_bounds__(T) void k_large_sweep(SweepArgs a) {
    __shared__ double smem[sweep_smem_doubles<T, MC>()];
    __shared__ double kst[2 * BlockTriG<T, MC>::LOGT * T];
    double* lds = smem;
    double* ftab = smem + 4 * T;
    if (stopped(a.stop)) return;
    BlockTriG<T, MC> S;
    S.load(a.tab, a.ptab, a.o.s2, a.o.r, a.dT / (double)a.coarse_steps, 0.0, a.M, kst);
    double dmax = 0.0;
    int bad = 0;
    sweep_slices<T, MC>(S, a.o, a.M, a.N, a.n0, a.coarse_steps, a.kind, a.predict != 0, a.dT, a.U,
                        a.U, a.Fv, a.Gold, a.Vt, lds, ftab, dmax, bad);
    if (!a.predict) {
        block_defect<T>(dmax, bad, lds);
        if (threadIdx.x == 0) sweep_record(a, dmax, bad);
    }
}

template <int T, int MC>
static int launch_large_setup(const OptionDev& o, int M, double h, double e, double* tab,
                              double* ptab, hipStream_t st) {
    hipLaunchKernelGGL((k_large_setup<T, MC>), dim3(1), dim3(T), 0, st, o.s2, o.r, h, e, M, tab,
                       ptab);
    BSP_LAUNCHED();
    return BS_OK;
}

size_t large_sweep_table_doubles(int M) {
    return is_large(shape_for(1, M)) ? (size_t)kLgFields * 32 * 512 + (size_t)kLgP * 512 : 0;
}

const double* large_sweep_ptab(const double* tab) { return tab + (size_t)kLgFields * 32 * 512; }

// Tables of the large-grid sweep's implicit-Euler solves, in tab (of
// large_sweep_table_doubles(M) doubles).
int launch_large_sweep_setup(const OptionDev& o, int M, double dT, int coarse_steps, double* tab,
                             hipStream_t stream) {
    const TriShape sh = shape_for(1, M);
    double* ptab = tab + (size_t)kLgFields * 32 * 512;
    const double h = dT / (double)coarse_steps;
    if (sh.MC == 16) return launch_large_setup<512, 16>(o, M, h, 0.0, tab, ptab, stream);
    return launch_large_setup<512, 32>(o, M, h, 0.0, tab, ptab, stream);
}


// ------------------------------------------ overlapped large-grid solve

// One launch for the prediction and iterations 1.. of a solve on a grid
// beyond 4096 nodes, after the fine propagation of slice 0's initial value
// (its iteration-1 result).  Block N-1 sweeps:
// iterations k = 1, 2, ... one after the other, slice by slice, each slice as
// soon as its fine result of iteration k is written; before them the coarse
// prediction (k = 0).  Blocks 0 .. N-2 are the fine blocks: block b owns
// slice n = b + 1 and propagates it for iterations k = 1 .. min(kmax, n + 1)
// (slice n is exact from iteration n + 1 on), each as soon as the sweep of
// iteration k-1 (the prediction for k = 1) has produced its initial value;
// slice 0's fine result of iteration 1 is computed before the launch.  So
// the sweep of iteration k runs beside the fine work of iteration k + 1 and
// an iteration costs about one fine propagation instead of one plus a sweep.
// Hand-offs go through the progress counters of PipeSync (ready: U[n] holds
// iterate j, stored as j + 1; taken: the fine block of iteration k has read
// U[n]; fdone: Fv[n] holds iteration k's result), exactly as in the solve
// that overlaps launches on side streams; the iterates are those of the
// one-iteration-at-a-time solve.  The fine blocks poll the stop flag every
// kRunSteps steps.  Every block must be resident (N blocks, one per compute
// unit): the host checks the device's capacity first.
constexpr int kLargePersistMaxN = 256;
// Slices per hand-off batch of the sweep block (one acquire and one release
// per batch: agent-scope fences write back / drop the compute unit's cached
// lines, which the sweep's solver re-reads every slice).
constexpr int kLargeSweepBatch = 8;

template <int MC>
constexpr int large_persist_lds() {  // doubles: the larger of the two roles
    constexpr int T = 512;
    constexpr int fine = (MC - 1) * T + 4 * T + 2 * kForceChunk;
    constexpr int sweep = 2 * BlockTriG<T, MC>::LOGT * T + sweep_smem_doubles<T, MC>();
    return fine > sweep ? fine : sweep;
}

template <int MC, bool HI>
__device__ __forceinline__ void large_fine_role(const LargePersistArgs& a, int n, double* smem,
                                                int* pslot) {
    constexpr int T = 512;
    double* kus = smem;
    double* lds = smem + (MC - 1) * T;
    double* ftab = lds + 4 * T;
    const double dt = a.dT / (double)a.fine_steps;
    RcFact<T, MC, HI> Fa;
    Fa.setup(a.o.s2, a.o.r, 0.5 * dt, 0.5 * dt, a.M, kus, lds);
    const bool slow = Fa.nst > kRcRegStages;  // the same in every thread
    const double tau0 = (double)n * a.dT;
    const int klast = min(a.kmax, n + 1);
    const PipeSync& ps = a.ps;
    for (int k = 1; k <= klast; ++k) {
        if (!pipe_wait(ps, ps.ready + n, k, a.stop, pslot)) return;
        double V[MC];
        load_cm<T, MC>(a.U + (long)n * (T * MC), V);
        pipe_signal(ps.taken + n, k);  // the loads have completed (release fence)
        const bool ok =
            slow ? theta_steps<T, MC, true, BlockTriR<T, MC, HI, true, true>, true>(
                       BlockTriR<T, MC, HI, true, true>(Fa), a.o, V, tau0, dt, a.fine_steps, 0.5,
                       false, lds, ftab, a.stop)
                 : theta_steps<T, MC, true, BlockTriR<T, MC, HI, true, false>, true>(
                       BlockTriR<T, MC, HI, true, false>(Fa), a.o, V, tau0, dt, a.fine_steps,
                       0.5, false, lds, ftab, a.stop);
        if (!ok) return;
        // Fv[n] of iteration k-1 has been used once the sweep of iteration k-1
        // has written U[n+1]
        if (!pipe_wait<false>(ps, ps.ready + n + 1, k, a.stop, pslot)) return;
        store_cm<T, MC>(a.Fv + (long)n * (T * MC), a.M, V);
        pipe_signal(ps.fdone + n, k);
    }
}

template <int MC>
__device__ __forceinline__ void large_sweep_role(const LargePersistArgs& a, double* smem,
                                                 int* pslot) {
    constexpr int T = 512;
    double* kst = smem;
    double* lds = smem + 2 * BlockTriG<T, MC>::LOGT * T;
    double* ftab = lds + 4 * T;
    BlockTriG<T, MC> S;
    S.load(a.tab, a.ptab, a.o.s2, a.o.r, a.dT / (double)a.coarse_steps, 0.0, a.M, kst);
    for (int k = 0; k <= a.kmax; ++k) {
        // k = 0: the coarse prediction, which the fine blocks' first
        // iteration follows slice by slice
        PipeSync ps = a.ps;
        ps.k = k;
        const int n0 = k == 0 ? 0 : min(k - 1, a.N - 1);
        double dmax = 0.0;
        int bad = 0;
        const bool ok = sweep_slices<T, MC, BlockTriG<T, MC>, true>(
            S, a.o, a.M, a.N, n0, a.coarse_steps, a.kind, k == 0, a.dT, a.U, a.U, a.Fv, a.Gold,
            a.Vt, lds, ftab, dmax, bad, ps, true, a.stop, pslot, 0, kLargeSweepBatch);
        if (!ok) return;
        if (k == 0) continue;
        block_defect<T>(dmax, bad, lds);
        if (threadIdx.x == 0) {
            SweepArgs sa{};
            sa.result = a.result;
            sa.stop = a.stop;
            sa.hist = a.hist;
            sa.tol = a.tol;
            sa.k = k;
            sa.growth = a.growth;
            sweep_record(sa, dmax, bad);
        }
        __syncthreads();
        if (__syncthreads_or(threadIdx.x == 0 && pipe_load(a.stop) != 0)) return;
    }
}

template <int MC, bool HI>
__global__ __launch_bounds__(512) void k_large_persist(LargePersistArgs a) {
    __shared__ double smem[large_persist_lds<MC>()];
    __shared__ int pslot;
    if ((int)blockIdx.x < (int)gridDim.x - 1)
        large_fine_role<MC, HI>(a, (int)blockIdx.x + 1, smem, &pslot);
    else
        large_sweep_role<MC>(a, smem, &pslot);
}

// Levels [levels][M] (node order) to and from the chunk-major layout
// [levels][T*MC] of the overlapped solve (zero past the grid).  One thread
// per chunk-major entry: the chunk-major side is coalesced, the node-order
// side reads or writes with stride MC (whole lines end up used through L2).
__global__ void k_to_cm(const double* __restrict__ src, double* __restrict__ dst, int M, int T,
                        int MC) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= T * MC) return;
    const long lev = blockIdx.y;
    const int node = (e % T) * MC + e / T;
    dst[lev * T * MC + e] = node < M ? src[lev * M + node] : 0.0;
}

__global__ void k_from_cm(const double* __restrict__ src, double* __restrict__ dst, int M, int T,
                          int MC) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= T * MC) return;
    const long lev = blockIdx.y;
    const int node = (e % T) * MC + e / T;
    if (node < M) dst[lev * M + node] = src[lev * T * MC + e];
}

long large_cm_level(int M) {
    const TriShape f = shape_for(0, M);
    return is_large(f) ? (long)f.T * f.MC : 0;
}

int launch_cm_convert(const double* src, double* dst, int levels, int M, bool to_cm,
                      hipStream_t stream) {
    const TriShape f = shape_for(0, M);
    if (!is_large(f) || levels < 0 || levels > 65535) {
        set_error("chunk-major levels: M = %d, %d levels", M, levels);
        return BS_ERR_ARG;
    }
    if (levels == 0) return BS_OK;
    const dim3 grid((f.T * f.MC + 255) / 256, levels), block(256);
    if (to_cm)
        hipLaunchKernelGGL(k_to_cm, grid, block, 0, stream, src, dst, M, f.T, f.MC);
    else
        hipLaunchKernelGGL(k_from_cm, grid, block, 0, stream, src, dst, M, f.T, f.MC);
    BSP_LAUNCHED();
    return BS_OK;
}

// The kernel instance for grid M and its slot in the residency cache.
static const void* large_persist_fn(int M, int& slot) {
    const TriShape f = shape_for(0, M);
    const bool hi = M % f.MC != 0;
    if (f.MC == 16) {
        slot = hi ? 4 : 5;
        return hi ? (const void*)k_large_persist<16, true> : (const void*)k_large_persist<16, false>;
    }
    slot = hi ? 6 : 7;
    return hi ? (const void*)k_large_persist<32, true> : (const void*)k_large_persist<32, false>;
}

// Shapes allow it, and the device holds all N blocks at once (they wait on
// each other).
bool large_persist_capable(int M, int N) {
    const TriShape f = shape_for(0, M), w = shape_for(1, M);
    if (!(is_large(f) && is_large(w) && f.MC == w.MC && N >= 2 && N <= kLargePersistMaxN))
        return false;
    int slot = 0;
    const void* fn = large_persist_fn(M, slot);
    return N <= resident_blocks(fn, 512, slot);
}

int launch_large_persist(const LargePersistArgs& a, hipStream_t stream) {
    if (!large_persist_capable(a.M, a.N)) {
        set_error("no overlapped large-grid solve for M = %d, N = %d", a.M, a.N);
        return BS_ERR_ARG;
    }
    const TriShape f = shape_for(0, a.M);
    const bool hi = a.M % f.MC != 0;
    int slot = 0;
    const void* fn = large_persist_fn(a.M, slot);
    const int cap = resident_blocks(fn, 512, slot);
    if (a.N > cap) {
        set_error("overlapped large-grid solve needs %d resident blocks, the device holds %d",
                  a.N, cap);
        return BS_ERR_HIP;
    }
    const dim3 grid(a.N), block(512);
    if (f.MC == 16) {
        if (hi) hipLaunchKernelGGL((k_large_persist<16, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((k_large_persist<16, false>), grid, block, 0, stream, a);
    } else {
        if (hi) hipLaunchKernelGGL((k_large_persist<32, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((k_large_persist<32, false>), grid, block, 0, stream, a);
    }
    BSP_LAUNCHED();
    return BS_OK;
}


// ------------------------------------------------------------ dispatch

// Default block shapes.  The F kernel favours one wavefront per system (no
// barriers) while its registers allow, then as few wavefronts of 16 nodes
// per lane as cover the grid; the serial sweep is one block for the whole
// grid and favours more threads per system.
static TriShape default_shape(int kernel, int M) {
    if (kernel == 0) {
        if (M <= 128) return {64, 2};
        if (M <= 256) return {64, 4};
        if (M <= 512) return {64, 8};
        if (M <= 1024) return {64, 16};
        if (M <= 2048) return {128, 16};
        if (M <= 4096) return {256, 16};
        if (M <= 8192) return {512, 16};
        if (M <= 16384) return {512, 32};
    } else {
        if (M <= 128) return {64, 2};
        if (M <= 256) return {64, 4};
        if (M <= 512) return {128, 4};
        if (M <= 1024) return {256, 4};
        if (M <= 2048) return {256, 8};
        if (M <= 4096) return {512, 8};
        if (M <= 8192) return {512, 16};
        if (M <= 16384) return {512, 32};
    }
    return {0, 0};
}

static bool shape_built(int T, int MC) {
#define BSP_IS(T_, MC_) if (T == T_ && MC == MC_) return true;
    BSP_TRI_SHAPES(BSP_IS)
#undef BSP_IS
    return false;
}

// Overrides installed by the autotuner: per kernel, M ranges -> shape.  The
// table is process-wide; a reader-writer lock makes concurrent lookups and
// updates from several host threads safe (a launch takes the shape current
// when it looks it up).
struct ShapeOverride {
    int M_lo, M_hi;
    TriShape sh;
};
constexpr int kMaxOverrides = 16;
static ShapeOverride g_over[2][kMaxOverrides];
static int g_nover[2] = {0, 0};
static std::shared_mutex g_over_mutex;

TriShape shape_for(int kernel, int M) {
    std::shared_lock<std::shared_mutex> lock(g_over_mutex);
    for (int i = g_nover[kernel] - 1; i >= 0; --i) {
        const ShapeOverride& o = g_over[kernel][i];
        if (M >= o.M_lo && M <= o.M_hi) return o.sh;
    }
    return default_shape(kernel, M);
}

TriShape tri_shape(int M) {
    const TriShape a = shape_for(0, M), b = shape_for(1, M);
    return (a.T && b.T) ? a : TriShape{0, 0};
}

int set_shape_override(int kernel, int M_lo, int M_hi, int T, int MC) {
    BSP_CHECK_ARG(kernel == 0 || kernel == 1, "kernel must be 0 (fine/coarse batch) or 1 (sweep)");
    BSP_CHECK_ARG(M_lo >= 1 && M_hi >= M_lo && M_hi <= kMaxM, "invalid M range");
    BSP_CHECK_ARG(shape_built(T, MC), "block shape (%d threads, %d nodes/thread) is not built", T,
                  MC);
    BSP_CHECK_ARG((long)T * MC >= M_hi, "shape covers %d nodes, range needs %d", T * MC, M_hi);
    std::unique_lock<std::shared_mutex> lock(g_over_mutex);
    BSP_CHECK_ARG(g_nover[kernel] < kMaxOverrides, "too many shape overrides");
    g_over[kernel][g_nover[kernel]++] = {M_lo, M_hi, {T, MC}};
    return BS_OK;
}

void reset_shape_overrides() {
    std::unique_lock<std::shared_mutex> lock(g_over_mutex);
    g_nover[0] = g_nover[1] = 0;
}

bool pipe_capable(int M) { return !is_large(shape_for(0, M)) && !is_large(shape_for(1, M)); }

int launch_theta_batch(const OptionDev& o, int M, int nsys, const double* tau0, double tau_start,
                       double tau_stride, int sys_offset, double dt, int steps, double theta,
                       const double* u_in, long ld_in, double* u_out, long ld_out,
                       hipStream_t stream, const int* stop, const PipeSync* ps) {
    if (nsys == 0) return BS_OK;
    const TriShape sh = shape_for(0, M);
    ThetaArgs a{o,          M,  steps, sys_offset, tau0,  tau_start, tau_stride,
                dt,         theta, u_in, ld_in,   u_out, ld_out,    stop};
    if (ps) {
        if (is_large(sh) || !stop) {
            set_error("overlapped fine launch needs a stop flag and a grid of at most 4096 nodes");
            return BS_ERR_ARG;
        }
        a.ps = *ps;
#define BSP_CASE(T_, MC_)                                                                  \
    if (sh.T == T_ && sh.MC == MC_) {                                                      \
        hipLaunchKernelGGL((k_theta_pipe<T_, MC_>), dim3(nsys), dim3(T_), 0, stream, a);   \
        BSP_LAUNCHED();                                                                    \
        return BS_OK;                                                                      \
    }
        BSP_TRI_SHAPES(BSP_CASE)
#undef BSP_CASE
        set_error("M = %d is beyond the supported range of the tridiagonal kernels", M);
        return BS_ERR_ARG;
    }
    if (is_large(sh)) {
        const bool hi = M % sh.MC != 0;
        if (sh.MC == 16) {
            if (hi) hipLaunchKernelGGL((k_rc_theta<512, 16, true>), dim3(nsys), dim3(512), 0, stream, a);
            else hipLaunchKernelGGL((k_rc_theta<512, 16, false>), dim3(nsys), dim3(512), 0, stream, a);
        } else {
            if (hi) hipLaunchKernelGGL((k_rc_theta<512, 32, true>), dim3(nsys), dim3(512), 0, stream, a);
            else hipLaunchKernelGGL((k_rc_theta<512, 32, false>), dim3(nsys), dim3(512), 0, stream, a);
        }
        BSP_LAUNCHED();
        return BS_OK;
    }
#define BSP_CASE(T_, MC_)                                                                   \
    if (sh.T == T_ && sh.MC == MC_) {                                                       \
        hipLaunchKernelGGL((k_theta_batch<T_, MC_>), dim3(nsys), dim3(T_), 0, stream, a);   \
        BSP_LAUNCHED();                                                                     \
        return BS_OK;                                                                       \
    }
    BSP_TRI_SHAPES(BSP_CASE)
#undef BSP_CASE
    set_error("M = %d is beyond the supported range of the tridiagonal kernels", M);
    return BS_ERR_ARG;
}

// One slice of the sweep with the flow-map coarse (one block): see
// launch_flow_correct.  Same arithmetic per node as sweep_slices.
__global__ __launch_bounds__(1024) void k_flow_correct(int M, int predict, int first,
                                                       const double* __restrict__ g,
                                                       const double* __restrict__ fv,
                                                       double* __restrict__ gold, double* un1,
                                                       double* __restrict__ result) {
    __shared__ double red[1024];
    __shared__ int rbad[1024];
    double dmax = 0.0;
    int bad = 0;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double gg = g[j];
        if (predict) {
            un1[j] = gg;
            gold[j] = gg;
        } else {
            const double uo = un1[j];
            const double unew = fv[j] + (gg - gold[j]);
            gold[j] = gg;
            un1[j] = unew;
            dmax = fmax(dmax, fabs(unew - uo));
            bad |= !isfinite(unew);
        }
    }
    if (predict) return;
    red[threadIdx.x] = dmax;
    rbad[threadIdx.x] = bad;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
            rbad[threadIdx.x] |= rbad[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        result[0] = first ? red[0] : fmax(result[0], red[0]);
        result[1] = (rbad[0] || (!first && result[1] != 0.0)) ? 1.0 : 0.0;
    }
}

int launch_flow_correct(int M, bool predict, bool first, const double* g, const double* fv,
                        double* gold, double* un1, double* result, hipStream_t stream) {
    hipLaunchKernelGGL(k_flow_correct, dim3(1), dim3(1024), 0, stream, M, predict ? 1 : 0,
                       first ? 1 : 0, g, fv, gold, un1, result);
    BSP_LAUNCHED();
    return BS_OK;
}

int launch_sweep(const SweepArgs& a, hipStream_t stream) {
    const TriShape sh = shape_for(1, a.M);
    if (is_large(sh)) {
        if (!a.tab) {
            set_error("the large-grid sweep needs its coefficient tables");
            return BS_ERR_ARG;
        }
        int rc = launch_large_sweep_setup(a.o, a.M, a.dT, a.coarse_steps, a.tab, stream);
        if (rc) return rc;
        SweepArgs b = a;
        b.ptab = a.tab + (size_t)kLgFields * 32 * 512;
        if (sh.MC == 16)
            hipLaunchKernelGGL((k_large_sweep<512, 16>), dim3(1), dim3(512), 0, stream, b);
        else
            hipLaunchKernelGGL((k_large_sweep<512, 32>), dim3(1), dim3(512), 0, stream, b);
        BSP_LAUNCHED();
        return BS_OK;
    }
#define BSP_CASE(T_, MC_)                                                        \
    if (sh.T == T_ && sh.MC == MC_) {                                            \
        hipLaunchKernelGGL((k_sweep<T_, MC_>), dim3(1), dim3(T_), 0, stream, a); \
        BSP_LAUNCHED();                                                          \
        return BS_OK;                                                            \
    }
    BSP_TRI_SHAPES(BSP_CASE)
#undef BSP_CASE
    set_error("M = %d is beyond the supported range of the tridiagonal kernels", a.M);
    return BS_ERR_ARG;
}

}  // namespace bsp
