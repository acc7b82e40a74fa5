// Internal declarations shared by the translation units of libbsparareal.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "bsparareal.h"

namespace bsp {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

#define BSP_CHECK_ARG(cond, ...)           \
    do {                                   \
        if (!(cond)) {                     \
            ::bsp::set_error(__VA_ARGS__); \
            return BS_ERR_ARG;             \
        }                                  \
    } while (0)

#define BSP_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::bsp::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                             __FILE__, __LINE__);                                       \
            return BS_ERR_HIP;                                                          \
        }                                                                               \
    } while (0)

#define BSP_LAUNCHED()                                                                 \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) {                                                        \
            ::bsp::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                      \
            return BS_ERR_HIP;                                                         \
        }                                                                              \
    } while (0)

constexpr int kMaxM = 16384;

// ------------------------------------------------------- model on device

// Coefficients a kernel needs about one option.
struct OptionDev {
    double K, r, s2, s_max, dS;
    int is_put;
};

inline OptionDev make_option(const bs_params& p, int M) {
    OptionDev o;
    o.K = p.K;
    o.r = p.r;
    o.s2 = p.sigma * p.sigma;
    o.s_max = p.s_max;
    o.dS = p.s_max / (double)(M + 1);
    o.is_put = p.is_put;
    return o;
}

// Row j (1-based) of the centred-difference operator in time to maturity,
// dV_j/dtau = al V_{j-1} + be V_j + ga V_{j+1}.  With S_j = j dS the mesh
// width cancels: al = (s2 j^2 - r j)/2, be = -(s2 j^2 + r), ga = (s2 j^2 + r j)/2.
__device__ __forceinline__ void op_row(double s2, double r, double j, double& al, double& be,
                                       double& ga) {
    double q = s2 * j * j;
    double p = r * j;
    al = 0.5 * (q - p);
    be = -(q + r);
    ga = 0.5 * (q + p);
}

// Dirichlet data at S = 0 (lo) and S = S_max (hi) for time to maturity tau.
__device__ __forceinline__ void dirichlet(const OptionDev& o, double disc, double& lo, double& hi) {
    if (o.is_put) {
        lo = o.K * disc;
        hi = 0.0;
    } else {
        lo = 0.0;
        hi = o.s_max - o.K * disc;
    }
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// ------------------------------------------------------- launch shapes

// Block shape of the tridiagonal kernels for M interior nodes: T threads,
// MC consecutive nodes per thread (T * MC >= M).
struct TriShape {
    int T, MC;
};
TriShape tri_shape(int M);  // {0, 0} if M has no kernel shape
TriShape shape_for(int kernel, int M);  // kernel 0: F/G batch, 1: sweep
int set_shape_override(int kernel, int M_lo, int M_hi, int T, int MC);
void reset_shape_overrides();

// ------------------------------------------- overlapped Parareal iterations
// Per-slice progress counters of a solve whose fine launch of iteration k+1
// runs alongside the sweep of iteration k (all zero at the start of a solve,
// in the caller's workspace):
//   ready[n] = j + 1 once U[n] holds iterate j (n = 0..N),
//   taken[n] = k once the fine launch of iteration k has read U[n],
//   fdone[n] = k once it has written Fv[n].
// Every wait names a counter that only earlier-queued work advances, so any
// serialisation of the launches completes.  A wait also ends when *stop is
// set (the solve has converged) or when *err is set; after kPipeSpinTicks of
// the constant-rate clock it sets *err itself.
struct PipeSync {
    int* ready;
    int* taken;
    int* fdone;
    int* err;
    int k;  // iteration of the launch (0: the prediction sweep)
};
constexpr long long kPipeSpinTicks = 200000000LL;  // 2 s at 100 MHz

__device__ __forceinline__ int pipe_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide wait for *f >= v: thread 0 polls and the outcome is shared
// through *slot (LDS).  ACQ: every thread then orders its later loads after
// the producer's stores (needed when the block reads what the producer
// wrote; a wait that only orders this block's later stores after the
// producer's loads needs no fence).  Returns false if the block must stop
// (stop or error).
template <bool ACQ = true>
__device__ inline bool pipe_wait(const PipeSync& ps, const int* f, int v, const int* stop,
                                 int* slot) {
    __syncthreads();  // slot may still be read from the previous wait
    if (threadIdx.x == 0) {
        int ok = 1;
        if (pipe_load(f) < v) {
            const long long t0 = wall_clock64();
            while (pipe_load(f) < v) {
                if ((stop && pipe_load(stop)) || pipe_load(ps.err)) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > kPipeSpinTicks) {
                    __hip_atomic_store(ps.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        *slot = ok;
    }
    __syncthreads();
    const bool ok = *slot != 0;
    if constexpr (ACQ) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

// The same for a wavefront working on its own (the block's other wavefronts
// do unrelated work): every lane polls the same counter, so the outcome is
// uniform without LDS or a barrier.
template <bool ACQ = true>
__device__ inline bool pipe_wait_wave(const PipeSync& ps, const int* f, int v, const int* stop) {
    bool ok = true;
    if (__builtin_amdgcn_readfirstlane(pipe_load(f)) < v) {
        const long long t0 = wall_clock64();
        while (__builtin_amdgcn_readfirstlane(pipe_load(f)) < v) {
            if ((stop && __builtin_amdgcn_readfirstlane(pipe_load(stop))) ||
                __builtin_amdgcn_readfirstlane(pipe_load(ps.err))) {
                ok = false;
                break;
            }
            if (wall_clock64() - t0 > kPipeSpinTicks) {
                if ((threadIdx.x & 63) == 0)
                    __hip_atomic_store(ps.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if constexpr (ACQ) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

__device__ inline void pipe_signal_wave(int* f, int v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & 63) == 0)
        __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Orders this wavefront's LDS accesses (lanes exchanging data through LDS
// without a block barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Publishes *f = v once the block's loads have completed (it wrote nothing
// the reader needs): after a barrier that follows their use.
__device__ inline void pipe_mark(int* f, int v) {
    if (threadIdx.x == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes *f = v after every thread's stores of the block.
__device__ inline void pipe_signal(int* f, int v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------- internal launchers

// theta-method on nsys independent systems: tau of system s = tau0[s] if
// tau0 != nullptr else tau_start + (s + sys_offset) * tau_stride.
int launch_theta_batch(const OptionDev& o, int M, int nsys, const double* tau0, double tau_start,
                       double tau_stride, int sys_offset, double dt, int steps, double theta,
                       const double* u_in, long ld_in, double* u_out, long ld_out,
                       hipStream_t stream, const int* stop = nullptr,
                       const PipeSync* ps = nullptr);

struct SweepArgs {
    OptionDev o;
    int M, N, n0, coarse_steps, kind, predict;
    double dT;                     // slice length
    double* U;                     // [N+1][M]
    const double* Fv;              // [N][M]
    double* Gold;                  // [N][M]
    const double* Vt;              // [N+1][M] or nullptr
    double* result;                // [0] defect, [1] status, [2] defect of iteration 1
    // Device-side stopping (asynchronous solve; all three may be null):
    // the sweep returns at once while *stop is set, and on finishing
    // iteration k it writes hist[2k] = defect, hist[2k+1] = status (0; 1
    // non-finite; 2 diverged: k >= 2 and defect > growth x the defect of
    // iteration 1) and sets *stop when the iteration is the last one
    // (defect <= tol or status != 0).
    int* stop;
    double* hist;
    double tol;
    int k;
    PipeSync ps;  // overlapped solve (ps.ready null: not overlapped)
    double growth = __builtin_inf();  // divergence guard (infinite: none)
    // grids beyond 4096 nodes: workspace space for the implicit-Euler tables
    // (large_sweep_table_doubles(M) doubles; ptab is set by launch_sweep)
    double* tab = nullptr;
    const double* ptab = nullptr;
};
size_t large_sweep_table_doubles(int M);  // 0 for grids the sweep solves in registers
const double* large_sweep_ptab(const double* tab);  // the per-thread part of the tables
int launch_large_sweep_setup(const OptionDev& o, int M, double dT, int coarse_steps, double* tab,
                             hipStream_t stream);
int launch_sweep(const SweepArgs& a, hipStream_t stream);

// Whole overlapped solve in one launch (see k_parareal_persist).  Iterate k
// lives in U (k even) or U2 (k odd); the launch leaves the last iterate in U.
struct PersistArgs {
    OptionDev o;
    int M, N, kmax, fine_steps, coarse_steps, kind, nfb, nsb;
    double dT, tol;
    double* U;
    double* U2;
    double* Fv;
    double* Gold;
    const double* Vt;
    double* result;
    int* stop;
    double* hist;     // host-mapped record [2 (kmax+1)]
    int* decided;     // [kmax+1]: the sweep of iteration k has recorded its defect
    int* exited;      // blocks that have finished
    int* stop_rank;   // kmax + 1 - (first iteration that met the stopping rule), 0: none
    PipeSync ps;
    double growth;    // divergence guard, as in SweepArgs
};
// Overlapped solve of a grid beyond 4096 nodes (see k_large_persist): after
// slice 0's iteration-1 fine propagation, one launch runs the prediction and
// the sweeps of every iteration in one block and the fine work of iterations
// 1, 2, ... in one block per slice n >= 1.
struct LargePersistArgs {
    OptionDev o;
    int M, N, kmax, fine_steps, coarse_steps, kind;
    double dT, tol, growth;
    // U, Fv, Gold, Vt: chunk-major levels (large_cm_level(M) doubles apart)
    double* U;
    double* Fv;
    double* Gold;
    const double* Vt;
    double* result;
    int* stop;
    double* hist;  // per-iteration record [2 (kmax+1)] (host-mapped or device)
    PipeSync ps;
    const double* tab;  // the sweep's implicit-Euler tables (launch_large_sweep_setup)
    const double* ptab;
};
bool large_persist_capable(int M, int N);
// Grids beyond 4096 nodes: doubles per chunk-major level (T * MC of the
// fine shape), 0 for smaller grids; conversion of `levels` levels between
// node order [levels][M] and chunk-major [levels][T*MC].
long large_cm_level(int M);
int launch_cm_convert(const double* src, double* dst, int levels, int M, bool to_cm,
                      hipStream_t stream);
int launch_large_persist(const LargePersistArgs& a, hipStream_t stream);

// The one-launch solve can cover this problem size (block shapes aside).
constexpr int kPersistMaxN = 512, kPersistMaxM = 1024;
inline bool persist_possible(int M, int N) { return M <= kPersistMaxM && N <= kPersistMaxN; }
bool persist_capable(int M, int N);
int launch_parareal_persist(const PersistArgs& a, hipStream_t stream);
int launch_set_int(int* p, int v, hipStream_t stream);  // *p = v in stream order
int launch_fill_int(int* p, int n, int v, hipStream_t stream);  // p[0..n) = v
int launch_fill_double(double* p, int n, double v, hipStream_t stream);  // p[0..n) = v
bool pipe_capable(int M);  // the overlapped solve covers grids of this size

int launch_initial(const OptionDev& o, int M, int payoff_mode, double* u0, hipStream_t stream);

// Network evaluated on the Parareal grid: Vt[n][j] = K v(n dT, (j+1) dS / K).
// Flow-map coarse of one slice: g[j] = K w(tau_s, tau_e, Us[j] / K, S_j / K).
int launch_flowmap(const pinn_net& net, const OptionDev& o, int M, double tau_s, double tau_e,
                   const double* Us, double* g, hipStream_t stream);
// The correction of one slice with the flow-map coarse (g = G(U[n]) given):
// predict: U[n+1] = Gold[n] = g; else U[n+1] = Fv[n] + (g - Gold[n]),
// Gold[n] = g, result[0] = max over the slices since `first` of
// max |U_new - U_old|, result[1] = 1 if a value is not finite.
int launch_flow_correct(int M, bool predict, bool first, const double* g, const double* fv,
                        double* gold, double* un1, double* result, hipStream_t stream);
int launch_pinn_grid(const pinn_net& net, const OptionDev& o, int M, int N, double dT, double* Vt,
                     hipStream_t stream);

// Batched options: one record per option (device), and the tiles of 32
// network-grid points (each inside one option's grid).
struct BatchOpt {
    OptionDev o;
    int M, N, fine_steps, coarse_steps;
    double dT;
    long u_off;   // option's U in the caller's packed array
    long w_off;   // option's Fv / Gold in the workspace (N*M each)
    long vt_off;  // option's network grid (N+1)*M in the packed grid array
};
struct BatchState {
    int done, iters, bad, pad;  // bad: 1 non-finite, 2 diverged (as SweepArgs' status)
    double defect, first;       // last defect, defect of iteration 1
};
struct BatchTile {
    int opt, pad;
    long base, count;  // packed index of the option's first grid point; (N+1)*M
};

int check_net(const pinn_net* net);
int release_batch_resources();  // class streams and events of this thread
long net_param_count(const pinn_net& net);

}  // namespace bsp
