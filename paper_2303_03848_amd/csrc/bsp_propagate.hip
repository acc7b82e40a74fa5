// Propagator kernels: expiry payoff, the batched theta-method (Crank-Nicolson
// fine F, implicit-Euler coarse G) and the serial Parareal correction sweep.
#include "bsp_common.hpp"
#include "bsp_tridiag.hpp"

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

// ------------------------------------------------------ shared helpers

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

// Steps per boundary-forcing table (two tables of this many doubles in LDS).
constexpr int kForceChunk = 1024;

// `steps` theta-steps of size dt from tau0 on the state V (this block's system).
// The boundary forcing of each step, (1-theta) dt g(tau_m) + theta dt g(tau_{m+1})
// at S = 0 and S = S_max, is tabulated in LDS for a chunk of steps by all
// threads in parallel, so the sequential step loop evaluates no exponential.
// ftab: 2 * kForceChunk doubles of LDS.
template <int T, int MC>
__device__ __forceinline__ void theta_steps(const BlockTri<T, MC>& S, const OptionDev& o,
                                            double (&V)[MC], double tau0, double dt, int steps,
                                            double theta, bool homog, double* lds, double* ftab) {
    double hl, hr;
    S.halo(V, hl, hr, lds);
    const double h = theta * dt, e = (1.0 - theta) * dt;
    for (int m0 = 0; m0 < steps; m0 += kForceChunk) {
        const int nch = min(kForceChunk, steps - m0);
        if (!homog) {
            __syncthreads();  // the previous chunk's table has been consumed
            for (int i = threadIdx.x; i < nch; i += T) {
                const int mm = m0 + i;
                double lo0, hi0, lo1, hi1;
                dirichlet(o, exp(-o.r * (tau0 + (double)mm * dt)), lo0, hi0);
                dirichlet(o, exp(-o.r * (tau0 + (double)(mm + 1) * dt)), lo1, hi1);
                ftab[i] = fma(e, lo0, h * lo1);
                ftab[kForceChunk + i] = fma(e, hi0, h * hi1);
            }
            __syncthreads();
        }
        double flo_n = homog ? 0.0 : ftab[0];
        double fhi_n = homog ? 0.0 : ftab[kForceChunk];
        for (int i = 0; i < nch; ++i) {
            const double flo = flo_n, fhi = fhi_n;
            if (!homog && i + 1 < nch) {
                flo_n = ftab[i + 1];
                fhi_n = ftab[kForceChunk + i + 1];
            }
            S.step(V, hl, hr, flo, fhi, lds);
        }
    }
}

// ------------------------------------------------ batched theta-method

struct ThetaArgs {
    OptionDev o;
    int M, steps, homog, sys_offset;
    const double* tau0;
    double tau_start, tau_stride, dt, theta;
    const double* u_in;
    long ld_in;
    double* u_out;
    long ld_out;
};

template <int T, int MC>
__global__ __launch_bounds__(T) void k_theta_batch(ThetaArgs a) {
    __shared__ double lds[4 * T];
    __shared__ double ftab[2 * kForceChunk];
    const int sys = blockIdx.x;
    BlockTri<T, MC> S;
    S.setup(a.o.s2, a.o.r, a.theta * a.dt, (1.0 - a.theta) * a.dt, a.M, lds);
    const double tau0 =
        a.tau0 ? a.tau0[sys] : a.tau_start + (double)(sys + a.sys_offset) * a.tau_stride;
    double V[MC];
    load_chunk<T, MC>(a.u_in + (long)sys * a.ld_in, a.M, V);
    theta_steps<T, MC>(S, a.o, V, tau0, a.dt, a.steps, a.theta, a.homog != 0, lds, ftab);
    store_chunk<T, MC>(a.u_out + (long)sys * a.ld_out, a.M, V);
}

// ---------------------------------------------------- Parareal sweep

// Serial over slices n = n0..N-1 in one block:
//   g = G(U[n])                       (state carried in registers)
//   predict: U[n+1] = g, Gold[n] = g
//   else:    U[n+1] = Fv[n] + (g - Gold[n]), Gold[n] = g,
//            defect = max |U_new[n+1] - U_old[n+1]|, non-finite flag.
template <int T, int MC>
__global__ __launch_bounds__(T) void k_sweep(SweepArgs a) {
    __shared__ double lds[4 * T];
    __shared__ double ftab[2 * kForceChunk];
    const int M = a.M;
    const double dtc = a.dT / (double)a.coarse_steps;
    BlockTri<T, MC> S;
    S.setup(a.o.s2, a.o.r, dtc, 0.0, M, lds);
    const int i0 = threadIdx.x * MC;
    const bool net = a.kind != BS_COARSE_IE;

    double V[MC];
    load_chunk<T, MC>(a.U + (long)a.n0 * M, M, V);
    double dmax = 0.0;
    int bad = 0;
    for (int n = a.n0; n < a.N; ++n) {
        double* un1 = a.U + (long)(n + 1) * M;
        double* go = a.Gold + (long)n * M;
        // Loads that do not depend on the coarse solve go first, so their
        // latency overlaps it (when registers allow: small chunks).
        constexpr bool kPrefetch = MC <= 4;
        double fv[MC], gold[MC], uold[MC], vt0[MC], vt1[MC];
        if (kPrefetch && !a.predict) {
            load_chunk<T, MC>(a.Fv + (long)n * M, M, fv);
            load_chunk<T, MC>(go, M, gold);
            load_chunk<T, MC>(un1, M, uold);
        }
        if (kPrefetch && net) {
            load_chunk<T, MC>(a.Vt + (long)(n + 1) * M, M, vt1);
            if (a.kind == BS_COARSE_PINN_IE) load_chunk<T, MC>(a.Vt + (long)n * M, M, vt0);
        }
        double g[MC];
        if (a.kind == BS_COARSE_IE) {
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = V[q];
            theta_steps<T, MC>(S, a.o, g, (double)n * a.dT, dtc, a.coarse_steps, 1.0, false, lds,
                               ftab);
        } else if (a.kind == BS_COARSE_PINN) {
            if (!kPrefetch) load_chunk<T, MC>(a.Vt + (long)(n + 1) * M, M, vt1);
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = vt1[q];
        } else {
            if (!kPrefetch) load_chunk<T, MC>(a.Vt + (long)n * M, M, vt0);
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = V[q] - vt0[q];
            theta_steps<T, MC>(S, a.o, g, (double)n * a.dT, dtc, a.coarse_steps, 1.0, true, lds,
                               ftab);
            if (!kPrefetch) load_chunk<T, MC>(a.Vt + (long)(n + 1) * M, M, vt1);
#pragma unroll
            for (int q = 0; q < MC; ++q) g[q] = vt1[q] + g[q];
        }
        if (!kPrefetch && !a.predict) {
            load_chunk<T, MC>(a.Fv + (long)n * M, M, fv);
            load_chunk<T, MC>(go, M, gold);
            load_chunk<T, MC>(un1, M, uold);
        }
        if (a.predict) {
            store_chunk<T, MC>(un1, M, g);
            store_chunk<T, MC>(go, M, g);
#pragma unroll
            for (int q = 0; q < MC; ++q) V[q] = g[q];
        } else {
#pragma unroll
            for (int q = 0; q < MC; ++q) {
                const double unew = fv[q] + (g[q] - gold[q]);
                if (i0 + q < M) {
                    go[i0 + q] = g[q];
                    un1[i0 + q] = unew;
                    dmax = fmax(dmax, fabs(unew - uold[q]));
                    bad |= !isfinite(unew);
                }
                V[q] = (i0 + q < M) ? unew : 0.0;
            }
        }
    }
    if (!a.predict) {
        // block max of the defect and OR of the flag
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
        if (threadIdx.x == 0) {
            a.result[0] = lds[0];
            a.result[1] = lds[T];
        }
    }
}

// ------------------------------------------------------------ dispatch

// Default block shapes.  The F kernel favours one wavefront per system (no
// barriers) while its registers allow; the serial sweep is one block for the
// whole grid and favours more threads per system.
static TriShape default_shape(int kernel, int M) {
    if (kernel == 0) {
        if (M <= 128) return {64, 2};
        if (M <= 256) return {64, 4};
        if (M <= 512) return {64, 8};
        if (M <= 1024) return {64, 16};
        if (M <= 2048) return {256, 8};
        if (M <= 4096) return {512, 8};
    } else {
        if (M <= 128) return {64, 2};
        if (M <= 256) return {64, 4};
        if (M <= 512) return {128, 4};
        if (M <= 1024) return {256, 4};
        if (M <= 2048) return {256, 8};
        if (M <= 4096) return {512, 8};
    }
    return {0, 0};
}

#define BSP_TRI_SHAPES(X) \
    X(64, 2) X(64, 4) X(64, 8) X(64, 16) X(128, 4) X(128, 8) X(256, 4) X(256, 8) X(512, 8)

static bool shape_built(int T, int MC) {
#define BSP_IS(T_, MC_) if (T == T_ && MC == MC_) return true;
    BSP_TRI_SHAPES(BSP_IS)
#undef BSP_IS
    return false;
}

// Overrides installed by the autotuner: per kernel, M ranges -> shape.
struct ShapeOverride {
    int M_lo, M_hi;
    TriShape sh;
};
constexpr int kMaxOverrides = 16;
static ShapeOverride g_over[2][kMaxOverrides];
static int g_nover[2] = {0, 0};

static TriShape shape_for(int kernel, int M) {
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
    BSP_CHECK_ARG(g_nover[kernel] < kMaxOverrides, "too many shape overrides");
    g_over[kernel][g_nover[kernel]++] = {M_lo, M_hi, {T, MC}};
    return BS_OK;
}

void reset_shape_overrides() { g_nover[0] = g_nover[1] = 0; }

int launch_theta_batch(const OptionDev& o, int M, int nsys, const double* tau0, double tau_start,
                       double tau_stride, int sys_offset, double dt, int steps, double theta,
                       int homog, const double* u_in, long ld_in, double* u_out, long ld_out,
                       hipStream_t stream) {
    if (nsys == 0) return BS_OK;
    const TriShape sh = shape_for(0, M);
    ThetaArgs a{o, M, steps, homog, sys_offset, tau0, tau_start, tau_stride, dt, theta, u_in, ld_in,
                u_out, ld_out};
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

int launch_sweep(const SweepArgs& a, hipStream_t stream) {
    const TriShape sh = shape_for(1, a.M);
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
