// Propagator kernels: expiry payoff, the batched theta-method (Crank-Nicolson
// fine F, implicit-Euler coarse G) and the serial Parareal correction sweep.
#include "bsp_common.hpp"
#include "bsp_steps.hpp"

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

template <int T, int MC>
__global__ __launch_bounds__(T) void k_sweep(SweepArgs a) {
    __shared__ double lds[4 * T];
    __shared__ double ftab[2 * kForceChunk];
    BlockTri<T, MC> S;
    S.setup(a.o.s2, a.o.r, a.dT / (double)a.coarse_steps, 0.0, a.M, lds);
    double dmax = 0.0;
    int bad = 0;
    sweep_slices<T, MC>(S, a.o, a.M, a.N, a.n0, a.coarse_steps, a.kind, a.predict != 0, a.dT, a.U,
                        a.Fv, a.Gold, a.Vt, lds, ftab, dmax, bad);
    if (!a.predict) {
        block_defect<T>(dmax, bad, lds);
        if (threadIdx.x == 0) {
            a.result[0] = dmax;
            a.result[1] = bad ? 1.0 : 0.0;
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

TriShape shape_for(int kernel, int M) {
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
