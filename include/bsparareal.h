/*
 * bsparareal: Parareal for the Black-Scholes equation on one AMD Instinct
 * MI355X (gfx950).  C ABI of libbsparareal.so.
 *
 * The method is the one of "Parareal with a physics-informed neural network
 * as coarse propagator" (Ibrahim, Goetschel, Ruprecht):
 *   - the model, eqs. (1)-(4): the Black-Scholes equation for a European
 *     option with expiry payoff and Dirichlet conditions at S = 0 and S_max;
 *   - the space discretisation, Sec. 3.2: second-order centred differences on
 *     S_j = j dS, j = 1..M, dS = S_max/(M+1); the problem is integrated in
 *     time to maturity tau = T - t (the paper solves backwards from T);
 *   - the propagators, Sec. 3.2: Crank-Nicolson as fine F, implicit Euler as
 *     numerical coarse G; Sec. 3.3: a physics-informed network as coarse G;
 *   - the iteration, Sec. 3.1 eq. (7):
 *       U^k_{n+1} = G(U^k_n) + F(U^{k-1}_n) - G(U^{k-1}_n),
 *     with F run on all N time slices concurrently;
 *   - the network loss, eqs. (11)-(14).
 *
 * Conventions for every call:
 *   - All array arguments are DEVICE pointers to caller-owned, contiguous,
 *     row-major memory unless marked "host".  The library never frees or
 *     keeps caller memory beyond the call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on it unless stated otherwise.
 *   - Return value: BS_OK (0) on success, a negative BS_ERR_* code on error
 *     (nothing has been launched when an argument check fails), or the
 *     positive warning BS_NOT_CONVERGED.  bs_last_error() gives a message.
 *     No C++ exception crosses the ABI.
 *   - Limits: 1 <= M <= 16384 interior nodes; 1 <= N; steps >= 1.
 */
#ifndef BSPARAREAL_H
#define BSPARAREAL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    BS_OK = 0,
    BS_NOT_CONVERGED = 1,  /* max_iter reached before tol; outputs are the last iterate */
    BS_ERR_ARG = -1,       /* invalid argument (null pointer, size out of range, ...) */
    BS_ERR_HIP = -2,       /* a HIP runtime call failed */
    BS_ERR_NONFINITE = -3, /* a NaN or Inf appeared in the Parareal state */
    BS_ERR_DIVERGED = -4,  /* the defect grew by bs_divergence_growth() over the first one */
    BS_ERR_WORKSPACE = -5  /* workspace pointer null or too small */
};

/* Divergence guard of parareal_solve and parareal_solve_batch.  Eq. (7)
 * reaches the serial fine solution after N iterations whatever G is (Sec.
 * 3.1), but an iteration whose defect grows instead of shrinking is not
 * converging and, in floating point, amplifies rounding errors: the solve
 * stops at the first iteration k >= 2 whose defect exceeds `growth` times
 * the defect of iteration 1 and returns BS_ERR_DIVERGED (the state is that
 * iterate).  Default BS_DIVERGENCE_GROWTH; bs_set_divergence_growth(g) sets
 * it for later solves of the whole process (g > 0, INFINITY turns the guard
 * off; BS_ERR_ARG otherwise). */
#define BS_DIVERGENCE_GROWTH 1.0e3
int bs_set_divergence_growth(double growth);
double bs_divergence_growth(void);

/* Option and model coefficients (eq. (1)): strike K, riskless rate r,
 * volatility sigma, expiry T, truncation S_max of the asset axis.
 * is_put = 0: call, V(tau,0) = 0, V(tau,S_max) = S_max - K exp(-r tau);
 * is_put = 1: put,  V(tau,0) = K exp(-r tau), V(tau,S_max) = 0. */
typedef struct bs_params {
    double K, r, sigma, T, s_max;
    int is_put;
} bs_params;

/* Space grid: M interior nodes.  payoff_mode 0 samples the expiry payoff
 * (eq. (2)) at S_j; payoff_mode 1 averages it over [S_j - dS/2, S_j + dS/2]. */
typedef struct bs_grid {
    int M;
    int payoff_mode;
} bs_grid;

/* Time slices (Sec. 3.1): N slices of length T/N; F takes fine_steps
 * Crank-Nicolson steps per slice, the numerical G coarse_steps implicit-Euler
 * steps per slice. */
typedef struct bs_slices {
    int N;
    int fine_steps;
    int coarse_steps;
} bs_slices;

/* Coarse propagator kinds (Sec. 3.3 for the network ones).
 *   BS_COARSE_IE      : coarse_steps implicit-Euler steps.
 *   BS_COARSE_PINN    : G(U_n) = Vt_{n+1}, the network's price at the end of
 *                       slice n, independent of U_n (the literal reading).
 *   BS_COARSE_PINN_IE : G(U_n) = Vt_{n+1} + E(U_n - Vt_n), E = coarse_steps
 *                       implicit-Euler steps with zero boundary data: the
 *                       network anchors the state, one cheap solve carries
 *                       the deviation.
 *   BS_COARSE_FLOWMAP : G(U_n)(S_j) = K * w(tau_n, tau_{n+1}, U_n(S_j) / K, S_j / K)
 *                       with w a network of 4 inputs: the coarse interface
 *                       of Sec. 3.3 (slice start and end, the state at the
 *                       start, the asset price) applied node by node to the
 *                       state.  Evaluated inside the sweep, slice after
 *                       slice; parareal_start, parareal_iterate and
 *                       parareal_solve only (iterations one after the other;
 *                       coarse_steps unused).
 * Vt_n(S_j) = K * v(tau_n, S_j / K) with v the network of `pinn_net`. */
enum { BS_COARSE_IE = 0, BS_COARSE_PINN = 1, BS_COARSE_PINN_IE = 2, BS_COARSE_FLOWMAP = 3 };

/* Network arithmetic. */
enum { BS_PREC_FP32 = 0, BS_PREC_BF16 = 1 };

/* A fully connected tanh network (Sec. 3.3) with n_in inputs (2: (tau, S/K);
 * 4: (tau, S/K, sigma, r)), `depth` hidden tanh layers of `width` units and
 * one linear output v = V/K.  `params` (device, float32) packs the layers in
 * torch.nn.Linear order: W1[width][n_in], b1[width], W2[width][width], b2,
 * ..., W_depth, b_depth, Wo[1][width], bo[1]; its length is
 *   width*n_in + width + (depth-1)*(width*width + width) + width + 1.
 * precision BS_PREC_BF16: matrix products take bfloat16 inputs on the matrix
 * cores with float32 accumulation; BS_PREC_FP32: float32 throughout.
 * Limits: n_in in {2, 4}; 1 <= depth <= 16; width in {16, 32, 64, 128, 256}. */
typedef struct pinn_net {
    int n_in, depth, width, precision;
    const float* params;
} pinn_net;

/* Message describing the last error of the calling thread ("" if none). */
const char* bs_last_error(void);

/* Expiry payoff at the interior nodes (eq. (2), or its put analogue):
 * u0[M] (device, out). */
int bs_initial(const bs_params* prm, const bs_grid* grid, double* u0, void* stream);

/* Fine propagator F on a batch of independent systems (Sec. 3.2):
 * system s starts at time to maturity tau0[s] (device, [nsys]) from state
 * u_in[s][0..M) and takes `steps` Crank-Nicolson steps of size dtau/steps
 * with the exact Dirichlet data of `prm` at every time level; the result goes
 * to u_out[s][0..M).  u_in and u_out may be the same array.
 * Errors: BS_ERR_ARG for null pointers, nsys < 0, steps < 1, dtau <= 0, M
 * out of range; BS_ERR_HIP if the launch fails. */
int bs_fine_propagate_batch(const bs_params* prm, const bs_grid* grid, int nsys,
                            const double* tau0, double dtau, int steps, const double* u_in,
                            double* u_out, void* stream);

/* Numerical coarse propagator G (Sec. 3.2): as bs_fine_propagate_batch with
 * implicit-Euler steps. */
int bs_coarse_numeric(const bs_params* prm, const bs_grid* grid, int nsys, const double* tau0,
                      double dtau, int steps, const double* u_in, double* u_out, void* stream);

/* Network forward pass (Sec. 3.3): v_out[i] = v(X[i][0..n_in)), i < n.
 * X: device float32 [n][n_in]; v_out: device float32 [n]. */
int pinn_forward(const pinn_net* net, int n, const float* X, float* v_out, void* stream);

/* *bytes (host, out) = bytes of device workspace pinn_residual_fwd_bwd needs
 * for these point counts.  BS_ERR_ARG on an invalid network or counts. */
int pinn_residual_workspace_size(const pinn_net* net, int n_f, int n_e, int n_b, size_t* bytes);

/* PINN loss and its gradient (eqs. (11)-(14)), one fused pass.
 * Interior points X_f [n_f][n_in]: residual
 *     f = v_tau - sigma^2 x^2 v_xx / 2 - r x v_x + r v   (eq. (1) in tau, x = S/K, v = V/K),
 *   with v_tau, v_x, v_xx differentiated through the network by hand-written
 *   forward-mode streams (the paper uses automatic differentiation).
 * Terminal points X_e [n_e][n_in]: target y_e[i] (device float32 [n_e]) or,
 *   with y_e NULL, the expiry condition of eq. (2) at tau = 0, max(x-1,0)
 *   (call) or max(1-x,0) (put).  With targets given the set is any set of
 *   value-matching points (e.g. fine-propagator data, and with n_f = n_b = 0
 *   the loss of a network trained on data alone).
 * Boundary points X_b [n_b][n_in]: target y_b[i] (device float32 [n_b]) or,
 *   with y_b NULL, eqs. (3)-(4): x == 0 is the lower boundary (call 0, put
 *   exp(-r tau)); any other x is the upper one (call x - exp(-r tau), put 0).
 * sigma and r come from `prm` when n_in == 2 and from columns 2, 3 of X when
 * n_in == 4; prm->is_put selects the targets (prm must not be NULL; K, T,
 * s_max are not used).
 * Outputs (device, float32): loss3[3] = (MSE_f, MSE_exp, MSE_b); grad[n_params]
 * = d(MSE_f + MSE_exp + MSE_b)/d params, packed like net->params.
 * ws: device workspace of pinn_residual_workspace_size() bytes.
 * n_f, n_e, n_b >= 0; an empty set contributes 0 to loss and gradient.
 * The sums over points run in a fixed order: the result is the same from
 * call to call.  Precision BS_PREC_BF16 (width 32, 64 or 128): the whole pass
 * is one launch plus a reduction, the hidden-layer products take bfloat16
 * operands (everything else float32); params and ws must then be 16-byte
 * aligned (BS_ERR_ARG otherwise).  BS_ERR_WORKSPACE if ws_bytes is too small. */
int pinn_residual_fwd_bwd(const pinn_net* net, const bs_params* prm, int n_f, const float* X_f,
                          int n_e, const float* X_e, const float* y_e, int n_b, const float* X_b,
                          const float* y_b, float* loss3, float* grad, void* ws, size_t ws_bytes,
                          void* stream);

/* *bytes (host, out) = bytes of device workspace one Parareal solve needs (F
 * and coarse values, progress counters, a second state buffer for the
 * one-launch solve, and the network grid for the network kinds).  BS_ERR_ARG
 * on an invalid grid, slice count or kind. */
int parareal_workspace_size(const bs_grid* grid, const bs_slices* sl, int coarse_kind,
                            size_t* bytes);

/* Start a Parareal solve: U[0] = expiry payoff; for the network kinds the
 * network is evaluated at every (tau_n, S_j), n = 0..N; then the coarse
 * prediction U[n+1] = G(U[n]), n = 0..N-1 (iteration k = 0).
 * U: device [N+1][M] (out).  ws: device workspace (state kept between calls). */
int parareal_start(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                   int coarse_kind, const pinn_net* net, void* ws, size_t ws_bytes, double* U,
                   void* stream);

/* One Parareal iteration k >= 1 (eq. (7)) on the state left by
 * parareal_start / the previous iteration: F on every slice n >= k-1
 * concurrently (slices n < k-1 already hold the serial fine solution and
 * their F values from the previous iteration are reused unchanged), then the
 * serial sweep U[n+1] = F_n + (G(U[n]) - G_old_n) with the max-norm change
 * of U.  SYNCHRONOUS: returns after the stream has drained.
 * defect (host, out): max_{n,j} |U^k - U^{k-1}|; nonfinite (host, out): 1 if
 * any NaN/Inf was produced (then BS_ERR_NONFINITE is returned). */
int parareal_iterate(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                     int coarse_kind, const pinn_net* net, void* ws, size_t ws_bytes, double* U,
                     int k, double* defect, int* nonfinite, void* stream);

/* Whole solve: parareal_start, then iterations until defect <= tol, k == N
 * (the iterate then equals serial fine integration) or k == max_iter.
 * SYNCHRONOUS.  iters (host, out): iterations done; defect_hist (host,
 * [max_iter] or NULL): defect of each iteration.  net may be NULL for
 * BS_COARSE_IE.  Returns BS_OK, BS_NOT_CONVERGED (max_iter hit first),
 * BS_ERR_NONFINITE, BS_ERR_DIVERGED (see bs_set_divergence_growth; U then
 * holds the iterate that tripped the guard) or another error.
 * For grids of up to 4096 nodes the iterations overlap (same iterates as
 * parareal_iterate called for k = 1, 2, ... with the same block shapes):
 * the fine propagation of iteration k starts each slice once the sweep of
 * iteration k-1 has produced its initial value, and the sweep of iteration
 * k takes each slice's F as soon as it is written.  With the one-wavefront
 * fine shapes and the 256 x 4 sweep shape (grids up to 1024 nodes by
 * default, N <= 512) the whole solve is one cooperative launch on `stream`;
 * otherwise F runs on one of two library-owned side streams of the calling
 * thread and the sweep on `stream`, which is joined with them before
 * returning.  The launches synchronise through progress counters in ws;
 * every wait also ends on the stop flag, and after about 2 s the solve
 * fails with BS_ERR_HIP.  Beyond 4096 nodes (block shapes of 512 threads)
 * with 2 <= N <= 256: slice 0's first fine propagation, then one launch in
 * which one block runs the prediction and the sweeps of all iterations and
 * one block per slice n >= 1 the fine work of iterations 1, 2, ... (network
 * grid and slice 0's propagation run side by side before it; when the
 * device holds all N blocks
 * at once; another kernel occupying compute units meanwhile makes the waits
 * time out: BS_ERR_HIP); otherwise the iterations run one after the other. */
int parareal_solve(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                   int coarse_kind, double tol, const pinn_net* net, int max_iter, void* ws,
                   size_t ws_bytes, double* U, int* iters, double* defect_hist, void* stream);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as parareal_solve without a caller workspace.  Its workspace and
 * per-iteration record live in a library-owned device array of
 * BS_NOALLOC_SCRATCH_BYTES bytes, one per GPU, created with the library's code
 * on that GPU and held until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call (the device address of the array is looked
 * up once per device, on the first call there).  Iterates, defects and
 * iteration counts are those of parareal_solve with the same block shapes:
 * grids covered by the one-launch solve run it; other grids run the
 * iterations one after the other on `stream` (no side streams).
 * Limits: M <= 4096, N <= 512, and the workspace of parareal_workspace_size()
 * plus 16 (min(max_iter, N) + 1) bytes of record must fit the array
 * (BS_ERR_ARG otherwise, with the sizes in bs_last_error()).  The array keeps
 * the last call's contents; every call initialises what it reads.  Calls on
 * one GPU share the array: calls that overlap in time on one GPU (another
 * thread, another stream) race and corrupt each other; order them.
 * SYNCHRONOUS.  Arguments and return values as parareal_solve. */
#define BS_NOALLOC_SCRATCH_BYTES (8u << 20)
int parareal_solve_noalloc(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                           int coarse_kind, double tol, const pinn_net* net, int max_iter,
                           double* U, int* iters, double* defect_hist, void* stream);

/* *bytes (host, out) = bytes of device workspace parareal_solve_batch needs
 * for these options (host arrays of n_opt entries).  BS_ERR_ARG if an option
 * is invalid (bs_last_error names it). */
int parareal_batch_workspace_size(int n_opt, const bs_params* prm, const bs_grid* grids,
                                  const bs_slices* sl, int coarse_kind, size_t* bytes);

/* Solve n_opt independent Parareal problems together (batched options with
 * uneven grids and slice counts).  Every phase of an iteration is one launch
 * per block-shape class covering all options of the class; options that have
 * converged, and slices that already hold the serial fine solution, are
 * skipped on the device, so iterations are queued ahead of their results:
 * `lookahead` iterations (1..16; 0 selects 4) stay in flight, each followed by
 * an asynchronous copy of the count of active options to pinned host memory,
 * and the host waits only for the oldest (no per-iteration round trip; at
 * most lookahead - 1 empty iterations run after the last option converges).
 * Stopping rule per option as in parareal_solve (defect <= tol, k == N, or
 * k == max_iter).
 * prm, grids, sl: host arrays [n_opt]; all options share payoff_mode; each
 *    grid has 1 <= M <= 4096 nodes (BS_ERR_ARG otherwise).
 * U: device FP64; option o's state [N_o+1][M_o] starts at element offsets[o]
 *    (host array); regions must not overlap.
 * Network kinds: the network is evaluated on every option's grid with inputs
 *    (tau, S/K, sigma, r) when n_in == 4 (its sigma, r come from the option)
 *    and prices calls: a put option takes put-call parity,
 *    V_put = K v - S + K exp(-r tau).
 * iters (host [n_opt], out): iterations per option; defects (host [n_opt] or
 * NULL, out): last defect per option.  SYNCHRONOUS.  Returns BS_OK,
 * BS_NOT_CONVERGED (some option hit max_iter first), BS_ERR_NONFINITE,
 * BS_ERR_DIVERGED (an option tripped the divergence guard; it stops there, the
 * others go on), or an argument / workspace / HIP error. */
int parareal_solve_batch(int n_opt, const bs_params* prm, const bs_grid* grids,
                         const bs_slices* sl, int coarse_kind, double tol, const pinn_net* net,
                         int max_iter, void* ws, size_t ws_bytes, double* U, const long* offsets,
                         int* iters, double* defects, int lookahead, void* stream);

/* Block shape of the tridiagonal kernels (for the autotuner).  Each system is
 * solved by one thread block of `threads` threads holding `nodes_per_thread`
 * consecutive nodes each.  kernel 0: the batched propagator kernel (F, and G
 * in bs_coarse_numeric); kernel 1: the serial Parareal sweep.  The setting
 * applies to grids with M_lo <= M <= M_hi (later settings win) until
 * bs_tune_reset().  Only built shapes are accepted (BS_ERR_ARG otherwise):
 * (64,2) (64,4) (64,8) (64,16) (128,4) (128,8) (256,4) (256,8) (512,8), and
 * threads * nodes_per_thread must cover M_hi.  Results do not depend on the
 * shape beyond rounding.  Process-wide (guarded by a lock: calls from several
 * threads are safe; a launch uses the setting current when it starts). */
int bs_tune_set_shape(int kernel, int M_lo, int M_hi, int threads, int nodes_per_thread);
int bs_tune_reset(void);

/* Kernel timing of the Parareal iteration, for measurement.
 * bs_profile_enable(1) resets the counters and makes parareal_iterate /
 * parareal_solve record HIP events on their stream around each launch of the
 * fine-propagator kernel, of the sweep kernel and of the one-launch solve
 * kernels; bs_profile_enable(0) stops recording.  Timing adds no
 * synchronisation beyond the per-iteration one.
 * bs_profile_read fills out[8] (host) with: total fine-kernel milliseconds,
 * number of fine launches, fine cell-updates of those launches (systems x
 * steps x M), total sweep milliseconds, number of sweep launches, total
 * milliseconds of one-launch solve kernels (fine work and sweeps of several
 * iterations in one launch), their number, and the fine cell-updates of the
 * iterations they ran.  Process-wide, not thread-safe: for a single
 * measuring thread. */
int bs_profile_enable(int on);
int bs_profile_read(double* out);

/* Releases what the library keeps between calls for the calling thread and
 * the current device (pinned per-iteration record, side streams and events,
 * coefficient tables of the large-grid solver, timing events).  The next call
 * that needs them creates them again.  Call it once no call of this thread is
 * in flight, before the HIP runtime shuts down (the Python binding does so at
 * interpreter exit). */
int bs_release_resources(void);

#ifdef __cplusplus
}
#endif

#endif /* BSPARAREAL_H */
