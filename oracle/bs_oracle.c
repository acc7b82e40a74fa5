/*
 * Plain FP64 CPU oracle for Parareal on the Black-Scholes equation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * What it follows (paper: "Parareal with a physics-informed neural network as
 * coarse propagator", Ibrahim, Goetschel, Ruprecht):
 *   - Sec. 3, eq. (1): the Black-Scholes operator, solved backwards from
 *     expiry; here written in time-to-maturity tau = T - t and integrated
 *     forward (Sec. 3.2 says the problem is solved backwards from T).
 *   - eqs. (2)-(4): expiry payoff and the two Dirichlet conditions; the upper
 *     one is read as V(S_max, tau) = S_max - K exp(-r tau) for a call (the
 *     prose of Sec. 3 says a deep in-the-money call is worth the asset).
 *   - Sec. 3.2, semi-discrete equation: second-order centred differences on
 *     the equidistant mesh S_j = j dS, j = 1..M, dS = S_max/(M+1).
 *   - Sec. 3.2: Crank-Nicolson as fine propagator F, implicit Euler as
 *     numerical coarse propagator G; both are the theta-method below.
 *   - Sec. 3.1, eq. (7): the Parareal iteration
 *       U^{k}_{n+1} = G(U^{k}_n) + F(U^{k-1}_n) - G(U^{k-1}_n),
 *     evaluated as F + (G_new - G_old).
 *   - The closed-form European price of the Black-Scholes model (cited in
 *     Sec. 3 as the reason the European call is used as a test problem).
 *
 * Compiled with -O2 -ffp-contract=off: no fused multiply-adds, IEEE
 * round-to-nearest everywhere.  The tridiagonal systems are solved with the
 * textbook Thomas algorithm, dividing anew at every step.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double K, r, sigma, T, s_max;
    int is_put;
} or_params;

enum { OR_COARSE_IE = 0, OR_COARSE_PINN = 1, OR_COARSE_PINN_IE = 2, OR_COARSE_CN = 3 };

/* ------------------------------------------------------------------ grid */

double or_dS(const or_params* p, int M) { return p->s_max / (double)(M + 1); }

/* Expiry condition, eq. (2) (call) and its put analogue, at interior nodes.
 * payoff_mode 0: sampled at S_j.  payoff_mode 1: averaged over the cell
 * [S_j - dS/2, S_j + dS/2] (removes the grid-dependent error from the kink). */
void or_initial(const or_params* p, int M, int payoff_mode, double* U0)
{
    double dS = or_dS(p, M);
    for (int j = 1; j <= M; ++j) {
        double S = j * dS;
        double v;
        if (payoff_mode == 0) {
            v = p->is_put ? fmax(p->K - S, 0.0) : fmax(S - p->K, 0.0);
        } else {
            double lo = S - 0.5 * dS, hi = S + 0.5 * dS;
            if (!p->is_put) {
                if (hi <= p->K) v = 0.0;
                else if (lo >= p->K) v = 0.5 * (lo + hi) - p->K;
                else v = (hi - p->K) * (hi - p->K) / (2.0 * dS);
            } else {
                if (lo >= p->K) v = 0.0;
                else if (hi <= p->K) v = p->K - 0.5 * (lo + hi);
                else v = (p->K - lo) * (p->K - lo) / (2.0 * dS);
            }
        }
        U0[j - 1] = v;
    }
}

/* Dirichlet data at S = 0 and S = S_max, eqs. (3)-(4). */
void or_boundary(const or_params* p, double tau, double* g_lo, double* g_hi)
{
    double disc = exp(-p->r * tau);
    if (p->is_put) {
        *g_lo = p->K * disc;
        *g_hi = 0.0;
    } else {
        *g_lo = 0.0;
        *g_hi = p->s_max - p->K * disc;
    }
}

/* Row j of the semi-discrete operator (Sec. 3.2), in tau:
 *   dV_j/dtau = al V_{j-1} + be V_j + ga V_{j+1}
 * with the diffusion term sigma^2 S_j^2 / (2 dS^2) and convection
 * r S_j / (2 dS). */
static void or_row(const or_params* p, double dS, int j, double* al, double* be, double* ga)
{
    double S = j * dS;
    double diff = 0.5 * p->sigma * p->sigma * S * S / (dS * dS);
    double conv = p->r * S / (2.0 * dS);
    *al = diff - conv;
    *be = -2.0 * diff - p->r;
    *ga = diff + conv;
}

/* -------------------------------------------------------- linear algebra */

/* Thomas algorithm for a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, i = 0..n-1
 * (a_0 and c_{n-1} unused).  cp is scratch of length n. */
void or_thomas(int n, const double* a, const double* b, const double* c, const double* d,
               double* x, double* cp)
{
    double denom = b[0];
    cp[0] = c[0] / denom;
    x[0] = d[0] / denom;
    for (int i = 1; i < n; ++i) {
        denom = b[i] - a[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? c[i] / denom : 0.0;
        x[i] = (d[i] - a[i] * x[i - 1]) / denom;
    }
    for (int i = n - 2; i >= 0; --i) x[i] = x[i] - cp[i] * x[i + 1];
}

/* One theta-method step of size dt from V^m to V^{m+1} (in place):
 *   (I - theta dt L) V^{m+1} = (I + (1-theta) dt L) V^m + boundary terms,
 * boundary values (g_lo, g_hi) given at both time levels.
 * theta = 1/2: Crank-Nicolson; theta = 1: implicit Euler.
 * work: 5*M doubles. */
void or_theta_step(const or_params* p, int M, double theta, double dt, double* V,
                   double glo_old, double ghi_old, double glo_new, double ghi_new, double* work)
{
    double dS = or_dS(p, M);
    double *a = work, *b = work + M, *c = work + 2 * M, *d = work + 3 * M, *cp = work + 4 * M;
    double ex = (1.0 - theta) * dt, im = theta * dt;
    for (int j = 1; j <= M; ++j) {
        double al, be, ga;
        or_row(p, dS, j, &al, &be, &ga);
        int i = j - 1;
        double left = (j == 1) ? glo_old : V[i - 1];
        double right = (j == M) ? ghi_old : V[i + 1];
        double rhs = V[i] + ex * (al * left + be * V[i] + ga * right);
        if (j == 1) rhs += im * al * glo_new;
        if (j == M) rhs += im * ga * ghi_new;
        a[i] = -im * al;
        b[i] = 1.0 - im * be;
        c[i] = -im * ga;
        d[i] = rhs;
    }
    or_thomas(M, a, b, c, d, V, cp);
}

/* `steps` theta-steps from tau0 over an interval of length dtau, with the
 * exact Dirichlet data of eqs. (3)-(4) at every time level.  u_in may alias
 * u_out. */
void or_propagate(const or_params* p, int M, double theta, double tau0, double dtau, int steps,
                  const double* u_in, double* u_out)
{
    double* work = (double*)malloc(sizeof(double) * 5 * (size_t)M);
    double dt = dtau / steps;
    if (u_out != u_in) memcpy(u_out, u_in, sizeof(double) * (size_t)M);
    for (int m = 0; m < steps; ++m) {
        double t_old = tau0 + m * dt, t_new = tau0 + (m + 1) * dt;
        double glo0, ghi0, glo1, ghi1;
        or_boundary(p, t_old, &glo0, &ghi0);
        or_boundary(p, t_new, &glo1, &ghi1);
        or_theta_step(p, M, theta, dt, u_out, glo0, ghi0, glo1, ghi1, work);
    }
    free(work);
}

/* Same, with the Dirichlet data supplied as sequences g_lo[m], g_hi[m],
 * m = 0..steps (used by the exact-discrete-solution checks). */
void or_propagate_bc(const or_params* p, int M, double theta, double dt, int steps,
                     const double* g_lo, const double* g_hi, const double* u_in, double* u_out)
{
    double* work = (double*)malloc(sizeof(double) * 5 * (size_t)M);
    if (u_out != u_in) memcpy(u_out, u_in, sizeof(double) * (size_t)M);
    for (int m = 0; m < steps; ++m)
        or_theta_step(p, M, theta, dt, u_out, g_lo[m], g_hi[m], g_lo[m + 1], g_hi[m + 1], work);
    free(work);
}

/* Fine propagator F over one time slice: fine_steps Crank-Nicolson steps. */
void or_fine(const or_params* p, int M, double tau0, double dtau, int steps, const double* u_in,
             double* u_out)
{
    or_propagate(p, M, 0.5, tau0, dtau, steps, u_in, u_out);
}

/* Numerical coarse propagator G over one slice: implicit Euler steps. */
void or_coarse_ie(const or_params* p, int M, double tau0, double dtau, int steps, const double* u_in,
                  double* u_out)
{
    or_propagate(p, M, 1.0, tau0, dtau, steps, u_in, u_out);
}

/* Implicit Euler steps with homogeneous Dirichlet data: propagates the
 * deviation of a state from the network's prediction (PINN-anchored coarse). */
static void or_coarse_ie_homog(const or_params* p, int M, double dtau, int steps, double* u)
{
    double* work = (double*)malloc(sizeof(double) * 5 * (size_t)M);
    double dt = dtau / steps;
    for (int m = 0; m < steps; ++m) or_theta_step(p, M, 1.0, dt, u, 0.0, 0.0, 0.0, 0.0, work);
    free(work);
}

/* Classical time stepping, eq. (6): U_{n+1} = F(U_n), n = 0..N-1.
 * U: (N+1)*M, U[0..M) must hold the initial value. */
void or_serial_fine(const or_params* p, int M, int N, int fine_steps, double* U)
{
    double dT = p->T / N;
    for (int n = 0; n < N; ++n)
        or_fine(p, M, n * dT, dT, fine_steps, U + (size_t)n * M, U + (size_t)(n + 1) * M);
}

/* Coarse propagator of slice n applied to u_in.
 *   IE      : coarse_steps implicit-Euler steps with the exact boundary data.
 *   PINN    : the network's prediction Vt[n+1], independent of the state.
 *   PINN_IE : Vt[n+1] + IE_0(u - Vt[n]), IE_0 with zero boundary data.
 *   CN      : coarse_steps Crank-Nicolson steps (a check: equals F when
 *             coarse_steps == fine_steps). */
static void or_coarse(const or_params* p, int M, int kind, int coarse_steps, const double* Vt,
                      int n, double dT, const double* u_in, double* u_out)
{
    switch (kind) {
    case OR_COARSE_IE:
        or_coarse_ie(p, M, n * dT, dT, coarse_steps, u_in, u_out);
        break;
    case OR_COARSE_CN:
        or_fine(p, M, n * dT, dT, coarse_steps, u_in, u_out);
        break;
    case OR_COARSE_PINN:
        memcpy(u_out, Vt + (size_t)(n + 1) * M, sizeof(double) * (size_t)M);
        break;
    case OR_COARSE_PINN_IE:
        for (int j = 0; j < M; ++j) u_out[j] = u_in[j] - Vt[(size_t)n * M + j];
        or_coarse_ie_homog(p, M, dT, coarse_steps, u_out);
        for (int j = 0; j < M; ++j) u_out[j] = Vt[(size_t)(n + 1) * M + j] + u_out[j];
        break;
    }
}

/* Parareal, eq. (7), in plain loops.
 *   k = 0      : coarse prediction U^0_{n+1} = G(U^0_n), Gold_n = U^0_{n+1}.
 *   k = 1, 2..: Fv_n = F(U^{k-1}_n) for all n (OpenMP over slices: the slices
 *               are independent, as the P = N processes of Sec. 3.1 are);
 *               then serially g = G(U^k_n), U^k_{n+1} = Fv_n + (g - Gold_n),
 *               Gold_n = g; defect_k = max |U^k - U^{k-1}| over all nodes.
 *   Stops at the first k with defect_k <= tol, or at k = N (after N
 *   iterations the iterate equals the serial fine solution), or at max_iter.
 * U (out): (N+1)*M.  iters: k at exit.  defects[k-1] = defect_k.
 * iterates (optional): (max_iter+1)*(N+1)*M, the iterate after each k.
 * Returns 0 if stopped by tol or k = N, 1 if max_iter was hit first. */
int or_parareal(const or_params* p, int M, int payoff_mode, int N, int fine_steps,
                int coarse_steps, int coarse_kind, const double* Vt, double tol, int max_iter,
                int nthreads, double* U, int* iters, double* defects, double* iterates)
{
    size_t slab = (size_t)(N + 1) * M;
    double dT = p->T / N;
    double* Fv = (double*)malloc(sizeof(double) * (size_t)N * M);
    double* Gold = (double*)malloc(sizeof(double) * (size_t)N * M);
    double* g = (double*)malloc(sizeof(double) * (size_t)M);
    double* Uprev = (double*)malloc(sizeof(double) * slab);
    int status = 1;

    or_initial(p, M, payoff_mode, U);
    for (int n = 0; n < N; ++n) {
        or_coarse(p, M, coarse_kind, coarse_steps, Vt, n, dT, U + (size_t)n * M,
                  U + (size_t)(n + 1) * M);
        memcpy(Gold + (size_t)n * M, U + (size_t)(n + 1) * M, sizeof(double) * (size_t)M);
    }
    if (iterates) memcpy(iterates, U, sizeof(double) * slab);

    int k = 0;
    int kmax = max_iter < N ? max_iter : N;
    while (k < kmax) {
        ++k;
        memcpy(Uprev, U, sizeof(double) * slab);
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
        for (int n = 0; n < N; ++n)
            or_fine(p, M, n * dT, dT, fine_steps, Uprev + (size_t)n * M, Fv + (size_t)n * M);
        (void)nthreads;

        double defect = 0.0;
        for (int n = 0; n < N; ++n) {
            or_coarse(p, M, coarse_kind, coarse_steps, Vt, n, dT, U + (size_t)n * M, g);
            double* un1 = U + (size_t)(n + 1) * M;
            double* go = Gold + (size_t)n * M;
            const double* fv = Fv + (size_t)n * M;
            for (int j = 0; j < M; ++j) {
                un1[j] = fv[j] + (g[j] - go[j]);
                go[j] = g[j];
            }
        }
        for (size_t i = 0; i < slab; ++i) {
            double e = fabs(U[i] - Uprev[i]);
            if (e > defect || e != e) defect = e;
        }
        if (defects) defects[k - 1] = defect;
        if (iterates) memcpy(iterates + (size_t)k * slab, U, sizeof(double) * slab);
        if (defect <= tol || k == N) {
            status = 0;
            break;
        }
    }
    *iters = k;
    free(Fv);
    free(Gold);
    free(g);
    free(Uprev);
    return status;
}

/* ----------------------------------------------------------- closed form */

/* Standard normal distribution function via the complementary error function. */
static double or_ncdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Closed-form European call / put price of the Black-Scholes model with time
 * to maturity tau. */
double or_bs_price(double S, double K, double r, double sigma, double tau, int is_put)
{
    if (tau <= 0.0) return is_put ? fmax(K - S, 0.0) : fmax(S - K, 0.0);
    if (S <= 0.0) return is_put ? K * exp(-r * tau) : 0.0;
    double st = sigma * sqrt(tau);
    double d1 = (log(S / K) + (r + 0.5 * sigma * sigma) * tau) / st;
    double d2 = d1 - st;
    if (is_put) return K * exp(-r * tau) * or_ncdf(-d2) - S * or_ncdf(-d1);
    return S * or_ncdf(d1) - K * exp(-r * tau) * or_ncdf(d2);
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
