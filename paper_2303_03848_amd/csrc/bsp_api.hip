// C ABI entry points: argument checks, workspace layout, and the host side of
// the Parareal iteration (one F launch over all unconverged slices, one sweep
// launch, one 16-byte read-back of the defect per iteration).
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <vector>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "bsp_common.hpp"

namespace bsp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

static int check_params(const bs_params* prm) {
    BSP_CHECK_ARG(prm != nullptr, "bs_params is NULL");
    BSP_CHECK_ARG(prm->K > 0 && prm->sigma > 0 && prm->r >= 0 && prm->T > 0 && prm->s_max > 0,
                  "bs_params out of range (need K > 0, sigma > 0, r >= 0, T > 0, s_max > 0)");
    BSP_CHECK_ARG(std::isfinite(prm->K) && std::isfinite(prm->sigma) && std::isfinite(prm->r) &&
                      std::isfinite(prm->T) && std::isfinite(prm->s_max),
                  "bs_params must be finite");
    return BS_OK;
}

static int check_grid(const bs_grid* g) {
    BSP_CHECK_ARG(g != nullptr, "bs_grid is NULL");
    BSP_CHECK_ARG(g->M >= 1 && g->M <= kMaxM, "M must be in [1, %d] (got %d)", kMaxM, g->M);
    BSP_CHECK_ARG(g->payoff_mode == 0 || g->payoff_mode == 1, "payoff_mode must be 0 or 1");
    BSP_CHECK_ARG(tri_shape(g->M).T > 0, "M = %d is not supported by the tridiagonal kernels",
                  g->M);
    return BS_OK;
}

static int check_slices(const bs_slices* s) {
    BSP_CHECK_ARG(s != nullptr, "bs_slices is NULL");
    BSP_CHECK_ARG(s->N >= 1 && s->N <= (1 << 20), "N must be >= 1 (got %d)", s->N);
    BSP_CHECK_ARG(s->fine_steps >= 1 && s->coarse_steps >= 1, "step counts must be >= 1");
    return BS_OK;
}

// Parareal workspace: [result 256 B | Fv N*M | Gold N*M | progress counters
// 4(N+1)+3 ints | U2 (N+1)*M (grids the one-launch solve may cover) | Vt
// (N+1)*M (network kinds) | the large-grid sweep's tables (grids beyond 4096
// nodes)].  result: [0] defect, [1] status of the last
// iteration (0, 1 non-finite, 2 diverged), [2] defect of iteration 1, int at
// [4]: stop flag of the asynchronous solve.
struct Workspace {
    double* result;
    double* Fv;
    double* Gold;
    int* flags;  // ready[N+1], taken[N+1], fdone[N+1], err, decided[N+1], exited, stop_rank
    double* U2;
    double* Vt;
    double* tab;  // grids beyond 4096 nodes: the sweep's implicit-Euler tables
    // grids beyond 4096 nodes: chunk-major copies of U, Fv, Gold and Vt for
    // the overlapped solve (large_cm_level(M) doubles per level)
    double* cm_U;
    double* cm_Fv;
    double* cm_Gold;
    double* cm_Vt;
};

// Doubles of the chunk-major region: U and Vt (N+1 levels), Fv and Gold (N).
static size_t cm_doubles(int M, int N, int kind) {
    const size_t L = (size_t)large_cm_level(M);
    return L * ((size_t)(N + 1) + 2 * (size_t)N + (kind != BS_COARSE_IE ? (size_t)(N + 1) : 0));
}

static int flag_count(int N) { return 4 * (N + 1) + 3; }

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t ws_bytes(int M, int N, int kind) {
    size_t b = 256;
    b += align256(sizeof(double) * (size_t)N * M);
    b += align256(sizeof(double) * (size_t)N * M);
    b += align256(sizeof(int) * (size_t)flag_count(N));
    if (persist_possible(M, N)) b += align256(sizeof(double) * (size_t)(N + 1) * M);
    if (kind != BS_COARSE_IE) b += align256(sizeof(double) * (size_t)(N + 1) * M);
    b += align256(sizeof(double) * large_sweep_table_doubles(M));
    b += align256(sizeof(double) * cm_doubles(M, N, kind));
    return b;
}

static Workspace ws_layout(void* ws, int M, int N, int kind) {
    char* p = (char*)ws;
    Workspace w;
    w.result = (double*)p;
    p += 256;
    w.Fv = (double*)p;
    p += align256(sizeof(double) * (size_t)N * M);
    w.Gold = (double*)p;
    p += align256(sizeof(double) * (size_t)N * M);
    w.flags = (int*)p;
    p += align256(sizeof(int) * (size_t)flag_count(N));
    w.U2 = nullptr;
    if (persist_possible(M, N)) {
        w.U2 = (double*)p;
        p += align256(sizeof(double) * (size_t)(N + 1) * M);
    }
    w.Vt = nullptr;
    if (kind != BS_COARSE_IE) {
        w.Vt = (double*)p;
        p += align256(sizeof(double) * (size_t)(N + 1) * M);
    }
    w.tab = large_sweep_table_doubles(M) ? (double*)p : nullptr;
    p += align256(sizeof(double) * large_sweep_table_doubles(M));
    w.cm_U = w.cm_Fv = w.cm_Gold = w.cm_Vt = nullptr;
    if (const long L = large_cm_level(M)) {
        w.cm_U = (double*)p;
        w.cm_Fv = w.cm_U + (size_t)(N + 1) * L;
        w.cm_Gold = w.cm_Fv + (size_t)N * L;
        if (kind != BS_COARSE_IE) w.cm_Vt = w.cm_Gold + (size_t)N * L;
    }
    return w;
}

static PipeSync pipe_sync(const Workspace& w, int N) {
    PipeSync ps{};
    ps.ready = w.flags;
    ps.taken = w.flags + (N + 1);
    ps.fdone = w.flags + 2 * (N + 1);
    ps.err = w.flags + 3 * (N + 1);
    return ps;
}

// Divergence guard (bs_set_divergence_growth).
static std::atomic<double> g_growth{BS_DIVERGENCE_GROWTH};

// Status of one iteration in the per-iteration record: 0, 1 non-finite, 2 diverged.
static int record_status(double flag) { return flag == 1.0 ? BS_ERR_NONFINITE
                                               : flag == 2.0 ? BS_ERR_DIVERGED : BS_OK; }

static int check_parareal(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                          int kind, const pinn_net* net, void* ws, size_t ws_size, double* U) {
    int rc;
    if ((rc = check_params(prm))) return rc;
    if ((rc = check_grid(grid))) return rc;
    if ((rc = check_slices(sl))) return rc;
    BSP_CHECK_ARG(kind == BS_COARSE_IE || kind == BS_COARSE_PINN || kind == BS_COARSE_PINN_IE ||
                      kind == BS_COARSE_FLOWMAP,
                  "unknown coarse kind %d", kind);
    if (kind != BS_COARSE_IE) {
        if ((rc = check_net(net))) return rc;
        BSP_CHECK_ARG(net->n_in == 2 || net->n_in == 4, "network inputs must be 2 or 4");
        BSP_CHECK_ARG(kind != BS_COARSE_FLOWMAP || net->n_in == 4,
                      "the flow-map coarse takes a network of 4 inputs");
    }
    BSP_CHECK_ARG(U != nullptr, "U is NULL");
    if (ws == nullptr || ws_size < ws_bytes(grid->M, sl->N, kind)) {
        set_error("workspace is NULL or smaller than parareal_workspace_size() = %zu bytes",
                  ws_bytes(grid->M, sl->N, kind));
        return BS_ERR_WORKSPACE;
    }
    return BS_OK;
}

static int propagate_checked(const bs_params* prm, const bs_grid* grid, int nsys,
                             const double* tau0, double dtau, int steps, const double* u_in,
                             double* u_out, double theta, void* stream) {
    clear_error();
    int rc;
    if ((rc = check_params(prm))) return rc;
    if ((rc = check_grid(grid))) return rc;
    BSP_CHECK_ARG(nsys >= 0, "nsys must be >= 0");
    BSP_CHECK_ARG(steps >= 1, "steps must be >= 1");
    BSP_CHECK_ARG(dtau > 0 && std::isfinite(dtau), "dtau must be positive");
    if (nsys == 0) return BS_OK;
    BSP_CHECK_ARG(tau0 && u_in && u_out, "tau0, u_in and u_out must be non-NULL");
    const OptionDev o = make_option(*prm, grid->M);
    return launch_theta_batch(o, grid->M, nsys, tau0, 0.0, 0.0, 0, dtau / steps, steps, theta,
                              u_in, grid->M, u_out, grid->M, (hipStream_t)stream);
}

// ----------------------------------------------------------- profiling
// F and sweep launches of parareal_iterate / parareal_solve are bracketed by
// events on the streams they run on (four per enqueued iteration), read back
// once the call has synchronised.
struct Profile {
    bool on = false;
    std::vector<hipEvent_t> ev;
    double fine_ms = 0, fine_launches = 0, fine_cells = 0, sweep_ms = 0, sweep_launches = 0;
    double solve_ms = 0, solve_launches = 0, solve_cells = 0;  // one-launch solve kernels
};
static Profile g_prof;

static int prof_reserve(int slots) {
    while ((int)g_prof.ev.size() < 4 * slots) {
        hipEvent_t e;
        BSP_HIP(hipEventCreate(&e));
        g_prof.ev.push_back(e);
    }
    return BS_OK;
}

// Adds iteration slot `slot` to the profile; cells: fine cell updates it did.
static int prof_collect(int slot, double cells) {
    float f_ms = 0.f, s_ms = 0.f;
    BSP_HIP(hipEventElapsedTime(&f_ms, g_prof.ev[4 * slot], g_prof.ev[4 * slot + 1]));
    BSP_HIP(hipEventElapsedTime(&s_ms, g_prof.ev[4 * slot + 2], g_prof.ev[4 * slot + 3]));
    g_prof.fine_ms += f_ms;
    g_prof.fine_launches += 1;
    g_prof.fine_cells += cells;
    g_prof.sweep_ms += s_ms;
    g_prof.sweep_launches += 1;
    return BS_OK;
}

// Initial state, network grid (network kinds) and (predict) the prediction
// sweep.  ps: progress counters of the overlapped solve (the sweep publishes
// U[n]).
static int start_impl(const bs_params* prm, const bs_grid* grid, const bs_slices* sl, int kind,
                      const pinn_net* net, void* ws, double* U, const PipeSync* ps,
                      hipStream_t st, bool predict = true) {
    int rc;
    const int M = grid->M, N = sl->N;
    const OptionDev o = make_option(*prm, M);
    const double dT = prm->T / N;
    Workspace w = ws_layout(ws, M, N, kind);
    if ((rc = launch_initial(o, M, grid->payoff_mode, U, st))) return rc;
    if (kind == BS_COARSE_FLOWMAP) {
        // the network sees the state: the prediction runs slice after slice
        // (g in the first M doubles of the network-grid area)
        for (int n = 0; n < N && predict; ++n) {
            if ((rc = launch_flowmap(*net, o, M, n * dT, (n + 1) * dT, U + (long)n * M, w.Vt,
                                     st)))
                return rc;
            if ((rc = launch_flow_correct(M, true, false, w.Vt, nullptr, w.Gold + (long)n * M,
                                          U + (long)(n + 1) * M, w.result, st)))
                return rc;
        }
        return BS_OK;
    }
    if (kind != BS_COARSE_IE) {
        if ((rc = launch_pinn_grid(*net, o, M, N, dT, w.Vt, st))) return rc;
    }
    if (!predict) return BS_OK;
    SweepArgs a{o, M, N, 0, sl->coarse_steps, kind, 1, dT, U, w.Fv, w.Gold, w.Vt, w.result};
    a.growth = INFINITY;
    a.tab = w.tab;
    if (ps) {
        a.ps = *ps;
        a.ps.k = 0;
    }
    return launch_sweep(a, st);
}

}  // namespace bsp

using namespace bsp;

extern "C" {

const char* bs_last_error(void) { return g_err; }

int bs_set_divergence_growth(double growth) {
    clear_error();
    BSP_CHECK_ARG(growth > 0 && !std::isnan(growth), "growth must be > 0 (got %g)", growth);
    g_growth.store(growth);
    return BS_OK;
}

double bs_divergence_growth(void) { return g_growth.load(); }

int bs_profile_enable(int on) {
    clear_error();
    if (on) {
        int rc = prof_reserve(1);
        if (rc) return rc;
    }
    g_prof.on = on != 0;
    if (on) {
        g_prof.fine_ms = g_prof.fine_launches = g_prof.fine_cells = 0;
        g_prof.sweep_ms = g_prof.sweep_launches = 0;
        g_prof.solve_ms = g_prof.solve_launches = g_prof.solve_cells = 0;
    }
    return BS_OK;
}

int bs_tune_set_shape(int kernel, int M_lo, int M_hi, int threads, int nodes_per_thread) {
    clear_error();
    return set_shape_override(kernel, M_lo, M_hi, threads, nodes_per_thread);
}

int bs_tune_reset(void) {
    clear_error();
    reset_shape_overrides();
    return BS_OK;
}

int bs_profile_read(double* out) {
    BSP_CHECK_ARG(out != nullptr, "out is NULL");
    out[0] = g_prof.fine_ms;
    out[1] = g_prof.fine_launches;
    out[2] = g_prof.fine_cells;
    out[3] = g_prof.sweep_ms;
    out[4] = g_prof.sweep_launches;
    out[5] = g_prof.solve_ms;
    out[6] = g_prof.solve_launches;
    out[7] = g_prof.solve_cells;
    return BS_OK;
}

int bs_initial(const bs_params* prm, const bs_grid* grid, double* u0, void* stream) {
    clear_error();
    int rc;
    if ((rc = check_params(prm))) return rc;
    if ((rc = check_grid(grid))) return rc;
    BSP_CHECK_ARG(u0 != nullptr, "u0 is NULL");
    return launch_initial(make_option(*prm, grid->M), grid->M, grid->payoff_mode, u0,
                          (hipStream_t)stream);
}

int bs_fine_propagate_batch(const bs_params* prm, const bs_grid* grid, int nsys,
                            const double* tau0, double dtau, int steps, const double* u_in,
                            double* u_out, void* stream) {
    return propagate_checked(prm, grid, nsys, tau0, dtau, steps, u_in, u_out, 0.5, stream);
}

int bs_coarse_numeric(const bs_params* prm, const bs_grid* grid, int nsys, const double* tau0,
                      double dtau, int steps, const double* u_in, double* u_out, void* stream) {
    return propagate_checked(prm, grid, nsys, tau0, dtau, steps, u_in, u_out, 1.0, stream);
}

int parareal_workspace_size(const bs_grid* grid, const bs_slices* sl, int coarse_kind,
                            size_t* bytes) {
    clear_error();
    int rc;
    BSP_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = 0;
    if ((rc = check_grid(grid))) return rc;
    if ((rc = check_slices(sl))) return rc;
    BSP_CHECK_ARG(coarse_kind == BS_COARSE_IE || coarse_kind == BS_COARSE_PINN ||
                      coarse_kind == BS_COARSE_PINN_IE || coarse_kind == BS_COARSE_FLOWMAP,
                  "unknown coarse kind %d", coarse_kind);
    *bytes = ws_bytes(grid->M, sl->N, coarse_kind);
    return BS_OK;
}

int parareal_start(const bs_params* prm, const bs_grid* grid, const bs_slices* sl, int kind,
                   const pinn_net* net, void* ws, size_t ws_size, double* U, void* stream) {
    clear_error();
    int rc = check_parareal(prm, grid, sl, kind, net, ws, ws_size, U);
    if (rc) return rc;
    return start_impl(prm, grid, sl, kind, net, ws, U, nullptr, (hipStream_t)stream);
}

}  // extern "C"

// Enqueues iteration k: F over the slices that still change on fst, then
// the sweep on st.  stop/hist/tol: device-side stopping of the asynchronous
// solve (null for a single synchronous iteration).  ps: progress counters of
// the overlapped solve (null: fst == st and the launches follow each other).
// slot: profiling slot.  growth: divergence guard (INFINITY: none).
static int enqueue_iteration(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                             int kind, const pinn_net* net, void* ws, double* U, int k,
                             int* stop, double* hist,
                             double tol, double growth, int slot, const PipeSync* ps,
                             hipStream_t fst, hipStream_t st) {
    const int M = grid->M, N = sl->N;
    const OptionDev o = make_option(*prm, M);
    const double dT = prm->T / N;
    Workspace w = ws_layout(ws, M, N, kind);
    const int first = k - 1 < N - 1 ? k - 1 : N - 1;
    const bool prof = g_prof.on && slot >= 0;
    PipeSync pk{};
    if (ps) {
        pk = *ps;
        pk.k = k;
    }
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[4 * slot], fst));
    int rc = launch_theta_batch(o, M, N - first, nullptr, 0.0, dT, first, dT / sl->fine_steps,
                                sl->fine_steps, 0.5, U + (long)first * M, M,
                                w.Fv + (long)first * M, M, fst, stop, ps ? &pk : nullptr);
    if (rc) return rc;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[4 * slot + 1], fst));
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[4 * slot + 2], st));
    if (kind == BS_COARSE_FLOWMAP) {
        // sweep: the network on U[n], then the correction, slice after slice
        for (int n = first; n < N; ++n) {
            if ((rc = launch_flowmap(*net, o, M, n * dT, (n + 1) * dT, U + (long)n * M, w.Vt,
                                     st)))
                return rc;
            if ((rc = launch_flow_correct(M, false, n == first, w.Vt, w.Fv + (long)n * M,
                                          w.Gold + (long)n * M, U + (long)(n + 1) * M, w.result,
                                          st)))
                return rc;
        }
        if (prof) BSP_HIP(hipEventRecord(g_prof.ev[4 * slot + 3], st));
        return BS_OK;
    }
    SweepArgs a{o,      M,      N,      first,    sl->coarse_steps, kind, 0, dT, U, w.Fv,
                w.Gold, w.Vt,   w.result, stop,   hist,             tol,  k,  pk};
    a.growth = growth;
    a.tab = w.tab;
    if ((rc = launch_sweep(a, st))) return rc;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[4 * slot + 3], st));
    return BS_OK;
}

// Fine cell updates of iteration k.
static double iteration_cells(const bs_grid* grid, const bs_slices* sl, int k) {
    const int first = k - 1 < sl->N - 1 ? k - 1 : sl->N - 1;
    return (double)(sl->N - first) * sl->fine_steps * grid->M;
}

static int iterate_impl(const bs_params* prm, const bs_grid* grid, const bs_slices* sl, int kind,
                        const pinn_net* net, void* ws, double* U, int k, double* defect,
                        int* nonfinite, hipStream_t st) {
    Workspace w = ws_layout(ws, grid->M, sl->N, kind);
    int rc = enqueue_iteration(prm, grid, sl, kind, net, ws, U, k, nullptr, nullptr, 0.0, INFINITY, 0,
                               nullptr, st, st);
    if (rc) return rc;
    double res[2];
    BSP_HIP(hipMemcpyAsync(res, w.result, sizeof(res), hipMemcpyDeviceToHost, st));
    BSP_HIP(hipStreamSynchronize(st));
    if (g_prof.on && (rc = prof_collect(0, iteration_cells(grid, sl, k)))) return rc;
    *defect = res[0];
    *nonfinite = res[1] == 1.0;
    if (*nonfinite) {
        set_error("non-finite value in the Parareal state at iteration %d", k);
        return BS_ERR_NONFINITE;
    }
    return BS_OK;
}

// Host-side state of the asynchronous solve, one per host thread (a solve
// is synchronous, so a thread runs one at a time): the per-iteration record
// in mapped pinned host memory that the sweep writes, completion events, and
// the two side streams (default priority, not synchronising with the null
// stream) on which the fine launches of the overlapped solve alternate.
struct SolveState {
    double* hist = nullptr;  // host view
    double* hist_dev = nullptr;
    size_t cap = 0;
    std::vector<hipEvent_t> done;
    int dev = -1;
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t go = nullptr, side_done[2] = {nullptr, nullptr};
};
static thread_local SolveState t_solve;

static int solve_reserve(int kmax) {
    SolveState& S = t_solve;
    const size_t need = 2 * (size_t)(kmax + 1);
    if (S.cap < need) {
        if (S.hist) BSP_HIP(hipHostFree(S.hist));
        S.hist = nullptr;
        S.cap = 0;
        BSP_HIP(hipHostMalloc((void**)&S.hist, need * sizeof(double),
                              hipHostMallocMapped | hipHostMallocCoherent));
        BSP_HIP(hipHostGetDevicePointer((void**)&S.hist_dev, S.hist, 0));
        S.cap = need;
    }
    while ((int)S.done.size() < kmax + 1) {
        hipEvent_t e;
        BSP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        S.done.push_back(e);
    }
    return BS_OK;
}

// Side streams and their events on the current device (those made for
// another device are released first).
static int solve_streams() {
    SolveState& S = t_solve;
    int dev = 0;
    BSP_HIP(hipGetDevice(&dev));
    if (S.dev == dev) return BS_OK;
    if (S.dev >= 0) {  // made on another device
        for (int i = 0; i < 2; ++i) {
            BSP_HIP(hipStreamDestroy(S.side[i]));
            BSP_HIP(hipEventDestroy(S.side_done[i]));
        }
        BSP_HIP(hipEventDestroy(S.go));
        S.dev = -1;
    }
    for (int i = 0; i < 2; ++i) {
        BSP_HIP(hipStreamCreateWithFlags(&S.side[i], hipStreamNonBlocking));
        BSP_HIP(hipEventCreateWithFlags(&S.side_done[i], hipEventDisableTiming));
    }
    BSP_HIP(hipEventCreateWithFlags(&S.go, hipEventDisableTiming));
    S.dev = dev;
    return BS_OK;
}

// Whole solve in one launch (grids covered by k_parareal_persist): initial
// state and network grid, then the persistent kernel, which runs the
// prediction and every iteration, records each iteration's defect in the
// host-mapped history and leaves the final iterate in U; the host reads the
// history once the stream has drained.  The stop flag must already be clear
// on st.
// rec_dev: the per-iteration record [2 (kmax+1)] the kernel writes; rec_host:
// where the host reads it after the stream has drained (the same memory when
// it is host-mapped; otherwise the record is copied there first).
static int solve_persistent(const bs_params* prm, const bs_grid* grid, const bs_slices* sl,
                            int kind, double tol, double growth, const pinn_net* net, int kmax,
                            void* ws, double* U, int* iters, double* defect_hist,
                            double* rec_dev, double* rec_host, bool rec_mapped, bool prof,
                            hipStream_t st) {
    int rc;
    const int M = grid->M, N = sl->N;
    const size_t nrec = 2 * (size_t)(kmax + 1);
    if (rec_mapped) {
        for (size_t i = 0; i < nrec; ++i) rec_host[i] = -1.0;  // not reached
    } else if ((rc = launch_fill_double(rec_dev, (int)nrec, -1.0, st))) {
        return rc;
    }
    Workspace w = ws_layout(ws, M, N, kind);
    const PipeSync ps = pipe_sync(w, N);
    if ((rc = launch_fill_int(w.flags, flag_count(N), 0, st))) return rc;
    if ((rc = start_impl(prm, grid, sl, kind, net, ws, U, nullptr, st, false))) return rc;
    PersistArgs a{};
    a.o = make_option(*prm, M);
    a.M = M;
    a.N = N;
    a.kmax = kmax;
    a.fine_steps = sl->fine_steps;
    a.coarse_steps = sl->coarse_steps;
    a.kind = kind;
    a.dT = prm->T / N;
    a.tol = tol;
    a.growth = growth;
    a.U = U;
    a.U2 = w.U2;
    a.Fv = w.Fv;
    a.Gold = w.Gold;
    a.Vt = w.Vt;
    a.result = w.result;
    a.stop = reinterpret_cast<int*>(w.result + 4);
    a.hist = rec_dev;
    a.decided = w.flags + 3 * (N + 1) + 1;
    a.exited = a.decided + (N + 1);
    a.stop_rank = a.exited + 1;
    a.ps = ps;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[0], st));
    if ((rc = launch_parareal_persist(a, st))) return rc;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[1], st));
    int err = 0;
    BSP_HIP(hipMemcpyAsync(&err, ps.err, sizeof(int), hipMemcpyDeviceToHost, st));
    if (!rec_mapped)
        BSP_HIP(hipMemcpyAsync(rec_host, rec_dev, nrec * sizeof(double), hipMemcpyDeviceToHost,
                               st));
    BSP_HIP(hipStreamSynchronize(st));
    if (err) {
        set_error("Parareal solve: a launch waited longer than its time limit");
        return BS_ERR_HIP;
    }
    // the first iteration that met the stopping rule (or kmax)
    const volatile double* hist = rec_host;
    int status = BS_NOT_CONVERGED, last = 0;
    for (int j = 1; j <= kmax; ++j) {
        const double d = hist[2 * j], flag = hist[2 * j + 1];
        if (d < 0.0) break;  // not reached
        if (defect_hist) defect_hist[j - 1] = d;
        last = j;
        if ((status = record_status(flag)) != BS_OK) break;
        if (d <= tol || j == N) {
            status = BS_OK;
            break;
        }
        status = BS_NOT_CONVERGED;
    }
    *iters = last;
    if (prof) {
        float ms = 0.f;
        BSP_HIP(hipEventElapsedTime(&ms, g_prof.ev[0], g_prof.ev[1]));
        g_prof.solve_ms += ms;
        g_prof.solve_launches += 1;
        for (int k = 1; k <= last; ++k) g_prof.solve_cells += iteration_cells(grid, sl, k);
    }
    if (status == BS_ERR_NONFINITE)
        set_error("non-finite value in the Parareal state at iteration %d", last);
    else if (status == BS_ERR_DIVERGED)
        set_error("Parareal diverging: defect of iteration %d above %g x the first", last, growth);
    return status;
}

// Overlapped solve of a grid beyond 4096 nodes (k_large_persist): initial
// state and network grid, slice 0's first fine propagation (on a side
// stream, beside the network grid), then one launch for the prediction and
// the sweeps of all iterations beside the fine work of iterations 1, 2, ...;
// the host reads the per-iteration record once the stream has drained.  The
// stop flag must already be clear on st.
static int solve_large(const bs_params* prm, const bs_grid* grid, const bs_slices* sl, int kind,
                       double tol, double growth, const pinn_net* net, int kmax, void* ws,
                       double* U, int* iters, double* defect_hist, hipStream_t st) {
    int rc;
    const int M = grid->M, N = sl->N;
    SolveState& S = t_solve;
    for (size_t i = 0; i < 2 * (size_t)(kmax + 1); ++i) S.hist[i] = -1.0;  // not reached
    Workspace w = ws_layout(ws, M, N, kind);
    const PipeSync ps = pipe_sync(w, N);
    int* stop = reinterpret_cast<int*>(w.result + 4);
    if ((rc = launch_fill_int(w.flags, flag_count(N), 0, st))) return rc;
    if ((rc = solve_streams())) return rc;
    const OptionDev o = make_option(*prm, M);
    const double dT = prm->T / N;
    const bool prof = g_prof.on;
    // U[0] = payoff; then slice 0's first fine propagation (iteration 1's
    // F of slice 0, the only one no fine block of the launch computes) on a
    // side stream beside the network grid
    if ((rc = launch_initial(o, M, grid->payoff_mode, U, st))) return rc;
    BSP_HIP(hipEventRecord(S.go, st));
    BSP_HIP(hipStreamWaitEvent(S.side[0], S.go, 0));
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[0], S.side[0]));
    if ((rc = launch_theta_batch(o, M, 1, nullptr, 0.0, dT, 0, dT / sl->fine_steps,
                                 sl->fine_steps, 0.5, U, M, w.Fv, M, S.side[0], stop, nullptr)))
        return rc;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[1], S.side[0]));
    if (kind != BS_COARSE_IE && (rc = launch_pinn_grid(*net, o, M, N, dT, w.Vt, st))) return rc;
    BSP_HIP(hipEventRecord(S.side_done[0], S.side[0]));
    BSP_HIP(hipStreamWaitEvent(st, S.side_done[0], 0));
    // counters: nothing produced yet except Fv[0] (the prediction publishes
    // U[0] and every U[n+1] as it goes)
    if ((rc = launch_fill_int(ps.fdone, 1, 1, st))) return rc;
    LargePersistArgs a{};
    if ((rc = launch_large_sweep_setup(o, M, dT, sl->coarse_steps, w.tab, st))) return rc;
    a.tab = w.tab;
    a.ptab = large_sweep_ptab(w.tab);
    a.o = o;
    a.M = M;
    a.N = N;
    a.kmax = kmax;
    a.fine_steps = sl->fine_steps;
    a.coarse_steps = sl->coarse_steps;
    a.kind = kind;
    a.dT = dT;
    a.tol = tol;
    a.growth = growth;
    // the launch works on chunk-major copies of U, Fv, Gold and Vt (of which
    // U[0], Fv[0] and Vt hold values so far)
    if ((rc = launch_cm_convert(U, w.cm_U, 1, M, true, st))) return rc;
    if ((rc = launch_cm_convert(w.Fv, w.cm_Fv, 1, M, true, st))) return rc;
    if (w.Vt && (rc = launch_cm_convert(w.Vt, w.cm_Vt, N + 1, M, true, st))) return rc;
    a.U = w.cm_U;
    a.Fv = w.cm_Fv;
    a.Gold = w.cm_Gold;
    a.Vt = w.cm_Vt;
    a.result = w.result;
    a.stop = stop;
    a.hist = S.hist_dev;
    a.ps = ps;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[2], st));
    if ((rc = launch_large_persist(a, st))) return rc;
    if (prof) BSP_HIP(hipEventRecord(g_prof.ev[3], st));
    // the iterate, the fine results and the coarse values back in node order
    if ((rc = launch_cm_convert(w.cm_U, U, N + 1, M, false, st))) return rc;
    if ((rc = launch_cm_convert(w.cm_Fv, w.Fv, N, M, false, st))) return rc;
    if ((rc = launch_cm_convert(w.cm_Gold, w.Gold, N, M, false, st))) return rc;
    int err = 0;
    BSP_HIP(hipMemcpyAsync(&err, ps.err, sizeof(int), hipMemcpyDeviceToHost, st));
    BSP_HIP(hipStreamSynchronize(st));
    if (err) {
        set_error("overlapped Parareal solve: a wait exceeded its time limit");
        return BS_ERR_HIP;
    }
    const volatile double* hist = S.hist;
    int status = BS_NOT_CONVERGED, last = 0;
    for (int j = 1; j <= kmax; ++j) {
        const double d = hist[2 * j], flag = hist[2 * j + 1];
        if (d < 0.0) break;  // not reached
        if (defect_hist) defect_hist[j - 1] = d;
        last = j;
        if ((status = record_status(flag)) != BS_OK) break;
        if (d <= tol || j == N) {
            status = BS_OK;
            break;
        }
        status = BS_NOT_CONVERGED;
    }
    *iters = last;
    if (prof) {
        float f_ms = 0.f, p_ms = 0.f;
        BSP_HIP(hipEventElapsedTime(&f_ms, g_prof.ev[0], g_prof.ev[1]));
        BSP_HIP(hipEventElapsedTime(&p_ms, g_prof.ev[2], g_prof.ev[3]));
        g_prof.fine_ms += f_ms;
        g_prof.fine_launches += 1;
        g_prof.fine_cells += (double)sl->fine_steps * M;  // slice 0, iteration 1
        g_prof.solve_ms += p_ms;
        g_prof.solve_launches += 1;
        for (int k = 1; k <= last; ++k) g_prof.solve_cells += iteration_cells(grid, sl, k);
        if (last >= 1) g_prof.solve_cells -= (double)sl->fine_steps * M;
    }
    if (status == BS_ERR_NONFINITE)
        set_error("non-finite value in the Parareal state at iteration %d", last);
    else if (status == BS_ERR_DIVERGED)
        set_error("Parareal diverging: defect of iteration %d above %g x the first", last, growth);
    return status;
}

extern "C" {

int parareal_iterate(const bs_params* prm, const bs_grid* grid, const bs_slices* sl, int kind,
                     const pinn_net* net, void* ws, size_t ws_size, double* U, int k,
                     double* defect, int* nonfinite, void* stream) {
    clear_error();
    int rc = check_parareal(prm, grid, sl, kind, net, ws, ws_size, U);
    if (rc) return rc;
    BSP_CHECK_ARG(k >= 1, "iteration index k must be >= 1");
    BSP_CHECK_ARG(defect && nonfinite, "defect and nonfinite must be non-NULL host pointers");
    return iterate_impl(prm, grid, sl, kind, net, ws, U, k, defect, nonfinite,
                        (hipStream_t)stream);
}

int parareal_solve(const bs_params* prm, const bs_grid* grid, const bs_slices* sl, int kind,
                   double tol, const pinn_net* net, int max_iter, void* ws, size_t ws_size,
                   double* U, int* iters, double* defect_hist, void* stream) {
    clear_error();
    int rc = check_parareal(prm, grid, sl, kind, net, ws, ws_size, U);
    if (rc) return rc;
    BSP_CHECK_ARG(iters != nullptr, "iters must be a non-NULL host pointer");
    BSP_CHECK_ARG(max_iter >= 1, "max_iter must be >= 1");
    BSP_CHECK_ARG(tol >= 0, "tol must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    const int N = sl->N;
    const int kmax = max_iter < N ? max_iter : N;
    const double growth = g_growth.load();
    *iters = 0;
    if ((rc = solve_reserve(kmax))) return rc;
    if (g_prof.on && (rc = prof_reserve(kmax))) return rc;
    SolveState& S = t_solve;
    for (size_t i = 0; i < 2 * (size_t)(kmax + 1); ++i) S.hist[i] = 0.0;
    Workspace w = ws_layout(ws, grid->M, N, kind);
    int* stop = reinterpret_cast<int*>(w.result + 4);
    if ((rc = launch_set_int(stop, 0, st))) return rc;
    if (kind == BS_COARSE_FLOWMAP) {
        // the coarse network sees the state: iterations one after the other,
        // the stopping rule and the divergence guard decided on the host
        if ((rc = start_impl(prm, grid, sl, kind, net, ws, U, nullptr, st))) return rc;
        double first = 0.0;
        for (int k = 1; k <= kmax; ++k) {
            double d = 0.0;
            int bad = 0;
            rc = iterate_impl(prm, grid, sl, kind, net, ws, U, k, &d, &bad, st);
            *iters = k;
            if (defect_hist) defect_hist[k - 1] = d;
            if (rc) return rc;
            if (k == 1) first = d;
            if (d <= tol || k == N) return BS_OK;
            if (k >= 2 && d > growth * first) {
                set_error("Parareal diverging: defect of iteration %d above %g x the first", k,
                          growth);
                return BS_ERR_DIVERGED;
            }
        }
        return BS_NOT_CONVERGED;
    }
    if (persist_capable(grid->M, N))
        return solve_persistent(prm, grid, sl, kind, tol, growth, net, kmax, ws, U, iters,
                                defect_hist, S.hist_dev, S.hist, true, g_prof.on, st);
    if (large_persist_capable(grid->M, N)) {
        if (g_prof.on && (rc = prof_reserve(1))) return rc;
        return solve_large(prm, grid, sl, kind, tol, growth, net, kmax, ws, U, iters,
                           defect_hist, st);
    }

    // Overlapped iterations (grids the one-block sweep and the per-system
    // fine kernel cover): the fine launch of iteration k runs on a side
    // stream and starts each slice as soon as the sweep of iteration k-1 has
    // produced its initial value, so the sweep of iteration k-1 and the fine
    // work of iteration k run at the same time; the sweep of iteration k
    // follows slice by slice.  The iterates are the same as one launch after
    // the other.  Consecutive fine launches alternate between two side
    // streams so that one may start while the previous one's last slices
    // still run.
    const bool pipe = pipe_capable(grid->M);
    PipeSync ps{};
    if (pipe) {
        if ((rc = solve_streams())) return rc;
        ps = pipe_sync(w, N);
        if ((rc = launch_fill_int(w.flags, flag_count(N), 0, st))) return rc;
        BSP_HIP(hipEventRecord(S.go, st));
        for (int i = 0; i < 2; ++i) BSP_HIP(hipStreamWaitEvent(S.side[i], S.go, 0));
    }
    if ((rc = start_impl(prm, grid, sl, kind, net, ws, U, pipe ? &ps : nullptr, st))) return rc;

    // Iteration k+1 is queued before the host looks at iteration k, so the
    // stream never waits for the host; the sweep that meets the stopping
    // rule sets the device flag, which turns the one queued iteration after
    // it into an empty launch pair.
    const volatile double* hist = S.hist;
    int status = BS_NOT_CONVERGED, last = 0, enq = 0;
    auto decide = [&](int j) {
        const double d = hist[2 * j];
        if (defect_hist) defect_hist[j - 1] = d;
        last = j;
        if ((status = record_status(hist[2 * j + 1])) != BS_OK) return true;
        if (d <= tol || j == N) {
            status = BS_OK;
            return true;
        }
        status = BS_NOT_CONVERGED;
        return j == kmax;
    };
    bool decided = false;
    for (int k = 1; k <= kmax && !decided; ++k) {
        if ((rc = enqueue_iteration(prm, grid, sl, kind, net, ws, U, k, stop, S.hist_dev, tol, growth,
                                    k - 1, pipe ? &ps : nullptr, pipe ? S.side[k & 1] : st, st)))
            return rc;
        BSP_HIP(hipEventRecord(S.done[k], st));
        enq = k;
        if (k >= 2) {
            BSP_HIP(hipEventSynchronize(S.done[k - 1]));
            decided = decide(k - 1);
        }
    }
    if (!decided) {
        BSP_HIP(hipEventSynchronize(S.done[enq]));
        decide(enq);
    }
    int err = 0;
    if (pipe) {  // the caller's stream ends after the side streams' work
        for (int i = 0; i < 2; ++i) {
            BSP_HIP(hipEventRecord(S.side_done[i], S.side[i]));
            BSP_HIP(hipStreamWaitEvent(st, S.side_done[i], 0));
        }
        BSP_HIP(hipMemcpyAsync(&err, ps.err, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    BSP_HIP(hipStreamSynchronize(st));
    *iters = last;
    if (err) {
        set_error("overlapped Parareal solve: a launch waited longer than its time limit");
        return BS_ERR_HIP;
    }
    if (g_prof.on) {
        for (int k = 1; k <= enq; ++k)
            if ((rc = prof_collect(k - 1, k <= last ? iteration_cells(grid, sl, k) : 0.0)))
                return rc;
    }
    if (status == BS_ERR_NONFINITE)
        set_error("non-finite value in the Parareal state at iteration %d", last);
    else if (status == BS_ERR_DIVERGED)
        set_error("Parareal diverging: defect of iteration %d above %g x the first", last, growth);
    return status;
}

int bs_release_resources(void) {
    clear_error();
    SolveState& S = t_solve;
    if (S.hist) BSP_HIP(hipHostFree(S.hist));
    S.hist = S.hist_dev = nullptr;
    S.cap = 0;
    for (hipEvent_t e : S.done) BSP_HIP(hipEventDestroy(e));
    S.done.clear();
    if (S.dev >= 0) {
        for (int i = 0; i < 2; ++i) {
            BSP_HIP(hipStreamDestroy(S.side[i]));
            BSP_HIP(hipEventDestroy(S.side_done[i]));
            S.side[i] = nullptr;
            S.side_done[i] = nullptr;
        }
        BSP_HIP(hipEventDestroy(S.go));
        S.go = nullptr;
        S.dev = -1;
    }
    for (hipEvent_t e : g_prof.ev) BSP_HIP(hipEventDestroy(e));
    g_prof.ev.clear();
    g_prof.on = false;
    return release_batch_resources();
}

}  // extern "C"

// ------------------------------------------------ solve without allocation
// parareal_solve_noalloc keeps its workspace and per-iteration record in a
// file-scope device array, `scratch` (one copy per GPU the library runs on,
// held until the process ends).  In host code the array's name stands for a
// host-side shadow, not a device address: kernels and copies get the address
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[BS_NOALLOC_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
constexpr int kNoallocMaxM = 4096;  // beyond: coefficient tables the library allocates
constexpr int kNoallocMaxN = 512;   // bounds the host copy of the record (on the stack)
static std::mutex g_scratch_mu;
static void* g_scratch[kScratchDevices] = {};

// Device address of this device's scratch (looked up on the first call on
// the device, with that device current).
static int scratch_address(void** out) {
    int dev = 0;
    BSP_HIP(hipGetDevice(&dev));
    BSP_CHECK_ARG(dev >= 0 && dev < kScratchDevices, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return BS_ERR_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return BS_OK;
}

extern "C" int parareal_solve_noalloc(const bs_params* prm, const bs_grid* grid,
                                      const bs_slices* sl, int kind, double tol,
                                      const pinn_net* net, int max_iter, double* U, int* iters,
                                      double* defect_hist, void* stream) {
    clear_error();
    int rc;
    if ((rc = check_params(prm))) return rc;
    if ((rc = check_grid(grid))) return rc;
    if ((rc = check_slices(sl))) return rc;
    BSP_CHECK_ARG(kind != BS_COARSE_FLOWMAP,
                  "parareal_solve_noalloc does not take the flow-map coarse");
    BSP_CHECK_ARG(kind == BS_COARSE_IE || kind == BS_COARSE_PINN || kind == BS_COARSE_PINN_IE,
                  "unknown coarse kind %d", kind);
    if (kind != BS_COARSE_IE) {
        if ((rc = check_net(net))) return rc;
        BSP_CHECK_ARG(net->n_in == 2 || net->n_in == 4, "network inputs must be 2 or 4");
    }
    BSP_CHECK_ARG(U != nullptr, "U is NULL");
    BSP_CHECK_ARG(iters != nullptr, "iters must be a non-NULL host pointer");
    BSP_CHECK_ARG(max_iter >= 1, "max_iter must be >= 1");
    BSP_CHECK_ARG(tol >= 0, "tol must be >= 0");
    const int M = grid->M, N = sl->N;
    BSP_CHECK_ARG(M <= kNoallocMaxM, "parareal_solve_noalloc covers grids of up to %d nodes (M = %d)",
                  kNoallocMaxM, M);
    BSP_CHECK_ARG(N <= kNoallocMaxN, "parareal_solve_noalloc covers up to %d slices (N = %d)",
                  kNoallocMaxN, N);
    const int kmax = max_iter < N ? max_iter : N;
    const size_t wsb = ws_bytes(M, N, kind);  // a multiple of 256
    const size_t nrec = 2 * (size_t)(kmax + 1);
    const size_t need = wsb + align256(sizeof(double) * nrec);
    if (need > (size_t)BS_NOALLOC_SCRATCH_BYTES) {
        set_error("parareal_solve_noalloc: M = %d, N = %d needs %zu bytes of scratch, the maximum "
                  "is %zu",
                  M, N, need, (size_t)BS_NOALLOC_SCRATCH_BYTES);
        return BS_ERR_ARG;
    }
    void* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    void* ws = base;
    double* rec_dev = reinterpret_cast<double*>(static_cast<char*>(base) + wsb);
    double rec[2 * (kNoallocMaxN + 1)];
    hipStream_t st = (hipStream_t)stream;
    const double growth = g_growth.load();
    *iters = 0;
    Workspace w = ws_layout(ws, M, N, kind);
    int* stop = reinterpret_cast<int*>(w.result + 4);
    if ((rc = launch_set_int(stop, 0, st))) return rc;
    if (persist_capable(M, N))
        return solve_persistent(prm, grid, sl, kind, tol, growth, net, kmax, ws, U, iters,
                                defect_hist, rec_dev, rec, false, false, st);

    // Otherwise the iterations one after the other on the caller's stream,
    // each decided from its 16-byte record before the next one is queued.
    if ((rc = start_impl(prm, grid, sl, kind, net, ws, U, nullptr, st))) return rc;
    int status = BS_NOT_CONVERGED, last = 0;
    for (int k = 1; k <= kmax; ++k) {
        if ((rc = enqueue_iteration(prm, grid, sl, kind, net, ws, U, k, stop, rec_dev, tol, growth, -1,
                                    nullptr, st, st)))
            return rc;
        BSP_HIP(hipMemcpyAsync(rec + 2 * k, rec_dev + 2 * k, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, st));
        BSP_HIP(hipStreamSynchronize(st));
        const double d = rec[2 * k];
        if (defect_hist) defect_hist[k - 1] = d;
        last = k;
        if ((status = record_status(rec[2 * k + 1])) != BS_OK) break;
        if (d <= tol || k == N) {
            status = BS_OK;
            break;
        }
        status = BS_NOT_CONVERGED;
    }
    *iters = last;
    if (status == BS_ERR_NONFINITE)
        set_error("non-finite value in the Parareal state at iteration %d", last);
    else if (status == BS_ERR_DIVERGED)
        set_error("Parareal diverging: defect of iteration %d above %g x the first", last, growth);
    return status;
}
