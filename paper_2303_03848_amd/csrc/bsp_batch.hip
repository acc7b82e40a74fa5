// Many independent options solved together: every kernel phase of a Parareal
// iteration is one launch per block-shape class covering every option of the
// class (uneven grids M and slice counts N are mixed within a launch).
//
// Work items live in device tables built once per solve: per option a record
// (coefficients, sizes, offsets) and a state (done flag, iterations, defect);
// per class the list of (option, slice) fine-propagator items and the list of
// options for the sweep.  Blocks of converged options, and fine items of
// slices that already hold the serial fine solution (n < k - 1), return at
// once, so the launch configuration never changes between iterations and the
// host can queue iterations ahead of their results: it keeps `lookahead`
// iterations in flight, each followed by an asynchronous copy of the count of
// still-active options into pinned host memory, and waits only for the
// oldest of them (the device never idles on a host round trip; at most
// lookahead - 1 empty iterations run after the last option converges).
#include <cmath>
#include <cstring>
#include <vector>

#include "bsp_steps.hpp"

namespace bsp {

// Largest grid of a batched option: the batch kernels keep the whole
// factorisation in registers (no streamed-coefficient variant).
constexpr int kMaxBatchM = 4096;

struct FItem {
    int opt, n;
};

// Expiry payoff of every option (one block per option).
__global__ void k_batch_initial(const BatchOpt* __restrict__ opts, int payoff_mode,
                                double* __restrict__ U) {
    const BatchOpt& b = opts[blockIdx.x];
    const OptionDev& o = b.o;
    for (int i = threadIdx.x; i < b.M; i += blockDim.x) {
        const double S = (double)(i + 1) * o.dS;
        const double K = o.K;
        double v;
        if (payoff_mode == 0) {
            v = o.is_put ? fmax(K - S, 0.0) : fmax(S - K, 0.0);
        } else {
            const double lo = S - 0.5 * o.dS, hi = S + 0.5 * o.dS;
            if (!o.is_put)
                v = (hi <= K) ? 0.0 : (lo >= K) ? 0.5 * (lo + hi) - K : (hi - K) * (hi - K) / (2.0 * o.dS);
            else
                v = (lo >= K) ? 0.0 : (hi <= K) ? K - 0.5 * (lo + hi) : (K - lo) * (K - lo) / (2.0 * o.dS);
        }
        U[b.u_off + i] = v;
    }
}

// Fine propagator on every unconverged (option, slice) item of one class.
template <int T, int MC>
__global__ __launch_bounds__(T) void k_batch_fine(const BatchOpt* __restrict__ opts,
                                                  const BatchState* __restrict__ state,
                                                  const FItem* __restrict__ items,
                                                  const int* __restrict__ kglob,
                                                  const double* __restrict__ U,
                                                  double* __restrict__ Fv) {
    __shared__ double smem[smem_doubles<T, MC>()];
    double* lds = smem;
    double* ftab = smem + 4 * T;
    const FItem it = items[blockIdx.x];
    if (state[it.opt].done) return;
    const int k = *kglob;
    if (it.n < k - 1) return;  // holds the serial fine solution; Fv unchanged
    const BatchOpt& b = opts[it.opt];
    const double dt = b.dT / (double)b.fine_steps;
    double V[MC];
    load_system<T, MC>(U + b.u_off + (long)it.n * b.M, b.M, V, smem);
    Solver<T, MC> S;
    S.setup(b.o.s2, b.o.r, 0.5 * dt, 0.5 * dt, b.M, lds);
    theta_steps<T, MC, true>(S, b.o, V, (double)it.n * b.dT, dt, b.fine_steps, 0.5, false, lds,
                             ftab);
    store_system<T, MC>(Fv + b.w_off + (long)it.n * b.M, b.M, V, smem);
}

// Serial sweep of every unconverged option of one class; decides convergence.
template <int T, int MC>
__global__ __launch_bounds__(T) void k_batch_sweep(const BatchOpt* __restrict__ opts,
                                                   BatchState* __restrict__ state,
                                                   const int* __restrict__ list,
                                                   const int* __restrict__ kglob, int predict,
                                                   int kind, double tol, double growth,
                                                   int max_iter,
                                                   double* __restrict__ U, const double* Fv,
                                                   double* Gold, const double* Vt,
                                                   int* __restrict__ active) {
    __shared__ double smem[sweep_smem_doubles<T, MC>()];
    double* lds = smem;
    double* ftab = smem + 4 * T;
    const int oi = list[blockIdx.x];
    BatchState& st = state[oi];
    if (st.done) return;
    const BatchOpt& b = opts[oi];
    const int k = predict ? 0 : *kglob;
    const int n0 = predict ? 0 : (k - 1 < b.N - 1 ? k - 1 : b.N - 1);
    Solver<T, MC> S;
    S.setup(b.o.s2, b.o.r, b.dT / (double)b.coarse_steps, 0.0, b.M, lds);
    double dmax = 0.0;
    int bad = 0;
    sweep_slices<T, MC>(S, b.o, b.M, b.N, n0, b.coarse_steps, kind, predict != 0, b.dT,
                        U + b.u_off, U + b.u_off, Fv + b.w_off, Gold + b.w_off,
                        Vt ? Vt + b.vt_off : nullptr,
                        lds, ftab, dmax, bad);
    if (predict) return;
    block_defect<T>(dmax, bad, lds);
    if (threadIdx.x == 0) {
        if (k == 1) st.first = dmax;
        // 1 non-finite; 2 diverged (the defect grew by `growth` over iteration 1's)
        const int status = bad ? 1 : (k >= 2 && dmax > growth * st.first) ? 2 : 0;
        st.defect = dmax;
        st.iters = k;
        st.bad = status;
        if (status || dmax <= tol || k >= b.N || k >= max_iter) {
            st.done = 1;
            atomicSub(active, 1);
        }
    }
}

__global__ void k_batch_set(int* __restrict__ kglob, int* __restrict__ active, int k, int n) {
    *kglob = k;
    *active = n;
}

__global__ void k_batch_tick(int* __restrict__ kglob) { *kglob += 1; }

// ------------------------------------------------------------------ host side

struct BatchPlan {
    int n_opt;
    std::vector<BatchOpt> opts;
    std::vector<TriShape> fine_cls, sweep_cls;              // distinct shapes
    std::vector<std::vector<FItem>> fine_items;             // per fine class
    std::vector<std::vector<int>> sweep_lists;              // per sweep class
    std::vector<BatchTile> tiles;
    long fw_total = 0, vt_total = 0;
};

static int class_of(std::vector<TriShape>& cls, TriShape s) {
    for (size_t i = 0; i < cls.size(); ++i)
        if (cls[i].T == s.T && cls[i].MC == s.MC) return (int)i;
    cls.push_back(s);
    return (int)cls.size() - 1;
}

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

struct BatchWs {
    BatchOpt* opts;
    BatchState* state;
    FItem* items;
    int* lists;
    BatchTile* tiles;
    int* counters;  // [0] k, [1] active
    double* Fv;
    double* Gold;
    double* Vt;
    size_t bytes;
};

static BatchWs batch_layout(const BatchPlan& P, long n_items, bool net, void* base) {
    BatchWs w{};
    char* p = (char*)base;
    size_t off = 0;
    auto take = [&](size_t b) {
        char* q = p ? p + off : nullptr;
        off += a256(b);
        return q;
    };
    w.opts = (BatchOpt*)take(sizeof(BatchOpt) * P.n_opt);
    w.state = (BatchState*)take(sizeof(BatchState) * P.n_opt);
    w.items = (FItem*)take(sizeof(FItem) * n_items);
    w.lists = (int*)take(sizeof(int) * P.n_opt);
    w.tiles = (BatchTile*)take(sizeof(BatchTile) * (net ? P.tiles.size() : 1));
    w.counters = (int*)take(sizeof(int) * 4);
    w.Fv = (double*)take(sizeof(double) * P.fw_total);
    w.Gold = (double*)take(sizeof(double) * P.fw_total);
    w.Vt = net ? (double*)take(sizeof(double) * P.vt_total) : nullptr;
    w.bytes = off;
    return w;
}

static int make_plan(int n_opt, const bs_params* prm, const bs_grid* grids, const bs_slices* sl,
                     const long* offsets, bool net, BatchPlan& P) {
    P.n_opt = n_opt;
    P.opts.resize(n_opt);
    long fw = 0, vt = 0;
    for (int i = 0; i < n_opt; ++i) {
        const bs_params& p = prm[i];
        BSP_CHECK_ARG(p.K > 0 && p.sigma > 0 && p.r >= 0 && p.T > 0 && p.s_max > 0,
                      "option %d: parameters out of range", i);
        const int M = grids[i].M, N = sl[i].N;
        BSP_CHECK_ARG(M >= 1 && M <= kMaxBatchM && tri_shape(M).T > 0,
                      "option %d: M = %d outside 1..%d", i, M, kMaxBatchM);
        BSP_CHECK_ARG(N >= 1 && sl[i].fine_steps >= 1 && sl[i].coarse_steps >= 1,
                      "option %d: slices out of range", i);
        BSP_CHECK_ARG(grids[i].payoff_mode == grids[0].payoff_mode,
                      "all options must share payoff_mode");
        BSP_CHECK_ARG(offsets[i] >= 0, "option %d: negative offset", i);
        BatchOpt& b = P.opts[i];
        b.o = make_option(p, M);
        b.M = M;
        b.N = N;
        b.fine_steps = sl[i].fine_steps;
        b.coarse_steps = sl[i].coarse_steps;
        b.dT = p.T / N;
        b.u_off = offsets[i];
        b.w_off = fw;
        fw += (long)N * M;
        b.vt_off = vt;
        const long cnt = (long)(N + 1) * M;
        if (net) {
            for (long t = 0; t < (cnt + 31) / 32; ++t) P.tiles.push_back({i, 0, vt, cnt});
            vt += (cnt + 31) / 32 * 32;
        }
        const int fc = class_of(P.fine_cls, shape_for(0, M));
        const int sc = class_of(P.sweep_cls, shape_for(1, M));
        if ((int)P.fine_items.size() <= fc) P.fine_items.resize(fc + 1);
        if ((int)P.sweep_lists.size() <= sc) P.sweep_lists.resize(sc + 1);
        for (int n = 0; n < N; ++n) P.fine_items[fc].push_back({i, n});
        P.sweep_lists[sc].push_back(i);
    }
    P.fw_total = fw;
    P.vt_total = vt;
    return BS_OK;
}

// Streams for the shape classes of one phase.  The launches of a phase touch
// disjoint items (fine) or options (sweep), so they run side by side: fork
// from the caller's stream, one stream per class, join back on it.
// Created once per thread and device, kept until the process ends.
constexpr int kMaxClasses = 16;
struct ClassStreams {
    int dev = -1;
    hipStream_t s[kMaxClasses] = {};
    hipEvent_t fork[2] = {}, join[2][kMaxClasses] = {};
};
static thread_local ClassStreams t_cls;

// Pinned slots for the active counts of the iterations in flight and their
// events; created once per thread and device, kept until released.
constexpr int kDefaultLookahead = 4, kMaxLookahead = 16;
struct LookaheadSlots {
    int dev = -1;
    int* active = nullptr;  // pinned host [kMaxLookahead]
    hipEvent_t ev[kMaxLookahead] = {};
};
static thread_local LookaheadSlots t_look;

static int release_lookahead() {
    LookaheadSlots& L = t_look;
    if (L.dev < 0) return BS_OK;
    for (int i = 0; i < kMaxLookahead; ++i) BSP_HIP(hipEventDestroy(L.ev[i]));
    BSP_HIP(hipHostFree(L.active));
    L = LookaheadSlots{};
    return BS_OK;
}

static int lookahead_slots() {
    LookaheadSlots& L = t_look;
    int dev = 0;
    BSP_HIP(hipGetDevice(&dev));
    if (L.dev == dev) return BS_OK;
    int rc = release_lookahead();
    if (rc) return rc;
    BSP_HIP(hipHostMalloc((void**)&L.active, sizeof(int) * kMaxLookahead, hipHostMallocDefault));
    for (int i = 0; i < kMaxLookahead; ++i)
        BSP_HIP(hipEventCreateWithFlags(&L.ev[i], hipEventDisableTiming));
    L.dev = dev;
    return BS_OK;
}

int release_batch_resources() {
    int rc = release_lookahead();
    if (rc) return rc;
    ClassStreams& C = t_cls;
    if (C.dev < 0) return BS_OK;
    for (int i = 0; i < kMaxClasses; ++i) {
        BSP_HIP(hipStreamDestroy(C.s[i]));
        for (int ph = 0; ph < 2; ++ph) BSP_HIP(hipEventDestroy(C.join[ph][i]));
    }
    for (int ph = 0; ph < 2; ++ph) BSP_HIP(hipEventDestroy(C.fork[ph]));
    C = ClassStreams{};
    return BS_OK;
}

static int class_streams() {
    ClassStreams& C = t_cls;
    int dev = 0;
    BSP_HIP(hipGetDevice(&dev));
    if (C.dev == dev) return BS_OK;
    if (C.dev >= 0) {  // made on another device: release them first
        int rc = release_batch_resources();
        if (rc) return rc;
    }
    for (int i = 0; i < kMaxClasses; ++i) {
        BSP_HIP(hipStreamCreateWithFlags(&C.s[i], hipStreamNonBlocking));
        for (int ph = 0; ph < 2; ++ph)
            BSP_HIP(hipEventCreateWithFlags(&C.join[ph][i], hipEventDisableTiming));
    }
    for (int ph = 0; ph < 2; ++ph) BSP_HIP(hipEventCreateWithFlags(&C.fork[ph], hipEventDisableTiming));
    C.dev = dev;
    return BS_OK;
}

// launch(c, stream) for the n classes of phase ph (0 fine, 1 sweep) on the
// class streams, joined on st before the call returns.
template <class F>
static int run_phase(int ph, int n, hipStream_t st, F&& launch) {
    if (n == 1) return launch(0, st);
    ClassStreams& C = t_cls;
    BSP_HIP(hipEventRecord(C.fork[ph], st));
    for (int c = 0; c < n; ++c) {
        BSP_HIP(hipStreamWaitEvent(C.s[c], C.fork[ph], 0));
        const int rc = launch(c, C.s[c]);
        if (rc) return rc;
        BSP_HIP(hipEventRecord(C.join[ph][c], C.s[c]));
        BSP_HIP(hipStreamWaitEvent(st, C.join[ph][c], 0));
    }
    return BS_OK;
}

static int launch_fine_class(TriShape sh, int nitems, const BatchWs& w, const FItem* items,
                             const double* U, hipStream_t st) {
#define BSP_CASE(T_, MC_)                                                                       \
    if (sh.T == T_ && sh.MC == MC_) {                                                           \
        hipLaunchKernelGGL((k_batch_fine<T_, MC_>), dim3(nitems), dim3(T_), 0, st, w.opts,     \
                           w.state, items, w.counters, U, w.Fv);                               \
        BSP_LAUNCHED();                                                                         \
        return BS_OK;                                                                           \
    }
    BSP_TRI_SHAPES(BSP_CASE)
#undef BSP_CASE
    set_error("unbuilt block shape");
    return BS_ERR_ARG;
}

static int launch_sweep_class(TriShape sh, int nopt, const BatchWs& w, const int* list,
                              int predict, int kind, double tol, double growth, int max_iter,
                              double* U, hipStream_t st) {
#define BSP_CASE(T_, MC_)                                                                      \
    if (sh.T == T_ && sh.MC == MC_) {                                                          \
        hipLaunchKernelGGL((k_batch_sweep<T_, MC_>), dim3(nopt), dim3(T_), 0, st, w.opts,     \
                           w.state, list, w.counters, predict, kind, tol, growth, max_iter,   \
                           U, w.Fv, w.Gold, w.Vt, w.counters + 1);                             \
        BSP_LAUNCHED();                                                                        \
        return BS_OK;                                                                          \
    }
    BSP_TRI_SHAPES(BSP_CASE)
#undef BSP_CASE
    set_error("unbuilt block shape");
    return BS_ERR_ARG;
}

int launch_pinn_batch_grid(const pinn_net& net, const BatchOpt* opts, const BatchTile* tiles,
                           long npts, double* Vt, hipStream_t stream);

}  // namespace bsp

using namespace bsp;

static int batch_checks(int n_opt, const bs_params* prm, const bs_grid* grids,
                        const bs_slices* sl, int kind, const pinn_net* net) {
    BSP_CHECK_ARG(n_opt >= 1, "n_opt must be >= 1");
    BSP_CHECK_ARG(prm && grids && sl, "host option arrays must be non-NULL");
    BSP_CHECK_ARG(kind != BS_COARSE_FLOWMAP, "the batched solve does not take the flow-map coarse");
    BSP_CHECK_ARG(kind == BS_COARSE_IE || kind == BS_COARSE_PINN || kind == BS_COARSE_PINN_IE,
                  "unknown coarse kind %d", kind);
    if (kind != BS_COARSE_IE) {
        int rc = check_net(net);
        if (rc) return rc;
    }
    return BS_OK;
}

extern "C" int parareal_batch_workspace_size(int n_opt, const bs_params* prm,
                                             const bs_grid* grids, const bs_slices* sl,
                                             int coarse_kind, size_t* bytes) {
    clear_error();
    BSP_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = 0;
    BSP_CHECK_ARG(n_opt >= 1, "n_opt must be >= 1");
    BSP_CHECK_ARG(prm && grids && sl, "host option arrays must be non-NULL");
    BSP_CHECK_ARG(coarse_kind == BS_COARSE_IE || coarse_kind == BS_COARSE_PINN ||
                      coarse_kind == BS_COARSE_PINN_IE,
                  "unknown coarse kind %d", coarse_kind);
    std::vector<long> offs(n_opt, 0);
    BatchPlan P;
    int rc = make_plan(n_opt, prm, grids, sl, offs.data(), coarse_kind != BS_COARSE_IE, P);
    if (rc) return rc;
    long n_items = 0;
    for (auto& v : P.fine_items) n_items += (long)v.size();
    *bytes = batch_layout(P, n_items, coarse_kind != BS_COARSE_IE, nullptr).bytes;
    return BS_OK;
}

extern "C" int parareal_solve_batch(int n_opt, const bs_params* prm, const bs_grid* grids,
                                    const bs_slices* sl, int kind, double tol,
                                    const pinn_net* net, int max_iter, void* ws, size_t ws_bytes,
                                    double* U, const long* offsets, int* iters, double* defects,
                                    int lookahead, void* stream) {
    clear_error();
    int rc = batch_checks(n_opt, prm, grids, sl, kind, net);
    if (rc) return rc;
    BSP_CHECK_ARG(U && offsets && iters, "U, offsets and iters must be non-NULL");
    BSP_CHECK_ARG(max_iter >= 1 && tol >= 0, "max_iter >= 1 and tol >= 0 required");
    BSP_CHECK_ARG(lookahead >= 0 && lookahead <= kMaxLookahead, "lookahead must be 0..%d",
                  kMaxLookahead);
    const bool is_net = kind != BS_COARSE_IE;
    BatchPlan P;
    if ((rc = make_plan(n_opt, prm, grids, sl, offsets, is_net, P))) return rc;
    long n_items = 0;
    for (auto& v : P.fine_items) n_items += (long)v.size();
    const BatchWs w = batch_layout(P, n_items, is_net, ws);
    if (!ws || ws_bytes < w.bytes) {
        set_error("workspace too small: need %zu bytes", w.bytes);
        return BS_ERR_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    const double growth = bs_divergence_growth();

    // tables -> device (one staging copy)
    std::vector<FItem> items_flat;
    std::vector<long> item_off, list_off;
    for (auto& v : P.fine_items) {
        item_off.push_back((long)items_flat.size());
        items_flat.insert(items_flat.end(), v.begin(), v.end());
    }
    std::vector<int> lists_flat;
    for (auto& v : P.sweep_lists) {
        list_off.push_back((long)lists_flat.size());
        lists_flat.insert(lists_flat.end(), v.begin(), v.end());
    }
    std::vector<BatchState> st0(n_opt);
    std::memset(st0.data(), 0, sizeof(BatchState) * n_opt);
    BSP_HIP(hipMemcpyAsync(w.opts, P.opts.data(), sizeof(BatchOpt) * n_opt, hipMemcpyHostToDevice, st));
    BSP_HIP(hipMemcpyAsync(w.state, st0.data(), sizeof(BatchState) * n_opt, hipMemcpyHostToDevice, st));
    BSP_HIP(hipMemcpyAsync(w.items, items_flat.data(), sizeof(FItem) * n_items, hipMemcpyHostToDevice, st));
    BSP_HIP(hipMemcpyAsync(w.lists, lists_flat.data(), sizeof(int) * n_opt, hipMemcpyHostToDevice, st));
    if (is_net)
        BSP_HIP(hipMemcpyAsync(w.tiles, P.tiles.data(), sizeof(BatchTile) * P.tiles.size(),
                               hipMemcpyHostToDevice, st));
    BSP_HIP(hipStreamSynchronize(st));  // the host tables may go out of scope

    // k = 0: payoff, network grid, coarse prediction
    hipLaunchKernelGGL(k_batch_initial, dim3(n_opt), dim3(256), 0, st, w.opts, grids[0].payoff_mode, U);
    BSP_LAUNCHED();
    if (is_net && (rc = launch_pinn_batch_grid(*net, w.opts, w.tiles, P.vt_total, w.Vt, st))) return rc;
    BSP_CHECK_ARG(P.fine_cls.size() <= (size_t)kMaxClasses && P.sweep_cls.size() <= (size_t)kMaxClasses,
                  "too many block-shape classes");
    if ((rc = class_streams())) return rc;
    rc = run_phase(1, (int)P.sweep_cls.size(), st, [&](int c, hipStream_t s) {
        return launch_sweep_class(P.sweep_cls[c], (int)P.sweep_lists[c].size(), w,
                                  w.lists + list_off[c], 1, kind, tol, growth, max_iter, U, s);
    });
    if (rc) return rc;
    hipLaunchKernelGGL(k_batch_set, dim3(1), dim3(1), 0, st, w.counters, w.counters + 1, 1, n_opt);
    BSP_LAUNCHED();

    int kmax = 0;
    for (int i = 0; i < n_opt; ++i) kmax = sl[i].N > kmax ? sl[i].N : kmax;
    kmax = max_iter < kmax ? max_iter : kmax;

    auto iteration = [&]() -> int {
        int r = run_phase(0, (int)P.fine_cls.size(), st, [&](int c, hipStream_t s) {
            return launch_fine_class(P.fine_cls[c], (int)P.fine_items[c].size(), w,
                                     w.items + item_off[c], U, s);
        });
        if (r) return r;
        r = run_phase(1, (int)P.sweep_cls.size(), st, [&](int c, hipStream_t s) {
            return launch_sweep_class(P.sweep_cls[c], (int)P.sweep_lists[c].size(), w,
                                      w.lists + list_off[c], 0, kind, tol, growth, max_iter,
                                      U, s);
        });
        if (r) return r;
        hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(1), 0, st, w.counters);
        BSP_LAUNCHED();
        return BS_OK;
    };

    // iterations queued ahead: after each one an asynchronous copy of the
    // active count to a pinned slot and an event; the host waits for the
    // oldest iteration in flight only, and stops queueing once a copied count
    // is zero (iterations already queued then return at once on the device)
    if ((rc = lookahead_slots())) return rc;
    const int L = lookahead == 0 ? kDefaultLookahead : lookahead;
    LookaheadSlots& LS = t_look;
    int queued = 0, checked = 0;
    bool finished = false;
    while (!finished && checked < kmax) {
        while (queued < kmax && queued - checked < L) {
            if ((rc = iteration())) return rc;
            BSP_HIP(hipMemcpyAsync(LS.active + queued % L, w.counters + 1, sizeof(int),
                                   hipMemcpyDeviceToHost, st));
            BSP_HIP(hipEventRecord(LS.ev[queued % L], st));
            ++queued;
        }
        BSP_HIP(hipEventSynchronize(LS.ev[checked % L]));
        finished = LS.active[checked % L] == 0;
        ++checked;
    }

    std::vector<BatchState> out(n_opt);
    BSP_HIP(hipMemcpyAsync(out.data(), w.state, sizeof(BatchState) * n_opt, hipMemcpyDeviceToHost, st));
    BSP_HIP(hipStreamSynchronize(st));
    // Worst outcome over the options: non-finite, then diverged, then not converged.
    int status = BS_OK;
    for (int i = 0; i < n_opt; ++i) {
        iters[i] = out[i].iters;
        if (defects) defects[i] = out[i].defect;
        if (out[i].bad == 1) {
            if (status != BS_ERR_NONFINITE) set_error("non-finite value in option %d", i);
            status = BS_ERR_NONFINITE;
        } else if (out[i].bad == 2) {
            if (status != BS_ERR_NONFINITE && status != BS_ERR_DIVERGED)
                set_error("option %d diverging: defect of iteration %d above %g x the first", i,
                          out[i].iters, growth);
            if (status != BS_ERR_NONFINITE) status = BS_ERR_DIVERGED;
        } else if (status == BS_OK && !(out[i].defect <= tol) && out[i].iters < P.opts[i].N) {
            status = BS_NOT_CONVERGED;
        }
    }
    return status;
}
