// Network forward pass (Sec. 3.3): (tau, S/K[, sigma, r]) -> v = V/K through
// `depth` tanh layers of `width` units and a linear output.
//
// FP32 path: one point per thread; the hidden activations of a block's 64
// points sit in LDS as [unit][point] (each thread reads its own column, no
// bank conflicts); weights are wave-uniform and arrive through scalar loads.
#include "bsp_common.hpp"
#include "bsp_net.hpp"

namespace bsp {

long net_param_count(const pinn_net& n) {
    const long w = n.width;
    return w * n.n_in + w + (long)(n.depth - 1) * (w * w + w) + w + 1;
}

int check_net(const pinn_net* net) {
    BSP_CHECK_ARG(net != nullptr, "pinn_net is NULL");
    BSP_CHECK_ARG(net->params != nullptr, "pinn_net.params is NULL");
    BSP_CHECK_ARG(net->n_in == 2 || net->n_in == 4, "pinn_net.n_in must be 2 or 4 (got %d)",
                  net->n_in);
    BSP_CHECK_ARG(net->depth >= 1 && net->depth <= 16, "pinn_net.depth must be in [1,16] (got %d)",
                  net->depth);
    const int w = net->width;
    BSP_CHECK_ARG(w == 16 || w == 32 || w == 64 || w == 128 || w == 256,
                  "pinn_net.width must be 16, 32, 64, 128 or 256 (got %d)", w);
    BSP_CHECK_ARG(net->precision == BS_PREC_FP32 || net->precision == BS_PREC_BF16,
                  "pinn_net.precision must be BS_PREC_FP32 or BS_PREC_BF16");
    return BS_OK;
}

// Output: out32[i] = v, or out64[i] = scale * v.
template <int W>
__global__ __launch_bounds__(64) void k_mlp_fp32(const float* __restrict__ prm, int depth, long n,
                                                 NetInput in, float* __restrict__ out32,
                                                 double* __restrict__ out64, double scale) {
    __shared__ float act[2][W][64];
    const int t = threadIdx.x;
    const long i = (long)blockIdx.x * 64 + t;
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    const bool valid = i < n && net_input(in, i, x);
    const int n_in = in.n_in;

    const float* Wl = prm;
    const float* bl = prm + W * n_in;
    for (int j = 0; j < W; ++j) {
        float z = bl[j];
        for (int c = 0; c < n_in; ++c) z = fmaf(Wl[j * n_in + c], x[c], z);
        act[0][j][t] = tanhf(z);
    }
    const float* base = bl + W;
    int cur = 0;
    constexpr int JC = 16;
    for (int l = 1; l < depth; ++l) {
        Wl = base;
        bl = base + W * W;
        for (int j0 = 0; j0 < W; j0 += JC) {
            float acc[JC];
#pragma unroll
            for (int jj = 0; jj < JC; ++jj) acc[jj] = bl[j0 + jj];
            for (int k = 0; k < W; ++k) {
                const float a = act[cur][k][t];
#pragma unroll
                for (int jj = 0; jj < JC; ++jj) acc[jj] = fmaf(Wl[(j0 + jj) * W + k], a, acc[jj]);
            }
#pragma unroll
            for (int jj = 0; jj < JC; ++jj) act[cur ^ 1][j0 + jj][t] = tanhf(acc[jj]);
        }
        cur ^= 1;
        base = bl + W;
    }
    float v = base[W];
    for (int k = 0; k < W; ++k) v = fmaf(base[k], act[cur][k][t], v);
    if (valid) net_store(in, i, v, out32, out64, scale);
}

int launch_mlp_bf16(const pinn_net& net, long n, const NetInput& in, float* out32, double* out64,
                    double scale, hipStream_t stream);

static int launch_mlp(const pinn_net& net, long n, const NetInput& in, float* out32,
                      double* out64, double scale, hipStream_t stream) {
    if (n == 0) return BS_OK;
    if (net.precision == BS_PREC_BF16) return launch_mlp_bf16(net, n, in, out32, out64, scale, stream);
    const dim3 grid((unsigned)((n + 63) / 64));
    switch (net.width) {
#define BSP_W(W_)                                                                            \
    case W_:                                                                                 \
        hipLaunchKernelGGL(k_mlp_fp32<W_>, grid, dim3(64), 0, stream, net.params, net.depth, \
                           n, in, out32, out64, scale);                                      \
        break;
        BSP_W(16) BSP_W(32) BSP_W(64) BSP_W(128) BSP_W(256)
#undef BSP_W
    default:
        set_error("unsupported width %d", net.width);
        return BS_ERR_ARG;
    }
    BSP_LAUNCHED();
    return BS_OK;
}

int launch_pinn_grid(const pinn_net& net, const OptionDev& o, int M, int N, double dT, double* Vt,
                     hipStream_t stream) {
    NetInput in{nullptr, net.n_in, M, dT, o.dS / o.K, sqrt(o.s2), o.r, nullptr, nullptr};
    return launch_mlp(net, (long)(N + 1) * M, in, nullptr, Vt, o.K, stream);
}

int launch_flowmap(const pinn_net& net, const OptionDev& o, int M, double tau_s, double tau_e,
                   const double* Us, double* g, hipStream_t stream) {
    NetInput in{nullptr, net.n_in, M, 0.0, o.dS / o.K, 0.0, 0.0, nullptr, nullptr};
    in.Us = Us;
    in.tau_s = tau_s;
    in.tau_e = tau_e;
    in.inv_K = 1.0 / o.K;
    return launch_mlp(net, M, in, nullptr, g, o.K, stream);
}

int launch_pinn_batch_grid(const pinn_net& net, const BatchOpt* opts, const BatchTile* tiles,
                           long npts, double* Vt, hipStream_t stream) {
    NetInput in{nullptr, net.n_in, 1, 0.0, 0.0, 0.0, 0.0, opts, tiles};
    return launch_mlp(net, npts, in, nullptr, Vt, 1.0, stream);
}

}  // namespace bsp

extern "C" int pinn_forward(const pinn_net* net, int n, const float* X, float* v_out,
                            void* stream) {
    bsp::clear_error();
    int rc = bsp::check_net(net);
    if (rc) return rc;
    BSP_CHECK_ARG(n >= 0, "n must be >= 0");
    BSP_CHECK_ARG(n == 0 || (X && v_out), "X and v_out must be non-NULL");
    bsp::NetInput in{X, net->n_in, 1, 0.0, 0.0, 0.0, 0.0, nullptr, nullptr};
    return bsp::launch_mlp(*net, n, in, v_out, nullptr, 1.0, (hipStream_t)stream);
}
