// Network forward pass on the matrix cores: bfloat16 operands, float32
// accumulation, tanh in float32 (the BS_PREC_BF16 path of pinn_forward and
// of the network coarse propagator).
//
// One block of 4 wavefronts takes 32 points through every layer without
// leaving the CU: activations ping-pong between two LDS tiles [32][W] (bf16),
// the layer's weights are staged in LDS in K-chunks of up to 128 columns, and
// each wavefront owns 32-unit column blocks of the layer output (one
// v_mfma_f32_32x32x16_bf16 per 16-wide K step).  The tiny first layer (2 or
// 4 inputs) and the output dot product run on the vector units.
#include "bsp_common.hpp"
#include "bsp_net.hpp"

namespace bsp {

template <int W>
__global__ __launch_bounds__(256) void k_mlp_bf16(const float* __restrict__ prm, int depth, long n,
                                                  NetInput in, float* __restrict__ out32,
                                                  double* __restrict__ out64, double scale) {
    constexpr int KC = W < 128 ? W : 128;  // weight columns staged per pass
    constexpr int LDA = W + 8;             // row stride of the activation tiles (bf16)
    constexpr int LDW = KC + 8;            // row stride of the staged weights (bf16)
    constexpr int NB = W >= 128 ? W / 128 : 1;  // output column blocks per wavefront
    __shared__ __align__(16) __bf16 act[2][32 * LDA];
    __shared__ __align__(16) __bf16 ws[W * LDW];
    __shared__ float xin[32][4];
    __shared__ int ok[32];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, h = lane >> 5;
    const long base = (long)blockIdx.x * 32;
    const int n_in = in.n_in;

    if (tid < 32) {
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        ok[tid] = base + tid < n && net_input(in, base + tid, x);
#pragma unroll
        for (int c = 0; c < 4; ++c) xin[tid][c] = x[c];
    }
    __syncthreads();
    for (int e = tid; e < 32 * W; e += 256) {
        const int i = e / W, j = e - i * W;
        float z = prm[W * n_in + j];
        for (int c = 0; c < n_in; ++c) z = fmaf(prm[j * n_in + c], xin[i][c], z);
        act[0][i * LDA + j] = (__bf16)tanh_f32(z);
    }
    long off = (long)W * n_in + W;
    int cur = 0;
    for (int l = 2; l <= depth; ++l) {
        const float* Wl = prm + off;
        const float* bl = Wl + (long)W * W;
        f32x16 acc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
        for (int kc = 0; kc < W; kc += KC) {
            __syncthreads();
            for (int e = tid; e < W * KC; e += 256) {
                const int j = e / KC, k = e - j * KC;
                ws[j * LDW + k] = (__bf16)Wl[(long)j * W + kc + k];
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int cb = wave + 4 * b;
                if (cb * 32 < W) {
#pragma unroll
                    for (int t = 0; t < KC / 16; ++t) {
                        const bf16x8 a = lds_frag(&act[cur][r32 * LDA + kc + 16 * t + 8 * h]);
                        const bf16x8 bb = lds_frag(&ws[(cb * 32 + r32) * LDW + 16 * t + 8 * h]);
                        acc[b] = mfma32x32x16(a, bb, acc[b]);
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int cb = wave + 4 * b;
            if (cb * 32 < W) {
                const int j = cb * 32 + r32;
                const float bj = bl[j];
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    act[cur ^ 1][mfma_row(v, lane) * LDA + j] = (__bf16)tanh_f32(acc[b][v] + bj);
            }
        }
        cur ^= 1;
        off += (long)W * W + W;
    }
    __syncthreads();
    // output layer: 8 threads per point, then a reduction over those 8 lanes
    const int i = tid >> 3, part = tid & 7;
    float s = 0.f;
    for (int j = part; j < W; j += 8) s = fmaf(prm[off + j], (float)act[cur][i * LDA + j], s);
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    if (part == 0 && ok[i]) net_store(in, base + i, s + prm[off + W], out32, out64, scale);
}

int launch_mlp_bf16(const pinn_net& net, long n, const NetInput& in, float* out32, double* out64,
                    double scale, hipStream_t stream) {
    const dim3 grid((unsigned)((n + 31) / 32));
    switch (net.width) {
#define BSP_W(W_)                                                                                 \
    case W_:                                                                                      \
        hipLaunchKernelGGL(k_mlp_bf16<W_>, grid, dim3(256), 0, stream, net.params, net.depth, n, \
                           in, out32, out64, scale);                                              \
        break;
        BSP_W(32) BSP_W(64) BSP_W(128) BSP_W(256)
#undef BSP_W
    default:
        set_error("the bfloat16 network path needs width >= 32 (got %d)", net.width);
        return BS_ERR_ARG;
    }
    BSP_LAUNCHED();
    return BS_OK;
}

}  // namespace bsp
