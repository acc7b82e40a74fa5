// Network forward pass on the matrix cores: bfloat16 operands, float32
// accumulation, tanh in float32 (the BS_PREC_BF16 path of pinn_forward and
// of the network coarse propagator).  tanh is evaluated through the
// exponential (tanh_bf16_act): the activations are rounded to bfloat16.
//
// One block of 4 wavefronts (8 for width 256) takes P = 256 points through
// every layer without leaving the CU: the activations [P][W] (bf16) sit in
// one LDS tile; a layer's products go to registers, and after a barrier its
// outputs overwrite its inputs (a second tile would halve P, and every block
// reads the weights once per layer, so points per block set the L2 traffic).
// Each wavefront owns 32-unit blocks of a layer's output and all P/32 point
// tiles; the products are taken as [unit][point] (weights as the first
// operand), so each lane ends with four consecutive units of one point and
// stores them together.  A weight fragment (8 consecutive inputs of one unit) is read
// from global memory (the layer stays in L2), converted to bf16 in
// registers and used for all row tiles before the next one, so weights are
// neither staged in LDS nor re-read per 32 points; the fragments are loaded
// eight K-steps ahead of their use.  One
// v_mfma_f32_32x32x16_bf16 per row tile and 16-wide K step.  The tiny first
// layer (2 or 4 inputs) and the output dot product run on the vector units.
#include "bsp_common.hpp"
#include "bsp_net.hpp"

namespace bsp {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpPoints = 256;  // points per block

// Wavefronts per block: 8 for the widest layers, so that two wavefronts share
// each SIMD and one's tanh epilogue overlaps the other's matrix products.
template <int W>
constexpr int mlp_waves() {
    return W >= 256 ? 8 : 4;
}

template <int W>
__global__ __launch_bounds__(64 * mlp_waves<W>()) void k_mlp_bf16(const float* __restrict__ prm, int depth, long n,
                                                  NetInput in, float* __restrict__ out32,
                                                  double* __restrict__ out64, double scale) {
    constexpr int P = kMlpPoints;
    constexpr int MT = P / 32;                  // row tiles
    constexpr int LDA = W + 8;                  // row stride of the activation tiles (bf16)
    constexpr int NW = mlp_waves<W>(), NT = 64 * NW;
    constexpr int NB = W >= 32 * NW ? W / (32 * NW) : 1;  // output column blocks per wavefront
    __shared__ __align__(16) __bf16 act[P * LDA];
    __shared__ float xin[P][4];
    __shared__ int ok[P];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, h = lane >> 5;
    const long base = (long)blockIdx.x * P;
    const int n_in = in.n_in;

    for (int t = tid; t < P; t += NT) {
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        ok[t] = base + t < n && net_input(in, base + t, x);
#pragma unroll
        for (int c = 0; c < 4; ++c) xin[t][c] = x[c];
    }
    __syncthreads();
    {
        // first layer: NT is a multiple of W, so a thread keeps one unit j
        // (its weights in registers) over the rows i0, i0 + NT/W, ...
        static_assert(NT % W == 0, "the first layer keeps one unit per thread");
        const int j = tid % W;
        float wj[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) wj[c] = c < n_in ? prm[j * n_in + c] : 0.f;
        const float bj = prm[W * n_in + j];
        for (int i = tid / W; i < P; i += NT / W) {
            float z = bj;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < n_in) z = fmaf(wj[c], xin[i][c], z);
            act[i * LDA + j] = (__bf16)tanh_bf16_act(z);
        }
    }
    long off = (long)W * n_in + W;
    for (int l = 2; l <= depth; ++l) {
        const float* Wl = prm + off;
        const float* bl = Wl + (long)W * W;
        __syncthreads();  // the layer's input complete
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int cb = wave + NW * b;
            const bool active = cb * 32 < W;  // (narrow layers leave wavefronts idle)
            f32x16 acc[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[mt][v] = 0.f;
            if (active) {
                // unit j = cb*32 + r32; this lane's inputs 16 t + 8 h .. + 7.
                // The weight fragments are loaded PD K-steps ahead of their use
                // (a ring of registers): with one wavefront per SIMD nothing else
                // hides the L2 latency.
                const float* wrow = Wl + (long)(cb * 32 + r32) * W + 8 * h;
                constexpr int KT = W / 16, PD = KT < 8 ? KT : 8;
                float4 wr0[PD], wr1[PD];
#pragma unroll
                for (int t = 0; t < PD; ++t) {
                    wr0[t] = *reinterpret_cast<const float4*>(wrow + 16 * t);
                    wr1[t] = *reinterpret_cast<const float4*>(wrow + 16 * t + 4);
                }
#pragma unroll
                for (int t = 0; t < KT; ++t) {
                    const float4 w0 = wr0[t % PD];
                    const float4 w1 = wr1[t % PD];
                    if (t + PD < KT) {
                        wr0[t % PD] = *reinterpret_cast<const float4*>(wrow + 16 * (t + PD));
                        wr1[t % PD] = *reinterpret_cast<const float4*>(wrow + 16 * (t + PD) + 4);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    bf16x8 bb;
                    bb[0] = (__bf16)w0.x; bb[1] = (__bf16)w0.y; bb[2] = (__bf16)w0.z; bb[3] = (__bf16)w0.w;
                    bb[4] = (__bf16)w1.x; bb[5] = (__bf16)w1.y; bb[6] = (__bf16)w1.z; bb[7] = (__bf16)w1.w;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const bf16x8 a = lds_frag(&act[(mt * 32 + r32) * LDA + 16 * t + 8 * h]);
                        acc[mt] = mfma32x32x16(bb, a, acc[mt]);  // [unit][point]
                    }
                }
            }
            __syncthreads();  // every wavefront is done reading the layer's input
            if (active) {
                // this lane: point mt*32 + r32, units cb*32 + 8 (v >> 2) + 4 h + (v & 3):
                // four consecutive units of one point per 8-byte store
                float bj[16];
#pragma unroll
                for (int v = 0; v < 16; ++v) bj[v] = bl[cb * 32 + mfma_row(v, lane)];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        bf16x4 q;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            q[e] = (__bf16)tanh_bf16_act(acc[mt][4 * m + e] + bj[4 * m + e]);
                        *reinterpret_cast<bf16x4*>(
                            &act[(mt * 32 + r32) * LDA + cb * 32 + 8 * m + 4 * h]) = q;
                    }
            }
        }
        off += (long)W * W + W;
    }
    __syncthreads();
    // output layer: 8 threads per point, then a reduction over those 8 lanes
    const int part = tid & 7;
    float wo[W / 8];  // this thread's output weights, units part, part + 8, ...
#pragma unroll
    for (int q = 0; q < W / 8; ++q) wo[q] = prm[off + part + 8 * q];
    for (int i = tid >> 3; i < P; i += NT / 8) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < W / 8; ++q) s = fmaf(wo[q], (float)act[i * LDA + part + 8 * q], s);
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        if (part == 0 && ok[i]) net_store(in, base + i, s + prm[off + W], out32, out64, scale);
    }
}

int launch_mlp_bf16(const pinn_net& net, long n, const NetInput& in, float* out32, double* out64,
                    double scale, hipStream_t stream) {
    const dim3 grid((unsigned)((n + kMlpPoints - 1) / kMlpPoints));
    switch (net.width) {
#define BSP_W(W_)                                                                                 \
    case W_:                                                                                      \
        hipLaunchKernelGGL(k_mlp_bf16<W_>, grid, dim3(64 * mlp_waves<W_>()), 0, stream,         \
                           net.params, net.depth, n,                                              \
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
