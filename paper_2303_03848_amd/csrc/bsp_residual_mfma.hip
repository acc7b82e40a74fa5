// Matrix-core (bfloat16 in, float32 accumulate) versions of the two
// GEMM-shaped steps of the PINN loss gradient, for widths 32, 64, 128.
//
// Forward hidden layer (k_res_fwd_bf16): a tile of 32 points carries its four
// input streams (value, d/dtau, d/dx, d2/dx2; recomputed from the previous
// layer's cache) in LDS; each wavefront owns 32-unit output blocks and runs
// one MFMA chain per stream against the staged weights; the epilogue applies
// the tanh stream rule and writes the layer cache.
//
// Backward hidden layer (k_res_bwd_bf16), persistent over point tiles:
//   abar_prev[s] = zbar[s] W                     (data adjoints, per tile)
//   dW += sum_s zbar[s]^T a_prev[s],  db += sum zbar[0]   (weights)
// The weight gradient is accumulated per block across its tiles in
// registers and written as one partial per block; k_res_reduce sums the
// partials in block order, so the result is deterministic.
#include "bsp_common.hpp"
#include "bsp_net.hpp"

namespace bsp {

constexpr int kResPartBlocksMfma = 64;

__device__ __forceinline__ void streams_of(const float* c, long plane, long idx, float (&a)[4]) {
    const float av = c[idx], zt = c[plane + idx], zx = c[2 * plane + idx], zxx = c[3 * plane + idx];
    const float s = 1.0f - av * av;
    a[0] = av;
    a[1] = s * zt;
    a[2] = s * zx;
    a[3] = s * zxx - 2.0f * av * s * zx * zx;
}

template <int W>
__global__ __launch_bounds__(256) void k_res_fwd_bf16(const float* __restrict__ Wl,
                                                      const float* __restrict__ bl,
                                                      const float* __restrict__ cprev,
                                                      float* __restrict__ cnext, long n_pad) {
    constexpr int LDA = W + 8;
    __shared__ __align__(16) __bf16 As[4][32 * LDA];
    __shared__ __align__(16) __bf16 Ws[W * LDA];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, h = lane >> 5;
    const long i0 = (long)blockIdx.x * 32;
    const long plane = n_pad * W;
    for (int e = tid; e < 32 * W; e += 256) {
        const int i = e / W, k = e - i * W;
        float a[4];
        streams_of(cprev, plane, (i0 + i) * W + k, a);
#pragma unroll
        for (int s = 0; s < 4; ++s) As[s][i * LDA + k] = (__bf16)a[s];
    }
    for (int e = tid; e < W * W; e += 256) {
        const int j = e / W, k = e - j * W;
        Ws[j * LDA + k] = (__bf16)Wl[e];
    }
    __syncthreads();
    for (int cb = wave; cb * 32 < W; cb += 4) {
        f32x16 acc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[s][v] = 0.f;
#pragma unroll
        for (int t = 0; t < W / 16; ++t) {
            const bf16x8 b = lds_frag(&Ws[(cb * 32 + r32) * LDA + 16 * t + 8 * h]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[s] = mfma32x32x16(lds_frag(&As[s][r32 * LDA + 16 * t + 8 * h]), b, acc[s]);
        }
        const int j = cb * 32 + r32;
        const float bj = bl[j];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const long idx = (i0 + mfma_row(v, lane)) * W + j;
            cnext[idx] = tanh_f32(acc[0][v] + bj);
            cnext[plane + idx] = acc[1][v];
            cnext[2 * plane + idx] = acc[2][v];
            cnext[3 * plane + idx] = acc[3][v];
        }
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_res_bwd_bf16(const float* __restrict__ Wl,
                                                      const float* __restrict__ zbar,
                                                      const float* __restrict__ cprev,
                                                      float* __restrict__ abar, long n_pad,
                                                      int ntiles, float* __restrict__ part) {
    constexpr int LDA = W + 8;   // [point][unit] tiles
    constexpr int LDT = 32 + 8;  // [unit][point] tiles
    constexpr int NBJ = W / 32;  // 32-wide blocks per dimension of dW
    constexpr int NBW = (NBJ * NBJ + 3) / 4;  // dW blocks per wavefront
    __shared__ __align__(16) __bf16 Zs[4][32 * LDA];
    __shared__ __align__(16) __bf16 ZT[4][W * LDT];
    __shared__ __align__(16) __bf16 aT[4][W * LDT];
    __shared__ __align__(16) __bf16 WT[W * LDA];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, h = lane >> 5;
    const long plane = n_pad * W;

    for (int e = tid; e < W * W; e += 256) {
        const int k = e / W, j = e - k * W;
        WT[k * LDA + j] = (__bf16)Wl[(long)j * W + k];
    }
    f32x16 gacc[NBW];
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) gacc[b][v] = 0.f;
    float gb = 0.f;

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long i0 = (long)tile * 32;
        __syncthreads();
        for (int e = tid; e < 32 * W; e += 256) {
            const int i = e / W, j = e - i * W;
            const long idx = (i0 + i) * W + j;
            float a[4];
            streams_of(cprev, plane, idx, a);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const __bf16 z = (__bf16)zbar[s * plane + idx];
                Zs[s][i * LDA + j] = z;
                ZT[s][j * LDT + i] = z;
                aT[s][j * LDT + i] = (__bf16)a[s];
            }
        }
        if (tid < W)
            for (int i = 0; i < 32; ++i) gb += zbar[(i0 + i) * W + tid];
        __syncthreads();
        // data adjoints of the previous layer: abar_prev[s][i][k] = sum_j zbar[s][i][j] W[j][k]
        for (int cb = wave; cb * 32 < W; cb += 4) {
            f32x16 acc[4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[s][v] = 0.f;
#pragma unroll
            for (int t = 0; t < W / 16; ++t) {
                const bf16x8 b = lds_frag(&WT[(cb * 32 + r32) * LDA + 16 * t + 8 * h]);
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc[s] = mfma32x32x16(lds_frag(&Zs[s][r32 * LDA + 16 * t + 8 * h]), b, acc[s]);
            }
            const int k = cb * 32 + r32;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const long idx = (i0 + mfma_row(v, lane)) * W + k;
#pragma unroll
                for (int s = 0; s < 4; ++s) abar[s * plane + idx] = acc[s][v];
            }
        }
        // weight gradient: dW[j][k] += sum_s sum_i zbar[s][i][j] a_prev[s][i][k]
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            const int blk = wave + 4 * b;
            if (blk < NBJ * NBJ) {
                const int jb = blk / NBJ, kb = blk - jb * NBJ;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        gacc[b] = mfma32x32x16(lds_frag(&ZT[s][(jb * 32 + r32) * LDT + 16 * t + 8 * h]),
                                               lds_frag(&aT[s][(kb * 32 + r32) * LDT + 16 * t + 8 * h]),
                                               gacc[b]);
            }
        }
    }
    float* out = part + (long)blockIdx.x * (W * W + W);
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
        const int blk = wave + 4 * b;
        if (blk < NBJ * NBJ) {
            const int jb = blk / NBJ, kb = blk - jb * NBJ;
#pragma unroll
            for (int v = 0; v < 16; ++v)
                out[(jb * 32 + mfma_row(v, lane)) * W + kb * 32 + r32] = gacc[b][v];
        }
    }
    if (tid < W) out[W * W + tid] = gb;
}

// grad[x] = sum over blocks b of part[b][x], x < count.  A block takes 32
// consecutive x; its 8 row groups sum the partials b = g, g + 8, ... (four
// running sums each, so the loads overlap), then the groups are added in
// order: a fixed summation order for every x, independent of timing.
__global__ __launch_bounds__(256) void k_res_reduce(const float* __restrict__ part, int nblk,
                                                    int count, float* __restrict__ grad) {
    __shared__ float acc[8][33];
    const int tx = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int x = blockIdx.x * 32 + tx;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (x < count) {
        int b = g;
        for (; b + 24 < nblk; b += 32) {
            s0 += part[(long)b * count + x];
            s1 += part[(long)(b + 8) * count + x];
            s2 += part[(long)(b + 16) * count + x];
            s3 += part[(long)(b + 24) * count + x];
        }
        for (; b < nblk; b += 8) s0 += part[(long)b * count + x];
    }
    acc[g][tx] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (g == 0 && x < count) {
        float s = acc[0][tx];
#pragma unroll
        for (int r = 1; r < 8; ++r) s += acc[r][tx];
        grad[x] = s;
    }
}

int launch_res_reduce(const float* part, int nblk, int count, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_res_reduce, dim3((count + 31) / 32), dim3(256), 0, st, part, nblk, count,
                       out);
    BSP_LAUNCHED();
    return BS_OK;
}

int launch_res_gemm_bf16(int which, const float* Wl, const float* bl, const float* cin,
                         float* cout_or_abar, const float* zbar, long n, long n_pad, int W,
                         float* gW, float* gb, float* part, hipStream_t st) {
    (void)n;
    const int ntiles = (int)(n_pad / 32);
    if (which == 0) {
        switch (W) {
#define BSP_W(W_)                                                                             \
    case W_:                                                                                  \
        hipLaunchKernelGGL(k_res_fwd_bf16<W_>, dim3(ntiles), dim3(256), 0, st, Wl, bl, cin,  \
                           cout_or_abar, n_pad);                                              \
        break;
            BSP_W(32) BSP_W(64) BSP_W(128)
#undef BSP_W
        default:
            set_error("bfloat16 residual path: width %d not supported (32, 64, 128)", W);
            return BS_ERR_ARG;
        }
        BSP_LAUNCHED();
        return BS_OK;
    }
    const int nblk = ntiles < kResPartBlocksMfma ? ntiles : kResPartBlocksMfma;
    switch (W) {
#define BSP_W(W_)                                                                                \
    case W_:                                                                                     \
        hipLaunchKernelGGL(k_res_bwd_bf16<W_>, dim3(nblk), dim3(256), 0, st, Wl, zbar, cin,     \
                           cout_or_abar, n_pad, ntiles, part);                                   \
        break;
        BSP_W(32) BSP_W(64) BSP_W(128)
#undef BSP_W
    default:
        set_error("bfloat16 residual path: width %d not supported (32, 64, 128)", W);
        return BS_ERR_ARG;
    }
    BSP_LAUNCHED();
    const int count = W * W + W;
    // dW and db are contiguous in the parameter packing (W_l then b_l)
    (void)gb;
    return launch_res_reduce(part, nblk, count, gW, st);
}

}  // namespace bsp
