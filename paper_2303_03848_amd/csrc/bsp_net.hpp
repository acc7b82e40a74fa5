// Device helpers for the network kernels: activation, bfloat16 conversion and
// the gfx950 matrix-core instruction used for every matrix product.
//
// v_mfma_f32_32x32x16_bf16 (one wavefront) computes C[32x32] += A[32x16] B[16x32]
// with bfloat16 inputs and float32 accumulation.  Lane l holds
//   A[l % 32][8 (l / 32) + e], e = 0..7        (8 bf16)
//   B[8 (l / 32) + e][l % 32], e = 0..7        (8 bf16)
//   C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32], v = 0..15   (16 f32)
// (layout checked on the device against a host product).
#pragma once

#include "bsp_common.hpp"

namespace bsp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float tanh_f32(float z) { return tanhf(z); }

// tanh z = 1 - 2 / (1 + e^{2z}) with the hardware base-2 exponential and
// reciprocal: a few instructions, absolute error about 1e-7 (relative error
// grows only for |z| below about 1e-3, where the value is that small).  For
// activations that are rounded to bfloat16 (8 significant bits) next.
// Saturates to +-1 (e^{2z} overflows to infinity or underflows to zero).
__device__ __forceinline__ float tanh_bf16_act(float z) {
    const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);  // e^{2z} = 2^{2z log2 e}
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

__device__ __forceinline__ f32x16 mfma32x32x16(const bf16x8& a, const bf16x8& b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Eight consecutive bf16 from LDS (16-byte aligned).
__device__ __forceinline__ bf16x8 lds_frag(const __bf16* p) {
    return *reinterpret_cast<const bf16x8*>(p);
}

// Where the inputs of point i come from: an explicit [n][n_in] array, or the
// Parareal grid (tau_n = n dT, x_j = (j+1) dS / K, i = n*M + j).
// Batch mode (tiles != nullptr): point i lies in tile i / 32, which names its
// option; the option's grid is packed from tiles[i/32].base on.
// Flow-map mode (Us != nullptr): point i is node i of the state Us of one
// slice, inputs (tau_s, tau_e, Us[i] / K, (i+1) dS / K).
struct NetInput {
    const float* X;
    int n_in;
    int M;
    double dT, dS_over_K, sigma, r;
    const BatchOpt* bopts;
    const BatchTile* tiles;
    const double* Us = nullptr;
    double tau_s = 0.0, tau_e = 0.0, inv_K = 0.0;
};

// Inputs of point i; false for the padding points of batch mode.
__device__ __forceinline__ bool net_input(const NetInput& in, long i, float (&x)[4]) {
    if (in.Us) {
        x[0] = (float)in.tau_s;
        x[1] = (float)in.tau_e;
        x[2] = (float)(in.Us[i] * in.inv_K);
        x[3] = (float)((double)(i + 1) * in.dS_over_K);
        return true;
    }
    if (in.X) {
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = (c < in.n_in) ? in.X[i * in.n_in + c] : 0.0f;
        return true;
    }
    if (in.tiles) {
        const BatchTile t = in.tiles[i >> 5];
        const long li = i - t.base;
        if (li >= t.count) {
            x[0] = x[1] = x[2] = x[3] = 0.0f;
            return false;
        }
        const BatchOpt& b = in.bopts[t.opt];
        const long n = li / b.M, j = li - n * b.M;
        x[0] = (float)((double)n * b.dT);
        x[1] = (float)((double)(j + 1) * (b.o.dS / b.o.K));
        x[2] = (float)sqrt(b.o.s2);
        x[3] = (float)b.o.r;
        return true;
    }
    const long n = i / in.M, j = i - n * in.M;
    x[0] = (float)((double)n * in.dT);
    x[1] = (float)((double)(j + 1) * in.dS_over_K);
    x[2] = (float)in.sigma;
    x[3] = (float)in.r;
    return true;
}

// Store the network value of point i: out32[i] = v, or out64[i] = scale * v;
// in batch mode out64[i] = K v, and for a put K v - S + K exp(-r tau) (the
// network prices calls; put-call parity gives the put).
__device__ __forceinline__ void net_store(const NetInput& in, long i, float v, float* out32,
                                          double* out64, double scale) {
    if (out32) out32[i] = v;
    if (!out64) return;
    if (in.tiles) {
        const BatchTile t = in.tiles[i >> 5];
        const BatchOpt& b = in.bopts[t.opt];
        const long li = i - t.base;
        double V = b.o.K * (double)v;
        if (b.o.is_put) {
            const long n = li / b.M, j = li - n * b.M;
            V = V - (double)(j + 1) * b.o.dS + b.o.K * exp(-b.o.r * ((double)n * b.dT));
        }
        out64[i] = V;
    } else {
        out64[i] = scale * (double)v;
    }
}

__device__ __forceinline__ int mfma_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

}  // namespace bsp
