// The PINN loss and its gradient (eqs. (11)-(14)) in one launch on the
// matrix cores (bfloat16 operands, float32 accumulation), for widths 32, 64
// and 128, plus one launch that reduces the per-block partial sums.
//
// Every step of the gradient is local to a point except the sums over
// points, so one block takes a few 32-point tiles through the whole pass:
//   first layer (vector units) -> hidden layers (one MFMA chain per
//   derivative stream) -> head (output layer, loss terms, output adjoints)
//   -> backward through the hidden layers (data adjoints W^T zbar per tile,
//   weight gradient sum_s zbar_s^T a_prev_s) -> first-layer gradient.
// Two kernels do this:
//   k_res_tile_bf16 (networks of 2 to 4 layers): wavefront w owns 32 units of
//     every layer and meets the adjoints in the matrix-core output layout;
//     each lane's cache fragments go to the workspace in its own order.
//   k_res_step_bf16 (any depth): point-major caches, adjoints and output
//     adjoints in the workspace, the weights staged in LDS once per layer.
// Each block writes one partial row: every parameter's gradient over its
// points, then the three loss sums by point type; k_res_reduce_step adds the
// rows in block order, so the result does not depend on timing.
#include "bsp_residual.hpp"

namespace bsp {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kResStepThreads = 256;
constexpr int kResStepMinTiles = 2;  // tiles per block: fewer partial rows to reduce

struct ResStepArgs {
    const float* prm;  // parameters, float32, nn.Linear order
    Points P;
    NetLayout L;
    long n, n_pad;     // points, points rounded up to whole tiles
    int ntiles, tiles_per_block;
    float* cache;      // depth x [4][n_pad][W]: (a, z_t, z_x, z_xx) per layer
    float* abar;       // [4][n_pad][W]: adjoints of the streams entering a layer
    float* g;          // [4][n_pad]: output adjoints
    float* part;       // [blocks][ldp]
    long ldp;          // L.total + 3
};

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

__device__ __forceinline__ void st4(float* p, float x, float y, float z, float w) {
    *reinterpret_cast<float4*>(p) = make_float4(x, y, z, w);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ld4(const __attribute__((address_space(1))) float* p) {
    const f32x4 v = *reinterpret_cast<const __attribute__((address_space(1))) f32x4*>(p);
    return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ void st4(__attribute__((address_space(1))) float* p, float x, float y,
                                    float z, float w) {
    const f32x4 v = {x, y, z, w};
    *reinterpret_cast<__attribute__((address_space(1))) f32x4*>(p) = v;
}

__device__ __forceinline__ void st_bf16x4(__bf16* p, const float (&v)[4]) {
    bf16x4 b;
    b[0] = (__bf16)v[0];
    b[1] = (__bf16)v[1];
    b[2] = (__bf16)v[2];
    b[3] = (__bf16)v[3];
    *reinterpret_cast<bf16x4*>(p) = b;
}

// Global-memory view of a pointer: loads and stores through it are global_*
// instructions, which, unlike flat ones, do not hold up waits on LDS.
#define BSP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ BSP_GLOBAL T* gmem(T* p) {
    return (BSP_GLOBAL T*)p;
}

__device__ __forceinline__ float comp(const float4& v, int q) {
    return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
}

template <int W>
__global__ __launch_bounds__(kResStepThreads) void k_res_step_bf16(ResStepArgs a) {
    constexpr int NT = kResStepThreads;
    constexpr int LDA = W + 8;            // [point][unit] tiles (bf16)
    constexpr int LDT = 32 + 8;           // [unit][point] tiles (bf16)
    constexpr int NCB = W / 32;           // 32-unit blocks of a layer
    constexpr int NBW = (NCB * NCB + 3) / 4;  // 32 x 32 blocks of dW per wavefront
    constexpr int G4 = W / 4;             // 4-unit groups of a row
    constexpr int RP = NT / G4;           // rows per pass of the elementwise phases
    constexpr int PASSES = 32 / RP;
    constexpr int NG8 = W * W / 8;        // 8-element groups of a weight matrix
    __shared__ __align__(16) __bf16 Wsh[W * LDA];     // W[j][k] forward, W[j][k] at [k][j] backward
    __shared__ __align__(16) __bf16 Xs[4][32 * LDA];  // input streams [i][k], or zbar [i][j]
    __shared__ __align__(16) __bf16 ZT[4][W * LDT];   // zbar [j][i]
    __shared__ __align__(16) __bf16 aT[4][W * LDT];   // previous layer's streams [k][i]
    __shared__ float gsh[4][32];
    __shared__ float lsh[32];
    float* red = reinterpret_cast<float*>(&ZT[0][0]);  // RP x W floats between phases

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, h = lane >> 5;
    const int u0 = 4 * (tid % G4), rr = tid / G4;  // units u0 .. u0 + 3, rows rr + RP p
    const NetLayout& L = a.L;
    const int d = L.depth, n_in = L.n_in;
    const long n = a.n, n_pad = a.n_pad, plane = n_pad * W;
    const int t0 = blockIdx.x * a.tiles_per_block;
    const int t1 = min(t0 + a.tiles_per_block, a.ntiles);
    // global-memory views (global_* rather than flat instructions)
    const BSP_GLOBAL float* prm = gmem(a.prm);
    const BSP_GLOBAL float* wo = prm + L.off_wo;
    BSP_GLOBAL float* out = gmem(a.part) + (long)blockIdx.x * a.ldp;
    BSP_GLOBAL float* const abar = gmem(a.abar);
    BSP_GLOBAL float* const gout = gmem(a.g);
    auto cache = [&](int l) { return gmem(a.cache) + (long)(l - 1) * 4 * plane; };

    // Per-thread partials acc[q] of unit u0 + q over rows rr + RP p, summed
    // over the RP row groups in order; unit u goes to dst[u * stride].
    auto combine = [&](const float (&acc)[4], BSP_GLOBAL float* dst, int stride) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) red[rr * W + u0 + q] = acc[q];
        __syncthreads();
        if (tid < W) {
            float s = red[tid];
            for (int r = 1; r < RP; ++r) s += red[r * W + tid];
            dst[(long)tid * stride] = s;
        }
    };

    // The same for one unit per thread (unit tid % W, row group tid / W).
    auto combine1 = [&](float acc, BSP_GLOBAL float* dst) {
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        if (tid < W) {
            float s = red[tid];
            for (int r = 1; r < NT / W; ++r) s += red[r * W + tid];
            dst[tid] = s;
        }
    };

    // ---- first layer: z = W1 x + b1, z_t = W1[:,0], z_x = W1[:,1], z_xx = 0
    {
        float w1[4][4], b1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            b1[q] = prm[L.offb[1] + u0 + q];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                w1[q][c] = c < n_in ? prm[L.offW[1] + (long)(u0 + q) * n_in + c] : 0.f;
        }
        BSP_GLOBAL float* c1 = cache(1);
        for (int t = t0; t < t1; ++t)
#pragma unroll
            for (int p = 0; p < PASSES; ++p) {
                const long i = (long)t * 32 + rr + RP * p;
                float av[4] = {0.f, 0.f, 0.f, 0.f}, zt[4] = {0.f, 0.f, 0.f, 0.f},
                      zx[4] = {0.f, 0.f, 0.f, 0.f};
                if (i < n) {
                    const float* xr = point_row(a.P, i);
                    float x[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) x[c] = c < n_in ? xr[c] : 0.f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float z = b1[q];
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (c < n_in) z = fmaf(w1[q][c], x[c], z);
                        av[q] = tanh_f32(z);
                        zt[q] = w1[q][0];
                        zx[q] = w1[q][1];
                    }
                }
                const long idx = i * W + u0;
                st4(c1 + idx, av[0], av[1], av[2], av[3]);
                st4(c1 + plane + idx, zt[0], zt[1], zt[2], zt[3]);
                st4(c1 + 2 * plane + idx, zx[0], zx[1], zx[2], zx[3]);
                st4(c1 + 3 * plane + idx, 0.f, 0.f, 0.f, 0.f);
            }
    }

    // ---- hidden layers: z_s = W a_s (+ b for the value), then the tanh streams
    for (int l = 2; l <= d; ++l) {
        const BSP_GLOBAL float* Wl = prm + L.offW[l];
        const BSP_GLOBAL float* bl = prm + L.offb[l];
        const BSP_GLOBAL float* cp = cache(l - 1);
        BSP_GLOBAL float* cn = cache(l);
        __syncthreads();  // the previous layer's products are done with Wsh and Xs
#pragma unroll
        for (int m = 0; m < (NG8 + NT - 1) / NT; ++m) {
            const int e = tid + NT * m;
            if (e < NG8) {
                const int j = e / (W / 8), k = (e - j * (W / 8)) * 8;
                const float4 w0 = ld4(Wl + (long)j * W + k), w1 = ld4(Wl + (long)j * W + k + 4);
                bf16x8 b;
                b[0] = (__bf16)w0.x; b[1] = (__bf16)w0.y; b[2] = (__bf16)w0.z; b[3] = (__bf16)w0.w;
                b[4] = (__bf16)w1.x; b[5] = (__bf16)w1.y; b[6] = (__bf16)w1.z; b[7] = (__bf16)w1.w;
                *reinterpret_cast<bf16x8*>(&Wsh[j * LDA + k]) = b;
            }
        }
        for (int t = t0; t < t1; ++t) {
            const long i0 = (long)t * 32;
            if (t > t0) __syncthreads();  // the previous tile's products are done with Xs
#pragma unroll
            for (int p = 0; p < PASSES; ++p) {
                const int i = rr + RP * p;
                const long idx = (i0 + i) * W + u0;
                const float4 c0 = ld4(cp + idx), c1 = ld4(cp + plane + idx),
                             c2 = ld4(cp + 2 * plane + idx), c3 = ld4(cp + 3 * plane + idx);
                float s0[4], s1[4], s2[4], s3[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    streams_of_values(comp(c0, q), comp(c1, q), comp(c2, q), comp(c3, q), s0[q],
                                      s1[q], s2[q], s3[q]);
                st_bf16x4(&Xs[0][i * LDA + u0], s0);
                st_bf16x4(&Xs[1][i * LDA + u0], s1);
                st_bf16x4(&Xs[2][i * LDA + u0], s2);
                st_bf16x4(&Xs[3][i * LDA + u0], s3);
            }
            __syncthreads();
            for (int cb = wave; cb < NCB; cb += 4) {
                f32x16 acc[4];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[s][v] = 0.f;
#pragma unroll
                for (int k = 0; k < W / 16; ++k) {
                    const bf16x8 b = lds_frag(&Wsh[(cb * 32 + r32) * LDA + 16 * k + 8 * h]);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[s] = mfma32x32x16(lds_frag(&Xs[s][r32 * LDA + 16 * k + 8 * h]), b,
                                              acc[s]);
                }
                const int j = cb * 32 + r32;
                const float bj = bl[j];
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const long idx = (i0 + mfma_row(v, lane)) * W + j;
                    cn[idx] = tanh_f32(acc[0][v] + bj);
                    cn[plane + idx] = acc[1][v];
                    cn[2 * plane + idx] = acc[2][v];
                    cn[3 * plane + idx] = acc[3][v];
                }
            }
        }
    }

    // ---- head: output layer, loss terms, output adjoints; output-layer gradient
    {
        const BSP_GLOBAL float* cd = cache(d);
        float lsum[3] = {0.f, 0.f, 0.f}, dbo = 0.f;
        float dwo[4] = {0.f, 0.f, 0.f, 0.f};
        const int u = tid & 7, pt = tid >> 3;  // eight lanes per point
        for (int t = t0; t < t1; ++t) {
            const long i0 = (long)t * 32;
            __syncthreads();  // cache(d) complete; gsh and lsh free
            const long i = i0 + pt;
            float v = 0.f, vt = 0.f, vx = 0.f, vxx = 0.f;
            if (i < n) {
#pragma unroll
                for (int jj = 0; jj < W / 8; ++jj) {
                    const int j = u + 8 * jj;
                    const long ij = i * W + j;
                    float s0, s1, s2, s3;
                    streams_of_values(cd[ij], cd[plane + ij], cd[2 * plane + ij],
                                      cd[3 * plane + ij], s0, s1, s2, s3);
                    v = fmaf(wo[j], s0, v);
                    vt = fmaf(wo[j], s1, vt);
                    vx = fmaf(wo[j], s2, vx);
                    vxx = fmaf(wo[j], s3, vxx);
                }
            }
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                v += __shfl_xor(v, o, 8);
                vt += __shfl_xor(vt, o, 8);
                vx += __shfl_xor(vx, o, 8);
                vxx += __shfl_xor(vxx, o, 8);
            }
            if (u == 0) {
                float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, lc = 0.f;
                if (i < n) head_point(a.P, i, v + prm[L.off_bo], vt, vx, vxx, g0, g1, g2, g3, lc);
                gsh[0][pt] = g0;
                gsh[1][pt] = g1;
                gsh[2][pt] = g2;
                gsh[3][pt] = g3;
                lsh[pt] = lc;
                gout[i] = g0;
                gout[n_pad + i] = g1;
                gout[2 * n_pad + i] = g2;
                gout[3 * n_pad + i] = g3;
            }
            __syncthreads();
            if (tid == 0)
                for (int q = 0; q < 32; ++q) {
                    const long iq = i0 + q;
                    if (iq < n) lsum[iq < a.P.nf ? 0 : iq < a.P.nf + a.P.ne ? 1 : 2] += lsh[q];
                    dbo += gsh[0][q];
                }
            // dwo[j] += sum_s g_s[i] a_s[i][j] over this tile's points
#pragma unroll
            for (int p = 0; p < PASSES; ++p) {
                const int ip = rr + RP * p;
                const long idx = (i0 + ip) * W + u0;
                const float4 c0 = ld4(cd + idx), c1 = ld4(cd + plane + idx),
                             c2 = ld4(cd + 2 * plane + idx), c3 = ld4(cd + 3 * plane + idx);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float s0, s1, s2, s3;
                    streams_of_values(comp(c0, q), comp(c1, q), comp(c2, q), comp(c3, q), s0, s1,
                                      s2, s3);
                    float tq = gsh[0][ip] * s0;
                    tq = fmaf(gsh[1][ip], s1, tq);
                    tq = fmaf(gsh[2][ip], s2, tq);
                    tq = fmaf(gsh[3][ip], s3, tq);
                    dwo[q] += tq;
                }
            }
        }
        combine(dwo, out + L.off_wo, 1);
        if (tid == 0) {
            out[L.off_bo] = dbo;
            out[L.total] = lsum[0];
            out[L.total + 1] = lsum[1];
            out[L.total + 2] = lsum[2];
        }
    }

    // ---- backward through the hidden layers
    for (int l = d; l >= 2; --l) {
        const BSP_GLOBAL float* Wl = prm + L.offW[l];
        const BSP_GLOBAL float* cl = cache(l);
        const BSP_GLOBAL float* cp = cache(l - 1);
        __syncthreads();  // the head / the previous layer are done with Wsh, Xs, ZT, aT
        // Wsh[k][j] = W[j][k]: rows j, j + 1 read together, one 4-byte store per k
#pragma unroll
        for (int m = 0; m < (NG8 + NT - 1) / NT; ++m) {
            const int e = tid + NT * m;
            if (e < NG8) {
                const int jp = e / (W / 4), k = (e - jp * (W / 4)) * 4, j = 2 * jp;
                const float4 r0 = ld4(Wl + (long)j * W + k), r1 = ld4(Wl + (long)(j + 1) * W + k);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x2 b;
                    b[0] = (__bf16)comp(r0, q);
                    b[1] = (__bf16)comp(r1, q);
                    *reinterpret_cast<bf16x2*>(&Wsh[(k + q) * LDA + j]) = b;
                }
            }
        }
        f32x16 gacc[NBW];
#pragma unroll
        for (int b = 0; b < NBW; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) gacc[b][v] = 0.f;
        // staging: thread (unit u = tid % W, row group rq = tid / W) takes
        // rows 4 (rq + NQ c) .. + 3; its transposed copies of four rows are
        // one 8-byte store per stream
        constexpr int NQ = NT / W, CH = 32 / (4 * NQ);
        const int u = tid % W, rq = tid / W;
        const float wou = wo[u];
        float db = 0.f;
        for (int t = t0; t < t1; ++t) {
            const long i0 = (long)t * 32;
            if (t > t0) __syncthreads();  // the previous tile's products are done
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int ib = 4 * (rq + NQ * c);
                float zq[4][4], aq[4][4];  // [stream][row]
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = ib + e;
                    const long idx = (i0 + i) * W + u;
                    float A[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        A[s] = l == d ? gout[s * n_pad + i0 + i] * wou : abar[s * plane + idx];
                    float zb[4];
                    tanh_adjoint(A[0], A[1], A[2], A[3], cl[idx], cl[plane + idx],
                                 cl[2 * plane + idx], cl[3 * plane + idx], zb[0], zb[1], zb[2],
                                 zb[3]);
                    streams_of_values(cp[idx], cp[plane + idx], cp[2 * plane + idx],
                                      cp[3 * plane + idx], aq[0][e], aq[1][e], aq[2][e], aq[3][e]);
                    db += zb[0];
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        zq[s][e] = zb[s];
                        Xs[s][i * LDA + u] = (__bf16)zb[s];
                    }
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    st_bf16x4(&ZT[s][u * LDT + ib], zq[s]);
                    st_bf16x4(&aT[s][u * LDT + ib], aq[s]);
                }
            }
            __syncthreads();
            // adjoints of the streams entering layer l: abar_s[i][k] = sum_j zbar_s[i][j] W[j][k]
            for (int cb = wave; cb < NCB; cb += 4) {
                f32x16 acc[4];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[s][v] = 0.f;
#pragma unroll
                for (int k = 0; k < W / 16; ++k) {
                    const bf16x8 b = lds_frag(&Wsh[(cb * 32 + r32) * LDA + 16 * k + 8 * h]);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[s] = mfma32x32x16(lds_frag(&Xs[s][r32 * LDA + 16 * k + 8 * h]), b,
                                              acc[s]);
                }
                const int kk = cb * 32 + r32;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const long idx = (i0 + mfma_row(v, lane)) * W + kk;
#pragma unroll
                    for (int s = 0; s < 4; ++s) abar[s * plane + idx] = acc[s][v];
                }
            }
            // dW[j][k] += sum_s sum_i zbar_s[i][j] a_prev_s[i][k]
#pragma unroll
            for (int b = 0; b < NBW; ++b) {
                const int blk = wave + 4 * b;
                if (blk < NCB * NCB) {
                    const int jb = blk / NCB, kb = blk - jb * NCB;
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int k = 0; k < 2; ++k)
                            gacc[b] = mfma32x32x16(
                                lds_frag(&ZT[s][(jb * 32 + r32) * LDT + 16 * k + 8 * h]),
                                lds_frag(&aT[s][(kb * 32 + r32) * LDT + 16 * k + 8 * h]), gacc[b]);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
            const int blk = wave + 4 * b;
            if (blk < NCB * NCB) {
                const int jb = blk / NCB, kb = blk - jb * NCB;
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    out[L.offW[l] + (long)(jb * 32 + mfma_row(v, lane)) * W + kb * 32 + r32] =
                        gacc[b][v];
            }
        }
        combine1(db, out + L.offb[l]);
    }

    // ---- first layer: dW1[j][c] = sum_i zb_ij x_ic (+ zb_t for c = 0, + zb_x
    // for c = 1), db1[j] = sum_i zb_ij, over the points i < n
    {
        const BSP_GLOBAL float* c1 = cache(1);
        float gw[4][4], gb1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) gw[c][q] = 0.f;
        __syncthreads();  // the data adjoints of the last layer are written
        for (int t = t0; t < t1; ++t)
#pragma unroll
            for (int p = 0; p < PASSES; ++p) {
                const long i = (long)t * 32 + rr + RP * p;
                if (i >= n) continue;
                const long idx = i * W + u0;
                float A[4][4];
                if (d == 1) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float gs = gout[s * n_pad + i];
#pragma unroll
                        for (int q = 0; q < 4; ++q) A[s][q] = gs * wo[u0 + q];
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float4 ab = ld4(abar + s * plane + idx);
#pragma unroll
                        for (int q = 0; q < 4; ++q) A[s][q] = comp(ab, q);
                    }
                }
                const float4 c0 = ld4(c1 + idx), cz1 = ld4(c1 + plane + idx),
                             c2 = ld4(c1 + 2 * plane + idx), c3 = ld4(c1 + 3 * plane + idx);
                const float* xr = point_row(a.P, i);
                float x[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) x[c] = c < n_in ? xr[c] : 0.f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float zb, zb_t, zb_x, zb_xx;
                    tanh_adjoint(A[0][q], A[1][q], A[2][q], A[3][q], comp(c0, q), comp(cz1, q),
                                 comp(c2, q), comp(c3, q), zb, zb_t, zb_x, zb_xx);
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (c < n_in) {
                            float tq = zb * x[c];
                            if (c == 0) tq += zb_t;
                            if (c == 1) tq += zb_x;
                            gw[c][q] += tq;
                        }
                    gb1[q] += zb;
                }
            }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < n_in) combine(gw[c], out + L.offW[1] + c, n_in);
        combine(gb1, out + L.offb[1], 1);
    }
}

// grad[x] = sum over blocks b of part[b][x] for x < total, and loss3[t] =
// (sum over blocks of part[b][total + t]) / (points of type t).  A block
// takes 32 consecutive x; its 8 row groups sum the partials b = g, g + 8, ...
// (four running sums each, so the loads overlap), then the groups are added
// in order: a fixed summation order, independent of timing.
__global__ __launch_bounds__(256) void k_res_reduce_step(const float* __restrict__ part, int nblk,
                                                         long ldp, long total, int nf, int ne,
                                                         int nb, float* __restrict__ grad,
                                                         float* __restrict__ loss3) {
    __shared__ float acc[8][33];
    const int tx = threadIdx.x & 31, g = threadIdx.x >> 5;
    const long x = (long)blockIdx.x * 32 + tx, count = total + 3;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (x < count) {
        int b = g;
        for (; b + 24 < nblk; b += 32) {
            s0 += part[(long)b * ldp + x];
            s1 += part[(long)(b + 8) * ldp + x];
            s2 += part[(long)(b + 16) * ldp + x];
            s3 += part[(long)(b + 24) * ldp + x];
        }
        for (; b < nblk; b += 8) s0 += part[(long)b * ldp + x];
    }
    acc[g][tx] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (g == 0 && x < count) {
        float s = acc[0][tx];
#pragma unroll
        for (int r = 1; r < 8; ++r) s += acc[r][tx];
        if (x < total) {
            grad[x] = s;
        } else {
            const int t = (int)(x - total);
            const int cnt = t == 0 ? nf : t == 1 ? ne : nb;
            loss3[t] = cnt > 0 ? s / (float)cnt : 0.f;
        }
    }
}

// grad[x] = sum over blocks b of part[b][x], x < count (row stride count),
// in the same fixed order; used by the float32 pass.
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

// Variant for networks of 2 to 4 layers.  A block of W/32 wavefronts takes
// its tiles one after the other; wavefront w owns units 32 w .. 32 w + 31 of
// every layer, and each lane holds the cache (a, z_t, z_x, z_xx) of its unit
// for the 16 rows of its matrix-core output fragment.  The backward product
// W^T zbar returns its result in that same fragment layout, so the adjoints
// meet the cache lane by lane: each lane writes its fragment of every
// layer's cache to the workspace as it is made (four 16-byte stores per
// stream, in the lane's own order) and reads it back one layer ahead of its
// use in the backward pass.  The weights come from bfloat16 copies
// (row-major and transposed, k_res_wbf16).  LDS holds the bfloat16 operands
// of the products: the input streams or zbar [i][j], zbar [j][i] and the
// previous layer's streams [k][i]; the head's float32 streams reuse the
// space of the latter two.
template <int W, int D>
__global__ __launch_bounds__(2 * W) void k_res_tile_bf16(ResStepArgs a,
                                                        const __bf16* __restrict__ wf,
                                                        const __bf16* __restrict__ wt) {
    constexpr int NW = W / 32, NT = 64 * NW;
    constexpr int LDA = W + 8, LDT = 32 + 8, LDH = W + 1;
    constexpr int KT = W / 16;  // K-steps of a hidden-layer product
    constexpr int ZT_ELEMS = 4 * W * LDT;
    constexpr int BIG = 2 * ZT_ELEMS * 2 > 4 * 32 * LDH * 4 ? 2 * ZT_ELEMS * 2 : 4 * 32 * LDH * 4;
    constexpr long SLOT = 4 * 32 * W;  // floats of one layer's cache of one tile
    __shared__ __align__(16) __bf16 Xs[4][32 * LDA];
    __shared__ __align__(16) unsigned char big[BIG];
    __shared__ float gsh[4][32];
    __shared__ float lsh[32];
    __shared__ float xsh[32][5];  // the tile's inputs and value targets
    __shared__ float wosh[W];     // output-layer weights
    __bf16* ZT = reinterpret_cast<__bf16*>(big);             // [4][W][LDT]
    __bf16* aT = ZT + ZT_ELEMS;                               // [4][W][LDT]
    float* hs = reinterpret_cast<float*>(big);                // [4][32][LDH]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r32 = lane & 31, h = lane >> 5;
    const int j = 32 * w + r32;  // this lane's unit in every layer
    const NetLayout& L = a.L;
    const int n_in = L.n_in;
    const long n = a.n;
    const int t0 = blockIdx.x * a.tiles_per_block;
    const int t1 = min(t0 + a.tiles_per_block, a.ntiles);
    const BSP_GLOBAL float* prm = gmem(a.prm);
    BSP_GLOBAL float* out = gmem(a.part) + (long)blockIdx.x * a.ldp;

    float w1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w1[c] = c < n_in ? prm[L.offW[1] + (long)j * n_in + c] : 0.f;
    const float b1 = prm[L.offb[1] + j], wo_j = prm[L.off_wo + j];
    for (int u = tid; u < W; u += NT) wosh[u] = prm[L.off_wo + u];
    float bl[D + 1];
#pragma unroll
    for (int l = 2; l <= D; ++l) bl[l] = prm[L.offb[l] + j];

    // per-lane sums over the block's rows (the lane pair h = 0, 1 is added at the end)
    float gW1[4] = {0.f, 0.f, 0.f, 0.f}, gb1 = 0.f, gwo = 0.f, gbl[D + 1];
#pragma unroll
    for (int l = 0; l <= D; ++l) gbl[l] = 0.f;
    float lsum[3] = {0.f, 0.f, 0.f}, dbo = 0.f;  // thread 0

    for (int t = t0; t < t1; ++t) {
        const long i0 = (long)t * 32;
        // this lane's fragment of layer l's cache: stream s, rows 4 m .. 4 m + 3 of
        // the fragment at frag(l) + (4 s + m) * 256
        BSP_GLOBAL float* const tile_cache =
            gmem(a.cache) + (long)t * D * SLOT + w * (SLOT / NW) + 4 * lane;
        auto frag = [&](int l) { return tile_cache + (long)(l - 1) * SLOT; };
        // the tile's inputs (and targets) into LDS: one load per value, not a
        // dependent load per row and lane
        __syncthreads();  // the previous tile's first-layer gradient is done with xsh
        if (tid < 32) {
            const long i = i0 + tid;
            float xv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            if (i < n) {
                const float* xr = point_row(a.P, i);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < n_in) xv[c] = xr[c];
                xv[4] = point_target(a.P, i);
            }
#pragma unroll
            for (int c = 0; c < 5; ++c) xsh[tid][c] = xv[c];
        }
        __syncthreads();
        // ---- first layer (vector units): z = W1 x + b1, z_t = W1[:,0], z_x = W1[:,1]
        f32x16 a1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int il = mfma_row(v, lane);
            const long i = i0 + il;
            // (w1[c] and the staged x are zero for c >= n_in: the terms add exact zeros)
            float z = b1;
#pragma unroll
            for (int c = 0; c < 4; ++c) z = fmaf(w1[c], xsh[il][c], z);
            const bool live = i < n;
            const float av = live ? tanh_f32(z) : 0.f, zt = live ? w1[0] : 0.f,
                        zx = live ? w1[1] : 0.f;
            a1[v] = av;
            float s0, s1, s2, s3;
            streams_of_values(av, zt, zx, 0.f, s0, s1, s2, s3);
            Xs[0][il * LDA + j] = (__bf16)s0;
            Xs[1][il * LDA + j] = (__bf16)s1;
            Xs[2][il * LDA + j] = (__bf16)s2;
            Xs[3][il * LDA + j] = (__bf16)s3;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            st4(frag(1) + m * 256, a1[4 * m], a1[4 * m + 1], a1[4 * m + 2], a1[4 * m + 3]);
        __syncthreads();
        // ---- hidden layers: z_s = W a_s (+ b for the value)
        f32x16 c0, c1, c2, c3;  // the cache of the layer just made
#pragma unroll
        for (int l = 2; l <= D; ++l) {
            // (an opaque base: the fragments are the same for every tile, and
            // loads hoisted out of the tile loop would hold registers for good)
            const __bf16* wl = wf + (size_t)(l - 2) * W * W;
            asm volatile("" : "+s"(wl));
            const BSP_GLOBAL __bf16* wrow = gmem(wl) + (size_t)j * W + 8 * h;
            bf16x8 bf[KT];
#pragma unroll
            for (int k = 0; k < KT; ++k)
                bf[k] = *reinterpret_cast<const BSP_GLOBAL bf16x8*>(wrow + 16 * k);
            f32x16 acc[4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[s][v] = 0.f;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                __builtin_amdgcn_sched_barrier(0);  // bound the loads hoisted ahead
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc[s] = mfma32x32x16(lds_frag(&Xs[s][r32 * LDA + 16 * k + 8 * h]), bf[k],
                                          acc[s]);
            }
            __syncthreads();  // every wavefront is done reading Xs
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                c0[v] = tanh_f32(acc[0][v] + bl[l]);
                c1[v] = acc[1][v];
                c2[v] = acc[2][v];
                c3[v] = acc[3][v];
            }
            BSP_GLOBAL float* fl = frag(l);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                st4(fl + m * 256, c0[4 * m], c0[4 * m + 1], c0[4 * m + 2], c0[4 * m + 3]);
                st4(fl + (4 + m) * 256, c1[4 * m], c1[4 * m + 1], c1[4 * m + 2], c1[4 * m + 3]);
                st4(fl + (8 + m) * 256, c2[4 * m], c2[4 * m + 1], c2[4 * m + 2], c2[4 * m + 3]);
                st4(fl + (12 + m) * 256, c3[4 * m], c3[4 * m + 1], c3[4 * m + 2], c3[4 * m + 3]);
            }
            if (l < D) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int il = mfma_row(v, lane);
                    float s0, s1, s2, s3;
                    streams_of_values(c0[v], c1[v], c2[v], c3[v], s0, s1, s2, s3);
                    Xs[0][il * LDA + j] = (__bf16)s0;
                    Xs[1][il * LDA + j] = (__bf16)s1;
                    Xs[2][il * LDA + j] = (__bf16)s2;
                    Xs[3][il * LDA + j] = (__bf16)s3;
                }
                __syncthreads();
            }
        }
        // ---- head: the last layer's streams (float32) through LDS, eight lanes per point
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int il = mfma_row(v, lane);
            float s0, s1, s2, s3;
            streams_of_values(c0[v], c1[v], c2[v], c3[v], s0, s1, s2, s3);
            hs[(0 * 32 + il) * LDH + j] = s0;
            hs[(1 * 32 + il) * LDH + j] = s1;
            hs[(2 * 32 + il) * LDH + j] = s2;
            hs[(3 * 32 + il) * LDH + j] = s3;
        }
        __syncthreads();
        for (int p0 = 0; p0 < 32; p0 += NT / 8) {
            const int u = tid & 7, pt = p0 + (tid >> 3);
            const long i = i0 + pt;
            // (padded rows hold finite values; their head is not evaluated)
            float v = 0.f, vt = 0.f, vx = 0.f, vxx = 0.f;
#pragma unroll
            for (int jj = 0; jj < W / 8; ++jj) {
                const int jx = u + 8 * jj;
                const float wj = wosh[jx];
                v = fmaf(wj, hs[(0 * 32 + pt) * LDH + jx], v);
                vt = fmaf(wj, hs[(1 * 32 + pt) * LDH + jx], vt);
                vx = fmaf(wj, hs[(2 * 32 + pt) * LDH + jx], vx);
                vxx = fmaf(wj, hs[(3 * 32 + pt) * LDH + jx], vxx);
            }
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                v += __shfl_xor(v, o, 8);
                vt += __shfl_xor(vt, o, 8);
                vx += __shfl_xor(vx, o, 8);
                vxx += __shfl_xor(vxx, o, 8);
            }
            if (u == 0) {
                float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, lc = 0.f;
                if (i < n)
                    head_point_x(a.P, i, xsh[pt], xsh[pt][4], v + prm[L.off_bo], vt, vx, vxx, g0,
                                 g1, g2, g3, lc);
                gsh[0][pt] = g0;
                gsh[1][pt] = g1;
                gsh[2][pt] = g2;
                gsh[3][pt] = g3;
                lsh[pt] = lc;
            }
        }
        __syncthreads();  // gsh and lsh complete; hs no longer read
        if (tid == 0) {
            // the tile's loss terms by point type and sum of g0, in point order
            // (padded points hold zeros)
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                const long iq = i0 + q;
                const float lc = lsh[q];
                lsum[0] += iq < a.P.nf ? lc : 0.f;
                lsum[1] += iq >= a.P.nf && iq < a.P.nf + a.P.ne ? lc : 0.f;
                lsum[2] += iq >= a.P.nf + a.P.ne ? lc : 0.f;
                dbo += gsh[0][q];
            }
        }
        // output-layer gradient and the adjoints of the last layer's streams
        f32x16 Ab[4];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int il = mfma_row(v, lane);
            float s0, s1, s2, s3;
            streams_of_values(c0[v], c1[v], c2[v], c3[v], s0, s1, s2, s3);
            float tq = gsh[0][il] * s0;
            tq = fmaf(gsh[1][il], s1, tq);
            tq = fmaf(gsh[2][il], s2, tq);
            tq = fmaf(gsh[3][il], s3, tq);
            gwo += tq;
#pragma unroll
            for (int s = 0; s < 4; ++s) Ab[s][v] = gsh[s][il] * wo_j;
        }
        // ---- backward through the hidden layers; (c0..c3) holds layer l's cache
#pragma unroll
        for (int l = D; l >= 2; --l) {
            // the previous layer's cache, read ahead of its use
            f32x16 p0, p1, p2, p3;
            const BSP_GLOBAL float* fp = frag(l - 1);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float4 q0 = ld4(fp + m * 256);
                p0[4 * m] = q0.x; p0[4 * m + 1] = q0.y; p0[4 * m + 2] = q0.z; p0[4 * m + 3] = q0.w;
                if (l - 1 >= 2) {
                    const float4 q1 = ld4(fp + (4 + m) * 256), q2 = ld4(fp + (8 + m) * 256),
                                 q3 = ld4(fp + (12 + m) * 256);
                    p1[4 * m] = q1.x; p1[4 * m + 1] = q1.y; p1[4 * m + 2] = q1.z; p1[4 * m + 3] = q1.w;
                    p2[4 * m] = q2.x; p2[4 * m + 1] = q2.y; p2[4 * m + 2] = q2.z; p2[4 * m + 3] = q2.w;
                    p3[4 * m] = q3.x; p3[4 * m + 1] = q3.y; p3[4 * m + 2] = q3.z; p3[4 * m + 3] = q3.w;
                }
            }
            if (l - 1 == 1) {  // layer 1: z_t, z_x from W1 (zero on padded rows), z_xx = 0
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const bool live = i0 + mfma_row(v, lane) < n;
                    p1[v] = live ? w1[0] : 0.f;
                    p2[v] = live ? w1[1] : 0.f;
                    p3[v] = 0.f;
                }
            }
            // zbar and the previous layer's streams, four rows (one fragment
            // group) at a time: [i][j] and [j][i] copies of zbar, [k][i] of
            // the streams (k = j, this lane's unit in layer l - 1)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                float zq[4][4], ap[4][4];  // [stream][row]
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int v = 4 * m + e;
                    tanh_adjoint(Ab[0][v], Ab[1][v], Ab[2][v], Ab[3][v], c0[v], c1[v], c2[v],
                                 c3[v], zq[0][e], zq[1][e], zq[2][e], zq[3][e]);
                    gbl[l] += zq[0][e];
                    const int il = mfma_row(v, lane);
#pragma unroll
                    for (int s = 0; s < 4; ++s) Xs[s][il * LDA + j] = (__bf16)zq[s][e];
                    streams_of_values(p0[v], p1[v], p2[v], p3[v], ap[0][e], ap[1][e], ap[2][e],
                                      ap[3][e]);
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    st_bf16x4(&ZT[(s * W + j) * LDT + 8 * m + 4 * h], zq[s]);
                    st_bf16x4(&aT[(s * W + j) * LDT + 8 * m + 4 * h], ap[s]);
                }
            }
            __syncthreads();
            // adjoints of the streams entering layer l: abar_s[i][k] = sum_j zbar_s[i][j] W[j][k]
            const __bf16* tl = wt + (size_t)(l - 2) * W * W;
            asm volatile("" : "+s"(tl));
            const BSP_GLOBAL __bf16* trow = gmem(tl) + (size_t)j * W + 8 * h;
            bf16x8 bt[KT];
#pragma unroll
            for (int k = 0; k < KT; ++k)
                bt[k] = *reinterpret_cast<const BSP_GLOBAL bf16x8*>(trow + 16 * k);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int v = 0; v < 16; ++v) Ab[s][v] = 0.f;
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    Ab[s] = mfma32x32x16(lds_frag(&Xs[s][r32 * LDA + 16 * k + 8 * h]), bt[k], Ab[s]);
            }
            // weight gradient, rows 32 w .. 32 w + 31: dW[j'][k'] += sum_s sum_i zbar_s[i][j'] a_s[i][k']
            float* olg = (float*)(out + L.offW[l]);
            asm volatile("" : "+s"(olg));  // addresses made here, not held across tiles
            BSP_GLOBAL float* ol = gmem(olg);
#pragma unroll
            for (int kb = 0; kb < NW; ++kb) {
                __builtin_amdgcn_sched_barrier(0);
                BSP_GLOBAL float* o = ol + (long)(32 * w + 4 * h) * W + 32 * kb + r32;
                // a later tile adds to the block's partial: its 16 loads go out
                // together, ahead of the products, not one behind each store
                f32x16 gacc;
                if (t == t0) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) gacc[v] = 0.f;
                } else {
#pragma unroll
                    for (int v = 0; v < 16; ++v) gacc[v] = o[(8 * (v >> 2) + (v & 3)) * W];
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int k = 0; k < 2; ++k)
                        gacc = mfma32x32x16(lds_frag(&ZT[(s * W + j) * LDT + 16 * k + 8 * h]),
                                            lds_frag(&aT[(s * W + 32 * kb + r32) * LDT + 16 * k + 8 * h]),
                                            gacc);
#pragma unroll
                for (int v = 0; v < 16; ++v) o[(8 * (v >> 2) + (v & 3)) * W] = gacc[v];
            }
            __syncthreads();  // every wavefront is done with Xs, ZT and aT
            c0 = p0;
            c1 = p1;
            c2 = p2;
            c3 = p3;
        }
        // ---- first layer: dW1[j][c] += zb x_c (+ zb_t for c = 0, + zb_x for c = 1), db1[j] += zb
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            // padded rows have zero adjoints and zero inputs: their terms are exact zeros
            const int il = mfma_row(v, lane);
            const bool live = i0 + il < n;
            float zb, zb_t, zb_x, zb_xx;
            tanh_adjoint(Ab[0][v], Ab[1][v], Ab[2][v], Ab[3][v], c0[v], live ? w1[0] : 0.f,
                         live ? w1[1] : 0.f, 0.f, zb, zb_t, zb_x, zb_xx);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                float tq = zb * xsh[il][c];
                if (c == 0) tq += zb_t;
                if (c == 1) tq += zb_x;
                gW1[c] += tq;
            }
            gb1 += zb;
        }
    }
    // the lane pair h = 0, 1 holds the two halves of each unit's rows
#pragma unroll
    for (int c = 0; c < 4; ++c) gW1[c] += __shfl_xor(gW1[c], 32);
    gb1 += __shfl_xor(gb1, 32);
    gwo += __shfl_xor(gwo, 32);
#pragma unroll
    for (int l = 2; l <= D; ++l) gbl[l] += __shfl_xor(gbl[l], 32);
    if (h == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < n_in) out[L.offW[1] + (long)j * n_in + c] = gW1[c];
        out[L.offb[1] + j] = gb1;
        out[L.off_wo + j] = gwo;
#pragma unroll
        for (int l = 2; l <= D; ++l) out[L.offb[l] + j] = gbl[l];
    }
    if (tid == 0) {
        out[L.off_bo] = dbo;
        out[L.total] = lsum[0];
        out[L.total + 1] = lsum[1];
        out[L.total + 2] = lsum[2];
    }
}

// The hidden layers' weights as bfloat16, row-major (wf) and transposed (wt),
// layer l at (l - 2) W^2.
__global__ void k_res_wbf16(const float* __restrict__ prm, NetLayout L, __bf16* __restrict__ wf,
                            __bf16* __restrict__ wt) {
    const long W = L.W, per = W * W, total = (long)(L.depth - 1) * per;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int l = 2 + (int)(e / per);
        const long r = e - (long)(l - 2) * per, jr = r / W, kc = r - jr * W;
        const float v = prm[L.offW[l] + r];
        wf[e] = (__bf16)v;
        wt[(long)(l - 2) * per + kc * W + jr] = (__bf16)v;
    }
}

// Blocks of the fused step for n_pad points: at least kResStepMinTiles
// tiles per block, at most max_blocks blocks.
int res_step_blocks(long n_pad, int max_blocks, int* tiles_per_block) {
    const long ntiles = n_pad / 32;
    long tpb = (ntiles + max_blocks - 1) / max_blocks;
    if (tpb < kResStepMinTiles) tpb = kResStepMinTiles;
    *tiles_per_block = (int)tpb;
    return (int)((ntiles + tpb - 1) / tpb);
}

int launch_res_step_bf16(const pinn_net& net, const Points& P, long n, long n_pad, float* cache,
                         float* abar, float* g, __bf16* wbf, float* part, long ldp, int max_blocks,
                         float* grad, float* loss3, hipStream_t st) {
    ResStepArgs a{};
    a.prm = net.params;
    a.P = P;
    a.L = net_layout(net);
    a.n = n;
    a.n_pad = n_pad;
    a.ntiles = (int)(n_pad / 32);
    const int nblk = res_step_blocks(n_pad, max_blocks, &a.tiles_per_block);
    a.cache = cache;
    a.abar = abar;
    a.g = g;
    a.part = part;
    a.ldp = ldp;
    if (net.width != 32 && net.width != 64 && net.width != 128) {
        set_error("bfloat16 residual path: width %d not supported (32, 64, 128)", net.width);
        return BS_ERR_ARG;
    }
    if (nblk > 0 && net.depth >= 2 && net.depth <= 4) {
        // caches in registers: the bfloat16 weight copies, then one launch
        const long per = (long)net.width * net.width;
        __bf16* wf = wbf;
        __bf16* wt = wbf + (net.depth - 1) * per;
        const long total = (net.depth - 1) * per;
        hipLaunchKernelGGL(k_res_wbf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           net.params, a.L, wf, wt);
        BSP_LAUNCHED();
        const int key = net.width * 8 + net.depth;
        switch (key) {
#define BSP_WD(W_, D_)                                                                        \
    case W_ * 8 + D_:                                                                         \
        hipLaunchKernelGGL((k_res_tile_bf16<W_, D_>), dim3(nblk), dim3(2 * W_), 0, st, a, wf, wt); \
        break;
            BSP_WD(32, 2) BSP_WD(32, 3) BSP_WD(32, 4) BSP_WD(64, 2) BSP_WD(64, 3) BSP_WD(64, 4)
            BSP_WD(128, 2) BSP_WD(128, 3) BSP_WD(128, 4)
#undef BSP_WD
        }
        BSP_LAUNCHED();
    } else if (nblk > 0) {
        switch (net.width) {
#define BSP_W(W_)                                                                             \
    case W_:                                                                                  \
        hipLaunchKernelGGL(k_res_step_bf16<W_>, dim3(nblk), dim3(kResStepThreads), 0, st, a); \
        break;
            BSP_W(32) BSP_W(64) BSP_W(128)
#undef BSP_W
        }
        BSP_LAUNCHED();
    }
    const long count = a.L.total + 3;
    hipLaunchKernelGGL(k_res_reduce_step, dim3((unsigned)((count + 31) / 32)), dim3(256), 0, st,
                       part, nblk, ldp, a.L.total, P.nf, P.ne, P.nb, grad, loss3);
    BSP_LAUNCHED();
    return BS_OK;
}

}  // namespace bsp
