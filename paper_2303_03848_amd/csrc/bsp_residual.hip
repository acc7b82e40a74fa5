// PINN loss and its gradient (eqs. (11)-(14)) with the input derivatives the
// residual of eq. (1) needs, differentiated by hand.
//
// Forward: every point carries four streams through the network,
//   value a, d/dtau a_t, d/dx a_x, d2/dx2 a_xx.
// For z = W a_prev + b (z_t = W a_prev_t, ...) and a = tanh(z), s = 1 - a^2:
//   a_t = s z_t,  a_x = s z_x,  a_xx = s z_xx - 2 a s z_x^2.
// Per layer the cache keeps (a, z_t, z_x, z_xx) for every (point, unit); the
// input streams of the next layer are recomputed from it.
//
// Head: v_* = wo . a_* (+ bo for the value); residual
//   f = v_t - sigma^2 x^2 v_xx / 2 - r x v_x + r v      (x = S/K, v = V/K),
// terminal and boundary mismatches; the output adjoints g_* of (v, v_t, v_x,
// v_xx) are (r, 1, -r x, -sigma^2 x^2 / 2) * 2 f / n_f at interior points and
// (1, 0, 0, 0) * 2 (v - y) / n at terminal / boundary points.
//
// Backward through a = tanh(z), given the adjoints (A, At, Ax, Axx) of
// (a, a_t, a_x, a_xx):
//   zb_t  = s At,  zb_x = s Ax - 4 a s z_x Axx,  zb_xx = s Axx,
//   zb    = s [A - 2 a (z_t At + z_x Ax + z_xx Axx) - 2 z_x^2 (1 - 3 a^2) Axx];
// through the linear layer: dW += sum_s zb_s a_prev_s^T, db += sum zb, and the
// adjoints of the previous streams are W^T zb_s.  In the first layer
// z_t = W[:,0], z_x = W[:,1], so dW[:,0] += sum zb_t, dW[:,1] += sum zb_x.
//
// Buffers (workspace, float32, stream-major [4][n_pad][W]): cache per layer,
// zbar, abar; g [4][n_pad]; per-point loss terms [n_pad].
// Every reduction over points is a fixed-order loop or tree: results are
// bitwise reproducible.
#include <cmath>

#include "bsp_residual.hpp"

namespace bsp {

// ------------------------------------------------------------------ layout

struct ResWs {
    long n_pad;
    float* cache;   // depth * 4 * n_pad * W
    float* zbar;    // 4 * n_pad * W
    float* abar;    // 4 * n_pad * W
    float* g;       // 4 * n_pad
    float* lossc;   // n_pad
    float* part;    // partial gradients: kPartRows rows of total + 3 floats
    __bf16* wbf;    // hidden-layer weights in bfloat16, row-major then transposed
    size_t bytes;
};

constexpr int kResPartBlocks = 256;
constexpr int kPartRows = 256;  // partial rows in the workspace: max over the split kernels

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

static ResWs res_layout(const pinn_net& n, long npts, void* base) {
    ResWs w{};
    w.n_pad = (npts + 31) / 32 * 32;
    const size_t plane = (size_t)4 * w.n_pad * n.width * sizeof(float);
    char* p = (char*)base;
    size_t off = 0;
    auto take = [&](size_t b) {
        char* q = p ? p + off : nullptr;
        off += a256(b);
        return q;
    };
    w.cache = (float*)take(plane * n.depth);
    w.zbar = (float*)take(plane);
    w.abar = (float*)take(plane);
    w.g = (float*)take(sizeof(float) * 4 * w.n_pad);
    w.lossc = (float*)take(sizeof(float) * w.n_pad);
    w.part = (float*)take(sizeof(float) * (size_t)kPartRows * (net_layout(n).total + 3));
    w.wbf = (__bf16*)take(sizeof(__bf16) * 2 * (size_t)(n.depth - 1) * n.width * n.width);
    w.bytes = off;
    return w;
}

// --------------------------------------------------------- forward kernels

// First layer: z = W1 x + b1, z_t = W1[:,0], z_x = W1[:,1], z_xx = 0.
__global__ void k_res_first(const float* __restrict__ prm, Points P, long n, long n_pad, int W,
                            float* __restrict__ cache) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_pad * W) return;
    const long i = t / W;
    const int j = (int)(t - i * W);
    const long plane = n_pad * W;
    float a = 0.f, zt = 0.f, zx = 0.f;
    if (i < n) {
        const float* x = point_row(P, i);
        const float* w = prm + (long)j * P.n_in;
        float z = prm[(long)W * P.n_in + j];
        for (int c = 0; c < P.n_in; ++c) z = fmaf(w[c], x[c], z);
        a = tanh_f32(z);
        zt = w[0];
        zx = w[1];
    }
    cache[t] = a;
    cache[plane + t] = zt;
    cache[2 * plane + t] = zx;
    cache[3 * plane + t] = 0.f;
}

// Layer epilogue: given z (with bias) and the three derivative streams,
// write the cache entry (a, z_t, z_x, z_xx).
__device__ __forceinline__ void tanh_epilogue(float z, float zt, float zx, float zxx, float* c,
                                              long plane, long idx) {
    c[idx] = tanh_f32(z);
    c[plane + idx] = zt;
    c[2 * plane + idx] = zx;
    c[3 * plane + idx] = zxx;
}

// Hidden-layer products of the FP32 residual pass, tiled: 32 points per
// block; the layer's weights and the points' four input streams go through
// LDS in K-chunks of up to 32; thread (tp, tu) of a 16 x 16 grid holds points
// tp, tp + 16 and units tu + 16 b (b < W/16) for the four streams.  Sums run
// over K in ascending order (bias first), as a plain per-output loop would.
//   MODE 0 (forward): z_s[i][j] = b_j [s = 0] + sum_k W[j][k] a_s[i][k], with
//                     a_s rebuilt from the cache of the layer below, then the
//                     tanh derivative streams into the next cache.
//   MODE 1 (adjoint): abar_s[i][k] = sum_j W[j][k] zbar_s[i][j].
template <int W, int MODE>
__global__ __launch_bounds__(256) void k_res_gemm_f32(const float* __restrict__ Wl,
                                                      const float* __restrict__ bl,
                                                      const float* __restrict__ in,
                                                      float* __restrict__ out, long n_pad) {
    constexpr int KC = W < 32 ? W : 32;
    constexpr int UB = W / 16;  // units per thread
    __shared__ float bs[KC][W + 1];     // B[k][u]: MODE 0 W[u][k], MODE 1 W[k][u]
    __shared__ float xs[4][32][KC + 1];  // inputs [stream][point][k]
    const int tid = threadIdx.x, tp = tid >> 4, tu = tid & 15;
    const long i0 = (long)blockIdx.x * 32;
    const long plane = n_pad * W;
    float acc[4][2][UB];
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < UB; ++b)
                acc[st][a][b] = (MODE == 0 && st == 0) ? bl[tu + 16 * b] : 0.f;
    for (int k0 = 0; k0 < W; k0 += KC) {
        __syncthreads();
        for (int e = tid; e < KC * W; e += 256) {
            if (MODE == 0) {  // row u of W, columns k0 .. k0 + KC
                const int u = e / KC, kk = e - u * KC;
                bs[kk][u] = Wl[(long)u * W + k0 + kk];
            } else {  // rows k0 .. k0 + KC of W
                const int kk = e / W, u = e - kk * W;
                bs[kk][u] = Wl[(long)(k0 + kk) * W + u];
            }
        }
        for (int e = tid; e < 32 * KC; e += 256) {
            const int c = e / KC, kk = e - c * KC;
            const long idx = (i0 + c) * W + k0 + kk;
            if (MODE == 0) {
                float a, at, ax, axx;
                streams_from_cache(in, plane, idx, a, at, ax, axx);
                xs[0][c][kk] = a;
                xs[1][c][kk] = at;
                xs[2][c][kk] = ax;
                xs[3][c][kk] = axx;
            } else {
#pragma unroll
                for (int st = 0; st < 4; ++st) xs[st][c][kk] = in[st * plane + idx];
            }
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KC; ++kk) {
            float x[4][2], wv[UB];
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int a = 0; a < 2; ++a) x[st][a] = xs[st][tp + 16 * a][kk];
#pragma unroll
            for (int b = 0; b < UB; ++b) wv[b] = bs[kk][tu + 16 * b];
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < UB; ++b)
                        acc[st][a][b] = fmaf(wv[b], x[st][a], acc[st][a][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < UB; ++b) {
            const long idx = (i0 + tp + 16 * a) * W + tu + 16 * b;
            if (MODE == 0) {
                tanh_epilogue(acc[0][a][b], acc[1][a][b], acc[2][a][b], acc[3][a][b], out, plane,
                              idx);
            } else {
#pragma unroll
                for (int st = 0; st < 4; ++st) out[st * plane + idx] = acc[st][a][b];
            }
        }
}

template <int MODE>
static int launch_res_gemm_f32(const float* Wl, const float* bl, const float* in, float* out,
                               long n_pad, int W, hipStream_t st) {
    const dim3 grid((unsigned)(n_pad / 32));
    switch (W) {
#define BSP_W(W_)                                                                              \
    case W_:                                                                                   \
        hipLaunchKernelGGL((k_res_gemm_f32<W_, MODE>), grid, dim3(256), 0, st, Wl, bl, in, out, \
                           n_pad);                                                             \
        break;
        BSP_W(16) BSP_W(32) BSP_W(64) BSP_W(128) BSP_W(256)
#undef BSP_W
        default:
            set_error("unsupported width %d", W);
            return BS_ERR_ARG;
    }
    BSP_LAUNCHED();
    return BS_OK;
}

// Output layer, loss terms and output adjoints (one thread per point).
__global__ void k_res_head(const float* __restrict__ prm, long off_wo, long off_bo, Points P,
                           long n, long n_pad, int W, const float* __restrict__ clast,
                           float* __restrict__ g, float* __restrict__ lossc) {
    // eight lanes per point: lane u sums units j = u, u + 8, ... (a point's
    // lanes read consecutive units of its row), then an xor tree over the
    // eight lanes; lane 0 finishes the point
    const int u = threadIdx.x & 7;
    const long i = (long)blockIdx.x * (blockDim.x >> 3) + (threadIdx.x >> 3);
    const long plane = n_pad * W;
    const float* wo = prm + off_wo;
    float v = 0.f, vt = 0.f, vx = 0.f, vxx = 0.f;
    if (i < n) {
        for (int j = u; j < W; j += 8) {
            float a, at, ax, axx;
            streams_from_cache(clast, plane, i * W + j, a, at, ax, axx);
            v = fmaf(wo[j], a, v);
            vt = fmaf(wo[j], at, vt);
            vx = fmaf(wo[j], ax, vx);
            vxx = fmaf(wo[j], axx, vxx);
        }
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
        v += __shfl_xor(v, o, 8);
        vt += __shfl_xor(vt, o, 8);
        vx += __shfl_xor(vx, o, 8);
        vxx += __shfl_xor(vxx, o, 8);
    }
    if (u != 0 || i >= n_pad) return;
    if (i >= n) {
        g[i] = g[n_pad + i] = g[2 * n_pad + i] = g[3 * n_pad + i] = 0.f;
        lossc[i] = 0.f;
        return;
    }
    v += prm[off_bo];
    float g0, g1, g2, g3, lc;
    head_point(P, i, v, vt, vx, vxx, g0, g1, g2, g3, lc);
    g[i] = g0;
    g[n_pad + i] = g1;
    g[2 * n_pad + i] = g2;
    g[3 * n_pad + i] = g3;
    lossc[i] = lc;
}

// loss3[t] = sum of lossc over the points of type t / count (one block).
__global__ void k_res_loss(const float* __restrict__ lossc, int nf, int ne, int nb,
                           float* __restrict__ loss3) {
    __shared__ float red[256];
    const int ranges[4] = {0, nf, nf + ne, nf + ne + nb};
    for (int t = 0; t < 3; ++t) {
        float s = 0.f;
        for (int i = ranges[t] + threadIdx.x; i < ranges[t + 1]; i += blockDim.x) s += lossc[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int cnt = ranges[t + 1] - ranges[t];
            loss3[t] = cnt > 0 ? red[0] / (float)cnt : 0.f;
        }
        __syncthreads();
    }
}

// --------------------------------------------------------- backward kernels

// zbar from the adjoints of the layer's output streams (abar, or g x wo for
// the last hidden layer) and the layer cache.  One thread per (point, unit).
__global__ void k_res_zbar(const float* __restrict__ c, const float* __restrict__ abar,
                           const float* __restrict__ g, const float* __restrict__ wo,
                           float* __restrict__ zbar, long n_pad, int W) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_pad * W) return;
    const long plane = n_pad * W;
    float A, At, Ax, Axx;
    if (abar) {
        A = abar[t];
        At = abar[plane + t];
        Ax = abar[2 * plane + t];
        Axx = abar[3 * plane + t];
    } else {
        const long i = t / W;
        const float w = wo[t - i * W];
        A = g[i] * w;
        At = g[n_pad + i] * w;
        Ax = g[2 * n_pad + i] * w;
        Axx = g[3 * n_pad + i] * w;
    }
    float zb, zb_t, zb_x, zb_xx;
    tanh_adjoint(A, At, Ax, Axx, c[t], c[plane + t], c[2 * plane + t], c[3 * plane + t], zb, zb_t,
                 zb_x, zb_xx);
    zbar[plane + t] = zb_t;
    zbar[2 * plane + t] = zb_x;
    zbar[3 * plane + t] = zb_xx;
    zbar[t] = zb;
}


// The gradient kernels below sum over points in chunks: block c of gridDim.x
// takes the points [c*chunk, (c+1)*chunk) and writes one partial per output
// to part[c][count]; k_res_reduce then sums the partials in block order.

__device__ __forceinline__ void chunk_range(long n, long& lo, long& hi) {
    const long chunk = (n + gridDim.x - 1) / gridDim.x;
    lo = (long)blockIdx.x * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
}

// Hidden-layer weight gradient, tiled (FP32):
//   dW[j][k] = sum_i sum_s zbar_s[i][j] a_s[i][k],  db[j] = sum_i zbar_0[i][j],
// s over the four derivative streams.  Split over points: each of the
// kGradwBlocks blocks sums a contiguous range of points into its own partial
// (reduced afterwards in a fixed order, so the result is deterministic).
// Points go through LDS in chunks of CH: the four adjoint streams and the
// four activation streams (rebuilt from the cache) of the chunk; thread
// (tj, tk) of a 16 x 16 grid accumulates rows j = tj + 16 a (a < JB) and
// columns k = tk + 16 b (b < W/16) in registers, JB rows per pass.
constexpr int kGradwBlocks = 256;

template <int W>
__global__ __launch_bounds__(256) void k_res_gradw_tiled(const float* __restrict__ zbar,
                                                         const float* __restrict__ cprev, long n,
                                                         long n_pad, float* __restrict__ part) {
    constexpr int CH = W >= 256 ? 8 : 16;
    constexpr int KB = W / 16 > 0 ? W / 16 : 1;  // columns per thread
    constexpr int JB = KB > 8 ? 8 : KB;          // rows per thread per pass
    constexpr int PASSES = KB / JB;
    __shared__ float zs[4][CH][W];
    __shared__ float as[4][CH][W];
    const int tid = threadIdx.x, tj = tid >> 4, tk = tid & 15;
    long lo, hi;
    chunk_range(n, lo, hi);
    const long plane = n_pad * W;
    const int count = W * W + W;
    float* out = part + (long)blockIdx.x * count;
    float dbacc = 0.f;  // thread t < W: db[t]
    for (int pass = 0; pass < PASSES; ++pass) {
        float acc[JB][KB];
#pragma unroll
        for (int a = 0; a < JB; ++a)
#pragma unroll
            for (int b = 0; b < KB; ++b) acc[a][b] = 0.f;
        for (long i0 = lo; i0 < hi; i0 += CH) {
            const int cnt = (int)(hi - i0 < CH ? hi - i0 : CH);
            __syncthreads();
            for (int e = tid; e < CH * W; e += 256) {
                const int c = e / W, k = e - c * W;
                float z0 = 0.f, z1 = 0.f, z2 = 0.f, z3 = 0.f, a = 0.f, at = 0.f, ax = 0.f, axx = 0.f;
                if (c < cnt) {
                    const long idx = (i0 + c) * W + k;
                    z0 = zbar[idx];
                    z1 = zbar[plane + idx];
                    z2 = zbar[2 * plane + idx];
                    z3 = zbar[3 * plane + idx];
                    streams_from_cache(cprev, plane, idx, a, at, ax, axx);
                }
                zs[0][c][k] = z0;
                zs[1][c][k] = z1;
                zs[2][c][k] = z2;
                zs[3][c][k] = z3;
                as[0][c][k] = a;
                as[1][c][k] = at;
                as[2][c][k] = ax;
                as[3][c][k] = axx;
            }
            __syncthreads();
            if (pass == 0 && tid < W)
                for (int c = 0; c < cnt; ++c) dbacc += zs[0][c][tid];
            for (int c = 0; c < cnt; ++c) {
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    float zj[JB], ak[KB];
#pragma unroll
                    for (int a = 0; a < JB; ++a) zj[a] = zs[st][c][(pass * JB + a) * 16 + tj];
#pragma unroll
                    for (int b = 0; b < KB; ++b) ak[b] = as[st][c][b * 16 + tk];
#pragma unroll
                    for (int a = 0; a < JB; ++a)
#pragma unroll
                        for (int b = 0; b < KB; ++b) acc[a][b] = fmaf(zj[a], ak[b], acc[a][b]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < JB; ++a) {
            const int j = (pass * JB + a) * 16 + tj;
            if (j < W && tk < W)
#pragma unroll
                for (int b = 0; b < KB; ++b) {
                    const int k = b * 16 + tk;
                    if (k < W) out[(long)j * W + k] = acc[a][b];
                }
        }
    }
    if (tid < W) out[W * W + tid] = dbacc;
}

// First-layer gradient: dW1[j][c] = sum_i zb_ij x_ic (+ sum zb_t for c = 0,
// + sum zb_x for c = 1), then db1[j] = sum_i zb_ij.
__global__ void k_res_grad_first(const float* __restrict__ zbar, Points P, long n, long n_pad,
                                 int W, float* __restrict__ part) {
    long lo, hi;
    chunk_range(n, lo, hi);
    const long plane = n_pad * W;
    const int nw = W * P.n_in, count = nw + W;
    // four running sums over the points i = lo + 4m + u (the loads of four
    // points are in flight together), added in a fixed order
    for (int x = threadIdx.x; x < count; x += blockDim.x) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        if (x < nw) {
            const int j = x / P.n_in, c = x - j * P.n_in;
            const long off = (c == 0) ? plane : (c == 1) ? 2 * plane : -1;
            for (long i0 = lo; i0 < hi; i0 += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const long i = i0 + u;
                    if (i < hi) {
                        const long idx = i * W + j;
                        float t = zbar[idx] * point_row(P, i)[c];
                        if (off >= 0) t += zbar[off + idx];
                        acc[u] += t;
                    }
                }
            }
        } else {
            const int j = x - nw;
            for (long i0 = lo; i0 < hi; i0 += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + u < hi) acc[u] += zbar[(i0 + u) * W + j];
            }
        }
        part[(long)blockIdx.x * count + x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
}

// Output-layer gradient: dwo[j] = sum_i sum_s g_s[i] a_s[i][j], then dbo = sum_i g_0[i].
__global__ void k_res_grad_out(const float* __restrict__ g, const float* __restrict__ clast,
                               long n, long n_pad, int W, float* __restrict__ part) {
    long lo, hi;
    chunk_range(n, lo, hi);
    const long plane = n_pad * W;
    const int count = W + 1;
    for (int x = threadIdx.x; x < count; x += blockDim.x) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        if (x < W) {
            for (long i0 = lo; i0 < hi; i0 += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const long i = i0 + u;
                    if (i < hi) {
                        float a, at, ax, axx;
                        streams_from_cache(clast, plane, i * W + x, a, at, ax, axx);
                        float t = g[i] * a;
                        t = fmaf(g[n_pad + i], at, t);
                        t = fmaf(g[2 * n_pad + i], ax, t);
                        t = fmaf(g[3 * n_pad + i], axx, t);
                        acc[u] += t;
                    }
                }
            }
        } else {
            for (long i0 = lo; i0 < hi; i0 += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (i0 + u < hi) acc[u] += g[i0 + u];
            }
        }
        part[(long)blockIdx.x * count + x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
}

int launch_res_reduce(const float* part, int nblk, int count, float* out, hipStream_t st);

int launch_res_step_bf16(const pinn_net& net, const Points& P, long n, long n_pad, float* cache,
                         float* abar, float* g, __bf16* wbf, float* part, long ldp, int max_blocks,
                         float* grad, float* loss3, hipStream_t st);

static dim3 grid_for(long work, int block) { return dim3((unsigned)((work + block - 1) / block)); }

}  // namespace bsp

using namespace bsp;

extern "C" int pinn_residual_workspace_size(const pinn_net* net, int n_f, int n_e, int n_b,
                                            size_t* bytes) {
    clear_error();
    BSP_CHECK_ARG(bytes != nullptr, "bytes is NULL");
    *bytes = 0;
    int rc = check_net(net);
    if (rc) return rc;
    BSP_CHECK_ARG(n_f >= 0 && n_e >= 0 && n_b >= 0, "point counts must be >= 0");
    *bytes = res_layout(*net, (long)n_f + n_e + n_b, nullptr).bytes;
    return BS_OK;
}

extern "C" int pinn_residual_fwd_bwd(const pinn_net* net, const bs_params* prm, int n_f,
                                     const float* X_f, int n_e, const float* X_e,
                                     const float* y_e, int n_b, const float* X_b,
                                     const float* y_b, float* loss3, float* grad, void* ws,
                                     size_t ws_bytes, void* stream) {
    clear_error();
    int rc = check_net(net);
    if (rc) return rc;
    BSP_CHECK_ARG(prm != nullptr, "bs_params is NULL");
    BSP_CHECK_ARG(n_f >= 0 && n_e >= 0 && n_b >= 0, "point counts must be >= 0");
    BSP_CHECK_ARG((n_f == 0 || X_f) && (n_e == 0 || X_e) && (n_b == 0 || X_b),
                  "point arrays must be non-NULL when their count is positive");
    BSP_CHECK_ARG(loss3 && grad, "loss3 and grad must be non-NULL");
    BSP_CHECK_ARG(net->width <= 128 || net->precision == BS_PREC_FP32,
                  "the bfloat16 residual path supports width <= 128");
    const long n = (long)n_f + n_e + n_b;
    const ResWs w = res_layout(*net, n, ws);
    if (!ws || ws_bytes < w.bytes) {
        set_error("workspace too small: need %zu bytes", w.bytes);
        return BS_ERR_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    const NetLayout L = net_layout(*net);
    const int W = net->width, d = net->depth;
    const long np = w.n_pad, plane = np * W, work = np * W;
    const float* P0 = net->params;
    Points P{X_f, X_e, X_b, n_f, n_e, n_b, net->n_in, (float)prm->sigma, (float)prm->r,
             prm->is_put, y_e, y_b};
    if (net->precision == BS_PREC_BF16) {
        // the whole pass in one launch, then the reduction of its partial rows
        BSP_CHECK_ARG(((uintptr_t)P0 & 15) == 0 && ((uintptr_t)ws & 15) == 0,
                      "the bfloat16 residual path needs 16-byte aligned parameters and workspace");
        return launch_res_step_bf16(*net, P, n, np, w.cache, w.abar, w.g, w.wbf, w.part,
                                    L.total + 3, kPartRows, grad, loss3, st);
    }
    auto cache = [&](int l) { return w.cache + (size_t)(l - 1) * 4 * plane; };

    hipLaunchKernelGGL(k_res_first, grid_for(work, 256), dim3(256), 0, st, P0, P, n, np, W,
                       cache(1));
    BSP_LAUNCHED();
    for (int l = 2; l <= d; ++l)
        if ((rc = launch_res_gemm_f32<0>(P0 + L.offW[l], P0 + L.offb[l], cache(l - 1), cache(l),
                                         np, W, st)))
            return rc;
    hipLaunchKernelGGL(k_res_head, grid_for(np, 32), dim3(256), 0, st, P0, L.off_wo, L.off_bo,
                       P, n, np, W, cache(d), w.g, w.lossc);
    BSP_LAUNCHED();
    hipLaunchKernelGGL(k_res_loss, dim3(1), dim3(256), 0, st, w.lossc, n_f, n_e, n_b, loss3);
    BSP_LAUNCHED();
    hipLaunchKernelGGL(k_res_grad_out, dim3(kResPartBlocks), dim3(256), 0, st, w.g, cache(d), n,
                       np, W, w.part);
    BSP_LAUNCHED();
    // wo and bo are contiguous in the parameter packing
    if ((rc = launch_res_reduce(w.part, kResPartBlocks, W + 1, grad + L.off_wo, st))) return rc;
    for (int l = d; l >= 1; --l) {
        hipLaunchKernelGGL(k_res_zbar, grid_for(work, 256), dim3(256), 0, st, cache(l),
                           l == d ? nullptr : w.abar, w.g, P0 + L.off_wo, w.zbar, np, W);
        BSP_LAUNCHED();
        if (l == 1) {
            hipLaunchKernelGGL(k_res_grad_first, dim3(kResPartBlocks), dim3(256), 0, st, w.zbar, P,
                               n, np, W, w.part);
            BSP_LAUNCHED();
            // W1 and b1 are contiguous in the parameter packing
            if ((rc = launch_res_reduce(w.part, kResPartBlocks, W * net->n_in + W,
                                        grad + L.offW[1], st)))
                return rc;
            break;
        }
        if ((rc = launch_res_gemm_f32<1>(P0 + L.offW[l], nullptr, w.zbar, w.abar, np, W, st)))
            return rc;
        switch (W) {
#define BSP_W(W_)                                                                             \
    case W_:                                                                                  \
        hipLaunchKernelGGL(k_res_gradw_tiled<W_>, dim3(kGradwBlocks), dim3(256), 0, st, w.zbar, \
                           cache(l - 1), n, np, w.part);                                      \
        break;
            BSP_W(16) BSP_W(32) BSP_W(64) BSP_W(128) BSP_W(256)
#undef BSP_W
            default:
                set_error("unsupported width %d", W);
                return BS_ERR_ARG;
        }
        BSP_LAUNCHED();
        if ((rc = launch_res_reduce(w.part, kGradwBlocks, W * W + W, grad + L.offW[l], st)))
            return rc;
    }
    return BS_OK;
}
