// gfx950 (CDNA4) kernels of the paper-faithful mapping loss of RT-GuIDE
// (arXiv 2409.18122, Sec. III eq. (4)): per view,
//   L = (1/P) sum_p ( w_d |D - D*| + l1 sum_ch |C - C*| ) + l2 (1 - SSIM(C, C*)),
// SSIM with an 11x11 Gaussian window (sigma 1.5, weights g(a) g(b)), zero
// padding, C1 = 0.01^2, C2 = 0.03^2, averaged over channels and pixels.
//
// Two passes over 16x16 output tiles, each staging a tile plus its 5-pixel
// halo through LDS and filtering separably (rows, then columns):
//   forward : per channel the local statistics mx, my, sx, sy, sxy, the
//             index S and its partial derivatives, folded into three maps
//             A = dS/dmx - 2 mx dS/dsx - my dS/dsxy, B = dS/dsx, C = dS/dsxy
//             so that the gradient is separable; per-block loss partials.
//   backward: dS/dx(q) = (g * A)(q) + 2 x(q) (g * B)(q) + y(q) (g * C)(q)
//             (the window is symmetric, so the adjoint filter is the filter),
//             plus the L1 signs.
// Compiled without floating-point contraction, like the rasterizer.
#include "rtg_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

namespace rtg {

namespace {

constexpr int SS_T = 16;                  // output tile edge
constexpr int SS_R = 5;                   // window radius
constexpr int SS_K = 2 * SS_R + 1;        // window taps
constexpr int SS_E = SS_T + 2 * SS_R;     // staged edge: tile plus halo
constexpr float SS_C1 = 0.01f * 0.01f;
constexpr float SS_C2 = 0.03f * 0.03f;

struct Win {
    float g[SS_K];
};

__device__ __forceinline__ float sgn(float e) { return e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Tile of this block within its view; false for the blocks past the view's last tile.
__device__ __forceinline__ bool tile_of(const ViewDev& V, int& x0, int& y0) {
    const int tx = (V.W + SS_T - 1) / SS_T, ty = (V.H + SS_T - 1) / SS_T;
    const int b = (int)blockIdx.x;
    if (b >= tx * ty) return false;
    x0 = (b % tx) * SS_T;
    y0 = (b / tx) * SS_T;
    return true;
}

// Stage the (SS_E x SS_E) window of a planar W x H image around the tile, 0 outside the image.
__device__ __forceinline__ void stage(float* __restrict__ dst, const float* __restrict__ img, int W, int H, int x0,
                                      int y0) {
    for (int i = threadIdx.x; i < SS_E * SS_E; i += SS_T * SS_T) {
        const int r = i / SS_E, c = i - r * SS_E;
        const int gu = x0 - SS_R + c, gv = y0 - SS_R + r;
        dst[i] = (gu >= 0 && gu < W && gv >= 0 && gv < H) ? img[(int64_t)gv * W + gu] : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const ViewDev* __restrict__ views, const float* __restrict__ rgb,
                                                  const float* __restrict__ depth, const float* __restrict__ trgb,
                                                  const float* __restrict__ tdepth, float w_depth, float l1, float l2,
                                                  Win w, uint64_t pix_total, float* __restrict__ maps,
                                                  double* __restrict__ partial) {
    __shared__ float s_x[SS_E * SS_E], s_y[SS_E * SS_E];
    __shared__ float s_h[5][SS_E][SS_T];
    __shared__ double s_w[4];
    const ViewDev& V = views[blockIdx.y];
    const uint64_t part = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    int x0, y0;
    if (!tile_of(V, x0, y0)) {
        if (threadIdx.x == 0) partial[part] = 0.0;
        return;
    }
    const int W = V.W, H = V.H;
    const int64_t P = (int64_t)W * H;
    const int lx = threadIdx.x & (SS_T - 1), ly = threadIdx.x >> 4;
    const int u = x0 + lx, v = y0 + ly;
    const bool inside = u < W && v < H;
    const int64_t p = (int64_t)v * W + u;
    const double invP = 1.0 / (double)P;
    double acc = 0.0;
    if (inside) {
        float row = 0.0f;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            const int64_t c = 3 * V.pix_off + ch * P + p;
            row += fabsf(rgb[c] - trgb[c]);
        }
        const int64_t q = V.pix_off + p;
        acc = ((double)w_depth * (double)fabsf(depth[q] - tdepth[q]) + (double)l1 * (double)row) * invP;
    }
    for (int ch = 0; ch < 3; ch++) {
        __syncthreads();
        stage(s_x, rgb + 3 * V.pix_off + ch * P, W, H, x0, y0);
        stage(s_y, trgb + 3 * V.pix_off + ch * P, W, H, x0, y0);
        __syncthreads();
        for (int i = threadIdx.x; i < SS_E * SS_T; i += SS_T * SS_T) {
            const int r = i >> 4, c = i & (SS_T - 1);
            float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, a4 = 0.0f;
#pragma unroll
            for (int k = 0; k < SS_K; k++) {
                const float xv = s_x[r * SS_E + c + k], yv = s_y[r * SS_E + c + k], g = w.g[k];
                a0 = fmaf(g, xv, a0);
                a1 = fmaf(g, yv, a1);
                a2 = fmaf(g, xv * xv, a2);
                a3 = fmaf(g, yv * yv, a3);
                a4 = fmaf(g, xv * yv, a4);
            }
            s_h[0][r][c] = a0;
            s_h[1][r][c] = a1;
            s_h[2][r][c] = a2;
            s_h[3][r][c] = a3;
            s_h[4][r][c] = a4;
        }
        __syncthreads();
        float mx = 0.0f, my = 0.0f, exx = 0.0f, eyy = 0.0f, exy = 0.0f;
#pragma unroll
        for (int k = 0; k < SS_K; k++) {
            const float g = w.g[k];
            mx = fmaf(g, s_h[0][ly + k][lx], mx);
            my = fmaf(g, s_h[1][ly + k][lx], my);
            exx = fmaf(g, s_h[2][ly + k][lx], exx);
            eyy = fmaf(g, s_h[3][ly + k][lx], eyy);
            exy = fmaf(g, s_h[4][ly + k][lx], exy);
        }
        if (inside) {
            const float sx = exx - mx * mx, sy = eyy - my * my, sxy = exy - mx * my;
            const float n1 = 2.0f * mx * my + SS_C1, n2 = 2.0f * sxy + SS_C2;
            const float d1 = mx * mx + my * my + SS_C1, d2 = sx + sy + SS_C2;
            const float den = d1 * d2;
            const float S = (n1 * n2) / den;
            const float dmx = (2.0f * my * n2 - S * 2.0f * mx * d2) / den;
            const float dsx = -S / d2;
            const float dsxy = 2.0f * n1 / den;
            const uint64_t o = V.pix_off + (uint64_t)p;
            maps[(uint64_t)(3 * ch + 0) * pix_total + o] = dmx - 2.0f * mx * dsx - my * dsxy;
            maps[(uint64_t)(3 * ch + 1) * pix_total + o] = dsx;
            maps[(uint64_t)(3 * ch + 2) * pix_total + o] = dsxy;
            acc -= (double)l2 * (double)S * invP / 3.0;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[part] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const ViewDev* __restrict__ views, const float* __restrict__ rgb,
                                                  const float* __restrict__ depth, const float* __restrict__ trgb,
                                                  const float* __restrict__ tdepth, float w_depth, float l1, float l2,
                                                  Win w, uint64_t pix_total, const float* __restrict__ maps,
                                                  float* __restrict__ d_rgb, float* __restrict__ d_depth) {
    __shared__ float s_m[3][SS_E * SS_E];
    __shared__ float s_h[3][SS_E][SS_T];
    const ViewDev& V = views[blockIdx.y];
    int x0, y0;
    if (!tile_of(V, x0, y0)) return;
    const int W = V.W, H = V.H;
    const int64_t P = (int64_t)W * H;
    const int lx = threadIdx.x & (SS_T - 1), ly = threadIdx.x >> 4;
    const int u = x0 + lx, v = y0 + ly;
    const bool inside = u < W && v < H;
    const int64_t p = (int64_t)v * W + u;
    const float invP = (float)(1.0 / (double)P);
    const float kS = (float)(-(double)l2 / (3.0 * (double)P));
    if (inside && d_depth) {
        const int64_t q = V.pix_off + p;
        d_depth[q] = w_depth * sgn(depth[q] - tdepth[q]) * invP;
    }
    if (!d_rgb) return;
    for (int ch = 0; ch < 3; ch++) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 3; j++) stage(s_m[j], maps + (uint64_t)(3 * ch + j) * pix_total + V.pix_off, W, H, x0, y0);
        __syncthreads();
        for (int i = threadIdx.x; i < SS_E * SS_T; i += SS_T * SS_T) {
            const int r = i >> 4, c = i & (SS_T - 1);
            float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
#pragma unroll
            for (int k = 0; k < SS_K; k++) {
                const float g = w.g[k];
                a0 = fmaf(g, s_m[0][r * SS_E + c + k], a0);
                a1 = fmaf(g, s_m[1][r * SS_E + c + k], a1);
                a2 = fmaf(g, s_m[2][r * SS_E + c + k], a2);
            }
            s_h[0][r][c] = a0;
            s_h[1][r][c] = a1;
            s_h[2][r][c] = a2;
        }
        __syncthreads();
        float cA = 0.0f, cB = 0.0f, cC = 0.0f;
#pragma unroll
        for (int k = 0; k < SS_K; k++) {
            const float g = w.g[k];
            cA = fmaf(g, s_h[0][ly + k][lx], cA);
            cB = fmaf(g, s_h[1][ly + k][lx], cB);
            cC = fmaf(g, s_h[2][ly + k][lx], cC);
        }
        if (inside) {
            const int64_t c = 3 * V.pix_off + ch * P + p;
            const float x = rgb[c], y = trgb[c];
            const float dS = fmaf(y, cC, fmaf(2.0f * x, cB, cA));
            d_rgb[c] = fmaf(kS, dS, l1 * sgn(x - y) * invP);
        }
    }
}

__global__ __launch_bounds__(256) void k_ssim_sum(const double* __restrict__ partial, int n, double add,
                                                  double* __restrict__ out) {
    __shared__ double s_w[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = ((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) + add;
}

Win window() {
    double g[SS_K], sum = 0.0;
    for (int k = -SS_R; k <= SS_R; k++) {
        g[k + SS_R] = std::exp(-(double)(k * k) / (2.0 * 1.5 * 1.5));
        sum += g[k + SS_R];
    }
    Win w;
    for (int k = 0; k < SS_K; k++) w.g[k] = (float)(g[k] / sum);
    return w;
}

}  // namespace

int ssim_blocks_per_view(int max_w, int max_h) { return ((max_w + SS_T - 1) / SS_T) * ((max_h + SS_T - 1) / SS_T); }

void loss_ssim(const ViewDev* views, int n_views, int blocks_per_view, uint64_t pix_total, const float* rgb,
               const float* depth, const float* trgb, const float* tdepth, float w_depth, float l1, float l2,
               float* maps, double* partial, float* d_rgb, float* d_depth, double* loss, hipStream_t s) {
    const Win w = window();
    dim3 grid((unsigned)blocks_per_view, (unsigned)n_views);
    k_ssim_fwd<<<grid, SS_T * SS_T, 0, s>>>(views, rgb, depth, trgb, tdepth, w_depth, l1, l2, w, pix_total, maps,
                                            partial);
    k_ssim_sum<<<1, 256, 0, s>>>(partial, blocks_per_view * n_views, (double)l2 * n_views, loss);
    if (d_rgb || d_depth)
        k_ssim_bwd<<<grid, SS_T * SS_T, 0, s>>>(views, rgb, depth, trgb, tdepth, w_depth, l1, l2, w, pix_total, maps,
                                                d_rgb, d_depth);
}

}  // namespace rtg
