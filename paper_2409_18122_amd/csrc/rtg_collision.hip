// gfx950 (CDNA4) collision check of RT-GuIDE's trajectory planner (arXiv
// 2409.18122, Sec. IV-B, trajectory planner, Collision Checking paragraph):
// points sampled on motion primitives against every Gaussian of the map, each taken as a sphere of lambda_g times its principal
// axis.  Compiled without floating-point contraction, like the rasterizer.
#include "rtg_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace rtg {

namespace {

inline unsigned grid_cap(uint64_t n, unsigned block, unsigned cap) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Sec. IV-B (trajectory planner, Collision Checking): a sampled point (a
// sphere of radius r_robot) collides with a Gaussian whose mean is closer than r_robot + lambda_g r, r = the Gaussian's
// principal axis exp(max log-scale).  Every point against every Gaussian:
// a prep pass packs each Gaussian as (mu, w = lambda_g r) plus the squared
// bound (r_robot + w)^2 widened down and up by a relative CC_BAND; the pair
// loop stages them through LDS in tiles and decides in binary32 outside the
// band, in binary64 (from the original parameters, in the oracle's order)
// inside it.  The clearance min_i (||p - mu_i|| - w_i) is binary32 (the
// hardware square root, within an ulp).

constexpr int CC_THREADS = 256;
constexpr int CC_TILE = 1024;            // Gaussians per LDS tile
constexpr double CC_BAND = 4e-6;         // relative band re-taken in binary64 (d^2 error < 4e-7)

__device__ __forceinline__ uint32_t ordered_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ordered_val(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// packed[i] = (mu, w); bound[i] = ((r_robot + w)^2 (1 - band), (r_robot + w)^2 (1 + band)), both
// formed in binary64 and rounded once.  Non-finite Gaussians: NaN mean (every comparison false), w 0.
__global__ __launch_bounds__(256) void k_collision_prep(GaussDev g, float r_robot, float lambda_g,
                                                        float4* __restrict__ packed, float2* __restrict__ bound) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float m0 = g.means[i], m1 = g.means[g.n + i], m2 = g.means[2 * g.n + i];
        const float l0 = g.log_scales[i], l1 = g.log_scales[g.n + i], l2 = g.log_scales[2 * g.n + i];
        const bool ok = isfinite(m0) && isfinite(m1) && isfinite(m2) && isfinite(l0) && isfinite(l1) && isfinite(l2);
        const double w = (double)lambda_g * exp((double)fmaxf(fmaxf(l0, l1), l2));
        const double gm = (double)r_robot + w;
        const double g2 = gm * gm;
        const float nan = __uint_as_float(0x7fc00000u);
        packed[i] = ok ? make_float4(m0, m1, m2, (float)w) : make_float4(nan, nan, nan, 0.0f);
        bound[i] = ok ? make_float2((float)(g2 * (1.0 - CC_BAND)), (float)(g2 * (1.0 + CC_BAND)))
                      : make_float2(0.0f, 0.0f);
    }
}

// binary64 test of point (px, py, pz) against Gaussian i, as the oracle takes it
__device__ __noinline__ bool collide64(const GaussDev& g, int64_t i, float px, float py, float pz, float r_robot,
                                       float lambda_g) {
    const double l0 = g.log_scales[i], l1 = g.log_scales[g.n + i], l2 = g.log_scales[2 * g.n + i];
    double lm = l0 > l1 ? l0 : l1;
    lm = lm > l2 ? lm : l2;
    const double r = exp(lm);
    const double dx = (double)px - (double)g.means[i];
    const double dy = (double)py - (double)g.means[g.n + i];
    const double dz = (double)pz - (double)g.means[2 * g.n + i];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double gm = (double)r_robot + (double)lambda_g * r;
    return d2 < gm * gm;
}

// grid: x over blocks of CC_THREADS points, y over chunks of `chunk` Gaussians.  The pair loop
// only notes a pair inside the band (`amb`); a tile with such a point is walked once more by the
// whole block, taking the binary64 test for those points alone.
__global__ __launch_bounds__(CC_THREADS) void k_collision(GaussDev g, const float4* __restrict__ packed,
                                                          const float2* __restrict__ bound,
                                                          const float* __restrict__ pts, int64_t np, int64_t chunk,
                                                          float r_robot, float lambda_g,
                                                          int32_t* __restrict__ collide,
                                                          uint32_t* __restrict__ clear_key) {
    __shared__ float4 s_c[CC_TILE];
    __shared__ float2 s_b[CC_TILE];
    const int64_t j = (int64_t)blockIdx.x * CC_THREADS + threadIdx.x;
    const bool live = j < np;
    const float px = live ? pts[j] : 0.0f, py = live ? pts[np + j] : 0.0f, pz = live ? pts[2 * np + j] : 0.0f;
    const int64_t c0 = (int64_t)blockIdx.y * chunk, c1 = min(c0 + chunk, g.n);
    bool hit = false;
    float best = __uint_as_float(0x7f800000u);  // +inf
    for (int64_t t0 = c0; t0 < c1; t0 += CC_TILE) {
        const int cnt = (int)min<int64_t>(CC_TILE, c1 - t0);
        __syncthreads();
        for (int k = threadIdx.x; k < cnt; k += CC_THREADS) {
            s_c[k] = packed[t0 + k];
            s_b[k] = bound[t0 + k];
        }
        __syncthreads();
        bool amb = false;
        if (live) {
#pragma unroll 4
            for (int k = 0; k < cnt; k++) {
                const float4 c = s_c[k];
                const float2 bd = s_b[k];
                const float dx = px - c.x, dy = py - c.y, dz = pz - c.z;
                const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                hit |= d2 < bd.x;
                amb |= d2 <= bd.y;
                // sqrt(d2) - w < best  <=>  d2 < (best + w) |best + w|   (false when best + w <= 0)
                const float tb = best + c.w;
                if (d2 < tb * fabsf(tb)) best = __builtin_amdgcn_sqrtf(d2) - c.w;
            }
        }
        const bool need = live && amb && !hit;
        if (__syncthreads_or(need) && need) {
            for (int k = 0; k < cnt && !hit; k++) {
                const float4 c = s_c[k];
                const float dx = px - c.x, dy = py - c.y, dz = pz - c.z;
                const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                if (d2 <= s_b[k].y && collide64(g, t0 + k, px, py, pz, r_robot, lambda_g)) hit = true;
            }
        }
    }
    if (!live) return;
    if (hit) atomicOr(&collide[j], 1);
    atomicMin(&clear_key[j], ordered_key(best));
}

__global__ __launch_bounds__(256) void k_collision_init(int64_t np, int32_t* __restrict__ collide,
                                                        uint32_t* __restrict__ clear_key) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
        collide[j] = 0;
        clear_key[j] = ordered_key(__uint_as_float(0x7f800000u));
    }
}

__global__ __launch_bounds__(256) void k_collision_finish(int64_t np, const uint32_t* __restrict__ clear_key,
                                                          float* __restrict__ clearance) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x)
        clearance[j] = ordered_val(clear_key[j]);
}

}  // namespace

void collision_check(const GaussDev& g, const float* pts, int64_t np, float r_robot, float lambda_g, float4* packed,
                     float2* bound, int32_t* collide, uint32_t* clear_key, float* clearance, hipStream_t s) {
    if (np <= 0) return;
    k_collision_init<<<grid_cap((uint64_t)np, 256, 4096), 256, 0, s>>>(np, collide, clear_key);
    if (g.n > 0) {
        k_collision_prep<<<grid_cap((uint64_t)g.n, 256, 1u << 16), 256, 0, s>>>(g, r_robot, lambda_g, packed, bound);
        const int64_t nbx = (np + CC_THREADS - 1) / CC_THREADS;
        // chunks sized for about 4096 blocks, whole tiles, at most 65535 rows
        int64_t chunk = (g.n * nbx + 4095) / 4096;
        chunk = std::max<int64_t>(CC_TILE, (chunk + CC_TILE - 1) / CC_TILE * CC_TILE);
        chunk = std::max<int64_t>(chunk, (g.n + 65534) / 65535);
        const int64_t nby = (g.n + chunk - 1) / chunk;
        dim3 grid((unsigned)nbx, (unsigned)nby);
        k_collision<<<grid, CC_THREADS, 0, s>>>(g, packed, bound, pts, np, chunk, r_robot, lambda_g, collide, clear_key);
    }
    if (clearance) k_collision_finish<<<grid_cap((uint64_t)np, 256, 4096), 256, 0, s>>>(np, clear_key, clearance);
}

}  // namespace rtg
