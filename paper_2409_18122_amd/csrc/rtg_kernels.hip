// gfx950 (CDNA4) kernels of the Gaussian-splatting rasterizer used by RT-GuIDE
// (arXiv 2409.18122): projection and culling, prefix sums, an LSD radix sort,
// tile binning, front-to-back compositing of RGB / depth / alpha /
// uncertainty, the L1 mapping loss, the reverse-mode kernels, and the
// persistent view scorer.
//
// The file is compiled without floating-point contraction: every fused
// multiply-add below is an explicit fmaf/fma, so a value computed in two
// kernels (a splat's alpha in the forward and the backward, the camera depth
// used as sort key) is bit-identical in both.
#include "rtg_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>

namespace rtg {

namespace {

constexpr double LOG2E = 1.4426950408889634;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ------------------------------------------------------------------ fill

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------- projection
// Sec. III (Gaussian Splatting paragraph): t = R^T (mu - T), d = t_z,
// mu_2D = (fx t_x / d + cx, fy t_y / d + cy); the 2D covariance is the EWA
// form J R^T Sigma R J^T of the cited 3DGS work, with Sigma = Rq S^2 Rq^T,
// or, for the paper's isotropic Gaussians, diag((fx r / d)^2, (fy r / d)^2)
// (r_2D = f r / d; one log-radius per Gaussian, no quaternion).

struct GPre {
    double mu[3];
    double Rq[9];
    double s[3];
    double o, rho2;
    float mu_f[3];
    float reach;           // rho * max scale: bound on the support radius in 3D
    float rho_f, rho2_f;   // binary32 rho = sqrt(2 ln(o / alpha_min)) and rho^2, for the bound
};

// The isotropic form: s = (r, r, r) and Rq = I; only the first n log-scale values are read.
__device__ inline bool pre_gauss_iso(const GaussDev& g, int64_t i, const SetDev& st, GPre& P) {
    const int64_t n = g.n;
    const float m0 = g.means[i], m1 = g.means[n + i], m2 = g.means[2 * n + i];
    const float lr = g.log_scales[i];
    const float op = g.opacity[i];
    if (!(isfinite(m0) && isfinite(m1) && isfinite(m2) && isfinite(lr) && isfinite(op))) return false;
    if (op < st.alpha_min) return false;
#pragma unroll
    for (int k = 0; k < 9; k++) P.Rq[k] = (k % 4 == 0) ? 1.0 : 0.0;
    const double r = exp((double)lr);
    P.s[0] = r;
    P.s[1] = r;
    P.s[2] = r;
    P.mu[0] = m0; P.mu[1] = m1; P.mu[2] = m2;
    P.mu_f[0] = m0; P.mu_f[1] = m1; P.mu_f[2] = m2;
    P.o = op;
    P.rho2 = 2.0 * log((double)op / (double)st.alpha_min);
    P.reach = (float)(sqrt(P.rho2) * r);
    P.rho_f = (float)sqrt(P.rho2);
    P.rho2_f = (float)P.rho2;
    return true;
}

__device__ inline bool pre_gauss(const GaussDev& g, int64_t i, const SetDev& st, GPre& P) {
    if (st.isotropic) return pre_gauss_iso(g, i, st, P);
    const int64_t n = g.n;
    float m0 = g.means[i], m1 = g.means[n + i], m2 = g.means[2 * n + i];
    float l0 = g.log_scales[i], l1 = g.log_scales[n + i], l2 = g.log_scales[2 * n + i];
    float q0 = g.quats[i], q1 = g.quats[n + i], q2 = g.quats[2 * n + i], q3 = g.quats[3 * n + i];
    float op = g.opacity[i];
    bool fin = isfinite(m0) && isfinite(m1) && isfinite(m2) && isfinite(l0) && isfinite(l1) &&
               isfinite(l2) && isfinite(q0) && isfinite(q1) && isfinite(q2) && isfinite(q3) &&
               isfinite(op);
    if (!fin) return false;
    if (op < st.alpha_min) return false;
    double w = q0, x = q1, y = q2, z = q3;
    double qn = sqrt(w * w + x * x + y * y + z * z);
    if (!(qn > 0.0)) return false;
    double inv = 1.0 / qn;
    w *= inv; x *= inv; y *= inv; z *= inv;
    double xx = x * x, yy = y * y, zz = z * z;
    double xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
    P.Rq[0] = 1.0 - 2.0 * (yy + zz); P.Rq[1] = 2.0 * (xy - wz);       P.Rq[2] = 2.0 * (xz + wy);
    P.Rq[3] = 2.0 * (xy + wz);       P.Rq[4] = 1.0 - 2.0 * (xx + zz); P.Rq[5] = 2.0 * (yz - wx);
    P.Rq[6] = 2.0 * (xz - wy);       P.Rq[7] = 2.0 * (yz + wx);       P.Rq[8] = 1.0 - 2.0 * (xx + yy);
    P.s[0] = exp((double)l0);
    P.s[1] = exp((double)l1);
    P.s[2] = exp((double)l2);
    P.mu[0] = m0; P.mu[1] = m1; P.mu[2] = m2;
    P.mu_f[0] = m0; P.mu_f[1] = m1; P.mu_f[2] = m2;
    P.o = op;
    P.rho2 = 2.0 * log((double)op / (double)st.alpha_min);
    double smax = fmax(P.s[0], fmax(P.s[1], P.s[2]));
    P.reach = (float)(sqrt(P.rho2) * smax);
    P.rho_f = (float)sqrt(P.rho2);
    P.rho2_f = (float)P.rho2;
    return true;
}

// Conservative binary32 test: false only if the exact binary64 projection is
// certain to be culled (behind the near plane, or its support box cannot meet
// the image).  The half extent of the support box is bounded through
// Sigma_xx <= s_max^2 |J_row0|^2 = s_max^2 fx^2 / t_z^2 (1 + t_x^2 / t_z^2).
// The binary32 camera values the test reads, packed in five 16-byte words:
// the columns of R with the camera centre, (fx, fy, cx, cy), (W - 1, H - 1).
struct CullView {
    float4 c0, c1, c2, k, wh;
};

__device__ __forceinline__ CullView cull_view(const ViewDev& V) {
    CullView f;
    f.c0 = make_float4(V.Rf[0], V.Rf[3], V.Rf[6], V.Tf[0]);
    f.c1 = make_float4(V.Rf[1], V.Rf[4], V.Rf[7], V.Tf[1]);
    f.c2 = make_float4(V.Rf[2], V.Rf[5], V.Rf[8], V.Tf[2]);
    f.k = make_float4(V.fxf, V.fyf, V.cxf, V.cyf);
    f.wh = make_float4((float)(V.W - 1), (float)(V.H - 1), 0.0f, 0.0f);
    return f;
}

__device__ inline bool may_be_visible(const GPre& P, const CullView& V, const SetDev& st) {
    float dx = P.mu_f[0] - V.c0.w;
    float dy = P.mu_f[1] - V.c1.w;
    float dz = P.mu_f[2] - V.c2.w;
    float mag = fabsf(dx) + fabsf(dy) + fabsf(dz) + 1.0f;
    float tz = dx * V.c2.x + dy * V.c2.y + dz * V.c2.z;
    float err = 1e-5f * mag;
    if (tz + err <= st.z_near) return false;
    if (tz <= 0.5f * st.z_near) return true;  // let the exact test decide
    float tx = dx * V.c0.x + dy * V.c0.y + dz * V.c0.z;
    float ty = dx * V.c1.x + dy * V.c1.y + dz * V.c1.z;
    // hardware reciprocal and square root (within an ulp or two): the slack
    // below is a relative 1e-3 plus a pixel
    float iz = __builtin_amdgcn_rcpf(tz);
    float ux = tx * iz, uy = ty * iz;
    float fx = V.k.x, fy = V.k.y;
    float ax = fx * ux + V.k.z;
    float ay = fy * uy + V.k.w;
    float rx = P.reach * fx * iz, ry = P.reach * fy * iz;
    const float ep = 2.0f * P.rho_f * st.eps2d + st.eps2d * P.rho2_f;
    float hx = __builtin_amdgcn_sqrtf(rx * rx * (1.0f + ux * ux) + ep);
    float hy = __builtin_amdgcn_sqrtf(ry * ry * (1.0f + uy * uy) + ep);
    float slack_x = 1e-3f * (fabsf(ax - V.k.z) + hx) + 1.0f + err * fx * iz * 4.0f;
    float slack_y = 1e-3f * (fabsf(ay - V.k.w) + hy) + 1.0f + err * fy * iz * 4.0f;
    if (ax + hx + slack_x < 0.0f) return false;
    if (ax - hx - slack_x > V.wh.x) return false;
    if (ay + hy + slack_y < 0.0f) return false;
    if (ay - hy - slack_y > V.wh.y) return false;
    return true;
}

struct GProj {
    double t[3];
    double A[9];  // R^T Rq
    double j0, j2, j4, j5;  // nonzero entries of the perspective Jacobian
    double cxx, cxy, cyy;
    double mx, my;
    int u0, u1, v0, v1;
};

// Exact binary64 projection.  The camera depth is evaluated in the fixed
// order ((dx R02 + dy R12) + dz R22): its binary32 rounding is the sort key.
__device__ inline bool project_exact(const GPre& P, const ViewDev& V, const SetDev& st, GProj& q) {
    double dx = P.mu[0] - V.T[0];
    double dy = P.mu[1] - V.T[1];
    double dz = P.mu[2] - V.T[2];
    const double* R = V.R;
    double tx = (dx * R[0] + dy * R[3]) + dz * R[6];
    double ty = (dx * R[1] + dy * R[4]) + dz * R[7];
    double tz = (dx * R[2] + dy * R[5]) + dz * R[8];
    if (!(tz > (double)st.z_near)) return false;
    q.t[0] = tx; q.t[1] = ty; q.t[2] = tz;
    double iz = 1.0 / tz;
    q.j0 = V.fx * iz;
    q.j4 = V.fy * iz;
    if (st.isotropic) {
        // Sigma_2D = diag(j0^2, j4^2) r^2: the EWA form below with A = I and
        // no off-axis Jacobian terms (which the backward then treats as constant)
#pragma unroll
        for (int k = 0; k < 9; k++) q.A[k] = (k % 4 == 0) ? 1.0 : 0.0;
        q.j2 = 0.0;
        q.j5 = 0.0;
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++)
                q.A[a * 3 + b] = fma(R[0 * 3 + a], P.Rq[0 * 3 + b],
                                     fma(R[1 * 3 + a], P.Rq[1 * 3 + b], R[2 * 3 + a] * P.Rq[2 * 3 + b]));
        q.j2 = -V.fx * tx * iz * iz;
        q.j5 = -V.fy * ty * iz * iz;
    }
    // B = J A scaled by s per column; cov = B S^2 B^T
    double cxx = 0.0, cxy = 0.0, cyy = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double b0 = fma(q.j0, q.A[0 * 3 + k], q.j2 * q.A[2 * 3 + k]) * P.s[k];
        double b1 = fma(q.j4, q.A[1 * 3 + k], q.j5 * q.A[2 * 3 + k]) * P.s[k];
        cxx = fma(b0, b0, cxx);
        cxy = fma(b0, b1, cxy);
        cyy = fma(b1, b1, cyy);
    }
    cxx += (double)st.eps2d;
    cyy += (double)st.eps2d;
    double det = cxx * cyy - cxy * cxy;
    if (!(det > 0.0) || !isfinite(det)) return false;
    q.cxx = cxx; q.cxy = cxy; q.cyy = cyy;
    q.mx = fma(V.fx * tx, iz, V.cx);
    q.my = fma(V.fy * ty, iz, V.cy);
    double hx = sqrt(P.rho2 * cxx), hy = sqrt(P.rho2 * cyy);
    double ulo = ceil(q.mx - hx), uhi = floor(q.mx + hx);
    double vlo = ceil(q.my - hy), vhi = floor(q.my + hy);
    if (!(ulo <= uhi) || !(vlo <= vhi)) return false;
    ulo = fmax(ulo, 0.0);
    vlo = fmax(vlo, 0.0);
    uhi = fmin(uhi, (double)(V.W - 1));
    vhi = fmin(vhi, (double)(V.H - 1));
    if (ulo > uhi || vlo > vhi) return false;
    q.u0 = (int)ulo; q.u1 = (int)uhi; q.v0 = (int)vlo; q.v1 = (int)vhi;
    return true;
}


// ------------------------------------------------------- support extents
// A splat's support {alpha >= alpha_min} in the whitened form is
// w1^2 + w2^2 <= log2(o / alpha_min) with w1 = a dx, w2 = b dx + c dy
// (geo1 = (a, b, c, o), d = pixel - mean): the ellipse with
// Q = [[a^2 + b^2, b c], [b c, c^2]], det Q = (a c)^2.  On a horizontal
// slice at offset dy it spans dx = (-B dy +/- sqrt(A l - D dy^2)) / A
// (A = a^2 + b^2, B = b c, D = det Q).  The right end is concave in dy with
// its maximum at dy_r = -(b / (a c)) sqrt(l), the left end convex with its
// minimum at -dy_r, so the x extent over a band of rows is the two slices at
// the offsets clamped into the band.
//
// The test is conservative in binary32: l exceeds log2(o / alpha_min) by the
// binary64 refinement band of the alpha_min test, by the binary32 rounding of
// a pixel's own exponent (which grows with |b dx| + c |dy|, bounded here
// through X and Y, the largest |dx| and |dy| in question) and by a relative
// 1e-4; the extents are widened by a relative 1e-3 plus 1e-3 pixel.
// Returns false if the rows [r0, r1] miss the support.
__device__ __forceinline__ bool support_span(float4 g0, float4 g1, float log2_amin, float X, int r0, int r1,
                                             float& xl, float& xr) {
    const float a = g1.x, b = g1.y, c = g1.z;
    const float mx = g0.x + g0.z, my = g0.y + g0.w;
    const float dy0 = (float)r0 - my, dy1 = (float)r1 - my;
    const float Y = fmaxf(fabsf(dy0), fabsf(dy1));
    const float l = (__builtin_amdgcn_logf(g1.w) - log2_amin) * 1.0001f + 0.004f + 4e-7f * fmaf(fabsf(b), X, c * Y);
    const float A = fmaf(a, a, b * b);
    const float ac = a * c;
    if (!(A > 0.0f) || !(ac > 0.0f) || !(l > 0.0f) || !(A < 3e38f)) {  // not expected: no culling
        xl = -3e38f;
        xr = 3e38f;
        return true;
    }
    const float D = ac * ac;
    const float B = b * c;
    const float dyr = -b * __builtin_amdgcn_rcpf(ac) * __builtin_amdgcn_sqrtf(l);
    const float yr = fminf(fmaxf(dyr, dy0), dy1);
    const float yl = fminf(fmaxf(-dyr, dy0), dy1);
    const float Al = A * l;
    const float dr = fmaf(-D * yr, yr, Al);
    const float dl = fmaf(-D * yl, yl, Al);
    if (dr < -1e-4f * Al) return false;
    const float ia = __builtin_amdgcn_rcpf(A);
    const float R = (__builtin_amdgcn_sqrtf(fmaxf(dr, 0.0f)) - B * yr) * ia;
    const float L = (-__builtin_amdgcn_sqrtf(fmaxf(dl, 0.0f)) - B * yl) * ia;
    const float mg = 1e-3f * (fabsf(R) + fabsf(L)) + 1e-3f;
    xl = mx + L - mg;
    xr = mx + R + mg;
    return true;
}

// Whether a splat's support can reach a pixel of the rectangle [c0, c1] x
// [r0, r1] (a prefilter; the per-pixel tests decide).  The mean (mx, my) and
// the rectangle are in any common pixel frame.
__device__ __forceinline__ bool support_meets_rect_xy(float mx, float my, float4 g1, float log2_amin, int c0,
                                                      int c1, int r0, int r1) {
    const float X = fmaxf(fabsf((float)c0 - mx), fabsf((float)c1 - mx));
    float xl, xr;
    if (!support_span(make_float4(mx, my, 0.0f, 0.0f), g1, log2_amin, X, r0, r1, xl, xr)) return false;
    return xl <= (float)c1 && xr >= (float)c0;
}

__device__ __forceinline__ bool support_meets_rect(float4 g0, float4 g1, float log2_amin, int c0, int c1, int r0,
                                                   int r1) {
    return support_meets_rect_xy(g0.x + g0.z, g0.y + g0.w, g1, log2_amin, c0, c1, r0, r1);
}

// Per-record constants of the support rows: on a slice at offset dy the
// ellipse spans [-sqrt(P - Qc dy^2) - Bc dy, sqrt(P - Qc dy^2) - Bc dy]
// (P = l / A, Qc = D / A^2, Bc = B / A in the notation of support_span), l
// taken with X and Y bounding |dx| and |dy| over the whole pixel box.
struct SupportRows {
    float mx, my, dyr, P, Qc, Bc;
    uint32_t pb_x, pb_y;  // pixel box
    int all;              // 1: no culling (degenerate form, not expected)
};

// Pair counting and pair emission both call support_setup and support_row,
// two non-inlined functions, on the same stored record values (geo0, geo1,
// pixel box), so they agree exactly.
__device__ __noinline__ SupportRows support_setup(float4 g0, float4 g1, uint2 pb, float log2_amin) {
    SupportRows S;
    const float a = g1.x, b = g1.y, c = g1.z;
    S.mx = g0.x + g0.z;
    S.my = g0.y + g0.w;
    S.pb_x = pb.x;
    S.pb_y = pb.y;
    const float u0 = (float)(pb.x & 0xffffu), u1 = (float)(pb.x >> 16);
    const float v0 = (float)(pb.y & 0xffffu), v1 = (float)(pb.y >> 16);
    const float X = fmaxf(fabsf(u0 - S.mx), fabsf(u1 - S.mx));
    const float Y = fmaxf(fabsf(v0 - S.my), fabsf(v1 - S.my));
    const float l = (__builtin_amdgcn_logf(g1.w) - log2_amin) * 1.0001f + 0.004f + 4e-7f * fmaf(fabsf(b), X, c * Y);
    const float A = fmaf(a, a, b * b);
    const float ac = a * c;
    S.all = !(A > 0.0f) || !(ac > 0.0f) || !(l > 0.0f) || !(A < 3e38f);
    const float ia = __builtin_amdgcn_rcpf(A);
    S.dyr = -b * __builtin_amdgcn_rcpf(ac) * __builtin_amdgcn_sqrtf(l);
    S.P = l * ia;
    S.Qc = (ac * ia) * (ac * ia);
    S.Bc = (b * c) * ia;
    return S;
}

// Tiles of tile row ty (tiles 2^tws x 2^ths) that a record's support meets
// inside its pixel box, as (first column, count).
__device__ __noinline__ uint2 support_row(SupportRows S, uint32_t ty, int tws, int ths) {
    const int u0 = (int)(S.pb_x & 0xffffu), u1 = (int)(S.pb_x >> 16);
    const int v0 = (int)(S.pb_y & 0xffffu), v1 = (int)(S.pb_y >> 16);
    const int y0 = max((int)(ty << ths), v0), y1 = min((int)((ty + 1) << ths) - 1, v1);
    const uint32_t f0 = (uint32_t)u0 >> tws;
    if (y0 > y1) return make_uint2(f0, 0u);
    if (S.all) return make_uint2(f0, ((uint32_t)u1 >> tws) - f0 + 1);
    const float dy0 = (float)y0 - S.my, dy1 = (float)y1 - S.my;
    const float yr = fminf(fmaxf(S.dyr, dy0), dy1);
    const float yl = fminf(fmaxf(-S.dyr, dy0), dy1);
    const float er = fmaf(-S.Qc * yr, yr, S.P);
    const float el = fmaf(-S.Qc * yl, yl, S.P);
    if (er < -1e-4f * S.P) return make_uint2(f0, 0u);  // the rows miss the support
    const float R = __builtin_amdgcn_sqrtf(fmaxf(er, 0.0f)) - S.Bc * yr;
    const float L = -__builtin_amdgcn_sqrtf(fmaxf(el, 0.0f)) - S.Bc * yl;
    const float mg = 1e-3f * (fabsf(R) + fabsf(L)) + 1e-3f;
    const float cl = fmaxf(ceilf(S.mx + L - mg), (float)u0);
    const float cr = fminf(floorf(S.mx + R + mg), (float)u1);
    if (!(cl <= cr)) return make_uint2(f0, 0u);
    const uint32_t first = (uint32_t)cl >> tws;
    return make_uint2(first, ((uint32_t)cr >> tws) - first + 1);
}

constexpr int PC_VIEWS = 256;

// STAGED (batches of at most PC_VIEWS views): the cameras' test values are
// read from LDS; otherwise from the view table in global memory.
template <bool STAGED>
__global__ __launch_bounds__(256) void k_project_count(GaussDev g, const ViewDev* __restrict__ views,
                                                       const Header* __restrict__ hdr, int words,
                                                       SetDev st, uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ mask) {
    // the cameras' test values, staged in LDS (every thread reads the same
    // camera at a time; from LDS it waits less than from the scalar cache,
    // which the cameras of a large batch overflow)
    __shared__ CullView s_vf[STAGED ? PC_VIEWS : 1];
    int nv = (int)hdr->n_views;
    if (STAGED) {
        for (int t = threadIdx.x; t < min(nv, PC_VIEWS); t += blockDim.x) s_vf[t] = cull_view(views[t]);
        __syncthreads();
    }
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    GPre P;
    bool ok = pre_gauss(g, i, st, P);
    uint32_t c = 0;
    for (int w = 0; w < words; w++) {
        uint32_t vis = 0;
        int base = 32 * w;
        if (ok && base < nv) {
            uint32_t cand = 0;
            int lim = min(32, nv - base);
            for (int b = 0; b < lim; b++) {
                const int vb = base + b;
                const CullView V = STAGED ? s_vf[vb] : cull_view(views[vb]);
                if (may_be_visible(P, V, st)) cand |= 1u << b;
            }
            while (cand) {
                int b = __ffs(cand) - 1;
                cand &= cand - 1;
                GProj q;
                if (project_exact(P, views[base + b], st, q)) vis |= 1u << b;
            }
        }
        mask[(int64_t)w * g.n + i] = vis;
        c += __popc(vis);
    }
    cnt[i] = c;
}

// -------------------------------------------------------------- prefix sum

constexpr int SC_THREADS = 256;
constexpr int SC_IPT = 8;
constexpr int SC_TILE = SC_THREADS * SC_IPT;
constexpr int SC_MAX_BLOCKS = 1024;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(v, o, 64);
        if (l >= (uint32_t)o) v += y;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* ws, uint32_t& total) {
    uint32_t inc = wave_incl_scan(x);
    int wv = threadIdx.x >> 6;
    if (lane_id() == 63) ws[wv] = inc;
    __syncthreads();
    uint32_t base = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < SC_THREADS / 64; k++) {
        uint32_t t = ws[k];
        if (k < wv) base += t;
        total += t;
    }
    __syncthreads();
    return base + inc - x;
}

__device__ __forceinline__ void chunk_of(uint32_t n, int nblocks, uint32_t& begin, uint32_t& end) {
    uint32_t per = (uint32_t)(((uint64_t)n + nblocks - 1) / nblocks);
    per = (per + SC_TILE - 1) / SC_TILE * SC_TILE;
    uint64_t b = (uint64_t)blockIdx.x * per;
    begin = (uint32_t)min<uint64_t>(b, n);
    end = (uint32_t)min<uint64_t>(b + per, n);
}

__device__ __forceinline__ uint32_t scan_in(const uint32_t* in, const uint32_t* gather, uint32_t i) {
    return gather ? in[gather[i]] : in[i];
}

// Multi-block exclusive scan of n = min(*n_dev, cap) items (n = cap when n_dev is
// null), in[gather[i]] when gather is given: per-block totals here, then
// k_scan_down.  Totals are formed in 64 bits; a block total is stored
// saturated at SCAN_LIMIT, so that k_scan_down can tell a sum of 2^31 or more
// from one that merely wrapped.
constexpr uint64_t SCAN_LIMIT = 0x80000000ull;

__device__ __forceinline__ uint64_t block_sum64(uint64_t x, uint64_t* ws) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += (uint64_t)__shfl_xor((unsigned long long)x, o, 64);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = x;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < SC_THREADS / 64; k++) t += ws[k];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                            const uint32_t* __restrict__ gather,
                                                            const uint32_t* __restrict__ n_dev,
                                                            uint32_t cap, uint32_t* __restrict__ partial) {
    __shared__ uint64_t ws[SC_THREADS / 64];
    const uint32_t n = n_dev ? min(*n_dev, cap) : cap;
    uint32_t begin, end;
    chunk_of(n, gridDim.x, begin, end);
    uint64_t acc = 0;
    for (uint32_t i = begin + threadIdx.x; i < end; i += SC_THREADS) acc += scan_in(in, gather, i);
    const uint64_t total = block_sum64(acc, ws);
    if (threadIdx.x == 0) partial[blockIdx.x] = (uint32_t)min(total, SCAN_LIMIT);
}


// partial[b] holds block b's total (k_scan_reduce); each block adds up the
// totals before it, and block 0 writes the grand total to *total (nullable).
// A grand total of 2^31 or more is not representable by the 32-bit offsets:
// then *total is 0, flags (nullable) gets FLAG_COUNT_OVERFLOW and nothing is
// written to out, so every consumer of the total sees an empty list.
// in and out may be the same array (each item is read and written by one thread).
__global__ __launch_bounds__(SC_THREADS) void k_scan_down(const uint32_t* in,
                                                          const uint32_t* __restrict__ gather,
                                                          uint32_t* out,
                                                          const uint32_t* __restrict__ n_dev, uint32_t cap,
                                                          const uint32_t* __restrict__ partial,
                                                          uint32_t* __restrict__ total_out,
                                                          uint32_t* __restrict__ flags) {
    __shared__ uint32_t ws[SC_THREADS / 64];
    __shared__ uint64_t ws64[SC_THREADS / 64];
    const uint32_t n = n_dev ? min(*n_dev, cap) : cap;
    uint32_t begin, end;
    chunk_of(n, gridDim.x, begin, end);
    uint64_t before = 0, all = 0;
    for (uint32_t t = threadIdx.x; t < gridDim.x; t += SC_THREADS) {
        const uint64_t p = partial[t];
        all += p;
        before += t < blockIdx.x ? p : 0u;
    }
    uint32_t run = (uint32_t)block_sum64(before, ws64);
    all = block_sum64(all, ws64);
    if (all >= SCAN_LIMIT) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (total_out) *total_out = 0u;
            if (flags) atomicOr(flags, FLAG_COUNT_OVERFLOW);
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = (uint32_t)all;
    for (uint32_t t0 = begin; t0 < end; t0 += SC_TILE) {
        // thread owns SC_IPT consecutive items
        uint32_t v[SC_IPT];
        uint32_t first = t0 + threadIdx.x * SC_IPT;
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < SC_IPT; j++) {
            uint32_t idx = first + j;
            v[j] = idx < end ? scan_in(in, gather, idx) : 0;
            sum += v[j];
        }
        uint32_t total;
        uint32_t ex = block_excl_scan(sum, ws, total) + run;
#pragma unroll
        for (int j = 0; j < SC_IPT; j++) {
            uint32_t idx = first + j;
            if (idx < end) out[idx] = ex;
            ex += v[j];
        }
        run += total;
    }
}

// ------------------------------------------------------------- radix sort
// Stable LSD sort with digits of up to 11 bits (2048 bins).  A fixed grid of
// blocks splits the input into equal chunks; per pass: per-block digit
// histograms (upsweep, one LDS atomic add per item into per-wave tables), the
// offsets of every (digit, block), and a scatter in
// which every wave ranks its items with 64-lane ballots (peers with the same
// digit), preserving input order within the block; with 8-bit digits the
// block then sorts its tile in LDS and writes each digit's run from
// consecutive lanes.  Up to 128 blocks compute their offsets themselves from
// the block-major histogram table; more blocks scan a digit-major table with
// the multi-block scan.

// 16 items per lane (a 4096-item tile per block step of 256 threads): each
// digit's run per step is twice as long as with 8, so fewer of the scatter's
// writes are partial cache lines (measured 3% faster on 192M pairs, 6% on
// 40M).  Inputs of at least RS_BIG_ITEMS take blocks of 512 threads (8192-item
// tiles, runs twice as long again); smaller ones keep 256, which gives them
// twice as many blocks.
constexpr int RS_THREADS = 256;
constexpr int RS_THREADS_BIG = 512;
constexpr int RS_IPT = 16;
constexpr int RS_SEG = 64 * RS_IPT;         // items per wave per tile
constexpr int RS_TILE = RS_THREADS * RS_IPT;  // items per block per tile (256 threads)
constexpr int RS_MAX_BLOCKS = 1024;
constexpr uint64_t RS_BIG_ITEMS = (uint64_t)RS_MAX_BLOCKS * RS_THREADS_BIG * RS_IPT;
constexpr int RS_FUSED_BLOCKS = 128;
constexpr int RS_MAX_DB = 11;

template <int DB>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, uint64_t valid) {
    uint64_t m = valid;
#pragma unroll
    for (int b = 0; b < DB; b++) {
        uint32_t bit = (d >> b) & 1u;
        uint64_t bal = __ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

template <int TILE>
__device__ __forceinline__ void rs_chunk(uint32_t n, uint32_t& begin, uint32_t& end) {
    uint32_t per = (uint32_t)(((uint64_t)n + gridDim.x - 1) / gridDim.x);
    per = (per + TILE - 1) / TILE * TILE;
    uint64_t b = (uint64_t)blockIdx.x * per;
    begin = (uint32_t)min<uint64_t>(b, n);
    end = (uint32_t)min<uint64_t>(b + per, n);
}

// Digit of this pass: `bits` (<= DB) bits from `shift`.
// hist layout: digit-major [d][block] when block_major == 0 (scanned as a
// whole), block-major [block][d] otherwise (read directly by the scatter).
template <int DB, int NT>
__global__ __launch_bounds__(NT) void k_rs_upsweep(const uint32_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ n_dev, uint32_t cap,
                                                           int shift, int bits, uint32_t* __restrict__ hist,
                                                           int block_major) {
    constexpr int NB = 1 << DB;
    constexpr int WAVES = NT / 64, TILE = NT * RS_IPT;
    // each wave counts into CP copies of its table (lane l into copy l % CP),
    // so that a skewed digit (few tiles or views dominating a pass) does not
    // serialise a whole wave's atomics on one LDS word
    constexpr int CP = DB <= 8 ? 4 : 1;
    __shared__ uint32_t h[WAVES * CP][NB];
    const int tid = threadIdx.x, wv = tid >> 6;
    const int cp = wv * CP + (int)(lane_id() % CP);
    const uint32_t mask = (1u << bits) - 1u;
    for (int i = tid; i < WAVES * CP * NB; i += NT) (&h[0][0])[i] = 0;
    __syncthreads();
    uint32_t n = min(*n_dev, cap);
    uint32_t begin, end;
    rs_chunk<TILE>(n, begin, end);
    // the scatter's tiling: RS_IPT coalesced loads per lane in flight, then
    // their RS_IPT additions to the wave's table
    for (uint32_t t0 = begin; t0 < end; t0 += TILE) {
        const uint32_t seg = t0 + wv * RS_SEG;
        uint32_t k[RS_IPT];
#pragma unroll
        for (int j = 0; j < RS_IPT; j++) {
            const uint32_t idx = seg + j * 64 + lane_id();
            k[j] = idx < end ? keys[idx] : 0u;
        }
#pragma unroll
        for (int j = 0; j < RS_IPT; j++) {
            const uint32_t idx = seg + j * 64 + lane_id();
            if (idx < end) atomicAdd(&h[cp][(k[j] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < NB; d += NT) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < WAVES * CP; w++) c += h[w][d];
        if (block_major)
            hist[(uint64_t)blockIdx.x * NB + d] = c;
        else
            hist[(uint64_t)d * gridDim.x + blockIdx.x] = c;
    }
}

// STAGE: a tile's items are first placed at their block-local sorted positions
// in LDS and written out in that order, so that consecutive lanes write the
// consecutive addresses of a digit's run; otherwise each item is written from
// where its wave ranked it.
template <int DB, bool STAGE, int NT>
__global__ __launch_bounds__(NT) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout,
                                                           const uint32_t* __restrict__ n_dev, uint32_t cap,
                                                           int shift, int bits, const uint32_t* __restrict__ hist,
                                                           int block_major, const uint32_t* __restrict__ gsrc,
                                                           uint32_t* __restrict__ gout) {
    constexpr int NB = 1 << DB;
    constexpr int WAVES = NT / 64, TILE = NT * RS_IPT;
    constexpr int DPT = NB / NT > 0 ? NB / NT : 1;  // digits per thread
    __shared__ uint32_t wh[WAVES][NB];
    __shared__ uint32_t bbase[NB];
    __shared__ uint32_t ws[WAVES];
    constexpr int SB = STAGE ? NB : 1, ST = STAGE ? TILE : 1;
    __shared__ uint32_t lst[SB], tcnt[SB];
    __shared__ uint32_t s_k[ST], s_v[ST];
    const int tid = threadIdx.x, wv = tid >> 6;
    const uint32_t lane = lane_id();
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t n = min(*n_dev, cap);
    uint32_t begin, end;
    rs_chunk<TILE>(n, begin, end);
    if (block_major) {
        // offset of digit d for this block = count of smaller digits in all
        // blocks + count of digit d in earlier blocks; thread tid owns the
        // DPT consecutive digits from tid * DPT
        uint32_t tot[DPT], pre[DPT];
#pragma unroll
        for (int j = 0; j < DPT; j++) tot[j] = pre[j] = 0;
        if (tid * DPT < NB) {
            // independent loads, unrolled so that many are in flight
#pragma unroll(DPT == 1 ? 32 : 8)
            for (uint32_t b = 0; b < gridDim.x; b++) {
                uint32_t c[DPT];
                if constexpr (DPT % 4 == 0) {
#pragma unroll
                    for (int j = 0; j < DPT; j += 4) {
                        const uint4 q = *reinterpret_cast<const uint4*>(hist + (uint64_t)b * NB + tid * DPT + j);
                        c[j] = q.x;
                        c[j + 1] = q.y;
                        c[j + 2] = q.z;
                        c[j + 3] = q.w;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < DPT; j++) c[j] = hist[(uint64_t)b * NB + tid * DPT + j];
                }
                const bool earlier = b < blockIdx.x;
#pragma unroll
                for (int j = 0; j < DPT; j++) {
                    tot[j] += c[j];
                    pre[j] += earlier ? c[j] : 0u;
                }
            }
        }
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < DPT; j++) mine += tot[j];
        const uint32_t inc = wave_incl_scan(mine);
        if (lane == 63) ws[wv] = inc;
        __syncthreads();
        uint32_t base = inc - mine;
#pragma unroll
        for (int w = 0; w < WAVES; w++)
            if (w < wv) base += ws[w];
        if (tid * DPT < NB) {
#pragma unroll
            for (int j = 0; j < DPT; j++) {
                bbase[tid * DPT + j] = base + pre[j];
                base += tot[j];
            }
        }
    } else {
        for (int d = tid; d < NB; d += NT) bbase[d] = hist[(uint64_t)d * gridDim.x + blockIdx.x];
    }
    for (uint32_t t0 = begin; t0 < end; t0 += TILE) {
        for (int i = tid; i < WAVES * NB; i += NT) (&wh[0][0])[i] = 0;
        __syncthreads();
        uint32_t seg = t0 + wv * RS_SEG;
        uint32_t k[RS_IPT], v[RS_IPT], pos[RS_IPT];
#pragma unroll
        for (int j = 0; j < RS_IPT; j++) {
            uint32_t idx = seg + j * 64 + lane;
            bool valid = idx < end;
            k[j] = valid ? kin[idx] : 0u;
            v[j] = valid ? vin[idx] : 0u;
        }
#pragma unroll
        for (int j = 0; j < RS_IPT; j++) {
            uint32_t idx = seg + j * 64 + lane;
            bool valid = idx < end;
            uint32_t d = (k[j] >> shift) & mask;
            uint64_t vm = __ballot(valid);
            uint64_t m = digit_peers<DB>(d, vm);
            uint32_t before = valid ? wh[wv][d] : 0u;
            pos[j] = before + (uint32_t)__popcll(m & lanemask_lt());
            if (valid && lane == (uint32_t)__builtin_ctzll(m)) wh[wv][d] = before + (uint32_t)__popcll(m);
        }
        __syncthreads();
        if constexpr (!STAGE) {
            for (int d = tid; d < NB; d += NT) {
                uint32_t run = bbase[d];
#pragma unroll
                for (int w = 0; w < WAVES; w++) {
                    uint32_t c = wh[w][d];
                    wh[w][d] = run;
                    run += c;
                }
                bbase[d] = run;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RS_IPT; j++) {
                uint32_t idx = seg + j * 64 + lane;
                if (idx < end) {
                    uint32_t d = (k[j] >> shift) & mask;
                    uint32_t dst = wh[wv][d] + pos[j];
                    kout[dst] = k[j];
                    vout[dst] = v[j];
                    if (gsrc) gout[dst] = gsrc[v[j]];
                }
            }
        } else {
            // per digit: the waves' offsets inside the tile's run of the digit, and the run length
            for (int d = tid; d < NB; d += NT) {
                uint32_t run = 0;
#pragma unroll
                for (int w = 0; w < WAVES; w++) {
                    uint32_t c = wh[w][d];
                    wh[w][d] = run;
                    run += c;
                }
                tcnt[d] = run;
            }
            __syncthreads();
            // lst[d]: start of digit d's run in the tile's sorted order (thread tid owns
            // the DPT consecutive digits from tid * DPT)
            {
                uint32_t c[DPT];
                uint32_t mine = 0;
#pragma unroll
                for (int j = 0; j < DPT; j++) {
                    c[j] = tid * DPT < NB ? tcnt[tid * DPT + j] : 0u;
                    mine += c[j];
                }
                const uint32_t inc = wave_incl_scan(mine);
                if (lane == 63) ws[wv] = inc;
                __syncthreads();
                uint32_t base = inc - mine;
#pragma unroll
                for (int w = 0; w < WAVES; w++)
                    if (w < wv) base += ws[w];
                if (tid * DPT < NB) {
#pragma unroll
                    for (int j = 0; j < DPT; j++) {
                        lst[tid * DPT + j] = base;
                        base += c[j];
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RS_IPT; j++) {
                uint32_t idx = seg + j * 64 + lane;
                if (idx < end) {
                    uint32_t d = (k[j] >> shift) & mask;
                    uint32_t lp = lst[d] + wh[wv][d] + pos[j];
                    s_k[lp] = k[j];
                    s_v[lp] = v[j];
                }
            }
            __syncthreads();
            const uint32_t tn = min<uint32_t>(TILE, end - t0);
            for (uint32_t i = tid; i < tn; i += NT) {
                const uint32_t kk = s_k[i];
                const uint32_t d = (kk >> shift) & mask;
                const uint32_t dst = bbase[d] + (i - lst[d]);
                const uint32_t vv = s_v[i];
                kout[dst] = kk;
                vout[dst] = vv;
                if (gsrc) gout[dst] = gsrc[vv];
            }
            __syncthreads();
            for (int d = tid; d < NB; d += NT) bbase[d] += tcnt[d];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- binning

// A block covers EM_ITEMS consecutive pairs and each thread EM_RUN
// consecutive ones.  The depth-ordered records spanning the block are found
// by one binary search over the pair offsets and their offsets staged in LDS.
// A record whose support meets every tile of its box is enumerated in
// row-major order directly.  For the others the block evaluates every tile
// row of their rectangles once, in parallel (one support_row call per row),
// into an LDS table of (first column, count) and its prefix; a thread then
// finds the row of each of its pairs by binary search.  A block whose records
// have more than EM_ROWS such rows falls back to a per-thread cursor that
// walks the rows up to its first pair.  Output is written in depth order,
// EM_RUN pairs per 16-byte store.
constexpr int EM_THREADS = 256;
constexpr int EM_RUN = 4;
constexpr int EM_ITEMS = EM_THREADS * EM_RUN;
constexpr int EM_ROWS = 2048;
constexpr int EM_ROWS_PT = EM_ROWS / EM_THREADS;

__device__ __forceinline__ uint32_t last_le(const uint32_t* a, uint32_t n, uint32_t x) {
    // largest i < n with a[i] <= x (a[0] == 0 <= x)
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (a[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same search over global memory by one wave in 64-way steps: the lanes
// probe 64 evenly spaced positions of the current range; the probes with
// a[p] <= x form a prefix of the lanes (a is non-decreasing), so their count
// narrows the range 64-fold per step.  All values are wave-uniform.
__device__ __forceinline__ uint32_t wave_last_le(const uint32_t* __restrict__ a, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n - 1;  // a[lo] <= x; the answer lies in [lo, hi]
    const uint32_t lane = lane_id();
    while (hi > lo) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint64_t p = (uint64_t)lo + (uint64_t)step * (lane + 1);
        const bool le = p <= hi && a[p] <= x;
        const uint32_t c = (uint32_t)__popcll(__ballot(le));
        const uint32_t nlo = lo + step * c;
        hi = (uint32_t)min<uint64_t>(hi, (uint64_t)lo + (uint64_t)step * (c + 1) - 1);
        lo = nlo;
    }
    return lo;
}

// Position within one record's pairs.
struct PairCursor {
    uint32_t r, tile_off, tiles_x, tx0, nx, ty0, ty1;
    bool full;       // every tile of the box
    SupportRows S;   // when !full
    uint32_t li;     // pair index within the record (full)
    uint32_t ty, first, cnt, rem;  // current support row (!full)
};

// Next row with a nonzero count at or after c.ty; false if none is left.
__device__ __forceinline__ bool cursor_row(PairCursor& c, int tws, int ths) {
    for (; c.ty <= c.ty1; c.ty++) {
        const uint2 fc = support_row(c.S, c.ty, tws, ths);
        if (fc.y) {
            c.first = fc.x;
            c.cnt = fc.y;
            return true;
        }
    }
    return false;
}

__device__ __forceinline__ void cursor_open(PairCursor& c, const Records& rec, const ViewDev* views, uint32_t r,
                                            uint32_t li, int tws, int ths, float log2_amin, uint32_t* flags) {
    c.r = r;
    const EmitRec e = rec.emit[r];
    const uint2 rc = e.rect;
    c.tx0 = rc.x & 0xffffu;
    c.nx = (rc.x >> 16) - c.tx0 + 1;
    c.ty0 = rc.y & 0xffffu;
    c.ty1 = rc.y >> 16;
    const ViewDev& V = views[e.view];
    c.tile_off = V.tile_off;
    c.tiles_x = (uint32_t)V.tiles_x;
    c.full = e.ntiles == c.nx * (c.ty1 - c.ty0 + 1);
    c.li = li;
    if (c.full) return;
    c.S = support_setup(e.g0, e.g1, e.pbox, log2_amin);
    c.ty = c.ty0;
    uint32_t rem = li;
    while (cursor_row(c, tws, ths)) {
        if (rem < c.cnt) {
            c.rem = rem;
            return;
        }
        rem -= c.cnt;
        c.ty++;
    }
    // a support that meets no tile still owns one pair, its box's first tile;
    // anything else would be a counting mismatch
    if (li != 0) atomicOr(flags, FLAG_BIN_MISMATCH);
    c.full = true;
    c.nx = 1;
    c.li = 0;
}

__device__ __forceinline__ uint32_t cursor_tile(const PairCursor& c) {
    if (c.full) return c.tile_off + (c.ty0 + c.li / c.nx) * c.tiles_x + c.tx0 + c.li % c.nx;
    return c.tile_off + c.ty * c.tiles_x + c.first + c.rem;
}

__device__ __forceinline__ void cursor_next(PairCursor& c, int tws, int ths) {
    c.li++;
    if (c.full) return;
    if (++c.rem < c.cnt) return;
    c.rem = 0;
    c.ty++;
    cursor_row(c, tws, ths);  // the caller knows the record has another pair
}

// Record emission, one thread per record so that the record arrays are
// written in contiguous runs: the records of Gaussian i are rec_off[i] ...
// rec_off[i] + cnt[i] - 1, one per visible view in view order.  A block finds
// the Gaussians spanning its records with two wave searches and stages their
// offsets in LDS (a span wider than PE_LDS, i.e. a long run of culled
// Gaussians, is searched in global memory instead).
constexpr int PE_THREADS = 256;
constexpr uint32_t PE_LDS = 2048;
constexpr uint32_t PE_PRE = 64;
// Records with more tile rows than this have their rows counted by the
// whole wave (a wave would otherwise loop as long as its tallest record).
constexpr uint32_t PE_ROWS_SELF = 4;
// Visibility mask words a record's view search loads at once.
constexpr int PE_MASK_WORDS = 8;

__device__ __forceinline__ float readlane_f(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Position of the k-th (from 0) set bit of x (k < popcount(x)), by halving.
__device__ __forceinline__ int nth_set_bit(uint32_t x, uint32_t k) {
    int pos = 0;
#pragma unroll
    for (int h = 16; h > 0; h >>= 1) {
        const uint32_t c = (uint32_t)__popc(x & ((1u << h) - 1u));
        const bool up = k >= c;
        k = up ? k - c : k;
        x = up ? x >> h : x;
        pos += up ? h : 0;
    }
    return pos;
}

static_assert(PE_THREADS == PE_CHUNK, "a block step of the record emission is one chunk");

// The Gaussians that own the first and the last record of every chunk of
// PE_CHUNK records (chunk_g[2c], chunk_g[2c + 1]): each Gaussian writes the
// chunk ends that fall among its records, so every entry has one writer.
// Record p is owned by the Gaussian i with rec_off[i] <= p < rec_off[i] +
// cnt[i], which is the last Gaussian whose first record is at or before p.
__global__ __launch_bounds__(256) void k_chunk_owners(const uint32_t* __restrict__ cnt,
                                                      const uint32_t* __restrict__ rec_off, int64_t n,
                                                      const uint32_t* __restrict__ R_dev, uint32_t rec_cap,
                                                      uint32_t* __restrict__ chunk_g) {
    const uint32_t R = min(*R_dev, rec_cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cnt[i];
        const uint32_t a = rec_off[i];
        if (c == 0 || a >= R) continue;
        const uint32_t b = (uint32_t)min<uint64_t>((uint64_t)a + c, R);  // records [a, b)
        for (uint32_t k = a / PE_CHUNK; k <= (b - 1) / PE_CHUNK; k++) {
            const uint32_t first = k * PE_CHUNK;
            const uint32_t last = (uint32_t)min<uint64_t>((uint64_t)first + PE_CHUNK - 1, R - 1);
            if (first >= a) chunk_g[2 * k] = (uint32_t)i;
            if (last < b) chunk_g[2 * k + 1] = (uint32_t)i;
        }
    }
}

__global__ __launch_bounds__(PE_THREADS) void k_project_emit(GaussDev g, const ViewDev* __restrict__ views,
                                                             int words, SetDev st, int tws, int ths,
                                                             const uint32_t* __restrict__ mask,
                                                             const uint32_t* __restrict__ rec_off,
                                                             const uint32_t* __restrict__ R_dev, uint32_t rec_cap,
                                                             Records rec, uint32_t* __restrict__ sortkey,
                                                             uint32_t* __restrict__ order, int write_attr,
                                                             const uint32_t* __restrict__ chunk_g,
                                                             uint32_t* __restrict__ flags) {
    __shared__ uint32_t s_off[PE_LDS];
    __shared__ GPre s_pre[PE_PRE];
    const uint32_t Rall = *R_dev;
    if (blockIdx.x == 0 && threadIdx.x == 0 && Rall > rec_cap) atomicOr(flags, FLAG_REC_OVERFLOW);
    const uint32_t R = min(Rall, rec_cap);
    const uint32_t n = (uint32_t)g.n;
    for (uint32_t k0 = blockIdx.x * PE_THREADS; k0 < R; k0 += gridDim.x * PE_THREADS) {
        const uint32_t k1 = min(k0 + PE_THREADS, R);  // exclusive
        __syncthreads();
        // the Gaussians owning the chunk's first and last records
        const uint32_t lo = chunk_g[2 * (k0 / PE_CHUNK)], ng = chunk_g[2 * (k0 / PE_CHUNK) + 1] - lo + 1;
        const bool staged = ng <= PE_LDS;
        if (staged)
            for (uint32_t j = threadIdx.x; j < ng; j += PE_THREADS) s_off[j] = rec_off[lo + j];
        // the per-Gaussian part of the projection, once per Gaussian when few
        // Gaussians own the block's records (many views see each)
        const bool shared_pre = ng <= PE_PRE;
        if (shared_pre && threadIdx.x < ng) pre_gauss(g, lo + threadIdx.x, st, s_pre[threadIdx.x]);
        __syncthreads();
        const uint32_t pos = k0 + threadIdx.x;
        const bool valid = pos < k1;
        // the record's support rows: a record with few tile rows counts its
        // own; the wave counts the rows of the others together below
        SupportRows S{};
        uint32_t nt = 0, ty0 = 0, ny = 0;
        if (valid) {
            // owner Gaussian: the last one whose first record is at or before pos
            const uint32_t ii = staged ? last_le(s_off, ng, pos) : last_le(rec_off + lo, ng, pos);
            const uint32_t i = lo + ii;
            // its (pos - rec_off[i])-th visible view; the mask words are
            // loaded eight at a time (256 views), all in flight together,
            // then scanned for the word that holds it
            uint32_t kk = pos - (staged ? s_off[ii] : rec_off[i]);
            int v = 0;
            bool found = false;
            for (int w0 = 0; w0 < words && !found; w0 += PE_MASK_WORDS) {
                uint32_t vis[PE_MASK_WORDS];
#pragma unroll
                for (int q = 0; q < PE_MASK_WORDS; q++)
                    vis[q] = w0 + q < words ? mask[(int64_t)(w0 + q) * n + i] : 0u;
                uint32_t word = 0;
                int wsel = 0;
#pragma unroll
                for (int q = 0; q < PE_MASK_WORDS; q++) {
                    const uint32_t c = (uint32_t)__popc(vis[q]);
                    const bool here = !found && kk < c;
                    word = here ? vis[q] : word;
                    wsel = here ? w0 + q : wsel;
                    kk = !found && !here ? kk - c : kk;
                    found = found || here;
                }
                if (found) v = 32 * wsel + nth_set_bit(word, kk);
            }
            GPre P;
            if (shared_pre) P = s_pre[i - lo];
            else pre_gauss(g, i, st, P);
            const ViewDev& V = views[v];
            GProj q;
            project_exact(P, V, st, q);
            float mxh = (float)q.mx, myh = (float)q.my;
            const float4 g0 = make_float4(mxh, myh, (float)(q.mx - (double)mxh), (float)(q.my - (double)myh));
            double det = q.cxx * q.cyy - q.cxy * q.cxy;
            // Sigma_2D = C C^T (Cholesky); M = sqrt(log2e / 2) C^-1
            double c00 = sqrt(q.cxx);
            double c10 = q.cxy / c00;
            double c11 = sqrt(det / q.cxx);
            double sl = sqrt(0.5 * LOG2E);
            const float4 g1 = make_float4((float)(sl / c00), (float)(-sl * c10 / (c00 * c11)), (float)(sl / c11),
                                          (float)P.o);
            rec.q64[pos] = make_double4(q.cyy / det, -q.cxy / det, q.cxx / det, 0.0);
            float depth = (float)q.t[2];
            const int64_t gi = i;
            if (write_attr) {
                if (g.colors)
                    rec.attr[pos] = make_float4(g.colors[gi], g.colors[g.n + gi], g.colors[2 * g.n + gi], depth);
                else
                    rec.attr[pos] = make_float4(0.0f, 0.0f, 0.0f, depth);
            }
            uint32_t tx0 = (uint32_t)q.u0 >> tws, tx1 = (uint32_t)q.u1 >> tws;
            ty0 = (uint32_t)q.v0 >> ths;
            const uint32_t ty1 = (uint32_t)q.v1 >> ths;
            ny = ty1 - ty0 + 1;
            const uint2 pb = make_uint2((uint32_t)q.u0 | ((uint32_t)q.u1 << 16),
                                        (uint32_t)q.v0 | ((uint32_t)q.v1 << 16));
            sortkey[pos] = __float_as_uint(depth);
            S = support_setup(g0, g1, pb, st.log2_amin);
            if (ny <= PE_ROWS_SELF)
                for (uint32_t ty = ty0; ty <= ty1; ty++) nt += support_row(S, ty, tws, ths).y;
            EmitRec e;
            e.g0 = g0;
            e.g1 = g1;
            e.pbox = pb;
            e.rect = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
            e.ntiles = 0;  // written below
            e.view = (uint32_t)v;
            e.unc = __float_as_uint(g.uncert ? g.uncert[gi] : 0.0f);
            e.gid = i;
            rec.emit[pos] = e;
            order[pos] = pos;
        }
        // every lane takes one row of the record at a time; the per-row
        // counts are integers, so their sum does not depend on the split
        uint64_t big = __ballot(valid && ny > PE_ROWS_SELF);
        while (big) {
            const int src = __builtin_ctzll(big);
            big &= big - 1;
            SupportRows B;
            B.mx = readlane_f(S.mx, src);
            B.my = readlane_f(S.my, src);
            B.dyr = readlane_f(S.dyr, src);
            B.P = readlane_f(S.P, src);
            B.Qc = readlane_f(S.Qc, src);
            B.Bc = readlane_f(S.Bc, src);
            B.pb_x = (uint32_t)__builtin_amdgcn_readlane((int)S.pb_x, src);
            B.pb_y = (uint32_t)__builtin_amdgcn_readlane((int)S.pb_y, src);
            B.all = __builtin_amdgcn_readlane(S.all, src);
            const uint32_t bty0 = (uint32_t)__builtin_amdgcn_readlane((int)ty0, src);
            const uint32_t bny = (uint32_t)__builtin_amdgcn_readlane((int)ny, src);
            uint32_t part = 0;
            for (uint32_t r = lane_id(); r < bny; r += 64) part += support_row(B, bty0 + r, tws, ths).y;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += (uint32_t)__shfl_xor((int)part, o, 64);
            if ((int)lane_id() == src) nt = part;
        }
        if (valid) {
            // pairs: the tiles the support meets (a subset of the box's
            // tiles); at least one, so that every record owns a pair
            rec.ntiles[pos] = max(nt, 1u);
            rec.emit[pos].ntiles = max(nt, 1u);
        }
    }
}

// Record offsets per thread for one chunk's EM_ITEMS + 1 entries.
constexpr int EM_OFF_PT = (EM_ITEMS + 1 + EM_THREADS - 1) / EM_THREADS;

// Loads (issues) a chunk's record offsets from its first record lo and the
// ids of the records the thread sets up; entries past the last record read as
// "after every pair" (offsets) and 0 (ids).
__device__ __forceinline__ void em_load_chunk(const uint32_t* __restrict__ inst_off,
                                              const uint32_t* __restrict__ order, uint32_t R, uint32_t lo,
                                              uint32_t (&off)[EM_OFF_PT], uint32_t (&rid)[EM_RUN]) {
    const uint32_t navail = min<uint32_t>(EM_ITEMS + 1, R - lo);
#pragma unroll
    for (int m = 0; m < EM_OFF_PT; m++) {
        const uint32_t q = threadIdx.x + m * EM_THREADS;
        off[m] = q < navail ? inst_off[lo + q] : 0xffffffffu;
    }
#pragma unroll
    for (int q = 0; q < EM_RUN; q++) {
        const uint32_t jr = threadIdx.x * EM_RUN + q;
        rid[q] = jr < R - lo ? order[lo + jr] : 0u;
    }
}

__global__ __launch_bounds__(EM_THREADS, 4) void k_emit_instances(const uint32_t* __restrict__ order,
                                                               const uint32_t* __restrict__ R_dev, uint32_t rec_cap,
                                                               const uint32_t* __restrict__ K_dev, Records rec,
                                                               const ViewDev* __restrict__ views,
                                                               const uint32_t* __restrict__ inst_off,
                                                               int tws, int ths, float log2_amin,
                                                               uint32_t inst_cap, uint32_t* __restrict__ tile_key,
                                                               uint32_t* __restrict__ inst_rec,
                                                               uint2* __restrict__ ranges, uint32_t tiles_cap,
                                                               uint32_t* __restrict__ flags) {
    __shared__ uint32_t s_off[EM_ITEMS + 1];
    __shared__ uint32_t s_roff[EM_ITEMS + 1];  // first table row of each record (prefix of row counts)
    __shared__ uint32_t s_row[EM_ROWS];        // first tile column | pairs of the row << 16
    __shared__ uint32_t s_rpre[EM_ROWS + 1];   // pairs of all table rows before this one
    // per record of the chunk: its id, its first tile row's global tile id
    // minus tx0, tx0 | nx << 16, and its view's tiles per row
    __shared__ uint32_t s_rid[EM_ITEMS], s_tbase[EM_ITEMS], s_tx[EM_ITEMS];
    __shared__ uint16_t s_tpr[EM_ITEMS];
    __shared__ uint32_t ws[SC_THREADS / 64];
    __shared__ uint32_t s_lo;
    // every tile starts empty; k_tile_ranges later fills the occupied ones
    // (nothing reads the ranges in between), and an overflow leaves them empty
    for (uint32_t t = blockIdx.x * EM_THREADS + threadIdx.x; t < tiles_cap; t += gridDim.x * EM_THREADS)
        ranges[t] = make_uint2(0u, 0u);
    if (*flags & (FLAG_REC_OVERFLOW | FLAG_COUNT_OVERFLOW)) return;
    const uint32_t R = min(*R_dev, rec_cap);
    const uint32_t Kall = *K_dev;
    if (threadIdx.x == 0 && blockIdx.x == 0 && Kall > inst_cap) atomicOr(flags, FLAG_INST_OVERFLOW);
    const uint32_t K = min(Kall, inst_cap);
    if (R == 0) return;
    // each block takes one contiguous run of whole EM_ITEMS chunks, so that
    // the records of a chunk follow those of the previous one: one search in
    // global memory per block, then one coalesced load of the next EM_ITEMS + 1
    // record offsets per chunk
    const uint32_t per = (uint32_t)(((uint64_t)K + (uint64_t)gridDim.x * EM_ITEMS - 1) /
                                    ((uint64_t)gridDim.x * EM_ITEMS)) * EM_ITEMS;
    const uint32_t kbeg = (uint32_t)min<uint64_t>((uint64_t)blockIdx.x * per, K);
    const uint32_t kend = (uint32_t)min<uint64_t>((uint64_t)kbeg + per, K);
    if (kbeg >= kend) return;
    if (threadIdx.x < 64) {
        const uint32_t lo0 = wave_last_le(inst_off, R, kbeg);
        if (threadIdx.x == 0) s_lo = lo0;
    }
    __syncthreads();
    uint32_t lo_chunk = s_lo;
    // the first chunk's record offsets and ids; every chunk then issues the
    // next one's loads before it sets up its own records, so that they arrive
    // while it works
    uint32_t pf_off[EM_OFF_PT], pf_rid[EM_RUN];
    em_load_chunk(inst_off, order, R, lo_chunk, pf_off, pf_rid);
    for (uint32_t k0 = kbeg; k0 < kend; k0 += EM_ITEMS) {
        const uint32_t k1 = min(k0 + EM_ITEMS, kend);  // exclusive
        const uint32_t lo = lo_chunk;
        __syncthreads();
        // the offsets of the records from the first one spanning the chunk
        // (every record owns at least one pair, so at most EM_ITEMS records
        // span it); entries past the last record read as "after every pair"
        const uint32_t navail = min<uint32_t>(EM_ITEMS + 1, R - lo);
#pragma unroll
        for (int m = 0; m < EM_OFF_PT; m++) {
            const uint32_t q = threadIdx.x + m * EM_THREADS;
            if (q < EM_ITEMS + 1) s_off[q] = pf_off[m];
        }
        __syncthreads();
        const uint32_t nrec = last_le(s_off, navail, k1 - 1) + 1;
        lo_chunk = lo + last_le(s_off, navail, k1);  // the next chunk's first record
        uint32_t rids[EM_RUN];
#pragma unroll
        for (int q = 0; q < EM_RUN; q++) rids[q] = pf_rid[q];
        if (k1 < kend) em_load_chunk(inst_off, order, R, lo_chunk, pf_off, pf_rid);
        // table rows of the records (EM_RUN records per thread): every tile
        // row of a record that is not enumerated directly
        uint32_t nr[EM_RUN];
        uint32_t nsum = 0;
#pragma unroll
        for (int q = 0; q < EM_RUN; q++) {
            const uint32_t jr = threadIdx.x * EM_RUN + q;
            nr[q] = 0;
            if (jr < nrec) {
                const uint32_t rid = rids[q];
                const EmitRec e = rec.emit[rid];
                const uint32_t tx0 = e.rect.x & 0xffffu, ty0 = e.rect.y & 0xffffu;
                const uint32_t nx = (e.rect.x >> 16) - tx0 + 1;
                const uint32_t ny = (e.rect.y >> 16) - ty0 + 1;
                nr[q] = e.ntiles == nx * ny ? 0u : ny;
                const ViewDev& V = views[e.view];
                s_rid[jr] = rid;
                s_tbase[jr] = V.tile_off + ty0 * (uint32_t)V.tiles_x;
                s_tx[jr] = tx0 | (nx << 16);
                s_tpr[jr] = (uint16_t)V.tiles_x;
            }
            nsum += nr[q];
        }
        uint32_t total_rows;
        uint32_t rbase = block_excl_scan(nsum, ws, total_rows);
#pragma unroll
        for (int q = 0; q < EM_RUN; q++) {
            const uint32_t jr = threadIdx.x * EM_RUN + q;
            if (jr < nrec) s_roff[jr] = rbase;
            rbase += nr[q];
        }
        if (threadIdx.x == 0) s_roff[nrec] = total_rows;
        const bool staged = total_rows <= (uint32_t)EM_ROWS;
        if (staged) {
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < total_rows; t += EM_THREADS) {
                const uint32_t jr = last_le(s_roff, nrec, t);
                const EmitRec e = rec.emit[s_rid[jr]];
                const SupportRows S = support_setup(e.g0, e.g1, e.pbox, log2_amin);
                const uint2 fc = support_row(S, (e.rect.y & 0xffffu) + (t - s_roff[jr]), tws, ths);
                s_row[t] = fc.x | (fc.y << 16);
            }
            __syncthreads();
            // exclusive prefix of the row counts over the whole table
            uint32_t c[EM_ROWS_PT];
            uint32_t csum = 0;
#pragma unroll
            for (int q = 0; q < EM_ROWS_PT; q++) {
                const uint32_t t = threadIdx.x * EM_ROWS_PT + q;
                c[q] = t < total_rows ? s_row[t] >> 16 : 0u;
                csum += c[q];
            }
            uint32_t all;
            uint32_t pre = block_excl_scan(csum, ws, all);
#pragma unroll
            for (int q = 0; q < EM_ROWS_PT; q++) {
                const uint32_t t = threadIdx.x * EM_ROWS_PT + q;
                if (t < total_rows) s_rpre[t] = pre;
                pre += c[q];
            }
            if (threadIdx.x == 0) s_rpre[total_rows] = all;
        }
        __syncthreads();
        const uint32_t kb = k0 + threadIdx.x * EM_RUN;
        if (kb >= k1) continue;
        uint32_t tk[EM_RUN], tr[EM_RUN];
        const int n = (int)min<uint32_t>(EM_RUN, k1 - kb);
        if (staged) {
            uint32_t j = last_le(s_off, nrec, kb);
            uint32_t jc = 0xffffffffu, r = 0, base = 0, t0 = 0, t1 = 0, tx0 = 0, nx = 1, tb = 0, tiles_x = 0;
#pragma unroll
            for (int q = 0; q < EM_RUN; q++) {
                if (q >= n) break;
                const uint32_t kq = kb + q;
                while (j + 1 < nrec && kq >= s_off[j + 1]) j++;
                if (j != jc) {
                    jc = j;
                    r = s_rid[j];
                    tx0 = s_tx[j] & 0xffffu;
                    nx = s_tx[j] >> 16;
                    tb = s_tbase[j];
                    tiles_x = s_tpr[j];
                    t0 = s_roff[j];
                    t1 = s_roff[j + 1];
                    base = s_rpre[t0];
                }
                const uint32_t li = kq - s_off[j];
                uint32_t tile;
                if (t0 == t1) {  // every tile of the rectangle
                    tile = tb + (li / nx) * tiles_x + tx0 + li % nx;
                } else if (s_rpre[t1] == base) {
                    // a support that meets no tile still owns one pair, its
                    // box's first tile; anything else is a counting mismatch
                    if (li != 0) atomicOr(flags, FLAG_BIN_MISMATCH);
                    tile = tb + tx0;
                } else {
                    // the last row whose pairs start at or before li (empty
                    // rows share the next row's start, so it is not empty)
                    uint32_t a = t0, b = t1 - 1;
                    while (a < b) {
                        const uint32_t m = a + (b - a + 1) / 2;
                        if (s_rpre[m] - base <= li) a = m;
                        else b = m - 1;
                    }
                    const uint32_t row = s_row[a];
                    const uint32_t col = (row & 0xffffu) + (li - (s_rpre[a] - base));
                    if (li - (s_rpre[a] - base) >= (row >> 16)) atomicOr(flags, FLAG_BIN_MISMATCH);
                    tile = tb + (a - t0) * tiles_x + col;
                }
                tk[q] = tile;
                tr[q] = r;
            }
        } else {
            uint32_t j = last_le(s_off, nrec, kb);
            PairCursor c;
            cursor_open(c, rec, views, order[lo + j], kb - s_off[j], tws, ths, log2_amin, flags);
#pragma unroll
            for (int q = 0; q < EM_RUN; q++) {
                if (q >= n) break;
                if (q > 0) {
                    if (j + 1 < nrec && kb + q >= s_off[j + 1]) {
                        j++;
                        cursor_open(c, rec, views, order[lo + j], 0, tws, ths, log2_amin, flags);
                    } else {
                        cursor_next(c, tws, ths);
                    }
                }
                tk[q] = cursor_tile(c);
                tr[q] = c.r;
            }
        }
        if (n == EM_RUN) {
#pragma unroll
            for (int q = 0; q < EM_RUN; q += 4) {
                *reinterpret_cast<uint4*>(tile_key + kb + q) = make_uint4(tk[q], tk[q + 1], tk[q + 2], tk[q + 3]);
                *reinterpret_cast<uint4*>(inst_rec + kb + q) = make_uint4(tr[q], tr[q + 1], tr[q + 2], tr[q + 3]);
            }
        } else {
            for (int q = 0; q < n; q++) {
                tile_key[kb + q] = tk[q];
                inst_rec[kb + q] = tr[q];
            }
        }
    }
}

// A tile's range starts where the sorted key changes from the previous one
// and ends where it changes to the next.  Each thread reads four consecutive
// keys with one 16-byte load; the neighbours across thread boundaries come
// from the adjacent lanes (lane 0 and lane 63 load theirs).  Keys are stored
// 16-byte aligned.
__device__ __forceinline__ void range_edges(uint32_t i, uint32_t t, uint32_t prev, uint32_t next, uint32_t K,
                                            uint2* __restrict__ ranges, uint32_t tiles_cap) {
    if (t >= tiles_cap) return;
    if (i == 0 || prev != t) ranges[t].x = i;
    if (i + 1 == K || next != t) ranges[t].y = i + 1;
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ K_dev, uint32_t cap,
                                                     uint2* __restrict__ ranges, uint32_t tiles_cap,
                                                     const uint32_t* __restrict__ flags) {
    if (*flags) return;  // an overflowed binning leaves the ranges empty
    const uint32_t K = min(*K_dev, cap);
    const uint32_t n4 = K / 4;  // whole groups of four keys
    const uint32_t lane = lane_id();
    const uint32_t stride = gridDim.x * blockDim.x;
    // the loop bound is rounded up to whole waves so that every lane of a
    // wave takes part in the shuffles of every round
    const uint32_t nwave = (n4 + 63) / 64 * 64;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nwave; g += stride) {
        const bool live = g < n4;
        const uint32_t i = 4 * g;
        const uint4 k = live ? *reinterpret_cast<const uint4*>(key + i) : make_uint4(0u, 0u, 0u, 0u);
        uint32_t prev = (uint32_t)__shfl_up((int)k.w, 1, 64);
        uint32_t next = (uint32_t)__shfl_down((int)k.x, 1, 64);
        if (live && lane == 0 && i > 0) prev = key[i - 1];
        if (live && (lane == 63 || g + 1 == n4)) next = i + 4 < K ? key[i + 4] : 0u;
        if (live) {
            range_edges(i, k.x, prev, k.y, K, ranges, tiles_cap);
            range_edges(i + 1, k.y, k.x, k.z, K, ranges, tiles_cap);
            range_edges(i + 2, k.z, k.y, k.w, K, ranges, tiles_cap);
            range_edges(i + 3, k.w, k.z, next, K, ranges, tiles_cap);
        }
    }
    // the last K % 4 keys
    const uint32_t i = 4 * n4 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K) range_edges(i, key[i], i > 0 ? key[i - 1] : 0u, i + 1 < K ? key[i + 1] : 0u, K, ranges, tiles_cap);
}

// ---------------------------------------------------------- tile order
// The compositing kernels take the tiles in descending order of their pair
// counts, bucketed by powers of two, so that long tiles start first and no
// long tile is left for the end of a launch.  A counting sort over 33
// buckets: bucket 0 holds the tiles with 2^31 or more pairs, bucket 31 those
// with one, bucket 32 the empty ones; within a bucket the order is
// arbitrary, since every tile's result is independent of when it runs.
constexpr int TO_BUCKETS = 33;
static_assert(TILE_ORDER_WS == 2 * TO_BUCKETS, "the scratch holds the bucket sizes and the cursors");

__device__ __forceinline__ int tile_bucket(uint2 rg) {
    const uint32_t c = rg.y - rg.x;
    return c ? __clz((int)c) : 32;
}

__global__ __launch_bounds__(256) void k_tile_order_count(const uint2* __restrict__ ranges,
                                                          const Header* __restrict__ hdr, uint32_t tiles_cap,
                                                          uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[TO_BUCKETS];
    for (int i = threadIdx.x; i < TO_BUCKETS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint32_t n = min(hdr->tiles_total, tiles_cap);
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        atomicAdd(&h[tile_bucket(ranges[t])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < TO_BUCKETS; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// hist: the bucket sizes; cursor: per bucket, the places already taken
// (zero before the launch).
__global__ __launch_bounds__(256) void k_tile_order_place(const uint2* __restrict__ ranges,
                                                          const Header* __restrict__ hdr, uint32_t tiles_cap,
                                                          const uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ cursor,
                                                          uint32_t* __restrict__ order) {
    __shared__ uint32_t start[TO_BUCKETS], h[TO_BUCKETS], base[TO_BUCKETS];
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < TO_BUCKETS; i++) {
            start[i] = run;
            run += hist[i];
        }
    }
    const uint32_t n = min(hdr->tiles_total, tiles_cap);
    for (uint32_t t0 = blockIdx.x * blockDim.x; t0 < n; t0 += gridDim.x * blockDim.x) {
        for (int i = threadIdx.x; i < TO_BUCKETS; i += blockDim.x) h[i] = 0;
        __syncthreads();
        const uint32_t t = t0 + threadIdx.x;
        int b = 0;
        uint32_t rank = 0;
        if (t < n) {
            b = tile_bucket(ranges[t]);
            rank = atomicAdd(&h[b], 1u);
        }
        __syncthreads();
        if (threadIdx.x < TO_BUCKETS && h[threadIdx.x]) base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]);
        __syncthreads();
        if (t < n) order[start[b] + base[b] + rank] = t;
        __syncthreads();
    }
}

// ------------------------------------------------------------ compositing
// Sec. III: C(p) = sum_i c_i a_i T_i with T_i = prod_{j<i} (1 - a_j); the
// depth image replaces c_i by d_i; the uncertainty image by u_i (Sec. IV-A).

__device__ __forceinline__ uint32_t view_of_tile(const ViewDev* views, int nv, uint32_t tile) {
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= tile) lo = mid;
        else hi = mid - 1;
    }
    return (uint32_t)lo;
}

// Pixel arithmetic of the compositing loops is done relative to an origin
// fixed per 32 x 16 pixel block (a multiple of every tile shape, so no
// pixel's arithmetic depends on the tile): a pixel's coordinates are then
// small exact integers and a splat's mean, staged once per tile as
// (mean hi - origin) + mean lo, is rounded at the magnitude of its distance
// from the block, far below what the alpha test needs.
__device__ __forceinline__ int origin_x(int x) { return x & ~31; }
__device__ __forceinline__ int origin_y(int y) { return y & ~15; }
__device__ __forceinline__ float4 rel_mean(float4 g0, int ox, int oy) {
    return make_float4((g0.x - (float)ox) + g0.z, (g0.y - (float)oy) + g0.w, 0.0f, 0.0f);
}

// alpha of one splat at the pixel (lx, ly) of the block whose origin the
// staged mean (mx, my) is relative to: G = exp2(-|M d|^2), d = p - mean.
// CLAMP = false leaves out the clamp at alpha_max, for splats whose opacity
// is at most alpha_max: G <= 1, so their rounded o G never exceeds it and
// the result is the same.
template <bool CLAMP = true>
__device__ __forceinline__ float splat_alpha(float mx, float my, float4 g1, float lx, float ly, float amax, float& G,
                                             float& dx, float& dy, float& w1, float& w2) {
    dx = lx - mx;
    dy = ly - my;
    w1 = g1.x * dx;
    w2 = fmaf(g1.y, dx, g1.z * dy);
    float pw = fmaf(w1, w1, w2 * w2);
    G = fast_exp2(-pw);
    // o G >= 0, so the median of (o G, 0, alpha_max) is min(alpha_max, o G)
    // (one instruction, with no quieting of its operands)
    return CLAMP ? __builtin_amdgcn_fmed3f(g1.w * G, 0.0f, amax) : g1.w * G;
}

template <bool V>
struct BoolC {
    static constexpr bool value = V;
};

// Splat box meets the pixel rectangle [c0, c1] x [r0, r1].
__device__ __forceinline__ bool box_meets(uint2 b, int c0, int c1, int r0, int r1) {
    return (int)(b.x & 0xffffu) <= c1 && (int)(b.x >> 16) >= c0 && (int)(b.y & 0xffffu) <= r1 &&
           (int)(b.y >> 16) >= r0;
}


// Where the support-ellipse prefilter runs.  It pays in scoring (many
// elongated splats seen close up from arbitrary poses); on mapping frames
// the box test alone is faster in the forward and backward passes.
constexpr bool FWD_ELL = false, BWD_ELL = false, SCORE_ELL = true;

// For a staged batch of `cnt` splats, bit k of m[k / 64] is set when splat k
// can reach the calling wave's pixel rectangle (wave-uniform result): its box
// meets the rectangle and, with ELL, so does its support ellipse.
template <int NT, bool ELL>
__device__ __forceinline__ void wave_masks(const uint2* s_pb, const float4* s_g0, const float4* s_g1,
                                           float log2_amin, int cnt, int c0, int c1, int r0, int r1,
                                           uint64_t (&m)[(NT + 63) / 64]) {
    const int lane = (int)lane_id();
#pragma unroll
    for (int c = 0; c < (NT + 63) / 64; c++) {
        const int e = c * 64 + lane;
        bool hit = e < cnt && box_meets(s_pb[e], c0, c1, r0, r1);
        if (ELL && hit) hit = support_meets_rect(s_g0[e], s_g1[e], log2_amin, c0, c1, r0, r1);
        m[c] = __ballot(hit);
    }
}
// The same selection as a list: the indices of the staged splats that can
// reach the wave's pixel rectangle, in ascending order, written to list[0, n)
// (n returned, wave-uniform).  A loop over the list needs no scalar
// bit-scanning per splat.
template <int NT, bool ELL>
__device__ __forceinline__ int wave_list(const uint2* s_pb, const float4* s_g0, const float4* s_g1,
                                         float log2_amin, int cnt, int c0, int c1, int r0, int r1,
                                         uint16_t* list) {
    const int lane = (int)lane_id();
    int n = 0;
#pragma unroll
    for (int c = 0; c < (NT + 63) / 64; c++) {
        const int e = c * 64 + lane;
        bool hit = e < cnt && box_meets(s_pb[e], c0, c1, r0, r1);
        if (ELL && hit) hit = support_meets_rect(s_g0[e], s_g1[e], log2_amin, c0, c1, r0, r1);
        const uint64_t m = __ballot(hit);
        if (hit) list[n + (int)__popcll(m & lanemask_lt())] = (uint16_t)e;
        n += (int)__popcll(m);
    }
    return n;
}

// Next P set bits of a wave-uniform mask (entries past the last are -1).
template <int P>
__device__ __forceinline__ void pop_n(uint64_t& mm, int base, int (&ks)[P]) {
#pragma unroll
    for (int q = 0; q < P; q++) {
        if (mm) {
            ks[q] = base + (int)__builtin_ctzll(mm);
            mm &= mm - 1;
        } else {
            ks[q] = -1;
        }
    }
}

// Splats evaluated per step of the front-to-back loops: their alphas are
// independent of the pixel state, so they overlap; the updates follow in order.
constexpr int FWD_STEP = 2;
// The scoring loop's (it keeps only T and one sum per pixel).
constexpr int SCORE_STEP = 2;
// Splats per step of the back-to-front backward loop (four measured slower:
// the registers cut occupancy); the reduction below is written for two.
constexpr int BWD_STEP = 2;
// Relative band around alpha_min inside which the skip decision is re-taken
// in binary64 (far wider than the binary32 error of alpha).
constexpr float REFINE = 2e-3f;

// Whether binary32 alpha a lies in that band: |a - alpha_min| <= band, with
// band = REFINE alpha_min (a subtraction and a compare of the magnitude).
__device__ __forceinline__ bool near_amin(float a, float amin, float band) { return fabsf(a - amin) <= band; }

// The alpha_min test: a splat with alpha < alpha_min at a pixel is skipped
// there.  Where binary32 alpha lies in [alpha_min (1 - REFINE), alpha_min
// (1 + REFINE)] the decision is re-taken in binary64 from the binary64 conic
// (kept64), as the definition states it.  No pixel box test is needed: the
// box is the exact bounding box of the support, so outside it alpha <
// alpha_min already.  The loops take the rare binary64 branch once per
// step, for all the splats of the step.

__device__ __forceinline__ bool kept64(float4 g0, float4 g1, const double4* __restrict__ q64, uint32_t r, float px,
                                       float py, const SetDev& st) {
    const float amin = st.alpha_min;
    const double4 q = q64[r];
    const double dx = ((double)px - (double)g0.x) - (double)g0.z;
    const double dy = ((double)py - (double)g0.y) - (double)g0.w;
    const double pw = (q.x * dx * dx + 2.0 * q.y * dx * dy) + q.z * dy * dy;
    const double ad = fmin((double)st.alpha_max, (double)g1.w * exp(-0.5 * pw));
    return ad >= (double)amin;
}

// Staged form of a splat for the pair loops of the forward and scoring
// kernels: p = (mean x, mean y relative to the block origin, M00, M10),
// q = (M11, opacity, u, log2 opacity).  Slot NB of the staged arrays holds
// the null splat (opacity 0, log2 opacity -3e38): alpha 0 at every pixel, far
// from alpha_min's band, so it never contributes.
__device__ __forceinline__ void stage_splat(const EmitRec& e, int ox, int oy, float4& p, float4& q) {
    const float4 m = rel_mean(e.g0, ox, oy);
    p = make_float4(m.x, m.y, e.g1.x, e.g1.y);
    q = make_float4(e.g1.z, e.g1.w, __uint_as_float(e.unc), __builtin_amdgcn_logf(e.g1.w));
}

template <int NB>
__device__ __forceinline__ void stage_null_splat(float4* s_p, float4* s_q) {
    if (threadIdx.x == 0) {
        s_p[NB] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        s_q[NB] = make_float4(0.0f, 0.0f, 0.0f, -3e38f);
    }
}

// The staged splats that can reach the calling wave's pixel rectangle
// [c0, c1] x [r0, r1] (relative to the block origin (ox, oy)): their box
// meets it and, with ELL, so does their support ellipse.  Written to list as
// LDS byte offsets of their staged entries, in ascending order (so a step
// reads its offsets with one load and no unpacking); two entries past the
// end name the null splat, so the loops run in whole steps of two without
// checks.  Returns the count (wave-uniform).
template <int NB, bool ELL>
__device__ __forceinline__ int splat_list(const uint2* s_pb, const float4* s_p, const float4* s_q, float log2_amin,
                                          int cnt, int c0, int c1, int r0, int r1, int ox, int oy,
                                          uint32_t* list) {
    const int lane = (int)lane_id();
    int n = 0;
#pragma unroll
    for (int c = 0; c < (NB + 63) / 64; c++) {
        const int e = c * 64 + lane;
        bool hit = e < cnt && box_meets(s_pb[e], c0 + ox, c1 + ox, r0 + oy, r1 + oy);
        if (ELL && hit) {
            const float4 p = s_p[e], q = s_q[e];
            hit = support_meets_rect_xy(p.x, p.y, make_float4(p.z, p.w, q.x, q.y), log2_amin, c0, c1, r0, r1);
        }
        const uint64_t m = __ballot(hit);
        if (hit) list[n + (int)__popcll(m & lanemask_lt())] = (uint32_t)(e * sizeof(float4));
        n += (int)__popcll(m);
    }
    if (lane < 2) list[n + lane] = (uint32_t)(NB * sizeof(float4));
    return n;
}

// The binary64 re-decision of a splat whose binary32 alpha fell within the
// band around alpha_min: a splat it keeps enters with alpha at least
// alpha_min (its binary32 alpha lies within the band, below the binary64
// value), one it drops with alpha 0.
__device__ __forceinline__ float redecide(float a, const Records& rec, uint32_t r, int u, int v, const SetDev& st) {
    const EmitRec& e = rec.emit[r];
    return kept64(e.g0, e.g1, rec.q64, r, (float)u, (float)v, st) ? fmaxf(a, st.alpha_min) : 0.0f;
}

// B splats are staged per batch (B <= TW * TH; threads below B load them).
// Register budget: at most 80 VGPRs, six waves per SIMD (a 640x480 frame of
// 16x16 tiles brings 4.7 waves per SIMD, larger frames many more).
// UNC: the uncertainty image is requested (otherwise it is not composited).
//
// Front to back over the wave's list, FWD_STEP splats per step: their alphas
// are independent of the pixel state, the updates follow in order.  A pixel
// whose next transmittance would fall below T_min stops there; its T is then
// kept negated (|T| is the final transmittance), which no later update
// passes, so the loop carries no per-pixel flags.  A splat below alpha_min
// enters with alpha 0 (T unchanged, exactly) and is not counted.
template <int TW, int TH, int B, bool UNC>
__global__ __launch_bounds__(TW * TH, 6) void k_render_fwd(const ViewDev* __restrict__ views, int n_views,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ tile_order,
                                                        const uint32_t* __restrict__ inst_rec,
                                                        Records rec, SetDev st, RenderOut out,
                                                        const uint32_t* __restrict__ flags) {
    constexpr int NT = TW * TH;
    static_assert(B <= NT, "batch larger than the tile");
    static_assert(32 % TW == 0 && 16 % TH == 0, "tiles must divide the 32 x 16 origin block");
    static_assert(FWD_STEP == 2, "the list is padded for steps of two");
    if (flags && *flags) return;
    __shared__ float4 s_p[B + 1], s_q[B + 1], s_at[B + 1];
    __shared__ uint32_t s_r[B];
    __shared__ uint2 s_pb[B];
    __shared__ __align__(8) uint32_t s_list[NT / 64 * (B + 2)];
    stage_null_splat<B>(s_p, s_q);
    if (threadIdx.x == 0) s_at[B] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const uint32_t tile = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
    const uint32_t vi = view_of_tile(views, n_views, tile);
    const ViewDev& V = views[vi];
    const int W = V.W, H = V.H;
    const uint32_t lt = tile - V.tile_off;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int u = tx * TW + (int)(threadIdx.x % TW), v = ty * TH + (int)(threadIdx.x / TW);
    const int ox = origin_x(tx * TW), oy = origin_y(ty * TH);
    // this wave's pixel rectangle (64 consecutive threads = 64 / TW rows of
    // the tile), relative to the origin
    const int wc0 = tx * TW - ox, wc1 = wc0 + TW - 1;
    const int wr0 = ty * TH + (int)(threadIdx.x >> 6) * (64 / TW) - oy, wr1 = wr0 + 64 / TW - 1;
    const bool inside = u < W && v < H;
    const float lx = (float)(u - ox), ly = (float)(v - oy);
    const float amin = st.alpha_min, amax = st.alpha_max, tmin = st.T_min;
    const float band = REFINE * amin;
    const char* sp = reinterpret_cast<const char*>(s_p);
    const char* sq = reinterpret_cast<const char*>(s_q);
    const char* sa = reinterpret_cast<const char*>(s_at);
    const uint2 rg = ranges[tile];
    float T = inside ? 1.0f : -1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, dd = 0.0f, uu = 0.0f;
    uint32_t last = 0, ncontrib = 0;
    for (uint32_t b = rg.x; b < rg.y; b += B) {
        if (__syncthreads_count(T > 0.0f) == 0) break;
        uint32_t idx = b + threadIdx.x;
        if (threadIdx.x < (uint32_t)B && idx < rg.y) {
            uint32_t r = inst_rec[idx];
            s_r[threadIdx.x] = r;
            const EmitRec e = rec.emit[r];
            s_pb[threadIdx.x] = e.pbox;
            stage_splat(e, ox, oy, s_p[threadIdx.x], s_q[threadIdx.x]);
            s_at[threadIdx.x] = rec.attr[r];
        }
        __syncthreads();
        const int cnt = (int)min<uint32_t>(B, rg.y - b);
        uint32_t* my = s_list + (threadIdx.x >> 6) * (B + 2);
        int nl = 0;
        if (__ballot(T > 0.0f))
            nl = splat_list<B, FWD_ELL>(s_pb, s_p, s_q, st.log2_amin, cnt, wc0, wc1, wr0, wr1, ox, oy, my);
        __syncthreads();  // the wave's list is in LDS
        // LDS offset of the last splat this lane took in this batch
        uint32_t lastoff = 0xffffffffu;
        for (int i = 0; i < nl; i += FWD_STEP) {
            if (!__ballot(T > 0.0f)) break;
            uint32_t ko[FWD_STEP];
            float as[FWD_STEP];
            bool need = false;
#pragma unroll
            for (int q = 0; q < FWD_STEP; q++) {
                ko[q] = my[i + q];
                const float4 pp = *reinterpret_cast<const float4*>(sp + ko[q]);
                const float4 qq = *reinterpret_cast<const float4*>(sq + ko[q]);
                float G, dx, dy, w1, w2;
                as[q] = splat_alpha(pp.x, pp.y, make_float4(pp.z, pp.w, qq.x, qq.y), lx, ly, amax, G, dx, dy, w1,
                                    w2);
                need = need | near_amin(as[q], amin, band);
            }
            if (__ballot(need)) {
#pragma unroll
                for (int q = 0; q < FWD_STEP; q++)
                    if (near_amin(as[q], amin, band) & (ko[q] < B * sizeof(float4)))
                        as[q] = redecide(as[q], rec, s_r[ko[q] / sizeof(float4)], u, v, st);
            }
#pragma unroll
            for (int q = 0; q < FWD_STEP; q++) {
                const bool ok = as[q] >= amin;
                const float a0 = ok ? as[q] : 0.0f;
                const float Tn = fmaf(-a0, T, T);
                const bool live = Tn >= tmin;
                const bool use = ok & live;
                // weight 0 where the splat is skipped (a0 = 0) or the pixel
                // stops: fmaf(x, 0, c) = c for the finite staged attributes,
                // so the sums need no per-channel select
                const float w = live ? a0 * T : 0.0f;
                const float4 at = *reinterpret_cast<const float4*>(sa + ko[q]);
                c0 = fmaf(at.x, w, c0);
                c1 = fmaf(at.y, w, c1);
                c2 = fmaf(at.z, w, c2);
                dd = fmaf(at.w, w, dd);
                if (UNC) {
                    const float uk = *reinterpret_cast<const float*>(sq + ko[q] + 8);
                    uu = fmaf(uk, w, uu);
                }
                lastoff = use ? ko[q] : lastoff;
                ncontrib += use ? 1u : 0u;
                T = live ? Tn : -fabsf(T);
            }
        }
        if (lastoff != 0xffffffffu) last = b - rg.x + 1 + lastoff / (uint32_t)sizeof(float4);
    }
    if (!inside) return;
    T = fabsf(T);
    const uint64_t P = (uint64_t)W * H;
    const uint64_t pix = V.pix_off + (uint64_t)v * W + u;
    if (out.rgb) {
        float* base = out.rgb + 3 * V.pix_off + (uint64_t)v * W + u;
        base[0] = c0;
        base[P] = c1;
        base[2 * P] = c2;
    }
    if (out.depth) out.depth[pix] = dd;
    if (out.alpha) out.alpha[pix] = 1.0f - T;
    if (out.unc) out.unc[pix] = uu;
    if (out.T_final) out.T_final[pix] = T;
    if (out.n_last) out.n_last[pix] = last;
    if (out.n_contrib) out.n_contrib[pix] = ncontrib;
}

// ----------------------------------------------------------------- loss
// Sec. III eq. (4), L1 terms: (1/P) sum_p (sum_ch |C - C*| + w_d |D - D*|).

__device__ __forceinline__ float sgnf(float e) { return e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f); }

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ float wave_sum_f(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__global__ __launch_bounds__(256) void k_loss(const ViewDev* __restrict__ views, const float* __restrict__ rgb,
                                              const float* __restrict__ depth, const float* __restrict__ trgb,
                                              const float* __restrict__ tdepth, float w_depth,
                                              float* __restrict__ d_rgb, float* __restrict__ d_depth,
                                              double* __restrict__ partial) {
    __shared__ double ws[4];
    const ViewDev& V = views[blockIdx.y];
    const uint64_t P = (uint64_t)V.W * V.H;
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (p < P) {
        const float invP = (float)(1.0 / (double)P);
        const uint64_t c = 3 * V.pix_off + p;
        const uint64_t q = V.pix_off + p;
        float acc = 0.0f;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float e = rgb[c + ch * P] - trgb[c + ch * P];
            acc += fabsf(e);
            if (d_rgb) d_rgb[c + ch * P] = sgnf(e) * invP;
        }
        float e = depth[q] - tdepth[q];
        if (d_depth) d_depth[q] = w_depth * sgnf(e) * invP;
        l = ((double)acc + (double)w_depth * (double)fabsf(e)) / (double)P;
    }
    l = wave_sum_d(l);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partial[(uint64_t)blockIdx.y * gridDim.x + blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// One block; each thread keeps four running sums over entries 4096 apart, so
// that four loads are in flight per step (the order is fixed: the total is
// the same on every run).
constexpr int SP_THREADS = 1024;
__global__ __launch_bounds__(SP_THREADS) void k_sum_partials(const double* __restrict__ partial, int n,
                                                             double* __restrict__ out) {
    __shared__ double ws[SP_THREADS / 64];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 4 * SP_THREADS) {
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (i + k * SP_THREADS < n) a[k] += partial[i + k * SP_THREADS];
    }
    double s = wave_sum_d((a[0] + a[1]) + (a[2] + a[3]));
    if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < SP_THREADS / 64; w++) t += ws[w];
        *out = t;
    }
}

// ------------------------------------------------------------ backward
// Reverse mode of the compositing, walking each tile back to front; the
// transmittance before splat i is recovered as T_{i+1} / (1 - a_i).

// Sum over the 64 lanes of a wave with DPP moves (result valid in lane 63,
// returned to every lane).  Rows of 16: quad swaps, rotations by 4 and 8,
// then row broadcasts 15 and 31 accumulate rows into row 3.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}

__device__ __forceinline__ float wave_sum_dpp(float x) {
    x += dpp_mov<0xb1>(x);        // quad_perm [1, 0, 3, 2]
    x += dpp_mov<0x4e>(x);        // quad_perm [2, 3, 0, 1]
    x += dpp_mov<0x124>(x);       // row_ror 4
    x += dpp_mov<0x128>(x);       // row_ror 8
    x += dpp_mov<0x142, 0xa>(x);  // row_bcast 15 into rows 1 and 3
    x += dpp_mov<0x143, 0xc>(x);  // row_bcast 31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Sums each of n per-lane values over the wave (the same DPP steps as
// wave_sum_dpp, applied to all values step by step so they overlap).
template <int N>
__device__ __forceinline__ void wave_sum_dpp_n(float* x) {
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp_mov<0xb1>(x[i]);
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp_mov<0x4e>(x[i]);
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp_mov<0x124>(x[i]);
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp_mov<0x128>(x[i]);
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp_mov<0x142, 0xa>(x[i]);
#pragma unroll
    for (int i = 0; i < N; i++) x[i] += dpp_mov<0x143, 0xc>(x[i]);
#pragma unroll
    for (int i = 0; i < N; i++) x[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[i]), 63));
}

// Sums 20 per-lane values over the wave by recursive halving: at each of six
// steps a lane keeps half of its values, sends the other half to its partner
// and adds the partner's copy of the kept half.  Partners must agree on every
// earlier choice, so the DPP pairings that flip several lane bits come first:
// row_mirror (decided by lane bit 3), row_half_mirror (bit 2), then quad
// swaps xor 2 (bit 1) and xor 1 (bit 0), then the row swaps of gfx950 across
// 16 lanes (bit 4) and 32 lanes (sum).  Lane l ends with the total of value
// v = 10 b3 + 5 b2 + 3 b1 + 2 b0 + b4, valid when 2 b0 + b4 < (b1 ? 2 : 3)
// (else v = -1); lanes l and l + 32 hold the same total.
//
// v_permlane16_swap(x, y) exchanges the odd 16-lane rows of x with the even
// rows of y, so the two results add up, in every lane, to x[l] + x[l ^ 16] on
// even rows and y[l ^ 16] + y[l] on odd rows; v_permlane32_swap(x, x) likewise
// gives x[l] + x[l ^ 32].  Both are VALU moves, not LDS round trips.
__device__ __forceinline__ float wave_sum_halving20(const float* x, int lane, int& v) {
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1,
               b4 = (lane >> 4) & 1;
    float a[10], c[5], d[3], e[2];
#pragma unroll
    for (int j = 0; j < 10; j++) {
        const float keep = b3 ? x[10 + j] : x[j], send = b3 ? x[j] : x[10 + j];
        a[j] = keep + dpp_mov<0x140>(send);  // row_mirror
    }
#pragma unroll
    for (int j = 0; j < 5; j++) {
        const float keep = b2 ? a[5 + j] : a[j], send = b2 ? a[j] : a[5 + j];
        c[j] = keep + dpp_mov<0x141>(send);  // row_half_mirror
    }
#pragma unroll
    for (int j = 0; j < 3; j++) {  // halves {0, 1, 2} and {3, 4, pad}
        const float hi = j + 3 < 5 ? c[j + 3] : 0.0f;
        const float keep = b1 ? hi : c[j], send = b1 ? c[j] : hi;
        d[j] = keep + dpp_mov<0x4e>(send);  // quad_perm [2, 3, 0, 1]
    }
#pragma unroll
    for (int j = 0; j < 2; j++) {  // halves {0, 1} and {2, pad}
        const float hi = j + 2 < 3 ? d[j + 2] : 0.0f;
        const float keep = b0 ? hi : d[j], send = b0 ? d[j] : hi;
        e[j] = keep + dpp_mov<0xb1>(send);  // quad_perm [1, 0, 3, 2]
    }
    const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(e[0]), __float_as_uint(e[1]), false, false);
    const float f = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
    const int pos = 2 * (int)b0 + (int)b4;
    v = pos < (b1 ? 2 : 3) ? 10 * (int)b3 + 5 * (int)b2 + 3 * (int)b1 + pos : -1;
    const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(f), __float_as_uint(f), false, false);
    return __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
}

// Highest set bit of a wave-uniform mask array, cleared; -1 if none.
template <int NW>
__device__ __forceinline__ int pop_high(uint64_t (&m)[NW]) {
    // static indices only, so that m stays in registers
    int k = -1;
#pragma unroll
    for (int c = 0; c < NW; c++)
        if (m[c]) k = c * 64 + 63 - (int)__builtin_clzll(m[c]);
#pragma unroll
    for (int c = 0; c < NW; c++)
        if (k >= 0 && c == (k >> 6)) m[c] &= ~(1ull << (k & 63));
    return k;
}

// One pixel's step of the reverse compositing recursion for a kept splat i.
// With T = T_{i+1} (transmittance behind it), T_i = T / (1 - a_i) and the
// splat's weight w = a_i T_i; for an image channel with colour c_i and pixel
// gradient g, dL/da_i = g (c_i T_i - S / (1 - a_i)), S = sum_{j > i} c_j w_j.
// The channels enter only through GA = sum_ch g_ch c_i,ch, so the pixel
// carries one running sum D = sum_ch g_ch S_ch (D += w GA) instead of one per
// channel: dL/da_i = T_i GA - D / (1 - a_i).  Since a_i <= alpha_max < 1,
// 1 - a_i is a normal number well away from zero and the hardware reciprocal
// (within 1 ulp) stands in for the correctly rounded division; T only scales
// gradient terms here and decides nothing.
// Per-lane sums acc (the record's gradient slots, in this order), with
// t = dL/da a_g, where a_g = o G is the splat's alpha where it is not clamped
// at alpha_max (then da/dpower = -a_g / 2 and da/do = a_g / o) and 0 where it
// is (no gradient flows through the clamp):
//   0, 1: sum t dx, sum t dy, with d = pixel - mean; the projection backward
//         scales them by -1/2 into sum dpow dx, sum dpow dy (dpow = dL/dpower,
//         power = d^T Q d, G = exp(-power / 2)) and forms the mean's gradient
//         -2 Q (sum dpow d) per record in binary64;
//   2, 3, 4: sum t dx^2, sum t dx dy, sum t dy^2, likewise (dL/dQ);
//   5: sum t, which the projection backward divides by o (dL/do);
//   6..9: sum g_ch w (colour and depth).
// A splat with a = 0 and a_g = 0 leaves T (1 / (1 - 0) = 1 exactly), D and
// every sum unchanged, for finite pixel gradients and colours.
// AU: the alpha and uncertainty images carry gradients too (colour 1 and u
// in GA; otherwise their terms are left out altogether).
template <bool AU, bool FIRST = false>
__device__ __forceinline__ void bwd_pixel(float a, float ag, float dx, float dy, float4 at, float ui, float gr,
                                          float gg, float gb, float gd, float ga, float gu, float& T, float& D,
                                          float* acc) {
    const float inv = __builtin_amdgcn_rcpf(1.0f - a);
    const float Ti = T * inv;
    const float w = a * Ti;
    float GA = gr * at.x;
    GA = fmaf(gg, at.y, GA);
    GA = fmaf(gb, at.z, GA);
    GA = fmaf(gd, at.w, GA);
    if constexpr (AU) {
        GA += ga;
        GA = fmaf(gu, ui, GA);
    }
    const float da = fmaf(Ti, GA, -(D * inv));
    D = fmaf(w, GA, D);
    T = Ti;
    const float t0 = da * ag;
    const float t1 = t0 * dx, t2 = t0 * dy;
    if constexpr (FIRST) {
        acc[6] = gr * w;
        acc[7] = gg * w;
        acc[8] = gb * w;
        acc[9] = gd * w;
        acc[5] = t0;
        acc[0] = t1;
        acc[1] = t2;
        acc[2] = t1 * dx;
        acc[3] = t1 * dy;
        acc[4] = t2 * dy;
    } else {
        acc[6] = fmaf(gr, w, acc[6]);
        acc[7] = fmaf(gg, w, acc[7]);
        acc[8] = fmaf(gb, w, acc[8]);
        acc[9] = fmaf(gd, w, acc[9]);
        acc[5] += t0;
        acc[0] += t1;
        acc[1] += t2;
        acc[2] = fmaf(t1, dx, acc[2]);
        acc[3] = fmaf(t1, dy, acc[3]);
        acc[4] = fmaf(t2, dy, acc[4]);
    }
}

// NW waves per tile; the tile's 8x8 pixel blocks are dealt to the waves in
// row-major order (PPT blocks each) and a lane owns one pixel per block.
// Splats are staged per batch for the whole workgroup; a wave visits only
// the splats whose support can reach its blocks (ballot masks per batch).  Per
// splat, the lane sums its pixels' contributions, the wave reduces them once
// with DPP and one lane adds the 10 totals to the record's binary64 gradient.
template <int TW, int TH, int NW, bool AU>
__global__ __launch_bounds__(64 * NW, AU ? 1 : 3) void k_render_bwd(const ViewDev* __restrict__ views, int n_views,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ tile_order,
                                                        const uint32_t* __restrict__ inst_rec, Records rec,
                                                        SetDev st, const float* __restrict__ T_final,
                                                        const uint32_t* __restrict__ n_last,
                                                        const float* __restrict__ d_rgb,
                                                        const float* __restrict__ d_depth,
                                                        const float* __restrict__ d_alpha,
                                                        const float* __restrict__ d_unc, double* __restrict__ g2d,
                                                        const uint32_t* __restrict__ flags) {
    constexpr int NB8 = TW * TH / 64;
    constexpr int PPT = NB8 / NW;
    constexpr int B = 64 * NW;
    static_assert(PPT >= 1 && PPT * NW == NB8, "waves must split the 8x8 blocks evenly");
    if (flags && *flags) return;
    __shared__ float4 s_g0[B], s_g1[B], s_at[B];
    __shared__ float s_u[B];
    __shared__ uint32_t s_r[B];
    __shared__ uint2 s_pb[B];
    __shared__ uint32_t s_max;
    const uint32_t tile = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
    const uint32_t vi = view_of_tile(views, n_views, tile);
    const ViewDev& V = views[vi];
    const int W = V.W, H = V.H;
    const uint32_t lt = tile - V.tile_off;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const uint2 rg = ranges[tile];
    const uint64_t P = (uint64_t)W * H;
    const int lane = (int)(threadIdx.x & 63), wave = NW == 1 ? 0 : (int)(threadIdx.x >> 6);

    // pixel j of this lane: (px0 + bx(j), py0 + by(j)) relative to the block
    // origin, block offsets that are constants when the tile has one wave
    const int ox = origin_x(tx * TW), oy = origin_y(ty * TH);
    const float px0 = (float)(tx * TW - ox + (lane & 7)), py0 = (float)(ty * TH - oy + (lane >> 3));
    auto bx = [&](int j) { return (float)(((wave * PPT + j) % (TW / 8)) * 8); };
    auto by = [&](int j) { return (float)(((wave * PPT + j) / (TW / 8)) * 8); };
    auto ux = [&](int j) { return tx * TW + ((wave * PPT + j) % (TW / 8)) * 8 + (lane & 7); };
    auto vy = [&](int j) { return ty * TH + ((wave * PPT + j) / (TW / 8)) * 8 + (lane >> 3); };
    float T[PPT];
    uint32_t last[PPT];
    float gr[PPT], gg[PPT], gb[PPT], gd[PPT], ga[PPT], gu[PPT];
    float D[PPT];
    uint32_t mylast = 0;
    int wc0 = 1 << 30, wc1 = -1, wr0 = 1 << 30, wr1 = -1;  // the wave's pixel rectangle
#pragma unroll
    for (int j = 0; j < PPT; j++) {
        const int blk = wave * PPT + j;
        const int bx0 = tx * TW + (blk % (TW / 8)) * 8, by0 = ty * TH + (blk / (TW / 8)) * 8;
        wc0 = min(wc0, bx0);
        wc1 = max(wc1, bx0 + 7);
        wr0 = min(wr0, by0);
        wr1 = max(wr1, by0 + 7);
        const int u = bx0 + (lane & 7), v = by0 + (lane >> 3);
        T[j] = 1.0f;
        last[j] = 0;
        gr[j] = gg[j] = gb[j] = gd[j] = ga[j] = gu[j] = 0.0f;
        D[j] = 0.0f;
        if (u < W && v < H) {
            const uint64_t pix = V.pix_off + (uint64_t)v * W + u;
            T[j] = T_final[pix];
            last[j] = n_last[pix];
            if (d_rgb) {
                const float* cb = d_rgb + 3 * V.pix_off + (uint64_t)v * W + u;
                gr[j] = cb[0];
                gg[j] = cb[P];
                gb[j] = cb[2 * P];
            }
            if (d_depth) gd[j] = d_depth[pix];
            if (AU && d_alpha) ga[j] = d_alpha[pix];
            if (AU && d_unc) gu[j] = d_unc[pix];
        }
        mylast = max(mylast, last[j]);
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (mylast) atomicMax(&s_max, mylast);
    __syncthreads();
    const uint32_t maxlast = s_max;
    uint32_t wave_last = mylast;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, o, 64));
    const float amax = st.alpha_max;
    const float band = REFINE * st.alpha_min;

    for (int64_t bend = maxlast; bend > 0; bend -= B) {
        const int64_t bstart = bend - B > 0 ? bend - B : 0;
        __syncthreads();
        {
            const int64_t e = bstart + threadIdx.x;
            if (e < bend) {
                const uint32_t r = inst_rec[rg.x + (uint32_t)e];
                s_r[threadIdx.x] = r;
                const EmitRec e = rec.emit[r];
                s_pb[threadIdx.x] = e.pbox;
                s_g0[threadIdx.x] = rel_mean(e.g0, ox, oy);
                s_g1[threadIdx.x] = e.g1;
                s_at[threadIdx.x] = rec.attr[r];
                if (AU) s_u[threadIdx.x] = __uint_as_float(e.unc);
            }
        }
        __syncthreads();
        uint64_t m[NW];
        // splats at or past every lane's last contributor cannot matter
        const int cnt = (int)(min<int64_t>(bend, (int64_t)wave_last) - bstart);
        wave_masks<B, BWD_ELL>(s_pb, s_g0, s_g1, st.log2_amin, cnt, wc0, wc1, wr0, wr1, m);
        // back to front over the splats that can reach this wave's pixels,
        // BWD_STEP per step: their alphas are independent of the pixel state,
        // and their wave reductions run interleaved
        for (;;) {
            int ks[BWD_STEP];
            ks[0] = pop_high<NW>(m);
            if (ks[0] < 0) break;
#pragma unroll
            for (int q = 1; q < BWD_STEP; q++) ks[q] = pop_high<NW>(m);
            float4 sg0[BWD_STEP], sg1[BWD_STEP], sat[BWD_STEP];
            float su[BWD_STEP];
            uint32_t sr[BWD_STEP], spos[BWD_STEP];
#pragma unroll
            for (int q = 0; q < BWD_STEP; q++) {
                const int k = ks[q] < 0 ? ks[0] : ks[q];
                sg0[q] = s_g0[k];
                sg1[q] = s_g1[k];
                sat[q] = s_at[k];
                su[q] = AU ? s_u[k] : 0.0f;
                sr[q] = s_r[k];
                spos[q] = ks[q] < 0 ? 0xffffffffu : (uint32_t)(bstart + ks[q]);
            }
            float acc[BWD_STEP][10];
            bool any[BWD_STEP];
#pragma unroll
            for (int q = 0; q < BWD_STEP; q++) {
                any[q] = false;
#pragma unroll
                for (int v = 0; v < 10; v++) acc[q][v] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < PPT; j++) {
                float a[BWD_STEP], G[BWD_STEP], dx[BWD_STEP], dy[BWD_STEP], w1[BWD_STEP], w2[BWD_STEP];
                bool need = false;
#pragma unroll
                for (int q = 0; q < BWD_STEP; q++) {
                    a[q] = splat_alpha(sg0[q].x, sg0[q].y, sg1[q], px0 + bx(j), py0 + by(j), amax, G[q], dx[q],
                                       dy[q], w1[q], w2[q]);
                    need = need | near_amin(a[q], st.alpha_min, band);
                }
                // the forward's binary64 re-decision, taken the same way
                if (__ballot(need)) {
#pragma unroll
                    for (int q = 0; q < BWD_STEP; q++)
                        if ((spos[q] < last[j]) & near_amin(a[q], st.alpha_min, band))
                            a[q] = redecide(a[q], rec, sr[q], ux(j), vy(j), st);
                }
                // predicated, not branched: a splat the pixel does not take
                // enters with alpha 0 and a_g 0, which leaves T, D and the
                // sums unchanged
#pragma unroll
                for (int q = 0; q < BWD_STEP; q++) {
                    const bool ok = (spos[q] < last[j]) & (a[q] >= st.alpha_min);
                    any[q] = any[q] | ok;
                    const float a0 = ok ? a[q] : 0.0f;
                    const float ag = sg1[q].w * G[q] <= amax ? a0 : 0.0f;
                    bwd_pixel<AU>(a0, ag, dx[q], dy[q], sat[q], su[q], gr[j], gg[j], gb[j], gd[j], ga[j],
                                  gu[j], T[j], D[j], acc[q]);
                }
            }
            bool t[BWD_STEP];
            bool tany = false;
#pragma unroll
            for (int q = 0; q < BWD_STEP; q++) {
                t[q] = __ballot(any[q]) != 0;
                tany = tany || t[q];
            }
            if (tany) {
                // lane l < 32 ends with the total of value v (splat v / 10,
                // gradient slot v % 10) and adds it: one 20-lane atomic
                int v;
                const float tot = wave_sum_halving20(&acc[0][0], lane, v);
                if (lane < 32 && v >= 0) {
                    const int q = v >= 10 ? 1 : 0;
                    const int slot = v - 10 * q;
                    if (q ? t[1] : t[0])
                        unsafeAtomicAdd(g2d + (uint64_t)(q ? sr[1] : sr[0]) * G2D_STRIDE + slot, (double)tot);
                }
            }
        }
    }
}

// The one-wave form of k_render_bwd (a tile per wave): the staging lanes
// keep only the splats whose box meets the tile and write them compacted, in
// ascending order, to LDS, so the walk back to front is a plain countdown
// with no mask scanning; the wave loads the next step's two splats while it
// computes the current one.  Every pixel sees the same splats in the same
// order, with the same arithmetic, as in k_render_bwd, and every splat's
// per-tile sums are reduced by the same lane tree, so the two kernels add
// identical partial gradients.  Slot B holds the null splat: position
// 0xffffffff (no pixel takes it), zero geometry and colour.
template <int TW, int TH, bool AU>
__global__ __launch_bounds__(64, AU ? 1 : 3) void k_render_bwd1(const ViewDev* __restrict__ views, int n_views,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ tile_order,
                                                        const uint32_t* __restrict__ inst_rec, Records rec,
                                                        SetDev st, const float* __restrict__ T_final,
                                                        const uint32_t* __restrict__ n_last,
                                                        const float* __restrict__ d_rgb,
                                                        const float* __restrict__ d_depth,
                                                        const float* __restrict__ d_alpha,
                                                        const float* __restrict__ d_unc, double* __restrict__ g2d,
                                                        const uint32_t* __restrict__ flags) {
    constexpr int PPT = TW * TH / 64;
    constexpr int B = 64;
    static_assert(PPT >= 1 && PPT * 64 == TW * TH, "the tile must be whole 8x8 blocks");
    if (flags && *flags) return;
    // s_p = (mean x, mean y relative to the origin, record id bits, position bits)
    __shared__ float4 s_p[B + 1], s_g1[B + 1], s_at[B + 1];
    __shared__ float s_u[B + 1];
    const uint32_t tile = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
    const uint32_t vi = view_of_tile(views, n_views, tile);
    const ViewDev& V = views[vi];
    const int W = V.W, H = V.H;
    const uint32_t lt = tile - V.tile_off;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const uint2 rg = ranges[tile];
    const uint64_t P = (uint64_t)W * H;
    const int lane = (int)threadIdx.x;
    if (lane == 0) {
        s_p[B] = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(0xffffffffu));
        s_g1[B] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        s_at[B] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        s_u[B] = 0.0f;
    }

    const int ox = origin_x(tx * TW), oy = origin_y(ty * TH);
    const float px0 = (float)(tx * TW - ox + (lane & 7)), py0 = (float)(ty * TH - oy + (lane >> 3));
    auto bx = [&](int j) { return (float)((j % (TW / 8)) * 8); };
    auto by = [&](int j) { return (float)((j / (TW / 8)) * 8); };
    auto ux = [&](int j) { return tx * TW + (j % (TW / 8)) * 8 + (lane & 7); };
    auto vy = [&](int j) { return ty * TH + (j / (TW / 8)) * 8 + (lane >> 3); };
    float T[PPT];
    uint32_t last[PPT];
    float gr[PPT], gg[PPT], gb[PPT], gd[PPT], ga[PPT], gu[PPT];
    float D[PPT];
    uint32_t mylast = 0;
    const int c0 = tx * TW, c1 = c0 + TW - 1, r0 = ty * TH, r1 = r0 + TH - 1;  // the tile's pixels
#pragma unroll
    for (int j = 0; j < PPT; j++) {
        const int u = ux(j), v = vy(j);
        T[j] = 1.0f;
        last[j] = 0;
        gr[j] = gg[j] = gb[j] = gd[j] = ga[j] = gu[j] = 0.0f;
        D[j] = 0.0f;
        if (u < W && v < H) {
            const uint64_t pix = V.pix_off + (uint64_t)v * W + u;
            T[j] = T_final[pix];
            last[j] = n_last[pix];
            if (d_rgb) {
                const float* cb = d_rgb + 3 * V.pix_off + (uint64_t)v * W + u;
                gr[j] = cb[0];
                gg[j] = cb[P];
                gb[j] = cb[2 * P];
            }
            if (d_depth) gd[j] = d_depth[pix];
            if (AU && d_alpha) ga[j] = d_alpha[pix];
            if (AU && d_unc) gu[j] = d_unc[pix];
        }
        mylast = max(mylast, last[j]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mylast = max(mylast, (uint32_t)__shfl_xor((int)mylast, o, 64));
    const uint32_t maxlast = mylast;
    const float amax = st.alpha_max;
    const float band = REFINE * st.alpha_min;

    for (int64_t bend = maxlast; bend > 0; bend -= B) {
        const int64_t bstart = bend - B > 0 ? bend - B : 0;
        __syncthreads();
        bool hit = false;
        float4 p, q1, at;
        float uv = 0.0f;
        {
            const int64_t e = bstart + lane;
            if (e < bend) {
                const uint32_t r = inst_rec[rg.x + (uint32_t)e];
                const EmitRec er = rec.emit[r];
                hit = box_meets(er.pbox, c0, c1, r0, r1);
                const float4 m = rel_mean(er.g0, ox, oy);
                p = make_float4(m.x, m.y, __uint_as_float(r), __uint_as_float((uint32_t)e));
                q1 = er.g1;
                at = rec.attr[r];
                if (AU) uv = __uint_as_float(er.unc);
            }
        }
        const uint64_t hm = __ballot(hit);
        const int n = (int)__popcll(hm);
        if (hit) {
            const int slot = (int)__popcll(hm & lanemask_lt());
            s_p[slot] = p;
            s_g1[slot] = q1;
            s_at[slot] = at;
            if (AU) s_u[slot] = uv;
        }
        __syncthreads();
        // back to front over slots n - 1, n - 2, ..., two per step
        for (int i = n - 1; i >= 0; i -= 2) {
            float4 cp[2], cg[2], ca[2];
            float cu[2];
#pragma unroll
            for (int q = 0; q < 2; q++) {
                const int k = i - q >= 0 ? i - q : B;
                cp[q] = s_p[k];
                cg[q] = s_g1[k];
                ca[q] = s_at[k];
                cu[q] = AU ? s_u[k] : 0.0f;
            }
            uint32_t sr[2], spos[2];
#pragma unroll
            for (int q = 0; q < 2; q++) {
                sr[q] = __float_as_uint(cp[q].z);
                spos[q] = __float_as_uint(cp[q].w);
            }
            float acc[2][10];
            bool any[2];
#pragma unroll
            for (int q = 0; q < 2; q++) any[q] = false;
            // every alpha of the step first (one block of independent work),
            // then the rare binary64 re-decisions, then the ordered updates.
            // CL: a splat of the step is more opaque than alpha_max, so its
            // alpha may be clamped and then carries no gradient; otherwise
            // alpha = o G carries it at every pixel (a_g = a)
            auto step = [&](auto clamp) {
                constexpr bool CL = decltype(clamp)::value;
                float a[PPT][2], G[PPT][2], dx[PPT][2], dy[PPT][2];
                bool need = false;
#pragma unroll
                for (int j = 0; j < PPT; j++)
#pragma unroll
                    for (int q = 0; q < 2; q++) {
                        float w1, w2;
                        a[j][q] = splat_alpha<CL>(cp[q].x, cp[q].y, cg[q], px0 + bx(j), py0 + by(j), amax, G[j][q],
                                                  dx[j][q], dy[j][q], w1, w2);
                        need = need | near_amin(a[j][q], st.alpha_min, band);
                    }
                if (__ballot(need)) {
#pragma unroll
                    for (int j = 0; j < PPT; j++)
#pragma unroll
                        for (int q = 0; q < 2; q++)
                            if ((spos[q] < last[j]) & near_amin(a[j][q], st.alpha_min, band))
                                a[j][q] = redecide(a[j][q], rec, sr[q], ux(j), vy(j), st);
                }
#pragma unroll
                for (int j = 0; j < PPT; j++) {
#pragma unroll
                    for (int q = 0; q < 2; q++) {
                        const bool ok = (spos[q] < last[j]) & (a[j][q] >= st.alpha_min);
                        any[q] = any[q] | ok;
                        const float a0 = ok ? a[j][q] : 0.0f;
                        const float ag = CL ? (cg[q].w * G[j][q] <= amax ? a0 : 0.0f) : a0;
                        if (j == 0)
                            bwd_pixel<AU, true>(a0, ag, dx[j][q], dy[j][q], ca[q], cu[q], gr[j], gg[j], gb[j],
                                                gd[j], ga[j], gu[j], T[j], D[j], acc[q]);
                        else
                            bwd_pixel<AU>(a0, ag, dx[j][q], dy[j][q], ca[q], cu[q], gr[j], gg[j], gb[j], gd[j],
                                          ga[j], gu[j], T[j], D[j], acc[q]);
                    }
                }
            };
            // opacities and alpha_max are positive: their bits order as they do
            const uint32_t amax_bits = __float_as_uint(amax);
            if (__ballot((__float_as_uint(cg[0].w) > amax_bits) | (__float_as_uint(cg[1].w) > amax_bits)))
                step(BoolC<true>{});
            else
                step(BoolC<false>{});
            bool t[2];
#pragma unroll
            for (int q = 0; q < 2; q++) t[q] = __ballot(any[q]) != 0;
            // reduced unconditionally (a step that no pixel takes is rare), so
            // that the per-pixel sums are formed pixel by pixel instead of
            // being held back behind a branch
            int v;
            const float tot = wave_sum_halving20(&acc[0][0], lane, v);
            if (lane < 32 && v >= 0) {
                const int q = v >= 10 ? 1 : 0;
                const int slot = v - 10 * q;
                if (q ? t[1] : t[0])
                    unsafeAtomicAdd(g2d + (uint64_t)(q ? sr[1] : sr[0]) * G2D_STRIDE + slot, (double)tot);
            }
        }
    }
}

// Chain rule from the screen-space gradients of a Gaussian's records to its
// parameters, in binary64, summed over the views that see it.
__global__ __launch_bounds__(256) void k_project_bwd(GaussDev g, const ViewDev* __restrict__ views, SetDev st,
                                                     const uint32_t* __restrict__ rec_off,
                                                     const uint32_t* __restrict__ cnt,
                                                     const EmitRec* __restrict__ emit,
                                                     const double* __restrict__ g2d,
                                                     float* __restrict__ d_means, float* __restrict__ d_ls,
                                                     float* __restrict__ d_quats, float* __restrict__ d_op,
                                                     float* __restrict__ d_col, const uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    if (flags && *flags) return;
    uint32_t c = cnt[i];
    if (c == 0) return;
    GPre P;
    if (!pre_gauss(g, i, st, P)) return;
    const int64_t n = g.n;
    double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double go = 0.0, gc[3] = {0, 0, 0};
    uint32_t r0 = rec_off[i];
    for (uint32_t r = r0; r < r0 + c; r++) {
        const ViewDev& V = views[emit[r].view];
        GProj q;
        project_exact(P, V, st, q);
        const double* G2 = g2d + (uint64_t)r * G2D_STRIDE;
        go += G2[5];  // divided by the opacity below
        gc[0] += G2[6];
        gc[1] += G2[7];
        gc[2] += G2[8];
        double gdepth = G2[9];
        double det = q.cxx * q.cyy - q.cxy * q.cxy;
        double Qxx = q.cyy / det, Qxy = -q.cxy / det, Qyy = q.cxx / det;
        // the 2D mean: power = d^T Q d with d = pixel - mean, so
        // dL/dmean = -2 Q sum_p dpow d, and slots 0 and 1 hold -2 times that
        // sum (dpow = -t / 2)
        double gmx = Qxx * G2[0] + Qxy * G2[1];
        double gmy = Qxy * G2[0] + Qyy * G2[1];
        // conic gradient (slots 2..4 times -1/2: dL/dQxx, dL/dQxy of the xy
        // term taken once, dL/dQyy) -> symmetric matrix gradient
        double Gq00 = -0.5 * G2[2], Gq01 = -0.5 * G2[3], Gq11 = -0.5 * G2[4];
        // G_cov = -Q G_Q Q
        double m00 = Gq00 * Qxx + Gq01 * Qxy, m01 = Gq00 * Qxy + Gq01 * Qyy;
        double m10 = Gq01 * Qxx + Gq11 * Qxy, m11 = Gq01 * Qxy + Gq11 * Qyy;
        double C00 = -(Qxx * m00 + Qxy * m10);
        double C01 = -(Qxx * m01 + Qxy * m11);
        double C11 = -(Qxy * m01 + Qyy * m11);
        // cov = Bs Bs^T with Bs = J A diag(s)
        double B0[3], B1[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            B0[k] = fma(q.j0, q.A[0 * 3 + k], q.j2 * q.A[2 * 3 + k]);
            B1[k] = fma(q.j4, q.A[1 * 3 + k], q.j5 * q.A[2 * 3 + k]);
        }
        double GB0[3], GB1[3];  // dL/dB (B = J A)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            double gbs0 = 2.0 * (C00 * B0[k] + C01 * B1[k]) * P.s[k];  // dL/dBs row 0
            double gbs1 = 2.0 * (C01 * B0[k] + C11 * B1[k]) * P.s[k];
            gs[k] += gbs0 * B0[k] + gbs1 * B1[k];
            GB0[k] = gbs0 * P.s[k];
            GB1[k] = gbs1 * P.s[k];
        }
        // B = J A:  G_J = G_B A^T, G_A = J^T G_B
        double GJ00 = 0, GJ02 = 0, GJ11 = 0, GJ12 = 0;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            GJ00 += GB0[k] * q.A[0 * 3 + k];
            GJ02 += GB0[k] * q.A[2 * 3 + k];
            GJ11 += GB1[k] * q.A[1 * 3 + k];
            GJ12 += GB1[k] * q.A[2 * 3 + k];
        }
        double GA[9];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            GA[0 * 3 + k] = q.j0 * GB0[k];
            GA[1 * 3 + k] = q.j4 * GB1[k];
            GA[2 * 3 + k] = q.j2 * GB0[k] + q.j5 * GB1[k];
        }
        // A = R^T Rq:  G_Rq = R G_A
        const double* R = V.R;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++)
                gR[a * 3 + b] += R[a * 3 + 0] * GA[0 * 3 + b] + R[a * 3 + 1] * GA[1 * 3 + b] +
                                 R[a * 3 + 2] * GA[2 * 3 + b];
        // camera-frame mean
        double tx = q.t[0], ty = q.t[1], tz = q.t[2];
        double iz = 1.0 / tz, iz2 = iz * iz;
        double gtx = 0, gty = 0, gtz = 0;
        gtz += GJ00 * (-V.fx * iz2);
        gtx += GJ02 * (-V.fx * iz2);
        gtz += GJ02 * (2.0 * V.fx * tx * iz2 * iz);
        gtz += GJ11 * (-V.fy * iz2);
        gty += GJ12 * (-V.fy * iz2);
        gtz += GJ12 * (2.0 * V.fy * ty * iz2 * iz);
        gtx += gmx * V.fx * iz;
        gtz -= gmx * V.fx * tx * iz2;
        gty += gmy * V.fy * iz;
        gtz -= gmy * V.fy * ty * iz2;
        gtz += gdepth;
#pragma unroll
        for (int a = 0; a < 3; a++) gm[a] += R[a * 3 + 0] * gtx + R[a * 3 + 1] * gty + R[a * 3 + 2] * gtz;
    }
    // slot 5 summed dL/da a_g = o dL/do over the pixels (o >= alpha_min > 0)
    go /= P.o;
    if (st.isotropic) {
        // one radius for the three axes; no rotation
        if (d_means) {
            d_means[i] += (float)gm[0];
            d_means[n + i] += (float)gm[1];
            d_means[2 * n + i] += (float)gm[2];
        }
        if (d_ls) d_ls[i] += (float)((gs[0] + gs[1] + gs[2]) * P.s[0]);
        if (d_op) d_op[i] += (float)go;
        if (d_col) {
            d_col[i] += (float)gc[0];
            d_col[n + i] += (float)gc[1];
            d_col[2 * n + i] += (float)gc[2];
        }
        return;
    }
    // rotation matrix -> normalised quaternion -> raw quaternion
    double w = g.quats[i], x = g.quats[n + i], y = g.quats[2 * n + i], z = g.quats[3 * n + i];
    double qn = sqrt(w * w + x * x + y * y + z * z);
    double inv = 1.0 / qn;
    w *= inv; x *= inv; y *= inv; z *= inv;
    double gw = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    double gx = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] +
                       w * gR[7] - 2.0 * x * gR[8]);
    double gy = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                       z * gR[7] - 2.0 * y * gR[8]);
    double gz = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] + y * gR[5] +
                       x * gR[6] + y * gR[7]);
    double dot = w * gw + x * gx + y * gy + z * gz;
    if (d_quats) {
        d_quats[i] += (float)((gw - w * dot) * inv);
        d_quats[n + i] += (float)((gx - x * dot) * inv);
        d_quats[2 * n + i] += (float)((gy - y * dot) * inv);
        d_quats[3 * n + i] += (float)((gz - z * dot) * inv);
    }
    if (d_means) {
        d_means[i] += (float)gm[0];
        d_means[n + i] += (float)gm[1];
        d_means[2 * n + i] += (float)gm[2];
    }
    if (d_ls) {
        d_ls[i] += (float)(gs[0] * P.s[0]);
        d_ls[n + i] += (float)(gs[1] * P.s[1]);
        d_ls[2 * n + i] += (float)(gs[2] * P.s[2]);
    }
    if (d_op) d_op[i] += (float)go;
    if (d_col) {
        d_col[i] += (float)gc[0];
        d_col[n + i] += (float)gc[1];
        d_col[2 * n + i] += (float)gc[2];
    }
}

// ---------------------------------------------------------------- scoring
// Rendered form of the trace proxy of Sec. IV-A eq. (7): per view, the sum
// over pixels of the composited uncertainty sum_i u_i a_i T_i.  Only alpha,
// transmittance and uncertainty are composited; nothing is written per pixel.

// mode 0: sum_i u_i a_i T_i (the rendered proxy); mode 1: sum of u_i over
// the contributing splats (the binary-J trace).
//
// The pair loop is cut to the arithmetic the proxy needs.  Staged per splat:
// the mean relative to an origin fixed per 32 x 16 pixel block (a multiple
// of every tile shape, so no pixel's arithmetic depends on the tile), the
// whitening M, log2(opacity) and u; a pixel's offset is then one subtraction
// from a small exact integer, and alpha = min(alpha_max, exp2(log2 o - |Md|^2)).
// Termination is carried by T itself: a pixel whose next transmittance
// would fall below T_min stops with T = 0, after which every splat leaves it
// unchanged, so the loop needs no per-pixel flags; a splat below alpha_min
// enters the update with alpha 0 (T unchanged, exactly).
template <int MODE>
__device__ __forceinline__ float score_weight(float a0, float T) {
    return MODE ? 1.0f : a0 * T;
}

template <int TW, int TH, int B, int MODE>
__device__ __forceinline__ void score_one_tile(const ViewDev* __restrict__ views, int n_views, uint32_t tile,
                                               const uint2* __restrict__ ranges,
                                               const uint32_t* __restrict__ inst_rec, const Records& rec,
                                               const SetDev& st, double* __restrict__ partial,
                                               float4* s_p, float4* s_q, uint32_t* s_r, uint2* s_pb,
                                               double* ws, uint32_t* s_list) {
    constexpr int NT = TW * TH;
    static_assert(32 % TW == 0 && 16 % TH == 0, "tiles must divide the 32 x 16 origin block");
    static_assert(SCORE_STEP == 2, "the list is padded for steps of two");
    const uint32_t vi = view_of_tile(views, n_views, tile);
    const ViewDev& V = views[vi];
    const uint32_t lt = tile - V.tile_off;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int u = tx * TW + (int)(threadIdx.x % TW), v = ty * TH + (int)(threadIdx.x / TW);
    const int ox = origin_x(tx * TW), oy = origin_y(ty * TH);
    // this wave's pixel rectangle (64 consecutive threads = 64 / TW rows of
    // the tile), relative to the origin
    const int wc0 = tx * TW - ox, wc1 = wc0 + TW - 1;
    const int wr0 = ty * TH + (int)(threadIdx.x >> 6) * (64 / TW) - oy, wr1 = wr0 + 64 / TW - 1;
    const bool inside = u < V.W && v < V.H;
    const float lx = (float)(u - ox), ly = (float)(v - oy);
    const float amin = st.alpha_min, amax = st.alpha_max, tmin = st.T_min;
    const float band = REFINE * amin;
    const uint2 rg = ranges[tile];
    const char* sp = reinterpret_cast<const char*>(s_p);
    const char* sq = reinterpret_cast<const char*>(s_q);
    float T = inside ? 1.0f : 0.0f, uu = 0.0f;
    for (uint32_t b = rg.x; b < rg.y; b += B) {
        if (__syncthreads_count(T > 0.0f) == 0) break;
        uint32_t idx = b + threadIdx.x;
        if (threadIdx.x < (uint32_t)B && idx < rg.y) {
            uint32_t r = inst_rec[idx];
            s_r[threadIdx.x] = r;
            const EmitRec e = rec.emit[r];
            s_pb[threadIdx.x] = e.pbox;
            stage_splat(e, ox, oy, s_p[threadIdx.x], s_q[threadIdx.x]);
        }
        __syncthreads();
        const int cnt = (int)min<uint32_t>(B, rg.y - b);
        uint32_t* my = s_list + (threadIdx.x >> 6) * (B + 2);
        int nl = 0;
        if (__ballot(T > 0.0f))
            nl = splat_list<B, SCORE_ELL>(s_pb, s_p, s_q, st.log2_amin, cnt, wc0, wc1, wr0, wr1, ox, oy, my);
        __syncthreads();  // the wave's list is in LDS
        for (int i = 0; i < nl; i += SCORE_STEP) {
            if (!__ballot(T > 0.0f)) break;
            uint32_t ko[SCORE_STEP];
            float as[SCORE_STEP], us[SCORE_STEP];
            bool need = false;
#pragma unroll
            for (int q = 0; q < SCORE_STEP; q++) {
                ko[q] = my[i + q];
                const float4 p = *reinterpret_cast<const float4*>(sp + ko[q]);
                const float4 g = *reinterpret_cast<const float4*>(sq + ko[q]);
                const float dx = lx - p.x, dy = ly - p.y;
                const float w1 = p.z * dx, w2 = fmaf(p.w, dx, g.x * dy);
                const float ex = fmaf(w1, w1, fmaf(w2, w2, -g.w));
                const float a = __builtin_amdgcn_fmed3f(fast_exp2(-ex), 0.0f, amax);
                as[q] = a;
                us[q] = g.z;
                need = need | near_amin(a, amin, band);
            }
            if (__ballot(need)) {
#pragma unroll
                for (int q = 0; q < SCORE_STEP; q++)
                    if (near_amin(as[q], amin, band) & (ko[q] < B * sizeof(float4)))
                        as[q] = redecide(as[q], rec, s_r[ko[q] / sizeof(float4)], u, v, st);
            }
#pragma unroll
            for (int q = 0; q < SCORE_STEP; q++) {
                const bool ok = as[q] >= amin;
                const float a0 = ok ? as[q] : 0.0f;
                const float Tn = fmaf(-a0, T, T);
                const bool live = Tn >= tmin;
                const float w = score_weight<MODE>(a0, T);
                uu = (ok & live) ? fmaf(us[q], w, uu) : uu;
                T = live ? Tn : 0.0f;
            }
        }
    }
    float s = wave_sum_f(uu);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = (double)s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int w = 0; w < NT / 64; w++) acc += ws[w];
        partial[tile] = acc;
    }
    __syncthreads();
}

template <int TW, int TH, int B>
__global__ __launch_bounds__(TW * TH) void k_score_plain(const ViewDev* __restrict__ views, int n_views,
                                                         uint32_t tile_begin, const uint2* __restrict__ ranges,
                                                         const uint32_t* __restrict__ inst_rec, Records rec,
                                                         SetDev st, int mode, double* __restrict__ partial) {
    constexpr int NT = TW * TH;
    static_assert(B <= NT, "batch larger than the tile");
    __shared__ float4 s_p[B + 1], s_q[B + 1];
    __shared__ uint32_t s_r[B];
    __shared__ uint2 s_pb[B];
    __shared__ double ws[NT / 64];
    __shared__ __align__(8) uint32_t s_list[NT / 64 * (B + 2)];
    stage_null_splat<B>(s_p, s_q);
    if (mode)
        score_one_tile<TW, TH, B, 1>(views, n_views, tile_begin + blockIdx.x, ranges, inst_rec, rec, st, partial,
                                     s_p, s_q, s_r, s_pb, ws, s_list);
    else
        score_one_tile<TW, TH, B, 0>(views, n_views, tile_begin + blockIdx.x, ranges, inst_rec, rec, st, partial,
                                     s_p, s_q, s_r, s_pb, ws, s_list);
}

template <int TW, int TH, int B>
__global__ __launch_bounds__(TW * TH) __attribute__((amdgpu_waves_per_eu(6))) void k_score_persistent(const ViewDev* __restrict__ views,
                                                              const Header* __restrict__ hdr,
                                                              const uint2* __restrict__ ranges,
                                                              const uint32_t* __restrict__ tile_order,
                                                              const uint32_t* __restrict__ inst_rec, Records rec,
                                                              SetDev st, int mode, double* __restrict__ partial,
                                                              uint32_t* __restrict__ queue,
                                                              const uint32_t* __restrict__ flags) {
    constexpr int NT = TW * TH;
    static_assert(B <= NT, "batch larger than the tile");
    if (*flags) return;  // overflowed binning: results are reported invalid
    __shared__ float4 s_p[B + 1], s_q[B + 1];
    __shared__ uint32_t s_r[B];
    __shared__ uint2 s_pb[B];
    __shared__ double ws[NT / 64];
    __shared__ __align__(8) uint32_t s_list[NT / 64 * (B + 2)];
    stage_null_splat<B>(s_p, s_q);
    __shared__ uint32_t s_item;
    const uint32_t total = hdr->tiles_total;
    const int nv = (int)hdr->n_views;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        const uint32_t tile = tile_order ? tile_order[item] : item;
        if (mode)
            score_one_tile<TW, TH, B, 1>(views, nv, tile, ranges, inst_rec, rec, st, partial, s_p, s_q, s_r, s_pb,
                                         ws, s_list);
        else
            score_one_tile<TW, TH, B, 0>(views, nv, tile, ranges, inst_rec, rec, st, partial, s_p, s_q, s_r, s_pb,
                                         ws, s_list);
    }
}

__global__ __launch_bounds__(256) void k_score_reduce(const ViewDev* __restrict__ views,
                                                      const Header* __restrict__ hdr,
                                                      const double* __restrict__ partial,
                                                      double* __restrict__ scores,
                                                      const uint32_t* __restrict__ flags) {
    __shared__ double ws[4];
    const uint32_t v = blockIdx.x;
    if (v >= hdr->n_views) return;
    if (*flags) {  // an overflowed or inconsistent binning: the scores are invalid
        if (threadIdx.x == 0) scores[v] = __builtin_nan("");
        return;
    }
    const ViewDev& V = views[v];
    const uint32_t nt = (uint32_t)(V.tiles_x * V.tiles_y);
    double s = 0.0;
    for (uint32_t t = threadIdx.x; t < nt; t += 256) s += partial[V.tile_off + t];
    s = wave_sum_d(s);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) scores[v] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void k_export(const uint32_t* __restrict__ tile_key,
                                                const uint32_t* __restrict__ inst_rec,
                                                const uint32_t* __restrict__ K_dev, uint32_t cap, Records rec,
                                                uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    uint32_t K = min(*K_dev, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) {
        uint32_t r = inst_rec[i];
        if (keys) keys[i] = ((uint64_t)tile_key[i] << 32) | __float_as_uint(rec.attr[r].w);
        if (vals) vals[i] = rec.emit[r].gid;
    }
}

// Planar copies of the record fields for inspection (all outputs nullable).
__global__ __launch_bounds__(256) void k_export_records(const uint32_t* __restrict__ R_dev, uint32_t cap, Records rec,
                                                        double* __restrict__ mean2d, double* __restrict__ conic,
                                                        int32_t* __restrict__ pbox, uint32_t* __restrict__ depth_bits,
                                                        uint32_t* __restrict__ gid, uint32_t* __restrict__ view,
                                                        uint32_t* __restrict__ ntiles) {
    const uint32_t R = min(*R_dev, cap);
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += gridDim.x * blockDim.x) {
        const EmitRec e = rec.emit[r];
        if (mean2d) {
            mean2d[r] = (double)e.g0.x + (double)e.g0.z;
            mean2d[(uint64_t)R + r] = (double)e.g0.y + (double)e.g0.w;
        }
        if (conic) {
            const double4 q = rec.q64[r];
            conic[r] = q.x;
            conic[(uint64_t)R + r] = q.y;
            conic[2 * (uint64_t)R + r] = q.z;
        }
        if (pbox) {
            pbox[r] = (int32_t)(e.pbox.x & 0xffffu);
            pbox[(uint64_t)R + r] = (int32_t)(e.pbox.x >> 16);
            pbox[2 * (uint64_t)R + r] = (int32_t)(e.pbox.y & 0xffffu);
            pbox[3 * (uint64_t)R + r] = (int32_t)(e.pbox.y >> 16);
        }
        if (depth_bits) depth_bits[r] = __float_as_uint(rec.attr[r].w);
        if (gid) gid[r] = e.gid;
        if (view) view[r] = e.view;
        if (ntiles) ntiles[r] = e.ntiles;
    }
}

__global__ __launch_bounds__(256) void k_sum_u32_pair(const uint32_t* __restrict__ a,
                                                      const uint32_t* __restrict__ b, uint64_t n,
                                                      unsigned long long* __restrict__ out) {
    __shared__ unsigned long long ws[2][4];
    unsigned long long sa = 0, sb = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        sa += a[i];
        sb += b[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sa += __shfl_xor(sa, o, 64);
        sb += __shfl_xor(sb, o, 64);
    }
    if (lane_id() == 0) {
        ws[0][threadIdx.x >> 6] = sa;
        ws[1][threadIdx.x >> 6] = sb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(out, ws[0][0] + ws[0][1] + ws[0][2] + ws[0][3]);
        atomicAdd(out + 1, ws[1][0] + ws[1][1] + ws[1][2] + ws[1][3]);
    }
}

// ------------------------------------------------ view utility of eq. (8)
// Sec. IV-B: v(x, g) = 1 when the Gaussian is in the field of view (camera
// depth in (z_near, range], projected mean inside the image, no occlusion);
// xi = |H visible| - lambda |L visible| with H / L the Gaussians above / below
// the uncertainty thresholds.  The visibility test runs in binary32 and falls
// back to the exact binary64 expression within a margin of every border.

constexpr int UT_THREADS = 256;
constexpr double FIX_SCALE = 1099511627776.0;  // 2^40: uncertainty sums in fixed point

__device__ __forceinline__ bool fov_exact(double mx0, double my0, double mz0, const ViewDev& V, double z_near,
                                          double range) {
    double dx = mx0 - V.T[0], dy = my0 - V.T[1], dz = mz0 - V.T[2];
    const double* R = V.R;
    double tx = (dx * R[0] + dy * R[3]) + dz * R[6];
    double ty = (dx * R[1] + dy * R[4]) + dz * R[7];
    double tz = (dx * R[2] + dy * R[5]) + dz * R[8];
    if (!(tz > z_near) || !(tz <= range)) return false;
    double mx = V.fx * tx / tz + V.cx;
    double my = V.fy * ty / tz + V.cy;
    return mx >= 0.0 && mx <= (double)(V.W - 1) && my >= 0.0 && my <= (double)(V.H - 1);
}

// A view's binary32 values for the field-of-view screen (the camera's own
// binary32 values: its binary64 fields are these, widened).
struct ViewF {
    float T[3], R[9], fx, fy, cx, cy, W1, H1, kf, pad;
};

__device__ __forceinline__ ViewF view_f(const ViewDev& V) {
    ViewF f;
#pragma unroll
    for (int k = 0; k < 3; k++) f.T[k] = V.Tf[k];
#pragma unroll
    for (int k = 0; k < 9; k++) f.R[k] = V.Rf[k];
    f.fx = V.fxf;
    f.fy = V.fyf;
    f.cx = V.cxf;
    f.cy = V.cyf;
    f.W1 = (float)(V.W - 1);
    f.H1 = (float)(V.H - 1);
    f.kf = 1e-3f * (V.fxf + V.fyf);
    f.pad = 0.0f;
    return f;
}

// Binary32 screen of the field-of-view test: 1 certainly visible, 0
// certainly not, -1 too close to a depth limit or an image border to tell
// (the binary64 test then decides).  Branch-free: every Gaussian of a wave
// takes the same instructions.
__device__ __forceinline__ int fov_fast(float x, float y, float z, const ViewF& V, float z_near, float range) {
    const float dx = x - V.T[0], dy = y - V.T[1], dz = z - V.T[2];
    const float mag = fabsf(dx) + fabsf(dy) + fabsf(dz) + 1.0f;
    const float tx = fmaf(dz, V.R[6], fmaf(dy, V.R[3], dx * V.R[0]));
    const float ty = fmaf(dz, V.R[7], fmaf(dy, V.R[4], dx * V.R[1]));
    const float tz = fmaf(dz, V.R[8], fmaf(dy, V.R[5], dx * V.R[2]));
    const float ez = 1e-5f * mag;
    // hardware reciprocal (within an ulp or two): far inside the margin m
    const float iz = __builtin_amdgcn_rcpf(tz);
    const float mx = fmaf(V.fx * tx, iz, V.cx);
    const float my = fmaf(V.fy * ty, iz, V.cy);
    const float m = fmaf(1e-3f, 1.0f + fabsf(mx) + fabsf(my), V.kf * mag * iz);
    const bool out = (tz <= z_near - ez) | (tz > range + ez) | (mx < -m) | (mx > V.W1 + m) | (my < -m) |
                     (my > V.H1 + m);
    const bool in = (tz > z_near + ez) & (tz <= range - ez) & (mx > m) & (mx < V.W1 - m) & (my > m) &
                    (my < V.H1 - m);
    return out ? 0 : (in ? 1 : -1);
}

__device__ __noinline__ bool fov_exact_call(float x, float y, float z, const ViewDev& V, float z_near, float range) {
    return fov_exact((double)x, (double)y, (double)z, V, (double)z_near, (double)range);
}

// Work split: a block takes UT_VB views (their screen values in LDS) and a
// share of the Gaussians, streamed UT_G per thread per step with coalesced
// loads; each thread keeps its counts and fixed-point sum per view in
// registers and the wave reduces them once at the end.  Counts and sums are
// integers: the result does not depend on the order.
constexpr int UT_VB = 8;
constexpr int UT_G = 4;

__global__ __launch_bounds__(UT_THREADS) void k_view_utility(GaussDev g, const ViewDev* __restrict__ views, int nv,
                                                             float z_near, float range,
                                                             const double* __restrict__ lo_hi,
                                                             unsigned long long* __restrict__ cnt_h,
                                                             unsigned long long* __restrict__ cnt_l,
                                                             unsigned long long* __restrict__ fix_u) {
    __shared__ ViewF s_v[UT_VB];
    const int v0 = (int)blockIdx.y * UT_VB;
    const int nvb = min(UT_VB, nv - v0);
    if ((int)threadIdx.x < nvb) s_v[threadIdx.x] = view_f(views[v0 + threadIdx.x]);
    __syncthreads();
    const double lo = lo_hi[0], hi = lo_hi[1];
    const int64_t n = g.n;
    uint32_t ch[UT_VB], cl[UT_VB];
    unsigned long long su[UT_VB];
#pragma unroll
    for (int b = 0; b < UT_VB; b++) {
        ch[b] = cl[b] = 0u;
        su[b] = 0ull;
    }
    constexpr int64_t CH = (int64_t)UT_THREADS * UT_G;
    for (int64_t base = (int64_t)blockIdx.x * CH; base < n; base += (int64_t)gridDim.x * CH) {
        float x[UT_G], y[UT_G], z[UT_G];
        unsigned long long fu[UT_G];
        uint32_t ok = 0, isH = 0, isL = 0;  // bit j: Gaussian j of this thread
#pragma unroll
        for (int j = 0; j < UT_G; j++) {
            const int64_t i = base + (int64_t)j * UT_THREADS + threadIdx.x;
            x[j] = y[j] = z[j] = 0.0f;
            fu[j] = 0ull;
            if (i < n) {
                x[j] = g.means[i];
                y[j] = g.means[n + i];
                z[j] = g.means[2 * n + i];
                const float u = g.uncert[i];
                if (isfinite(x[j]) && isfinite(y[j]) && isfinite(z[j])) ok |= 1u << j;
                if ((double)u > hi) isH |= 1u << j;
                if ((double)u < lo) isL |= 1u << j;
                fu[j] = (isfinite(u) && u > 0.0f) ? (unsigned long long)((double)u * FIX_SCALE) : 0ull;
            }
        }
        // the views' values are read from LDS in every step (a compiler
        // barrier keeps them from being hoisted into registers, which would
        // cost occupancy)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int b = 0; b < UT_VB; b++) {
            if (b >= nvb) break;
            const ViewF V = s_v[b];
            uint32_t vis = 0, unsure = 0;
#pragma unroll
            for (int j = 0; j < UT_G; j++) {
                const int f = fov_fast(x[j], y[j], z[j], V, z_near, range);
                vis |= (uint32_t)(f == 1) << j;
                unsure |= (uint32_t)(f < 0) << j;
            }
            unsure &= ok;
            // near a border or the depth limits the binary64 test decides
            if (__ballot(unsure != 0)) {
#pragma unroll
                for (int j = 0; j < UT_G; j++)
                    if (((unsure >> j) & 1u) && fov_exact_call(x[j], y[j], z[j], views[v0 + b], z_near, range))
                        vis |= 1u << j;
            }
            vis &= ok;
            ch[b] += __popc(vis & isH);
            cl[b] += __popc(vis & isL);
#pragma unroll
            for (int j = 0; j < UT_G; j++) su[b] += ((vis >> j) & 1u) ? fu[j] : 0ull;
        }
    }
#pragma unroll
    for (int b = 0; b < UT_VB; b++) {
        if (b >= nvb) break;
        unsigned long long h = ch[b], l = cl[b], t = su[b];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            h += __shfl_xor(h, o, 64);
            l += __shfl_xor(l, o, 64);
            t += __shfl_xor(t, o, 64);
        }
        if (lane_id() == 0) {
            if (h) atomicAdd(cnt_h + v0 + b, h);
            if (l) atomicAdd(cnt_l + v0 + b, l);
            if (t) atomicAdd(fix_u + v0 + b, t);
        }
    }
}

__global__ void k_utility_finish(int nv, const unsigned long long* __restrict__ cnt_h,
                                 const unsigned long long* __restrict__ cnt_l,
                                 const unsigned long long* __restrict__ fix_u, double lambda,
                                 int64_t* __restrict__ n_high, int64_t* __restrict__ n_low,
                                 double* __restrict__ sum_u, double* __restrict__ xi) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        if (n_high) n_high[v] = (int64_t)cnt_h[v];
        if (n_low) n_low[v] = (int64_t)cnt_l[v];
        if (sum_u) sum_u[v] = (double)fix_u[v] / FIX_SCALE;
        if (xi) xi[v] = (double)cnt_h[v] - lambda * (double)cnt_l[v];
    }
}

// mean and population standard deviation of u, binary64, fixed reduction order
__global__ __launch_bounds__(256) void k_moments(const float* __restrict__ u, int64_t n, int pass,
                                                 const double* __restrict__ mean_in, double* __restrict__ partial) {
    __shared__ double ws[4];
    const double mean = pass ? *mean_in : 0.0;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double d = (double)u[i] - mean;
        s += pass ? d * d : (double)u[i];
    }
    s = wave_sum_d(s);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ void k_moments_finish(const double* __restrict__ partial, int nb, int64_t n, int pass, double k,
                                 double* __restrict__ mean_io, double* __restrict__ lo_hi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += partial[b];
    if (pass == 0) {
        *mean_io = n > 0 ? s / (double)n : 0.0;
    } else {
        double sd = n > 0 ? sqrt(s / (double)n) : 0.0;
        lo_hi[0] = *mean_io - k * sd;
        lo_hi[1] = *mean_io + k * sd;
    }
}

// eq. (10): utility of trajectory t = sum of xi over its states
// [off[t], off[t+1]) in order; best = first trajectory of maximal utility.
__global__ void k_traj_select(const double* __restrict__ xi, const int32_t* __restrict__ off, int n_traj,
                              double* __restrict__ util, int32_t* __restrict__ best) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int b = -1;
    double bv = 0.0;
    for (int t = 0; t < n_traj; t++) {
        double s = 0.0;
        for (int k = off[t]; k < off[t + 1]; k++) s += xi[k];
        if (util) util[t] = s;
        if (b < 0 || s > bv) {
            b = t;
            bv = s;
        }
    }
    *best = b;
}

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 65535u * 16u) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ------------------------------------------------- uncertainty bookkeeping
// Sec. IV-A: the uncertainty of a Gaussian is the magnitude of the change of
// its mean over a map update (squared for the -sq variant); a Gaussian whose
// mean did not change keeps its previous value.  Formed in binary64 as
// sqrt((dx dx + dy dy) + dz dz) and rounded once to binary32.

__global__ __launch_bounds__(256) void k_uncertainty_update(int64_t n, const float* __restrict__ prev,
                                                            const float* __restrict__ cur,
                                                            const float* u_prev, int squared, float* u_out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double dx = (double)cur[i] - (double)prev[i];
        const double dy = (double)cur[n + i] - (double)prev[n + i];
        const double dz = (double)cur[2 * n + i] - (double)prev[2 * n + i];
        float u;
        if (dx == 0.0 && dy == 0.0 && dz == 0.0) {
            u = u_prev[i];
        } else {
            const double s2 = (dx * dx + dy * dy) + dz * dz;
            u = (float)(squared ? s2 : sqrt(s2));
        }
        u_out[i] = u;
    }
}

// ---------------------------------------------------------- region utility
// Sec. IV-B (high-level planner; the 2.5 m edge is set in Sec. IV-C): cuboid
// regions of edge `size` over the box [lo, lo + dims size);
// a Gaussian belongs to region (ix, iy, iz), index ix + nx (iy + ny iz), with
// i = floor((mu - lo) / size) in binary64.  Counts are exact; sums are in
// fixed point with 2^-32 resolution (|u| < 2^20 per value), so the result
// does not depend on the order of the atomics.  A non-finite or out-of-range
// u marks its region (its sum and mean become NaN).

constexpr double RG_FIX = 4294967296.0;  // 2^32
constexpr int RG_LDS = 2048;             // regions privatised in LDS per block

__device__ __forceinline__ int64_t region_of(const float* __restrict__ means, int64_t n, int64_t i, double lx,
                                             double ly, double lz, double size, int nx, int ny, int nz) {
    const double fx = floor(((double)means[i] - lx) / size);
    const double fy = floor(((double)means[n + i] - ly) / size);
    const double fz = floor(((double)means[2 * n + i] - lz) / size);
    if (!(fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny && fz >= 0.0 && fz < (double)nz)) return -1;
    return (int64_t)fx + (int64_t)nx * ((int64_t)fy + (int64_t)ny * (int64_t)fz);
}

__global__ __launch_bounds__(256) void k_region_utility(int64_t n, const float* __restrict__ means,
                                                        const float* __restrict__ u, double lx, double ly,
                                                        double lz, double size, int nx, int ny, int nz,
                                                        unsigned long long* __restrict__ cnt,
                                                        unsigned long long* __restrict__ fix,
                                                        unsigned int* __restrict__ bad) {
    __shared__ unsigned long long s_cnt[RG_LDS], s_fix[RG_LDS];
    const int64_t nr = (int64_t)nx * ny * nz;
    const bool lds = nr <= RG_LDS;
    if (lds) {
        for (int r = threadIdx.x; r < nr; r += blockDim.x) s_cnt[r] = s_fix[r] = 0ull;
        __syncthreads();
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = region_of(means, n, i, lx, ly, lz, size, nx, ny, nz);
        if (r < 0) continue;
        const float v = u[i];
        const bool ok = isfinite(v) && fabsf(v) < 1048576.0f;
        const long long f = ok ? __double2ll_rn((double)v * RG_FIX) : 0ll;
        if (!ok) atomicOr(&bad[r], 1u);
        if (lds) {
            atomicAdd(&s_cnt[r], 1ull);
            atomicAdd(&s_fix[r], (unsigned long long)f);  // two's complement: signed sums wrap correctly
        } else {
            atomicAdd(&cnt[r], 1ull);
            atomicAdd(&fix[r], (unsigned long long)f);
        }
    }
    if (lds) {
        __syncthreads();
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {
            if (s_cnt[r]) {
                atomicAdd(&cnt[r], s_cnt[r]);
                atomicAdd(&fix[r], s_fix[r]);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_region_finish(int64_t nr, const unsigned long long* __restrict__ cnt,
                                                       const unsigned long long* __restrict__ fix,
                                                       const unsigned int* __restrict__ bad,
                                                       int64_t* __restrict__ count, double* __restrict__ sum,
                                                       double* __restrict__ mean) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nr; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = (int64_t)cnt[r];
        const double sm = bad[r] ? __longlong_as_double(0x7ff8000000000000ll) : (double)(long long)fix[r] / RG_FIX;
        if (count) count[r] = c;
        if (sum) sum[r] = sm;
        if (mean) mean[r] = c ? sm / (double)c : 0.0;
    }
}

}  // namespace

// ================================================================ launchers

#define RTG_TILE_DISPATCH(TW_, TH_, CALL)                      \
    if (tw == 8 && th == 8) {                                  \
        constexpr int TW_ = 8, TH_ = 8;                        \
        CALL;                                                  \
    } else if (tw == 32 && th == 8) {                          \
        constexpr int TW_ = 32, TH_ = 8;                       \
        CALL;                                                  \
    } else {                                                   \
        constexpr int TW_ = 16, TH_ = 16;                      \
        CALL;                                                  \
    }


// Tile and staging batch: batch 0 means one splat per thread of the tile;
// otherwise one of 32, 64, 128, 256 not above the tile's pixel count
// (checked by the library before any launch).
#define RTG_BATCH_DISPATCH(TW_, TH_, B_, CALL)                 \
    RTG_TILE_DISPATCH(TW_, TH_, {                              \
        const int bsel_ = batch > 0 ? batch : TW_ * TH_;       \
        if (bsel_ == 32) {                                     \
            constexpr int B_ = 32;                             \
            CALL;                                              \
        } else if (bsel_ == 64 || TW_ * TH_ == 64) {           \
            constexpr int B_ = 64;                             \
            CALL;                                              \
        } else if (bsel_ == 128) {                             \
            constexpr int B_ = (TW_ * TH_ >= 128) ? 128 : 64;  \
            CALL;                                              \
        } else {                                               \
            constexpr int B_ = (TW_ * TH_ >= 256) ? 256 : 64;  \
            CALL;                                              \
        }                                                      \
    })

int score_persistent_blocks(int tw, int th, int batch) {
    int per_cu = 0;
    hipError_t e = hipSuccess;
    RTG_BATCH_DISPATCH(TW, TH, B,
                       (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_score_persistent<TW, TH, B>,
                                                                         TW * TH, 0)));
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * device_cu_count();
}

void view_utility(const GaussDev& g, const ViewDev* views, int nv, float z_near, float range, const double* lo_hi,
                  unsigned long long* acc, double lambda, int64_t* n_high, int64_t* n_low, double* sum_u, double* xi,
                  hipStream_t s) {
    fill_u32(reinterpret_cast<uint32_t*>(acc), 0u, (uint64_t)6 * nv, s);
    if (g.n > 0) {
        // about 2048 blocks over (Gaussian shares) x (groups of UT_VB views)
        const unsigned gy = (unsigned)((nv + UT_VB - 1) / UT_VB);
        const unsigned gmax = grid_for(((uint64_t)g.n + UT_G - 1) / UT_G, UT_THREADS, 1u << 20);
        const unsigned gx = std::max(1u, std::min(gmax, (2048u + gy - 1) / gy));
        k_view_utility<<<dim3(gx, gy), UT_THREADS, 0, s>>>(g, views, nv, z_near, range, lo_hi, acc, acc + nv,
                                                           acc + 2 * nv);
    }
    k_utility_finish<<<(nv + 255) / 256, 256, 0, s>>>(nv, acc, acc + nv, acc + 2 * nv, lambda, n_high, n_low, sum_u,
                                                      xi);
}

void uncertainty_thresholds(const float* u, int64_t n, double k, double* scratch, double* lo_hi, hipStream_t s) {
    const int nb = (int)grid_for((uint64_t)std::max<int64_t>(n, 1), 256, 512);
    double* mean = scratch;
    double* partial = scratch + 1;
    k_moments<<<nb, 256, 0, s>>>(u, n, 0, mean, partial);
    k_moments_finish<<<1, 64, 0, s>>>(partial, nb, n, 0, k, mean, lo_hi);
    k_moments<<<nb, 256, 0, s>>>(u, n, 1, mean, partial);
    k_moments_finish<<<1, 64, 0, s>>>(partial, nb, n, 1, k, mean, lo_hi);
}

void trajectory_select(const double* xi, const int32_t* offsets, int n_traj, double* util, int32_t* best,
                       hipStream_t s) {
    k_traj_select<<<1, 64, 0, s>>>(xi, offsets, n_traj, util, best);
}

int device_cu_count() {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cu;
}

void fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    k_fill_u32<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, v, n);
}

void project_count(const GaussDev& g, const ViewDev* views, const Header* hdr, int n_views_cap, SetDev st,
                   uint32_t* cnt, uint32_t* mask, hipStream_t s) {
    if (g.n == 0) return;
    int words = (n_views_cap + 31) / 32;
    // one thread per Gaussian: the grid covers every n below 2^31
    if (n_views_cap <= PC_VIEWS)
        k_project_count<true><<<grid_for(g.n, 256, 0xffffffffu), 256, 0, s>>>(g, views, hdr, words, st, cnt, mask);
    else
        k_project_count<false><<<grid_for(g.n, 256, 0xffffffffu), 256, 0, s>>>(g, views, hdr, words, st, cnt, mask);
}

// log2 of a power-of-two tile side (8, 16 or 32)
static int ilog2(int x) {
    int k = 0;
    while ((1 << (k + 1)) <= x) k++;
    return k;
}

void project_emit(const GaussDev& g, const ViewDev* views, const Header* hdr, int n_views_cap, SetDev st,
                  int tw, int th, const uint32_t* mask, const uint32_t* cnt, const uint32_t* rec_off,
                  const uint32_t* R_dev, uint32_t rec_cap, Records rec, uint32_t* sortkey, uint32_t* order,
                  bool write_attr, uint32_t* chunk_g, uint32_t* flags, hipStream_t s) {
    (void)hdr;
    if (g.n == 0 || rec_cap == 0) return;
    int words = (n_views_cap + 31) / 32;
    k_chunk_owners<<<grid_for(g.n, 256, 16384), 256, 0, s>>>(cnt, rec_off, g.n, R_dev, rec_cap, chunk_g);
    k_project_emit<<<grid_for(rec_cap, PE_THREADS, 32768), PE_THREADS, 0, s>>>(
        g, views, words, st, ilog2(tw), ilog2(th), mask, rec_off, R_dev, rec_cap, rec, sortkey, order,
        write_attr ? 1 : 0, chunk_g, flags);
}

int scan_blocks(uint64_t cap) {
    uint64_t b = (cap + SC_TILE - 1) / SC_TILE;
    if (b < 1) b = 1;
    if (b > SC_MAX_BLOCKS) b = SC_MAX_BLOCKS;
    return (int)b;
}

void scan_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, const uint32_t* n_dev, uint32_t cap,
              uint32_t* total, uint32_t* flags, ScanWs ws, hipStream_t s) {
    int nb = scan_blocks(cap);
    k_scan_reduce<<<nb, SC_THREADS, 0, s>>>(in, gather, n_dev, cap, ws.partial);
    k_scan_down<<<nb, SC_THREADS, 0, s>>>(in, gather, out, n_dev, cap, ws.partial, total, flags);
}

// Grid of a pass with digits of db bits: one block per tile of input, up to
// RS_MAX_BLOCKS.  Wide digits make the per-block offset computation cost
// 2^db x blocks loads per block, so for them inputs of up to
// RS_FUSED_BLOCKS * 8 tiles use at most RS_FUSED_BLOCKS blocks, each walking
// several tiles, and need no separate offset scan.
static int sort_blocks_tile(uint64_t cap, int db, int tile) {
    uint64_t t = (cap + tile - 1) / tile;
    if (t < 1) t = 1;
    if (db > 8 && t <= (uint64_t)RS_FUSED_BLOCKS * 8) return (int)std::min<uint64_t>(t, RS_FUSED_BLOCKS);
    return (int)std::min<uint64_t>(t, RS_MAX_BLOCKS);
}

// The block count of the 256-thread form (at least that of the 512-thread one).
int sort_blocks(uint64_t cap, int db) { return sort_blocks_tile(cap, db, RS_TILE); }

size_t sort_hist_words(uint64_t cap) {
    return (size_t)(1u << RS_MAX_DB) * (size_t)std::max(sort_blocks(cap, 8), sort_blocks(cap, RS_MAX_DB));
}

template <int DB, int NT>
static void rs_pass(uint32_t* ki, uint32_t* vi, uint32_t* ko, uint32_t* vo, const uint32_t* n_dev, uint32_t cap,
                    int shift, int bits, SortWs ws, const uint32_t* gsrc, uint32_t* gout, hipStream_t s) {
    const int nb = sort_blocks_tile(cap, DB, NT * RS_IPT);
    const int fused = nb <= RS_FUSED_BLOCKS;
    k_rs_upsweep<DB, NT><<<nb, NT, 0, s>>>(ki, n_dev, cap, shift, bits, ws.hist, fused);
    if (!fused) {
        // table of 2^DB * nb counts, a size known here: the multi-block scan,
        // in place
        const uint32_t count = (uint32_t)((1u << DB) * nb);
        int sb = scan_blocks(count);
        k_scan_reduce<<<sb, SC_THREADS, 0, s>>>(ws.hist, nullptr, nullptr, count, ws.partial);
        k_scan_down<<<sb, SC_THREADS, 0, s>>>(ws.hist, nullptr, ws.hist, nullptr, count, ws.partial, nullptr,
                                              nullptr);
    }
    // 8-bit passes stage their scatter in LDS; the 11-bit one writes directly (its
    // per-wave tables already take 32 KB of LDS)
    k_rs_scatter<DB, DB == 8, NT><<<nb, NT, 0, s>>>(ki, vi, ko, vo, n_dev, cap, shift, bits, ws.hist, fused,
                                                     gsrc, gout);
}

// The nbits are split into the fewest passes of at most max_db bits, as
// evenly as possible; passes of up to 8 bits use 256 bins.
int radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev, uint32_t cap,
               int nbits, int max_db, SortWs ws, hipStream_t s, const uint32_t* gsrc, uint32_t* gout) {
    max_db = std::max(1, std::min(max_db, RS_MAX_DB));
    const int passes = std::max(1, (nbits + max_db - 1) / max_db);
    uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
    int shift = 0;
    for (int p = 0; p < passes; p++) {
        const int bits = nbits / passes + (p < nbits % passes ? 1 : 0);
        const bool last = p + 1 == passes;
        const uint32_t* gs = last ? gsrc : nullptr;
        uint32_t* go = last ? gout : nullptr;
        if (bits <= 8 && cap >= RS_BIG_ITEMS)
            rs_pass<8, RS_THREADS_BIG>(ki, vi, ko, vo, n_dev, cap, shift, std::max(bits, 1), ws, gs, go, s);
        else if (bits <= 8)
            rs_pass<8, RS_THREADS>(ki, vi, ko, vo, n_dev, cap, shift, std::max(bits, 1), ws, gs, go, s);
        else
            rs_pass<RS_MAX_DB, RS_THREADS>(ki, vi, ko, vo, n_dev, cap, shift, bits, ws, gs, go, s);
        shift += bits;
        uint32_t* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    return passes & 1;
}

void emit_instances(const uint32_t* order, const uint32_t* R_dev, uint32_t rec_cap, const uint32_t* K_dev,
                    Records rec, const ViewDev* views, const uint32_t* inst_off, int tw, int th, SetDev st,
                    uint32_t inst_cap, uint32_t* tile_key, uint32_t* inst_rec, uint2* ranges, uint32_t tiles_cap,
                    uint32_t* flags, hipStream_t s) {
    unsigned grid = grid_for(std::max<uint32_t>(inst_cap, 1), EM_ITEMS, 16384);
    k_emit_instances<<<grid, EM_THREADS, 0, s>>>(order, R_dev, rec_cap, K_dev, rec, views, inst_off, ilog2(tw),
                                                 ilog2(th), st.log2_amin, inst_cap, tile_key, inst_rec, ranges,
                                                 tiles_cap, flags);
}

void tile_ranges(const uint32_t* tile_key, const uint32_t* K_dev, uint32_t inst_cap, uint2* ranges,
                 uint32_t tiles_cap, const uint32_t* flags, hipStream_t s) {
    k_tile_ranges<<<grid_for((inst_cap + 3) / 4, 256, 16384), 256, 0, s>>>(tile_key, K_dev, inst_cap, ranges,
                                                                           tiles_cap, flags);
}

void tile_order(const uint2* ranges, const Header* hdr, uint32_t tiles_cap, uint32_t* ws, uint32_t* order,
                hipStream_t s) {
    if (tiles_cap == 0) return;
    fill_u32(ws, 0u, 2 * TO_BUCKETS, s);
    const unsigned grid = grid_for(tiles_cap, 256, 1024);
    k_tile_order_count<<<grid, 256, 0, s>>>(ranges, hdr, tiles_cap, ws);
    k_tile_order_place<<<grid, 256, 0, s>>>(ranges, hdr, tiles_cap, ws, ws + TO_BUCKETS, order);
}

void render_forward(int tw, int th, int batch, const ViewDev* views, int n_views,
                    uint32_t tiles_total, const uint2* ranges, const uint32_t* tile_order, const uint32_t* inst_rec,
                    Records rec, SetDev st, RenderOut out, const uint32_t* flags, hipStream_t s) {
    if (tiles_total == 0) return;
    if (out.unc) {
        RTG_BATCH_DISPATCH(TW, TH, B, (k_render_fwd<TW, TH, B, true><<<tiles_total, TW * TH, 0, s>>>(
                                          views, n_views, ranges, tile_order, inst_rec, rec, st, out, flags)));
    } else {
        RTG_BATCH_DISPATCH(TW, TH, B, (k_render_fwd<TW, TH, B, false><<<tiles_total, TW * TH, 0, s>>>(
                                          views, n_views, ranges, tile_order, inst_rec, rec, st, out, flags)));
    }
}

void loss_l1(const ViewDev* views, int n_views, int max_pix, const float* rgb, const float* depth,
             const float* trgb, const float* tdepth, float w_depth, float* d_rgb, float* d_depth, double* partial,
             int partial_cap, double* loss, hipStream_t s) {
    unsigned bx = grid_for((uint64_t)max_pix, 256, 1u << 30);
    (void)partial_cap;
    dim3 grid(bx, n_views);
    k_loss<<<grid, 256, 0, s>>>(views, rgb, depth, trgb, tdepth, w_depth, d_rgb, d_depth, partial);
    k_sum_partials<<<1, SP_THREADS, 0, s>>>(partial, (int)(bx * n_views), loss);
}

// Waves per tile for the backward: enough workgroups to fill the chip on
// frames with few tiles, one wave per tile otherwise (RTG_BWD_WAVES overrides).
static int backward_waves(int tw, int th, uint32_t tiles) {
    static int forced = -1;
    if (forced < 0) {
        const char* e = getenv("RTG_BWD_WAVES");
        forced = e ? atoi(e) : 0;
    }
    const int nb8 = tw * th / 64;
    int nw = 1;
    if (forced == 1 || forced == 2 || forced == 4) nw = forced;
    else {
        const uint32_t cu = (uint32_t)std::max(device_cu_count(), 1);
        if (tiles < 16 * cu) nw = 2;
    }
    while (nw > nb8) nw >>= 1;
    return nw;
}

// One wave per tile runs the compacted form; two or four the masked one.
template <int TW, int TH, int NW>
static void launch_bwd(bool au, uint32_t tiles_total, hipStream_t s, const ViewDev* views, int n_views,
                       const uint2* ranges, const uint32_t* tile_order, const uint32_t* inst_rec, Records rec,
                       SetDev st, const float* T_final,
                       const uint32_t* n_last, const float* d_rgb, const float* d_depth, const float* d_alpha,
                       const float* d_unc, double* g2d, const uint32_t* flags) {
    if constexpr (NW == 1) {
        if (au)
            k_render_bwd1<TW, TH, true><<<tiles_total, 64, 0, s>>>(views, n_views, ranges, tile_order, inst_rec, rec, st, T_final,
                                                                   n_last, d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
        else
            k_render_bwd1<TW, TH, false><<<tiles_total, 64, 0, s>>>(views, n_views, ranges, tile_order, inst_rec, rec, st, T_final,
                                                                    n_last, d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
    } else {
        if (au)
            k_render_bwd<TW, TH, NW, true><<<tiles_total, 64 * NW, 0, s>>>(views, n_views, ranges, tile_order, inst_rec, rec, st,
                                                                          T_final, n_last, d_rgb, d_depth, d_alpha,
                                                                          d_unc, g2d, flags);
        else
            k_render_bwd<TW, TH, NW, false><<<tiles_total, 64 * NW, 0, s>>>(views, n_views, ranges, tile_order, inst_rec, rec, st,
                                                                           T_final, n_last, d_rgb, d_depth, d_alpha,
                                                                           d_unc, g2d, flags);
    }
}

void render_backward(int tw, int th, int batch, const ViewDev* views, int n_views, uint32_t tiles_total,
                     const uint2* ranges, const uint32_t* tile_order, const uint32_t* inst_rec, Records rec,
                     SetDev st, const float* T_final,
                     const uint32_t* n_last, const float* d_rgb, const float* d_depth, const float* d_alpha,
                     const float* d_unc, double* g2d, const uint32_t* flags, hipStream_t s) {
    (void)batch;  // the backward stages 64 splats per wave of the tile
    if (tiles_total == 0) return;
    const int nw = backward_waves(tw, th, tiles_total);
    const bool au = d_alpha != nullptr || d_unc != nullptr;
    if (tw == 8 && th == 8) {
        launch_bwd<8, 8, 1>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last, d_rgb,
                            d_depth, d_alpha, d_unc, g2d, flags);
    } else if (tw == 32 && th == 8) {
        if (nw == 4)
            launch_bwd<32, 8, 4>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last,
                                 d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
        else if (nw == 2)
            launch_bwd<32, 8, 2>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last,
                                 d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
        else
            launch_bwd<32, 8, 1>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last,
                                 d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
    } else {
        if (nw == 4)
            launch_bwd<16, 16, 4>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last,
                                  d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
        else if (nw == 2)
            launch_bwd<16, 16, 2>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last,
                                  d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
        else
            launch_bwd<16, 16, 1>(au, tiles_total, s, views, n_views, ranges, tile_order, inst_rec, rec, st, T_final, n_last,
                                  d_rgb, d_depth, d_alpha, d_unc, g2d, flags);
    }
}

void project_backward(const GaussDev& g, const ViewDev* views, SetDev st, const uint32_t* rec_off,
                      const uint32_t* cnt, const EmitRec* emit, const double* g2d, float* d_means,
                      float* d_log_scales, float* d_quats, float* d_opacity, float* d_colors, const uint32_t* flags,
                      hipStream_t s) {
    if (g.n == 0) return;
    k_project_bwd<<<grid_for(g.n, 256, 0xffffffffu), 256, 0, s>>>(g, views, st, rec_off, cnt, emit, g2d, d_means,
                                                     d_log_scales, d_quats, d_opacity, d_colors, flags);
}

void score_tiles(int tw, int th, int batch, int mode, bool persistent, int grid_persistent, const ViewDev* views,
                 int n_views, const Header* hdr, uint32_t tile_begin, uint32_t n_tiles,
                 const uint2* ranges, const uint32_t* tile_order, const uint32_t* inst_rec, Records rec, SetDev st,
                 double* partial, uint32_t* queue, const uint32_t* flags, hipStream_t s) {
    if (persistent) {
        fill_u32(queue, 0u, 1, s);
        RTG_BATCH_DISPATCH(TW, TH, B,
                           (k_score_persistent<TW, TH, B><<<grid_persistent, TW * TH, 0, s>>>(views, hdr, ranges,
                                                                                             tile_order, inst_rec,
                                                                                             rec, st,
                                                                                             mode, partial, queue,
                                                                                             flags)));
    } else {
        if (n_tiles == 0) return;
        RTG_BATCH_DISPATCH(TW, TH, B,
                           (k_score_plain<TW, TH, B><<<n_tiles, TW * TH, 0, s>>>(views, n_views, tile_begin,
                                                                                ranges, inst_rec, rec, st, mode,
                                                                                partial)));
    }
}

void score_reduce(const ViewDev* views, const Header* hdr, int n_views_cap, const double* partial,
                  double* scores, const uint32_t* flags, hipStream_t s) {
    k_score_reduce<<<n_views_cap, 256, 0, s>>>(views, hdr, partial, scores, flags);
}

void sum_u32_pair(const uint32_t* a, const uint32_t* b, uint64_t n, unsigned long long* out, hipStream_t s) {
    if (n == 0) return;
    k_sum_u32_pair<<<grid_for(n, 256, 2048), 256, 0, s>>>(a, b, n, out);
}

void uncertainty_update(int64_t n, const float* prev, const float* cur, const float* u_prev, int squared,
                        float* u_out, hipStream_t s) {
    if (n <= 0) return;
    k_uncertainty_update<<<grid_for((uint64_t)n, 256, 1u << 20), 256, 0, s>>>(n, prev, cur, u_prev, squared, u_out);
}

void region_utility(int64_t n, const float* means, const float* u, const double* lo, double size, const int* dims,
                    unsigned long long* cnt, unsigned long long* fix, unsigned int* bad, int64_t* count, double* sum,
                    double* mean, hipStream_t s) {
    const int64_t nr = (int64_t)dims[0] * dims[1] * dims[2];
    fill_u32(reinterpret_cast<uint32_t*>(cnt), 0u, 2 * (uint64_t)nr, s);
    fill_u32(reinterpret_cast<uint32_t*>(fix), 0u, 2 * (uint64_t)nr, s);
    fill_u32(bad, 0u, (uint64_t)nr, s);
    if (n > 0) {
        const unsigned grid = grid_for((uint64_t)n, 256 * 16, 2048);  // blocks walk 16 x 256 Gaussians
        k_region_utility<<<grid, 256, 0, s>>>(n, means, u, lo[0], lo[1], lo[2], size, dims[0], dims[1], dims[2], cnt,
                                              fix, bad);
    }
    k_region_finish<<<grid_for((uint64_t)nr, 256, 4096), 256, 0, s>>>(nr, cnt, fix, bad, count, sum, mean);
}

void export_pairs(const uint32_t* tile_key, const uint32_t* inst_rec, const uint32_t* K_dev, Records rec,
                  uint64_t* keys, uint32_t* vals, uint32_t cap, hipStream_t s) {
    k_export<<<grid_for(cap, 256, 8192), 256, 0, s>>>(tile_key, inst_rec, K_dev, cap, rec, keys, vals);
}

void export_records(const uint32_t* R_dev, uint32_t cap, Records rec, double* mean2d, double* conic, int32_t* pbox,
                    uint32_t* depth_bits, uint32_t* gid, uint32_t* view, uint32_t* ntiles, hipStream_t s) {
    k_export_records<<<grid_for(std::max<uint32_t>(cap, 1), 256, 8192), 256, 0, s>>>(
        R_dev, cap, rec, mean2d, conic, pbox, depth_bits, gid, view, ntiles);
}

}  // namespace rtg
