// Internal declarations shared by the gfx950 kernels (rtg_kernels.hip) and the
// host runtime behind the C ABI (rtg_abi.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtg {

// Per-view camera and layout, resident in device memory.  Camera values are
// the binary32 inputs promoted to binary64.
struct ViewDev {
    double R[9];  // camera-to-world rotation, row-major
    double T[3];  // camera centre in the world
    double fx, fy, cx, cy;
    float Rf[9], Tf[3], fxf, fyf, cxf, cyf;  // the same in binary32 (the camera's own values)
    int32_t W, H, tiles_x, tiles_y;
    uint32_t tile_off;  // first global tile id of this view
    uint32_t pad;
    uint64_t pix_off;   // first pixel of this view in the packed images
};

// Device-side sizes of a batch of views (read by kernels so that captured
// graphs can be replayed with other cameras).
struct Header {
    uint32_t n_views;
    uint32_t tiles_total;
    uint64_t pix_total;
};

struct SetDev {
    float T_min, alpha_min, alpha_max, z_near, eps2d;
    float log2_amin;  // log2(alpha_min)
    int32_t isotropic;  // 1: one log-radius per Gaussian, no quaternion, r_2D = f r / d
};

struct GaussDev {
    int64_t n;
    const float *means, *log_scales, *quats, *opacity, *colors, *uncert;
};

// The fields pair emission and the compositing kernels' staging read, packed
// in one 64-byte line per record (both visit records at random: emission in
// depth order, compositing through the tile lists).
struct alignas(16) EmitRec {
    float4 g0, g1;
    uint2 pbox;
    uint2 rect;  // tile rectangle: x = tx0 | tx1 << 16, y = ty0 | ty1 << 16
    uint32_t ntiles, view;
    uint32_t unc;  // binary32 bits of the uncertainty
    uint32_t gid;  // Gaussian index
};

// Projected (view, Gaussian) records, structure of arrays.
//   emit = EmitRec: geo0, geo1, pixel box, tile rectangle, pair count, view,
//          uncertainty, Gaussian index, where
//          geo0 = (mean_x hi, mean_y hi, mean_x lo, mean_y lo): the binary64
//          mean as a sum of two binary32 values, so per-pixel offsets are exact;
//          geo1 = (m00, m10, m11, opacity): the lower-triangular whitening M
//          with M^T M = log2(e)/2 * Sigma_2D^-1, so that with w = M d the splat
//          is G = exp2(-|w|^2) = exp(-d^T Sigma_2D^-1 d / 2) (no cancellation
//          between terms for elongated splats);
//          pixel box of alpha >= alpha_min: x = u0 | u1 << 16, y = v0 | v1 << 16;
//   q64  = binary64 Sigma_2D^-1 (xx, xy, yy, 0), read only to re-take the
//          alpha_min decision in binary64 when binary32 alpha is near it;
//   attr = (r, g, b, binary32 camera depth, whose bits are the sort key);
//          written only for frames that composite colour and depth (not
//          for scoring);
//   ntiles = pairs (support tiles) of the record, also in emit, here dense
//          for the pair scan.
struct Records {
    EmitRec* emit;
    double4* q64;
    float4* attr;
    uint32_t* ntiles;
};

// Screen-space gradient per record, binary64, 16 entries (one 128-byte line):
// [0,1] sums toward d mean_2D, [2..4] toward d conic (xx, xy counted as one
// parameter, yy), [5] toward d opacity, [6..8] d colour, [9] d depth, rest
// unused.  Slots 0..5 hold pixel sums of dL/da times the unclamped alpha
// o G (times the pixel offsets for 0..4); the projection backward scales
// 0..4 by -1/2 and divides 5 by the opacity.  Per-tile partial
// sums are added in binary64 because a splat's mean / conic gradient is a sum
// of terms of both signs over its footprint that cancel to a small total.
constexpr int G2D_STRIDE = 16;

constexpr int MAX_VIEWS = 1024;

// Status bits written by kernels into a device word.
constexpr uint32_t FLAG_REC_OVERFLOW = 1u;
constexpr uint32_t FLAG_INST_OVERFLOW = 2u;
// Pair emission found fewer support tiles than were counted (never expected).
constexpr uint32_t FLAG_BIN_MISMATCH = 4u;
// A count scan summed to 2^31 or more (records or pairs beyond the 32-bit
// offsets); the scan then reports a total of 0.
constexpr uint32_t FLAG_COUNT_OVERFLOW = 8u;

// ---------------------------------------------------------------- launchers
// All take device pointers and enqueue on `s`.  n_dev arguments are device
// counters; *_cap are the capacities of the buffers those counts index.
// `flags` (nullable) is the overflow word of a capacity-sized pipeline: when
// it is non-zero, kernels that would index past a capacity exit at once.

void fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);

// cnt[i] = visible views of Gaussian i; mask[w * n + i] bit b = view 32w+b.
void project_count(const GaussDev& g, const ViewDev* views, const Header* hdr, int n_views_cap,
                   SetDev st, uint32_t* cnt, uint32_t* mask, hipStream_t s);
// Writes records at rec_off[i] .. for the visible views of Gaussian i (attr
// only when write_attr).
// chunk_g: workspace of pe_chunk_words(rec_cap) entries (the owners of each
// chunk's first and last records, found before the records are written).
constexpr int PE_CHUNK = 256;  // records per block step of the record emission
inline size_t pe_chunk_words(uint32_t rec_cap) { return 2 * ((size_t)rec_cap / PE_CHUNK + 2); }
void project_emit(const GaussDev& g, const ViewDev* views, const Header* hdr, int n_views_cap,
                  SetDev st, int tw, int th, const uint32_t* mask, const uint32_t* cnt, const uint32_t* rec_off,
                  const uint32_t* R_dev, uint32_t rec_cap, Records rec, uint32_t* sortkey, uint32_t* order,
                  bool write_attr, uint32_t* chunk_g, uint32_t* flags, hipStream_t s);

// Exclusive prefix sum of in[0..n) (n = min(*n_dev, cap)) into out; *total =
// the full sum.  If gather != NULL the input is in[gather[i]].  A sum of 2^31
// or more sets FLAG_COUNT_OVERFLOW in *flags (nullable) and gives *total = 0.
struct ScanWs {
    uint32_t* partial;  // >= scan_blocks(cap) entries
};
int scan_blocks(uint64_t cap);
void scan_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, const uint32_t* n_dev,
              uint32_t cap, uint32_t* total, uint32_t* flags, ScanWs ws, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on bits [0, nbits) of the key.
// Result lands in (k1, v1) if the number of 8-bit passes is odd, else (k0, v0);
// returns 1 or 0 accordingly.
struct SortWs {
    uint32_t* hist;     // sort_hist_words(cap) entries
    uint32_t* partial;  // scan workspace: >= 1024 + 1 entries
};
int sort_blocks(uint64_t cap, int db);
size_t sort_hist_words(uint64_t cap);
// Stable sort of (key, value) pairs on the low nbits of the keys, in passes of
// at most max_db (<= 11) bits; returns 1 if the result is in (k1, v1).  With
// gsrc, the last pass also writes gout[i] = gsrc[value at sorted position i].
int radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
               uint32_t cap, int nbits, int max_db, SortWs ws, hipStream_t s, const uint32_t* gsrc = nullptr,
               uint32_t* gout = nullptr);

// Instances of the depth-ordered records: tile keys and record ids, one per
// tile a record's support meets (tiles tw x th).  Also empties ranges[0,
// tiles_cap) for tile_ranges.
void emit_instances(const uint32_t* order, const uint32_t* R_dev, uint32_t rec_cap, const uint32_t* K_dev,
                    Records rec, const ViewDev* views, const uint32_t* inst_off, int tw, int th, SetDev st,
                    uint32_t inst_cap, uint32_t* tile_key, uint32_t* inst_rec, uint2* ranges, uint32_t tiles_cap,
                    uint32_t* flags, hipStream_t s);
// ranges[t] = [start, end) over the tile-sorted keys, for the occupied tiles;
// emit_instances has emptied them all.
void tile_ranges(const uint32_t* tile_key, const uint32_t* K_dev, uint32_t inst_cap,
                 uint2* ranges, uint32_t tiles_cap, const uint32_t* flags, hipStream_t s);
// order[0 .. tiles_total) = the tiles in descending order of their pair
// counts (by powers of two; any order within one); ws: TILE_ORDER_WS words
// of scratch.  The compositing kernels take their tiles through it.
constexpr int TILE_ORDER_WS = 66;
void tile_order(const uint2* ranges, const Header* hdr, uint32_t tiles_cap, uint32_t* ws, uint32_t* order,
                hipStream_t s);

struct RenderOut {
    float *rgb, *depth, *alpha, *unc;
    float* T_final;      // per pixel
    uint32_t* n_last;    // per pixel: list position after the last contributor
    uint32_t* n_contrib; // per pixel: number of contributing splats
};

// out[0] += sum a[i], out[1] += sum b[i] over i < n (64-bit).
void sum_u32_pair(const uint32_t* a, const uint32_t* b, uint64_t n, unsigned long long* out, hipStream_t s);
void render_forward(int tw, int th, int batch, const ViewDev* views, int n_views,
                    uint32_t tiles_total, const uint2* ranges, const uint32_t* tile_order,
                    const uint32_t* inst_rec, Records rec, SetDev st, RenderOut out, const uint32_t* flags,
                    hipStream_t s);

void loss_l1(const ViewDev* views, int n_views, int max_pix, const float* rgb, const float* depth,
             const float* trgb, const float* tdepth, float w_depth, float* d_rgb, float* d_depth,
             double* partial, int partial_cap, double* loss, hipStream_t s);

void render_backward(int tw, int th, int batch, const ViewDev* views, int n_views,
                     uint32_t tiles_total, const uint2* ranges, const uint32_t* tile_order, const uint32_t* inst_rec,
                     Records rec, SetDev st, const float* T_final, const uint32_t* n_last,
                     const float* d_rgb, const float* d_depth, const float* d_alpha,
                     const float* d_unc, double* g2d, const uint32_t* flags, hipStream_t s);

void project_backward(const GaussDev& g, const ViewDev* views, SetDev st, const uint32_t* rec_off,
                      const uint32_t* cnt, const EmitRec* emit, const double* g2d,
                      float* d_means, float* d_log_scales, float* d_quats, float* d_opacity,
                      float* d_colors, const uint32_t* flags, hipStream_t s);

// Scoring: per-(view, tile) partial sums of the composited uncertainty.
// mode 0 sums u a T per pixel, mode 1 sums u over the contributing splats.
// persistent: a fixed grid pulls tiles from an atomic queue (counter must be
// zeroed; done inside).  Otherwise one workgroup per tile of [tile_begin,
// tile_begin + n_tiles).
void score_tiles(int tw, int th, int batch, int mode, bool persistent, int grid_persistent,
                 const ViewDev* views, int n_views, const Header* hdr,
                 uint32_t tile_begin, uint32_t n_tiles, const uint2* ranges, const uint32_t* tile_order,
                 const uint32_t* inst_rec, Records rec, SetDev st, double* partial,
                 uint32_t* queue, const uint32_t* flags, hipStream_t s);
int score_persistent_blocks(int tw, int th, int batch);
// Mapping loss of eq. (4) with SSIM over packed views: blocks_per_view from
// ssim_blocks_per_view(widest, tallest view); maps: 9 x pix_total floats of
// scratch; partial: blocks_per_view x n_views doubles; d_rgb / d_depth may be
// NULL; loss: one device double.
int ssim_blocks_per_view(int max_w, int max_h);
void loss_ssim(const ViewDev* views, int n_views, int blocks_per_view, uint64_t pix_total, const float* rgb,
               const float* depth, const float* trgb, const float* tdepth, float w_depth, float l1, float l2,
               float* maps, double* partial, float* d_rgb, float* d_depth, double* loss, hipStream_t s);
// Collision check of np points (planar 3 x np) against the map; packed,
// bound: n float4 / float2 scratch, collide: np int32 (required), clear_key:
// np uint32 scratch, clearance: np floats or NULL.
void collision_check(const GaussDev& g, const float* pts, int64_t np, float r_robot, float lambda_g, float4* packed,
                     float2* bound, int32_t* collide, uint32_t* clear_key, float* clearance, hipStream_t s);
// Uncertainty bookkeeping (n Gaussians, planar 3 x n means).
void uncertainty_update(int64_t n, const float* prev, const float* cur, const float* u_prev, int squared,
                        float* u_out, hipStream_t s);
// Region utility over dims[0] x dims[1] x dims[2] cuboids from lo (host
// values) with edge size; cnt/fix (u64) and bad (u32) are nr-entry scratch.
void region_utility(int64_t n, const float* means, const float* u, const double* lo, double size, const int* dims,
                    unsigned long long* cnt, unsigned long long* fix, unsigned int* bad, int64_t* count, double* sum,
                    double* mean, hipStream_t s);
// scores[v] = sum of view v's tile partials, in a fixed order; NaN when
// *flags is non-zero.
void score_reduce(const ViewDev* views, const Header* hdr, int n_views_cap, const double* partial,
                  double* scores, const uint32_t* flags, hipStream_t s);

void export_pairs(const uint32_t* tile_key, const uint32_t* inst_rec, const uint32_t* K_dev,
                  Records rec, uint64_t* keys, uint32_t* vals, uint32_t cap, hipStream_t s);
// Planar copies of the first min(*R_dev, cap) records' fields (outputs nullable):
// mean2d 2 x R, conic 3 x R (binary64), pbox 4 x R (u0, u1, v0, v1), depth
// bits, Gaussian index, view and pair count.
void export_records(const uint32_t* R_dev, uint32_t cap, Records rec, double* mean2d, double* conic, int32_t* pbox,
                    uint32_t* depth_bits, uint32_t* gid, uint32_t* view, uint32_t* ntiles, hipStream_t s);

// Paper-literal view utility: per-view counts of visible high / low
// uncertainty Gaussians, their uncertainty sum and xi.  acc: 3 * nv u64
// scratch.  thresholds: scratch of 1 + 512 doubles.
void view_utility(const GaussDev& g, const ViewDev* views, int nv, float z_near, float range, const double* lo_hi,
                  unsigned long long* acc, double lambda, int64_t* n_high, int64_t* n_low, double* sum_u, double* xi,
                  hipStream_t s);
void uncertainty_thresholds(const float* u, int64_t n, double k, double* scratch, double* lo_hi, hipStream_t s);
void trajectory_select(const double* xi, const int32_t* offsets, int n_traj, double* util, int32_t* best,
                       hipStream_t s);

int device_cu_count();

}  // namespace rtg
