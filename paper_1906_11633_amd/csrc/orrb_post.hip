// Post-processing and 3 x 8-bit encoding of the rendered rgb (Sec. 4.3.1
// PostprocessingRandomizer: colour grading hue, saturation, contrast, temperature and
// tint, and grain; Sec. 5 measures 200 x 200 images in 3 x 8-bit RGB).
//
// k_post reads the linear fp32 rgb planes the render call has just written and writes
// the graded, grained, sRGB-encoded 8-bit planes (same planar layout): 12 bytes read
// and 3 written per pixel, plus the grain texture, which stays in the caches.  A thread
// handles groups of four horizontally consecutive pixels (one 16-byte load and one
// 4-byte store per plane when aligned); it issues the loads of all its groups before
// anything else and computes the frame's grading constants itself while they are in
// flight, so no workgroup waits on a shared prologue.
#include <algorithm>

#include "orrb_post.h"

namespace orrb {

constexpr int kPostBlock = 256;
constexpr int kPostPix = 4;     // pixels per group
constexpr int kPostGroups = 4;  // groups per thread, a workgroup's width apart
constexpr int kPostChunk = kPostBlock * kPostPix * kPostGroups;  // pixels per workgroup

// Whole aligned groups take 16-byte loads and 4-byte stores per plane.
ORRB_INLINE bool post_vec(const RenderArgs &a, int64_t P, int64_t po) {
    return ((po | P) & 3) == 0 && (((uintptr_t)a.out_rgb | (uintptr_t)a.out_rgb8) & 15) == 0;
}

// The linear rgb of the n <= 4 pixels p0.. of a frame (P pixels, planes at rgb).
ORRB_INLINE void post_load(const float *rgb, int64_t P, int64_t p0, int n, bool vec, float v[3][kPostPix]) {
    if (vec && n == kPostPix) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 x = *reinterpret_cast<const float4 *>(rgb + c * P + p0);
            v[c][0] = x.x; v[c][1] = x.y; v[c][2] = x.z; v[c][3] = x.w;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < kPostPix; ++k) v[c][k] = k < n ? rgb[c * P + p0 + k] : 0.f;
    }
}

// Grain texels of the n <= 4 pixels p0.. of any group (a row change recomputes).
ORRB_INLINE void grain_any(const RenderArgs &a, const PostFrame &q, int W, int64_t p0, int n, float g[3][kPostPix]) {
    int j, i;
    pixel_rc(p0, W, j, i);
    int tx = grain_coord(i, q.gs, q.gx, a.grain_w), ty = grain_coord(j, q.gs, q.gy, a.grain_h), sub = i % q.gs;
#pragma unroll
    for (int k = 0; k < kPostPix; ++k) {
        const unsigned t = k < n ? (unsigned)(ty * a.grain_w + tx) * 4u : 0u;
        g[0][k] = grain_at(q.g0, t);
        g[1][k] = grain_at(q.g1, t);
        g[2][k] = grain_at(q.g2, t);
        if (++i == W) {
            i = 0;
            ++j;
            tx = grain_coord(0, q.gs, q.gx, a.grain_w);
            ty = grain_coord(j, q.gs, q.gy, a.grain_h);
            sub = 0;
        } else if (++sub == q.gs) {
            sub = 0;
            if (++tx == a.grain_w) tx = 0;
        }
    }
}

// Encode and store the n <= 4 pixels p0.. (linear rgb v, grain texels g) of a frame of
// P pixels whose 8-bit planes start at dst.
ORRB_INLINE void post_finish(const PostFrame &q, int64_t P, int64_t p0, int n, bool vec, const float v[3][kPostPix],
                             const float g[3][kPostPix], uint8_t *dst) {
    unsigned char o[3][kPostPix];
#pragma unroll
    for (int k = 0; k < kPostPix; ++k) {
        const uchar3 u = post_pixel(q, v[0][k], v[1][k], v[2][k], g[0][k], g[1][k], g[2][k]);
        o[0][k] = u.x; o[1][k] = u.y; o[2][k] = u.z;
    }
    if (vec && n == kPostPix) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            *reinterpret_cast<unsigned *>(dst + c * P + p0) =
                (unsigned)o[c][0] | ((unsigned)o[c][1] << 8) | ((unsigned)o[c][2] << 16) | ((unsigned)o[c][3] << 24);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < kPostPix; ++k)
                if (k < n) dst[c * P + p0 + k] = o[c][k];
    }
}

// Grid: y over frames, x over the frame's kPostChunk-pixel chunks.  Thread t of chunk c
// takes the groups starting at pixels c * kPostChunk + (g * kPostBlock + t) * kPostPix.
__global__ __launch_bounds__(kPostBlock) void k_post(RenderArgs a, int f_base) {
    const int f = f_base + (int)blockIdx.y;
    const FrameInfo fi = a.frames[f];
    const int W = fi.width;
    const int64_t P = (int64_t)W * fi.height, po = fi.pixel_offset;
    const int64_t c0 = (int64_t)blockIdx.x * kPostChunk;
    if (c0 >= P) return;  // the whole chunk is past the frame
    const bool vec = post_vec(a, P, po);
    const float *rgb = a.out_rgb + 3 * po;
    uint8_t *dst = a.out_rgb8 + 3 * po;
    // groups stay inside a row when the width is a multiple of 4; a chunk whose groups
    // are all whole issues the loads of all of them first, the frame's last chunk goes
    // group by group
    const bool rows = (W & 3) == 0;
    if (rows && c0 + kPostChunk <= P) {
        float v[kPostGroups][3][kPostPix];
#pragma unroll
        for (int g = 0; g < kPostGroups; ++g)
            post_load(rgb, P, c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix, kPostPix, vec, v[g]);
        const PostFrame q = post_frame(a, f);  // uniform: while the loads are in flight
        // every grain texel of the chunk's groups gathered before any is used
        float gr[kPostGroups][3][kPostPix] = {};
        if (q.gi != 0.f) {
#pragma unroll
            for (int g = 0; g < kPostGroups; ++g)
                grain_row(a, q, W, c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix, gr[g]);
        }
#pragma unroll
        for (int g = 0; g < kPostGroups; ++g)
            post_finish(q, P, c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix, kPostPix, vec, v[g], gr[g], dst);
        return;
    }
    const PostFrame q = post_frame(a, f);
#pragma unroll 1
    for (int g = 0; g < kPostGroups; ++g) {
        const int64_t p0 = c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix;
        const int n = (int)max<int64_t>(0, min<int64_t>(kPostPix, P - p0));
        if (n == 0) continue;
        float v[3][kPostPix], gr[3][kPostPix] = {};
        post_load(rgb, P, p0, n, vec, v);
        if (q.gi != 0.f) {
            if (rows && n == kPostPix)
                grain_row(a, q, W, p0, gr);
            else
                grain_any(a, q, W, p0, n, gr);
        }
        post_finish(q, P, p0, n, vec, v, gr, dst);
    }
}

hipError_t launch_post(const RenderArgs &a, hipStream_t stream, int n_frames, int64_t max_frame_pixels) {
    if (n_frames <= 0 || !a.out_rgb8) return hipSuccess;
    const int64_t gx = (max_frame_pixels + kPostChunk - 1) / kPostChunk;
    constexpr int kMaxY = 32768;  // frames per launch (grid y)
    for (int f0 = 0; f0 < n_frames; f0 += kMaxY) {
        const int nf = min(kMaxY, n_frames - f0);
        hipLaunchKernelGGL(k_post, dim3((unsigned)gx, (unsigned)nf), dim3(kPostBlock), 0, stream, a, f0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace orrb
