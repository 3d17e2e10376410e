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

#include "orrb_primitives.h"

namespace orrb {

constexpr int kPostBlock = 256;
constexpr int kPostPix = 4;     // pixels per group
constexpr int kPostGroups = 4;  // groups per thread, a workgroup's width apart
constexpr int kPostChunk = kPostBlock * kPostPix * kPostGroups;  // pixels per workgroup

// sRGB transfer function (IEC 61966-2-1) of x in [0, 1]: x^(1/2.4) through the
// hardware log2 / exp2 (x = 0 gives exp2(-inf) = 0), both pieces evaluated and one
// selected, so the wave does not branch per channel.
ORRB_INLINE float srgb_encode(float x) {
    const float lin = 12.92f * x;
    const float pw = 1.055f * __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 2.4f)) - 0.055f;
    return x <= 0.0031308f ? lin : pw;
}

struct PostFrame {
    float wb0, wb1, wb2;  // white-balance gains
    float sat, con;
    float H[9];           // hue rotation about the grey axis, row-major
    float gi, gk;         // grain intensity, coloration
    int gs, gx, gy;       // grain size (pixels per texel), texel offsets in [0, n)
    float rs, rw, rh;     // 1 / gs, 1 / grain_w, 1 / grain_h (fp32)
    const float *g0, *g1, *g2;  // grain planes
};

ORRB_INLINE PostFrame post_frame(const RenderArgs &a, int f) {
    PostFrame q;
    float T = 0.f, G = 0.f, h = 0.f, s = 1.f, k = 1.f, I = 0.f, kap = 0.f, S = 1.f, ox = 0.f, oy = 0.f;
    if (a.post) {
        const float *p = a.post + (int64_t)ORRB_POST_WORDS * f;
        T = p[ORRB_POST_TEMPERATURE];
        G = p[ORRB_POST_TINT];
        h = p[ORRB_POST_HUE];
        s = p[ORRB_POST_SATURATION];
        k = p[ORRB_POST_CONTRAST];
        I = p[ORRB_POST_GRAIN];
        kap = p[ORRB_POST_GRAIN_COLOR];
        S = p[ORRB_POST_GRAIN_SIZE];
        ox = p[ORRB_POST_GRAIN_X];
        oy = p[ORRB_POST_GRAIN_Y];
    }
    q.wb0 = 1.0f + T / 5.0f;
    q.wb1 = 1.0f - G / 5.0f;
    q.wb2 = 1.0f - T / 5.0f;
    q.sat = s;
    q.con = k;
    // Rodrigues rotation about u = (1, 1, 1) / sqrt(3): cos h I + sin h [u]x + (1 - cos h) u u^T
    float sn, c;
    sincosf(h, &sn, &c);
    const float u = 0.57735026918962576f, t = (1.0f - c) / 3.0f;
    q.H[0] = c + t;      q.H[1] = t - sn * u; q.H[2] = t + sn * u;
    q.H[3] = t + sn * u; q.H[4] = c + t;      q.H[5] = t - sn * u;
    q.H[6] = t - sn * u; q.H[7] = t + sn * u; q.H[8] = c + t;
    q.gi = a.grain ? I : 0.f;
    q.gk = kap;
    q.gs = max(1, (int)floorf(S));
    // texel offsets reduced to [0, n) once, so a pixel's texel needs one remainder
    q.gx = a.grain ? (((int)ox % a.grain_w) + a.grain_w) % a.grain_w : 0;
    q.gy = a.grain ? (((int)oy % a.grain_h) + a.grain_h) % a.grain_h : 0;
    q.rs = 1.0f / (float)q.gs;
    q.rw = a.grain ? 1.0f / (float)a.grain_w : 0.f;
    q.rh = a.grain ? 1.0f / (float)a.grain_h : 0.f;
    const int plane = a.grain_w * a.grain_h;  // < 2^26 (checked by the host)
    q.g0 = a.grain;
    q.g1 = a.grain ? a.grain + plane : nullptr;
    q.g2 = a.grain ? a.grain + 2 * plane : nullptr;
    return q;
}

// The 8-bit codes of one linear pixel (r, g, b) whose grain texel holds (n0, n1, n2).
ORRB_INLINE uchar3 post_pixel(const PostFrame &q, float r, float g, float b, float n0, float n1, float n2) {
    const float e0 = srgb_encode(fminf(fmaxf(r * q.wb0, 0.f), 1.f));
    const float e1 = srgb_encode(fminf(fmaxf(g * q.wb1, 0.f), 1.f));
    const float e2 = srgb_encode(fminf(fmaxf(b * q.wb2, 0.f), 1.f));
    const float Y = 0.2126f * e0 + 0.7152f * e1 + 0.0722f * e2;
    const float c0 = 0.5f + q.con * (Y + q.sat * (e0 - Y) - 0.5f);
    const float c1 = 0.5f + q.con * (Y + q.sat * (e1 - Y) - 0.5f);
    const float c2 = 0.5f + q.con * (Y + q.sat * (e2 - Y) - 0.5f);
    float o0 = q.H[0] * c0 + q.H[1] * c1 + q.H[2] * c2;
    float o1 = q.H[3] * c0 + q.H[4] * c1 + q.H[5] * c2;
    float o2 = q.H[6] * c0 + q.H[7] * c1 + q.H[8] * c2;
    if (q.gi != 0.f) {
        const float m = (1.0f - q.gk) * n0;
        o0 = o0 + q.gi * (m + q.gk * n0 - 0.5f);
        o1 = o1 + q.gi * (m + q.gk * n1 - 0.5f);
        o2 = o2 + q.gi * (m + q.gk * n2 - 0.5f);
    }
    const float v0 = 255.0f * fminf(fmaxf(o0, 0.f), 1.f);
    const float v1 = 255.0f * fminf(fmaxf(o1, 0.f), 1.f);
    const float v2 = 255.0f * fminf(fmaxf(o2, 0.f), 1.f);
    // floor(v + 1/2) of a non-negative value: the truncating conversion
    return make_uchar3((unsigned char)(unsigned)(v0 + 0.5f), (unsigned char)(unsigned)(v1 + 0.5f),
                       (unsigned char)(unsigned)(v2 + 0.5f));
}

// Grain texel coordinate along one axis for pixel coordinate x >= 0: (x div S + o) mod n,
// with the offset o already in [0, n).
ORRB_INLINE int grain_coord(int x, int S, int o, int n) { return (x / S + o) % n; }

// x div d for 0 <= x < 2^20 and d >= 1, r = fp32 1 / d: the truncated fp32 product is
// within one of the quotient (its relative error is below 2^-22, so the absolute
// error is below 2^-2 for d >= 2; d = 1 gives r = 1 exactly), corrected once each way.
ORRB_INLINE int div_small(int x, int d, float r) {
    int k = (int)((float)x * r);
    k -= k * d > x;
    k += (k + 1) * d <= x;
    return k;
}

// grain_coord for x < 2^19, S and n below 2^19 (so x div S + o < 2^20).
ORRB_INLINE int grain_coord_small(int x, int S, float rs, int o, int n, float rn) {
    const int t = div_small(x, S, rs) + o;
    return t - n * div_small(t, n, rn);
}

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

// Row and column of pixel p of a frame W wide: 32-bit division when p fits.
ORRB_INLINE void pixel_rc(int64_t p, int W, int &j, int &i) {
    if (p <= 0xffffffffll) {
        const unsigned u = (unsigned)p, jj = u / (unsigned)W;
        j = (int)jj;
        i = (int)(u - jj * (unsigned)W);
    } else {
        j = (int)(p / W);
        i = (int)(p - (int64_t)j * W);
    }
}

// Plane value at byte offset `off` (a 32-bit offset from a uniform base: one
// scalar-based load, no per-lane 64-bit address arithmetic).
ORRB_INLINE float grain_at(const float *base, unsigned off) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off);
}

// Grain texels of the group of four pixels p0.. of a frame W wide when the group lies
// inside one row and coordinates are below 2^19: the first pixel's texel by division
// (fp32 reciprocals), the next ones by stepping, without branches.
ORRB_INLINE void grain_row(const RenderArgs &a, const PostFrame &q, int W, int64_t p0, float g[3][kPostPix]) {
    int j, i;
    pixel_rc(p0, W, j, i);
    const int qi = div_small(i, q.gs, q.rs);
    int sub = i - qi * q.gs;
    const int t = qi + q.gx;
    int tx = t - a.grain_w * div_small(t, a.grain_w, q.rw);
    const int row = grain_coord_small(j, q.gs, q.rs, q.gy, a.grain_h, q.rh) * a.grain_w;
#pragma unroll
    for (int k = 0; k < kPostPix; ++k) {
        const unsigned t = (unsigned)(row + tx) * 4u;  // < 2^28 bytes: texels per plane < 2^26
        g[0][k] = grain_at(q.g0, t);
        g[1][k] = grain_at(q.g1, t);
        g[2][k] = grain_at(q.g2, t);
        const bool step = ++sub == q.gs;  // next texel column
        sub = step ? 0 : sub;
        tx += step;
        tx = tx == a.grain_w ? 0 : tx;
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
    const bool rows = (W & 3) == 0 && fi.height < (1 << 19) && a.grain_w < (1 << 19) && a.grain_h < (1 << 19);
    if (rows && c0 + kPostChunk <= P) {
        float v[kPostGroups][3][kPostPix];
#pragma unroll
        for (int g = 0; g < kPostGroups; ++g)
            post_load(rgb, P, c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix, kPostPix, vec, v[g]);
        const PostFrame q = post_frame(a, f);  // uniform: while the loads are in flight
        if (q.gs < (1 << 19)) {
            // every grain texel of the chunk's groups gathered before any is used
            float gr[kPostGroups][3][kPostPix] = {};
            if (q.gi != 0.f) {
#pragma unroll
                for (int g = 0; g < kPostGroups; ++g)
                    grain_row(a, q, W, c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix, gr[g]);
            }
#pragma unroll
            for (int g = 0; g < kPostGroups; ++g)
                post_finish(q, P, c0 + (int64_t)(g * kPostBlock + (int)threadIdx.x) * kPostPix, kPostPix, vec, v[g], gr[g],
                            dst);
            return;
        }
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
            if (rows && n == kPostPix && q.gs < (1 << 19))
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
