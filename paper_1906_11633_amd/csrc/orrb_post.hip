// Post-processing and 3 x 8-bit encoding of the rendered rgb (Sec. 4.3.1
// PostprocessingRandomizer: colour grading hue, saturation, contrast, temperature and
// tint, and grain; Sec. 5 measures 200 x 200 images in 3 x 8-bit RGB).
//
// k_post reads the linear fp32 rgb planes the render call has just written and writes
// the graded, grained, sRGB-encoded 8-bit planes (same planar layout).  It is bound by
// HBM traffic: 12 bytes read and 3 written per pixel, plus the grain texture, which
// stays in the caches.  One thread handles four horizontally consecutive pixels of a
// frame (one 16-byte load and one 4-byte store per plane when aligned).
#include <algorithm>

#include "orrb_primitives.h"

namespace orrb {

constexpr int kPostBlock = 256;
constexpr int kPostPix = 4;  // pixels per thread

// sRGB transfer function (IEC 61966-2-1) of x in [0, 1]: x^(1/2.4) through the
// hardware log2 / exp2.
ORRB_INLINE float srgb_encode(float x) {
#pragma clang fp contract(off)
    if (x <= 0.0031308f) return 12.92f * x;
    return 1.055f * __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 2.4f)) - 0.055f;
}

struct PostFrame {
    float wb0, wb1, wb2;  // white-balance gains
    float sat, con;
    float H[9];           // hue rotation about the grey axis, row-major
    float gi, gk;         // grain intensity, coloration
    int gs, gx, gy;       // grain size (pixels per texel), texel offsets
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
    q.gx = (int)ox;
    q.gy = (int)oy;
    return q;
}

// The 8-bit codes of one linear pixel (r, g, b) whose grain texel is t0 (row-major in
// plane 0 of the grain texture).
ORRB_INLINE uchar3 post_pixel(const RenderArgs &a, const PostFrame &q, float r, float g, float b, int64_t t0) {
#pragma clang fp contract(off)
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
        const int64_t plane = (int64_t)a.grain_w * a.grain_h;
        const float g0 = a.grain[t0];
        const float m = (1.0f - q.gk) * g0;
        o0 = o0 + q.gi * (m + q.gk * g0 - 0.5f);
        o1 = o1 + q.gi * (m + q.gk * a.grain[plane + t0] - 0.5f);
        o2 = o2 + q.gi * (m + q.gk * a.grain[2 * plane + t0] - 0.5f);
    }
    const float v0 = 255.0f * fminf(fmaxf(o0, 0.f), 1.f);
    const float v1 = 255.0f * fminf(fmaxf(o1, 0.f), 1.f);
    const float v2 = 255.0f * fminf(fmaxf(o2, 0.f), 1.f);
    return make_uchar3((unsigned char)floorf(v0 + 0.5f), (unsigned char)floorf(v1 + 0.5f), (unsigned char)floorf(v2 + 0.5f));
}

// Grain texel coordinate along one axis for pixel coordinate x: (x div S + o) mod n,
// non-negative whatever the offset holds.
ORRB_INLINE int grain_coord(int x, int S, int o, int n) { return ((x / S + o) % n + n) % n; }

// Four consecutive pixels p0.. of frame f (W wide, P pixels, first pixel po).
ORRB_INLINE void post_group(const RenderArgs &a, const PostFrame &q, int f, int W, int64_t P, int64_t po, int64_t p0) {
    const int n = (int)min<int64_t>(kPostPix, P - p0);
    const float *rgb = a.out_rgb + 3 * po;
    uint8_t *dst = a.out_rgb8 + 3 * po;
    // whole aligned groups: 16-byte loads and 4-byte stores per plane
    const bool vec = n == kPostPix && ((po | P) & 3) == 0 && (((uintptr_t)a.out_rgb | (uintptr_t)a.out_rgb8) & 15) == 0;
    float v[3][kPostPix];
    if (vec) {
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
    // pixel coordinates and grain texel of the first pixel (one division per thread);
    // the next pixels step the texel column (a row change recomputes)
    int j = (int)(p0 / W), i = (int)(p0 - (int64_t)j * W);
    int tx = 0, ty = 0, sub = 0;
    const bool grain = q.gi != 0.f;
    if (grain) {
        tx = grain_coord(i, q.gs, q.gx, a.grain_w);
        ty = grain_coord(j, q.gs, q.gy, a.grain_h);
        sub = i % q.gs;
    }
    unsigned char o[3][kPostPix];
#pragma unroll
    for (int k = 0; k < kPostPix; ++k) {
        const uchar3 u = post_pixel(a, q, v[0][k], v[1][k], v[2][k], (int64_t)ty * a.grain_w + tx);
        o[0][k] = u.x; o[1][k] = u.y; o[2][k] = u.z;
        if (++i == W) {
            i = 0;
            ++j;
            if (grain) {
                tx = grain_coord(0, q.gs, q.gx, a.grain_w);
                ty = grain_coord(j, q.gs, q.gy, a.grain_h);
                sub = 0;
            }
        } else if (grain && ++sub == q.gs) {
            sub = 0;
            if (++tx == a.grain_w) tx = 0;
        }
    }
    if (vec) {
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

// Grid: y over frames, x over blocks that stride through the frame's 1024-pixel chunks.
__global__ __launch_bounds__(kPostBlock) void k_post(RenderArgs a, int f_base) {
    const int f = f_base + (int)blockIdx.y;
    const FrameInfo fi = a.frames[f];
    const int W = fi.width;
    const int64_t P = (int64_t)W * fi.height, po = fi.pixel_offset;
    if ((int64_t)blockIdx.x * kPostBlock * kPostPix >= P) return;  // the whole block is past the frame
    __shared__ PostFrame sq;
    if (threadIdx.x == 0) sq = post_frame(a, f);  // once per block
    __syncthreads();
    const PostFrame q = sq;
    for (int64_t p0 = ((int64_t)blockIdx.x * kPostBlock + threadIdx.x) * kPostPix; p0 < P;
         p0 += (int64_t)gridDim.x * kPostBlock * kPostPix)
        post_group(a, q, f, W, P, po, p0);
}

hipError_t launch_post(const RenderArgs &a, hipStream_t stream, int n_frames, int64_t max_frame_pixels) {
    if (n_frames <= 0 || !a.out_rgb8) return hipSuccess;
    const int64_t per_block = (int64_t)kPostBlock * kPostPix;
    const int64_t gx = (max_frame_pixels + per_block - 1) / per_block;  // one 1024-pixel chunk per block
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
