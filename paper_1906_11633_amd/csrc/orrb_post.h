// Colour grading, grain and 3 x 8-bit sRGB encoding of linear rgb (Sec. 4.3.1
// PostprocessingRandomizer: colour grading hue, saturation, contrast, temperature and
// tint, and grain; Sec. 5 benchmarks 200 x 200 images in 3 x 8-bit RGB): the epilogue of
// the render kernels, which encode each pixel as they write it.  Evaluated without
// contraction, so every kernel that inlines it produces the same bytes.
#pragma once

#include "orrb_primitives.h"

namespace orrb {

// sRGB transfer function (IEC 61966-2-1) of x in [0, 1]: x^(1/2.4) through the
// hardware log2 / exp2 (x = 0 gives exp2(-inf) = 0), both pieces evaluated and one
// selected, so the wave does not branch per channel.
ORRB_INLINE float srgb_encode(float x) {
#pragma clang fp contract(off)
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
#pragma clang fp contract(off)
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
    // pixels per texel; beyond 8192 (ORRB_MAX_DIM) every pixel of a row or column maps
    // to the same texel, so the clamp changes no result
    q.gs = (int)fminf(fmaxf(floorf(S), 1.0f), 8192.0f);
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

// Steps 1-4 of one linear pixel (r, g, b): white balance, clamp and sRGB encoding,
// saturation and contrast, hue rotation.  The result depends on the pixel only through
// (r, g, b), so background pixels share one value per frame.
ORRB_INLINE float3 post_grade(const PostFrame &q, float r, float g, float b) {
#pragma clang fp contract(off)
    const float e0 = srgb_encode(fminf(fmaxf(r * q.wb0, 0.f), 1.f));
    const float e1 = srgb_encode(fminf(fmaxf(g * q.wb1, 0.f), 1.f));
    const float e2 = srgb_encode(fminf(fmaxf(b * q.wb2, 0.f), 1.f));
    const float Y = 0.2126f * e0 + 0.7152f * e1 + 0.0722f * e2;
    const float c0 = 0.5f + q.con * (Y + q.sat * (e0 - Y) - 0.5f);
    const float c1 = 0.5f + q.con * (Y + q.sat * (e1 - Y) - 0.5f);
    const float c2 = 0.5f + q.con * (Y + q.sat * (e2 - Y) - 0.5f);
    return make_float3(q.H[0] * c0 + q.H[1] * c1 + q.H[2] * c2, q.H[3] * c0 + q.H[4] * c1 + q.H[5] * c2,
                       q.H[6] * c0 + q.H[7] * c1 + q.H[8] * c2);
}

// Steps 5-6: grain from the pixel's texel (n0, n1, n2), clamp and rounding to 8 bits.
ORRB_INLINE uchar3 post_final(const PostFrame &q, float3 o, float n0, float n1, float n2) {
#pragma clang fp contract(off)
    float o0 = o.x, o1 = o.y, o2 = o.z;
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

// The 8-bit codes of one linear pixel (r, g, b) whose grain texel holds (n0, n1, n2).
ORRB_INLINE uchar3 post_pixel(const PostFrame &q, float r, float g, float b, float n0, float n1, float n2) {
    return post_final(q, post_grade(q, r, g, b), n0, n1, n2);
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

// Plane value at byte offset `off` (a 32-bit offset from a uniform base: one
// scalar-based load, no per-lane 64-bit address arithmetic).
ORRB_INLINE float grain_at(const float *base, unsigned off) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off);
}

// Grain texels of four consecutive pixels (i .. i + 3, j) of one row, 0 <= i, j < 2^13
// (frames are at most ORRB_MAX_DIM = 8192 wide and high; pixels past the row's end get
// texels that are never used): the first pixel's texel by division (fp32 reciprocals
// unless the texture is 2^19 or more texels wide or high), the next ones by stepping,
// without branches.
ORRB_INLINE void grain_ij(const RenderArgs &a, const PostFrame &q, int i, int j, float g[3][4]) {
    int qi, tx, ty;
    if (a.grain_w < (1 << 19) && a.grain_h < (1 << 19)) {
        qi = div_small(i, q.gs, q.rs);
        const int t = qi + q.gx;
        tx = t - a.grain_w * div_small(t, a.grain_w, q.rw);
        ty = grain_coord_small(j, q.gs, q.rs, q.gy, a.grain_h, q.rh);
    } else {
        qi = i / q.gs;
        tx = (qi + q.gx) % a.grain_w;
        ty = grain_coord(j, q.gs, q.gy, a.grain_h);
    }
    int sub = i - qi * q.gs;
    const int row = ty * a.grain_w;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
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

// Byte offset of pixel (i, j)'s grain texel in each plane (one pixel, by division).
ORRB_INLINE unsigned grain_texel(const RenderArgs &a, const PostFrame &q, int i, int j) {
    const int tx = grain_coord(i, q.gs, q.gx, a.grain_w), ty = grain_coord(j, q.gs, q.gy, a.grain_h);
    return (unsigned)(ty * a.grain_w + tx) * 4u;
}

// The 8-bit codes of four consecutive pixels of one row starting at (i, j), linear rgb v
// (zero for background), packed little-endian per plane: byte k is pixel i + k.
ORRB_INLINE void post_codes_row(const RenderArgs &a, const PostFrame &q, int i, int j, const float v[3][4],
                                unsigned code[3]) {
    float g[3][4] = {};
    if (q.gi != 0.f) grain_ij(a, q, i, j, g);
    code[0] = code[1] = code[2] = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uchar3 u = post_pixel(q, v[0][k], v[1][k], v[2][k], g[0][k], g[1][k], g[2][k]);
        code[0] |= (unsigned)u.x << (8 * k);
        code[1] |= (unsigned)u.y << (8 * k);
        code[2] |= (unsigned)u.z << (8 * k);
    }
}

// The same for four background pixels, whose graded value o_bg = post_grade(q, 0, 0, 0)
// the caller computed once for the frame: only the grain differs between them.
ORRB_INLINE void post_codes_row_bg(const RenderArgs &a, const PostFrame &q, float3 o_bg, int i, int j,
                                   unsigned code[3]) {
    float g[3][4] = {};
    if (q.gi != 0.f) grain_ij(a, q, i, j, g);
    code[0] = code[1] = code[2] = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uchar3 u = post_final(q, o_bg, g[0][k], g[1][k], g[2][k]);
        code[0] |= (unsigned)u.x << (8 * k);
        code[1] |= (unsigned)u.y << (8 * k);
        code[2] |= (unsigned)u.z << (8 * k);
    }
}

}  // namespace orrb
