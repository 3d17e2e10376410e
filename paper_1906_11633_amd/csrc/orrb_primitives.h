// Device arithmetic primitives shared by every kernel of the batched renderer (vertex
// snapping, exact edge functions, fragment depth, shading, stores).  All kernels use
// these same inline functions, compiled with contraction off where the result bits
// matter, so every path produces bit-identical results.
#pragma once

#include "orrb_device.h"

namespace orrb {

#define ORRB_INLINE __device__ __attribute__((always_inline)) inline

// ------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------

ORRB_INLINE int lane_id() { return __lane_id(); }

ORRB_INLINE int lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// floor(a / 256) and ceil(a / 256) for int32 (arithmetic shift floors)
ORRB_INLINE int floor256(int a) { return a >> 8; }
ORRB_INLINE int ceil256(int a) { return -((-a) >> 8); }

ORRB_INLINE float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
ORRB_INLINE float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

ORRB_INLINE int find_slot(const int *base, int n, int x) {  // largest k < n with base[k] <= x
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------------------------
// vertex stage (FP64, the oracle's fma order, no contraction)
// ------------------------------------------------------------------------------------

// One entry e = 4 i + j of M = V o W (3x4 affine, row-major).
ORRB_INLINE double compose_entry(const float *V, const float *Wp, int e) {
#pragma clang fp contract(off)
    const int i = e >> 2, j = e & 3;
    const double v0 = V[i * 4 + 0], v1 = V[i * 4 + 1], v2 = V[i * 4 + 2], v3 = V[i * 4 + 3];
    if (j < 3) {
        double t = v2 * (double)Wp[2 * 4 + j];
        t = fma(v1, (double)Wp[1 * 4 + j], t);
        return fma(v0, (double)Wp[0 * 4 + j], t);
    }
    return fma(v0, (double)Wp[3], fma(v1, (double)Wp[7], fma(v2, (double)Wp[11], v3)));
}

struct Snapped {
    int X, Y, valid;
    int cull;  // invalid vertices: 1 nearer than the near plane, 2 beyond the guard band
    float iw;  // fp32 1 / w
};

// Transform, project and snap one vertex: X = rint(256 sx), Y = rint(256 sy), valid if
// w >= near and both inside the +-2^24 guard band.
ORRB_INLINE Snapped snap_vertex(const double *M, float4 p, double fx, double fy, double cx, double cy, double nearp) {
#pragma clang fp contract(off)
    const double x = p.x, y = p.y, z = p.z;
    const double e0 = fma(M[0], x, fma(M[1], y, fma(M[2], z, M[3])));
    const double e1 = fma(M[4], x, fma(M[5], y, fma(M[6], z, M[7])));
    const double e2 = fma(M[8], x, fma(M[9], y, fma(M[10], z, M[11])));
    const double w = -e2;
    Snapped s;
    s.valid = 0;
    s.cull = 1;
    s.X = s.Y = 0;
    s.iw = 0.f;
    if (w >= nearp) {
        const double qx = e0 / w, qy = e1 / w;  // IEEE division, round to nearest
        const double sx = fma(fx, qx, cx), sy = fma(-fy, qy, cy);
        const double Xd = rint(256.0 * sx), Yd = rint(256.0 * sy);  // half to even
        s.cull = 2;
        if (fabs(Xd) <= (double)kGuard && fabs(Yd) <= (double)kGuard) {
            s.valid = 1;
            s.cull = 0;
            s.X = (int)Xd;
            s.Y = (int)Yd;
            s.iw = 1.0f / (float)w;
        }
    }
    return s;
}

// ------------------------------------------------------------------------------------
// triangle set-up and edge functions
// ------------------------------------------------------------------------------------

// Exact edge functions of the positive-area triangle a, b, c at pixel centre (PX, PY).
// Small triangles (extent <= 2^14) use 24-bit integer products, larger ones FP64
// products (exact below 2^53).  E_k is the edge opposite vertex k.
struct Edges {
    float e0, e1, e2;
    bool covered;
};

ORRB_INLINE Edges edge_eval(int xa, int ya, int xb, int yb, int xc, int yc, int PX, int PY, int flags) {
    Edges r;
    const int b0 = (flags & 1) ? 0 : 1, b1 = (flags & 2) ? 0 : 1, b2 = (flags & 4) ? 0 : 1;
    if (!(flags & 8)) {
        const int E0 = __mul24(xc - xb, PY - yb) - __mul24(yc - yb, PX - xb);
        const int E1 = __mul24(xa - xc, PY - yc) - __mul24(ya - yc, PX - xc);
        const int E2 = __mul24(xb - xa, PY - ya) - __mul24(yb - ya, PX - xa);
        r.covered = ((E0 - b0) | (E1 - b1) | (E2 - b2)) >= 0;  // top-left rule
        r.e0 = (float)E0;
        r.e1 = (float)E1;
        r.e2 = (float)E2;
    } else {
        const double E0 = fma((double)(xc - xb), (double)(PY - yb), -((double)(yc - yb) * (double)(PX - xb)));
        const double E1 = fma((double)(xa - xc), (double)(PY - yc), -((double)(ya - yc) * (double)(PX - xc)));
        const double E2 = fma((double)(xb - xa), (double)(PY - ya), -((double)(yb - ya) * (double)(PX - xa)));
        r.covered = (E0 - b0) >= 0 && (E1 - b1) >= 0 && (E2 - b2) >= 0;
        r.e0 = (float)E0;
        r.e1 = (float)E1;
        r.e2 = (float)E2;
    }
    return r;
}

// The integer edge functions of edge_eval (small triangles) at pixel centre (PX, PY)
// and their steps per pixel in x and y.  Stepping adds exact int32 differences, so at
// every pixel centre of the triangle's range the values equal edge_eval's.
struct EdgeStep {
    int e0, e1, e2;
    int dx0, dx1, dx2, dy0, dy1, dy2;
};

ORRB_INLINE EdgeStep edge_start(int xa, int ya, int xb, int yb, int xc, int yc, int PX, int PY) {
    EdgeStep s;
    s.e0 = __mul24(xc - xb, PY - yb) - __mul24(yc - yb, PX - xb);
    s.e1 = __mul24(xa - xc, PY - yc) - __mul24(ya - yc, PX - xc);
    s.e2 = __mul24(xb - xa, PY - ya) - __mul24(yb - ya, PX - xa);
    s.dx0 = (yb - yc) * 256;
    s.dx1 = (yc - ya) * 256;
    s.dx2 = (ya - yb) * 256;
    s.dy0 = (xc - xb) * 256;
    s.dy1 = (xa - xc) * 256;
    s.dy2 = (xb - xa) * 256;
    return s;
}

ORRB_INLINE int top_left(int dX, int dY) { return dY < 0 || (dY == 0 && dX > 0); }

ORRB_INLINE int extent_flag(int xa, int ya, int xb, int yb, int xc, int yc) {
    const int ext = max(max(xa, max(xb, xc)) - min(xa, min(xb, xc)), max(ya, max(yb, yc)) - min(ya, min(yb, yc)));
    return ext > kSmallExtent ? 8 : 0;
}

// bit k = the edge opposite vertex k is top-left; bit 3 = large triangle (FP64 edges)
ORRB_INLINE int tri_flags(int xa, int ya, int xb, int yb, int xc, int yc) {
    return top_left(xc - xb, yc - yb) | (top_left(xa - xc, ya - yc) << 1) | (top_left(xb - xa, yb - ya) << 2) |
           extent_flag(xa, ya, xb, yb, xc, yc);
}

// Perspective-correct eye depth of a covered fragment: z = A / sum_k E_k / w_k.  All
// terms are non-negative, so the only error is rounding (< 3e-7 relative with the
// hardware reciprocal).
ORRB_INLINE float fragment_depth(const Edges &e, float iwa, float iwb, float iwc, float area) {
#pragma clang fp contract(off)
    const float T = fmaf(e.e0, iwa, fmaf(e.e1, iwb, e.e2 * iwc));
    return area * __builtin_amdgcn_rcpf(T);
}

ORRB_INLINE unsigned long long vis_key(float z, int tri) {
    return ((unsigned long long)__float_as_uint(z) << 32) | (unsigned)tri;
}

// ------------------------------------------------------------------------------------
// shading (shared by both paths)
// ------------------------------------------------------------------------------------

// A scene light in the frame's view space: point lights as a position, directional
// lights as the unit direction toward the light; w = intensity.
ORRB_INLINE float4 view_light(const float *V, const float *u, int type, float intensity) {
    double q[3];
    for (int r = 0; r < 3; ++r) {
        const double d = (double)V[r * 4 + 0] * u[0] + (double)V[r * 4 + 1] * u[1] + (double)V[r * 4 + 2] * u[2];
        q[r] = type == 0 ? d + (double)V[r * 4 + 3] : -d;
    }
    if (type != 0) {
        const double inv = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        q[0] *= inv;
        q[1] *= inv;
        q[2] *= inv;
    }
    return make_float4((float)q[0], (float)q[1], (float)q[2], intensity);
}

struct Material {
    float rough, ks, al0, al1, al2;
};

struct CamF {
    float cx, cy, ifx, ify, expo;
};

// A spot light (light type 2) in a frame's view space, with its shadow map: unit
// axis, cosines of the inner and outer half-angles, T = shadow camera o view^-1 (view
// space -> shadow camera space, row-major 3x4), the shadow camera's intrinsics and the
// map's slot.  A light's type word holds 2 | (index of this record << 4).
struct SpotLight {
    float ax, ay, az;
    float cin, cout;
    float T[12];
    float fx, fy, cx, cy;
    int slot;
};
constexpr float kShadowBias = 0.02f;  // lit if (1 - bias) w <= the map's depth

// The view-space record of global spot light l for a frame with world->camera view V
// (fp32 inputs, FP64 arithmetic, rounded once).
ORRB_INLINE SpotLight spot_setup(const RenderArgs &a, const float *V, int l) {
    SpotLight r;
    const float *d = a.light_dir + 3 * (int64_t)l;
    double ax[3];
    for (int k = 0; k < 3; ++k)
        ax[k] = (double)V[k * 4 + 0] * d[0] + (double)V[k * 4 + 1] * d[1] + (double)V[k * 4 + 2] * d[2];
    const double inv = 1.0 / sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    r.ax = (float)(ax[0] * inv);
    r.ay = (float)(ax[1] * inv);
    r.az = (float)(ax[2] * inv);
    r.cin = a.light_cone[2 * (int64_t)l];
    r.cout = a.light_cone[2 * (int64_t)l + 1];
    // V^-1 of the rigid view [R | t] is [R^T | -R^T t]
    double Vi[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) Vi[i * 4 + j] = V[j * 4 + i];
        Vi[i * 4 + 3] = -((double)V[0 * 4 + i] * V[3] + (double)V[1 * 4 + i] * V[7] + (double)V[2 * 4 + i] * V[11]);
    }
    const float *Sv = a.shadow_view + 12 * (int64_t)l;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) {
            double t = (double)Sv[i * 4 + 0] * Vi[0 * 4 + j] + (double)Sv[i * 4 + 1] * Vi[1 * 4 + j] +
                       (double)Sv[i * 4 + 2] * Vi[2 * 4 + j];
            if (j == 3) t += Sv[i * 4 + 3];
            r.T[i * 4 + j] = (float)t;
        }
    const float *K = a.shadow_intr + 4 * (int64_t)l;
    r.fx = K[0];
    r.fy = K[1];
    r.cx = K[2];
    r.cy = K[3];
    r.slot = a.spot_slot[l];
    return r;
}

// Fraction of the 3 x 3 shadow-map texels around view-space point p's texel that see
// it (percentage-closer filtering; empty and off-map texels count as lit, a point not
// in front of the shadow camera is lit).
ORRB_INLINE float shadow_pcf(const SpotLight &sp, const float *maps, int N, float px, float py, float pz) {
#pragma clang fp contract(off)
    const float qx = sp.T[0] * px + sp.T[1] * py + sp.T[2] * pz + sp.T[3];
    const float qy = sp.T[4] * px + sp.T[5] * py + sp.T[6] * pz + sp.T[7];
    const float qz = sp.T[8] * px + sp.T[9] * py + sp.T[10] * pz + sp.T[11];
    const float w = -qz;
    if (!(w > 0.f)) return 1.0f;
    const float u = sp.fx * (qx / w) + sp.cx, v = -sp.fy * (qy / w) + sp.cy;
    const float fu = floorf(u), fv = floorf(v);
    if (!(fu > -2.f && fu < (float)N + 1.f && fv > -2.f && fv < (float)N + 1.f)) return 1.0f;  // every texel off the map
    const int ti = (int)fu, tj = (int)fv;
    const float wb = (1.0f - kShadowBias) * w;
    const float *map = maps + (int64_t)sp.slot * N * N;
    int lit = 0;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
            const int x = ti + di, y = tj + dj;
            float z = 0.f;
            if (x >= 0 && y >= 0 && x < N && y < N) z = map[(int64_t)y * N + x];
            lit += (z == 0.f || wb <= z) ? 1 : 0;
        }
    return (float)lit * (1.0f / 9.0f);
}

struct PixelOut {
    float r0, r1, r2, n0, n1, n2;
};

ORRB_INLINE float3 rotate_normal(const float *R, float4 q) {
#pragma clang fp contract(off)
    const float3 r = f3(fmaf(R[0], q.x, fmaf(R[1], q.y, R[2] * q.z)), fmaf(R[3], q.x, fmaf(R[4], q.y, R[5] * q.z)),
                        fmaf(R[6], q.x, fmaf(R[7], q.y, R[8] * q.z)));
    const float s = rsqrtf(dot3(r, r));
    return f3(r.x * s, r.y * s, r.z * s);
}

// (1 - u)^m for 0 <= u < 1, m > 0, as 2^(m log2(1 - u)).  log2(1 - u) comes from the
// Taylor series of ln(1 - u) (through u^7, truncation below 5e-10 relative) when
// u < 1/16, where forming 1 - u would lose the low bits of u, and from the hardware
// log2 otherwise (1 - u is then within 2^-25 of exact).  Against the exact power the
// error stays below 3e-7 absolute and, where the power exceeds 1e-5, 1e-5 relative.
// log2(1 - u) for 0 <= u < 1, as spec_pow forms it (series below 1/16).
ORRB_INLINE float log2_one_minus(float u) {
#pragma clang fp contract(off)
    float l2;
    if (u < 0.0625f) {
        float p = fmaf(u, 1.0f / 7.0f, 1.0f / 6.0f);
        p = fmaf(u, p, 0.2f);
        p = fmaf(u, p, 0.25f);
        p = fmaf(u, p, 1.0f / 3.0f);
        p = fmaf(u, p, 0.5f);
        p = fmaf(u, p, 1.0f);
        l2 = -(u * p) * 1.44269504088896341f;
    } else {
        l2 = __builtin_amdgcn_logf(1.0f - u);
    }
    return l2;
}

ORRB_INLINE float spec_pow(float u, float m) {
#pragma clang fp contract(off)
    return __builtin_amdgcn_exp2f(m * log2_one_minus(u));
}

// A pixel's material inputs beyond the LDS material (textured / emissive shading):
// the winning triangle's vertex UVs (positive-area order), the object's texture id,
// UV transform and emissive power.
struct MatTex {
    float2 uva, uvb, uvc;
    int tex, ntex;              // pattern and normal texture (-1 none)
    float su, sv, ou, ov;
    float emit;
    float4 pa, pb, pc;          // object-space positions (normal texture only)
};

// Material inputs of global object o whose mesh vertices start at mvb, for the mesh
// triangle tv (a, b, c = tv.x, tv.z, tv.y in positive-area order).
ORRB_INLINE MatTex mat_inputs(const RenderArgs &a, int o, int mvb, int4 tv) {
    MatTex t;
    t.tex = a.obj_tex ? a.obj_tex[o] : -1;
    if (t.tex >= a.n_tex) t.tex = -1;  // not a resident texture: none
    t.ntex = a.obj_ntex ? a.obj_ntex[o] : -1;
    if (t.ntex >= a.n_tex) t.ntex = -1;
    t.su = t.sv = 1.f;
    t.ou = t.ov = 0.f;
    t.uva = t.uvb = t.uvc = make_float2(0.f, 0.f);
    if (t.ntex >= 0) {
        t.pa = a.mesh_pos[mvb + tv.x];
        t.pb = a.mesh_pos[mvb + tv.z];
        t.pc = a.mesh_pos[mvb + tv.y];
    }
    if (t.tex >= 0 || t.ntex >= 0) {
        const float4 x = *reinterpret_cast<const float4 *>(a.tex_xform + 4 * (int64_t)o);
        t.su = x.x;
        t.sv = x.y;
        t.ou = x.z;
        t.ov = x.w;
        t.uva = a.mesh_uv[mvb + tv.x];
        t.uvb = a.mesh_uv[mvb + tv.z];
        t.uvc = a.mesh_uv[mvb + tv.y];
    }
    t.emit = a.emission ? a.emission[o] : 0.f;
    return t;
}

// Bilinear sample of a texture at (u, v), repeating: texel (i, j) is centred at
// ((i + 1/2) / W, (j + 1/2) / H), row 0 first.
ORRB_INLINE float3 tex_bilinear(const float4 *texels, int4 info, double u, double v) {
#pragma clang fp contract(off)
    // texel coordinates and weights in FP64: a bright pixel on a contrasting texel edge
    // would otherwise carry the fp32 rounding of u W into its colour
    const int W = info.y, H = info.z;
    const double x = u * (double)W - 0.5, y = v * (double)H - 0.5;
    const double fx = floor(x), fy = floor(y);
    const float ax = (float)(x - fx), ay = (float)(y - fy);
    int i0 = (int)((long long)fx % W), j0 = (int)((long long)fy % H);
    if (i0 < 0) i0 += W;
    if (j0 < 0) j0 += H;
    const int i1 = i0 + 1 == W ? 0 : i0 + 1, j1 = j0 + 1 == H ? 0 : j0 + 1;
    const float4 *T = texels + info.x;
    const float4 t00 = T[j0 * W + i0], t01 = T[j0 * W + i1], t10 = T[j1 * W + i0], t11 = T[j1 * W + i1];
    const float b0 = 1.f - ax, b1 = 1.f - ay;
    return f3(b1 * (b0 * t00.x + ax * t01.x) + ay * (b0 * t10.x + ax * t11.x),
              b1 * (b0 * t00.y + ax * t01.y) + ay * (b0 * t10.y + ax * t11.y),
              b1 * (b0 * t00.z + ax * t01.z) + ay * (b0 * t10.z + ax * t11.z));
}

// The shading normal from a normal texture's bilinear sample rgb at a fragment with
// unit interpolated normal n: t = normalize(2 rgb - 1) in the triangle's tangent frame.
// T and B solve e1 = du1 T + dv1 B, e2 = du2 T + dv2 B for the object-space edges and
// UV differences (vertex order does not matter), rotated with the object by R; T is
// orthogonalized against n, B' = n x T' flipped to the side of B (the UV mapping's
// handedness).  Degenerate UVs, a tangent along n or t = 0 leave n.
ORRB_INLINE float3 normal_mapped(float3 n, float3 rgb, const MatTex &mt, const float *R) {
#pragma clang fp contract(off)
    const float3 t = f3(2.0f * rgb.x - 1.0f, 2.0f * rgb.y - 1.0f, 2.0f * rgb.z - 1.0f);
    const float tl2 = dot3(t, t);
    const float du1 = mt.uvb.x - mt.uva.x, dv1 = mt.uvb.y - mt.uva.y;
    const float du2 = mt.uvc.x - mt.uva.x, dv2 = mt.uvc.y - mt.uva.y;
    const float det = du1 * dv2 - du2 * dv1;
    if (!(tl2 > 0.f) || det == 0.f) return n;
    const float id = 1.0f / det;
    const float3 e1 = f3(mt.pb.x - mt.pa.x, mt.pb.y - mt.pa.y, mt.pb.z - mt.pa.z);
    const float3 e2 = f3(mt.pc.x - mt.pa.x, mt.pc.y - mt.pa.y, mt.pc.z - mt.pa.z);
    const float3 To = f3((e1.x * dv2 - e2.x * dv1) * id, (e1.y * dv2 - e2.y * dv1) * id, (e1.z * dv2 - e2.z * dv1) * id);
    const float3 Bo = f3((e2.x * du1 - e1.x * du2) * id, (e2.y * du1 - e1.y * du2) * id, (e2.z * du1 - e1.z * du2) * id);
    const float3 T = f3(R[0] * To.x + R[1] * To.y + R[2] * To.z, R[3] * To.x + R[4] * To.y + R[5] * To.z,
                        R[6] * To.x + R[7] * To.y + R[8] * To.z);
    const float3 B = f3(R[0] * Bo.x + R[1] * Bo.y + R[2] * Bo.z, R[3] * Bo.x + R[4] * Bo.y + R[5] * Bo.z,
                        R[6] * Bo.x + R[7] * Bo.y + R[8] * Bo.z);
    const float nt = dot3(n, T);
    float3 Tp = f3(T.x - nt * n.x, T.y - nt * n.y, T.z - nt * n.z);
    const float tp2 = dot3(Tp, Tp);
    if (!(tp2 > 0.f)) return n;
    const float tpi = rsqrtf(tp2);
    Tp = f3(Tp.x * tpi, Tp.y * tpi, Tp.z * tpi);
    float3 Bp = f3(n.y * Tp.z - n.z * Tp.y, n.z * Tp.x - n.x * Tp.z, n.x * Tp.y - n.y * Tp.x);
    if (dot3(Bp, B) < 0.f) Bp = f3(-Bp.x, -Bp.y, -Bp.z);
    const float ti = rsqrtf(tl2);
    const float3 s = f3((t.x * Tp.x + t.y * Bp.x + t.z * n.x) * ti, (t.x * Tp.y + t.y * Bp.y + t.z * n.y) * ti,
                        (t.x * Tp.z + t.y * Bp.z + t.z * n.z) * ti);
    const float si = rsqrtf(dot3(s, s));
    return f3(s.x * si, s.y * si, s.z * si);
}

// Shade the covered pixel (i, j) at eye depth z of the positive-area triangle a, b, c:
// perspective-correct smooth normal from the unit object-space vertex normals and R,
// then exposure * sum over lights of A * max(0, n.l) * (albedo + k_s * max(0, n.h)^m).
template <bool SPOT = false, bool MAT = false>
ORRB_INLINE PixelOut shade_pixel(int xa, int ya, int xb, int yb, int xc, int yc, float iwa, float iwb, float iwc,
                                 float4 na4, float4 nb4, float4 nc4, const float *R, int i, int j, float z,
                                 const CamF &cam, const float4 *light, const int *ltype, int nl, const Material &m,
                                 const SpotLight *spot = nullptr, const float *maps = nullptr, int shadow_res = 0,
                                 const MatTex *mt = nullptr, const float4 *texels = nullptr,
                                 const int4 *tex_info = nullptr) {
#pragma clang fp contract(off)
    const Edges e = edge_eval(xa, ya, xb, yb, xc, yc, (i << 8) + 128, (j << 8) + 128, extent_flag(xa, ya, xb, yb, xc, yc));
    // perspective-correct weights are proportional to E_k / w_k
    const float t0 = e.e0 * iwa, t1 = e.e1 * iwb, t2 = e.e2 * iwc;
    // R = s * Rotation (rigid + uniform scale) and unit object-space vertex normals, so
    // normalize(sum t_k normalize(R n_k)) = normalize(R sum t_k n_k): interpolate in
    // object space, rotate once, normalize once.
    const float4 no = make_float4(fmaf(t0, na4.x, fmaf(t1, nb4.x, t2 * nc4.x)), fmaf(t0, na4.y, fmaf(t1, nb4.y, t2 * nc4.y)),
                                  fmaf(t0, na4.z, fmaf(t1, nb4.z, t2 * nc4.z)), 0.f);
    const float3 n = rotate_normal(R, no);
    const float3 pp = f3(z * (((float)i + 0.5f - cam.cx) * cam.ifx), -z * (((float)j + 0.5f - cam.cy) * cam.ify), -z);
    const float pinv = rsqrtf(dot3(pp, pp));
    const float3 v = f3(-pp.x * pinv, -pp.y * pinv, -pp.z * pinv);
    const float mexp = 2.0f * __builtin_amdgcn_rcpf(m.rough * m.rough) - 2.0f;
    float al0 = m.al0, al1 = m.al1, al2 = m.al2;
    float r0 = 0.f, r1 = 0.f, r2 = 0.f;
    float3 ns = n;  // the normal the lights see
    if (MAT) {  // textures at the perspective-correct, transformed UV, then emission
        if (mt->tex >= 0 || mt->ntex >= 0) {
            // the UV as vertex a's plus the weighted differences (fp32 rounding relative to
            // the triangle's UV extent), then the tiling transform in FP64
            const float inv = 1.0f / (t0 + t1 + t2);
            const float du = (t1 * (mt->uvb.x - mt->uva.x) + t2 * (mt->uvc.x - mt->uva.x)) * inv;
            const float dv = (t1 * (mt->uvb.y - mt->uva.y) + t2 * (mt->uvc.y - mt->uva.y)) * inv;
            const double u = ((double)mt->uva.x + du) * mt->su + mt->ou;
            const double v = ((double)mt->uva.y + dv) * mt->sv + mt->ov;
            if (mt->tex >= 0) {
                const float3 tx = tex_bilinear(texels, tex_info[mt->tex], u, v);
                al0 *= tx.x;
                al1 *= tx.y;
                al2 *= tx.z;
            }
            if (mt->ntex >= 0) ns = normal_mapped(n, tex_bilinear(texels, tex_info[mt->ntex], u, v), *mt, R);
        }
        r0 = mt->emit * al0;
        r1 = mt->emit * al1;
        r2 = mt->emit * al2;
    }
    for (int l = 0; l < nl; ++l) {
        const float4 Lq = light[l];
        const int lt = ltype[l];
        float3 ld;
        float A;
        if (lt == 0 || (SPOT && (lt & 15) == 2)) {
            const float3 d = f3(Lq.x - pp.x, Lq.y - pp.y, Lq.z - pp.z);
            const float D = dot3(d, d);
            const float dinv = rsqrtf(D);
            ld = f3(d.x * dinv, d.y * dinv, d.z * dinv);
            A = Lq.w * __builtin_amdgcn_rcpf(fmaxf(D, 1e-4f));
        } else {
            ld = f3(Lq.x, Lq.y, Lq.z);
            A = Lq.w;
        }
        const float ndl = dot3(ns, ld);
        if (ndl <= 0.f) continue;
        if (SPOT && (lt & 15) == 2) {  // cone (smoothstep) and filtered shadow
            const SpotLight &sp = spot[lt >> 4];
            const float c = -(ld.x * sp.ax + ld.y * sp.ay + ld.z * sp.az);
            const float t = fminf(fmaxf((c - sp.cout) / (sp.cin - sp.cout), 0.f), 1.f);
            const float cone = t * t * (3.0f - 2.0f * t);
            if (cone <= 0.f) continue;
            A = A * cone * shadow_pcf(sp, maps, shadow_res, pp.x, pp.y, pp.z);
        }
        float s = 0.f;
        const float3 hh = f3(ld.x + v.x, ld.y + v.y, ld.z + v.z);
        const float H2 = dot3(hh, hh);
        if (H2 >= 1e-12f) {
            const float hinv = rsqrtf(H2);
            const float3 dd = f3(ns.x - hh.x * hinv, ns.y - hh.y * hinv, ns.z - hh.z * hinv);
            // 1 - n.h evaluated as |n - h|^2 / 2: no cancellation near the highlight
            const float u = 0.5f * dot3(dd, dd);
            if (u < 1.0f) s = (mexp == 0.f) ? 1.0f : spec_pow(u, mexp);
        }
        const float An = A * ndl;
        r0 = fmaf(An, fmaf(m.ks, s, al0), r0);
        r1 = fmaf(An, fmaf(m.ks, s, al1), r1);
        r2 = fmaf(An, fmaf(m.ks, s, al2), r2);
    }
    PixelOut o;
    o.r0 = r0 * cam.expo;
    o.r1 = r1 * cam.expo;
    o.r2 = r2 * cam.expo;
    o.n0 = n.x;
    o.n1 = n.y;
    o.n2 = n.z;
    return o;
}

// Plain stores: non-temporal ones bypass the L2 merging of neighbouring row segments
// and measured at about half the write bandwidth for tiled output.
ORRB_INLINE void store_pixel(const RenderArgs &a, int64_t po, int64_t HW, int64_t pix, const PixelOut &o, float z, int seg,
                             int tri, unsigned long long key) {
    if (a.out_rgb) {
        a.out_rgb[3 * po + pix] = o.r0;
        a.out_rgb[3 * po + HW + pix] = o.r1;
        a.out_rgb[3 * po + 2 * HW + pix] = o.r2;
    }
    if (a.out_depth) a.out_depth[po + pix] = z;
    if (a.out_normal) {
        a.out_normal[3 * po + pix] = o.n0;
        a.out_normal[3 * po + HW + pix] = o.n1;
        a.out_normal[3 * po + 2 * HW + pix] = o.n2;
    }
    if (a.out_seg) a.out_seg[po + pix] = seg;
    if (a.out_tri) a.out_tri[po + pix] = tri;
    if (a.out_vis) a.out_vis[po + pix] = key;
    if (a.out_alpha) a.out_alpha[po + pix] = key != kEmptyKey ? 1.0f : 0.0f;
}

// ------------------------------------------------------------------------------------
// tracker records (Sec. 4.3.2 Tracker)
// ------------------------------------------------------------------------------------

// Empty record of an object whose composed matrix M = V o W (FP64, row-major 3x4) puts
// its origin at eye coordinates (M[3], M[7], M[11]); the origin projected with the
// frame's pinhole camera, NaN when it is not in front of the camera.
ORRB_INLINE void track_init(orrb_track *t, double e0, double e1, double e2, double fx, double fy, double cx,
                            double cy) {
    const double w = -e2;
    float x = __builtin_nanf(""), y = __builtin_nanf("");
    if (w > 0.0) {
        x = (float)fma(fx, e0 / w, cx);
        y = (float)fma(-fy, e1 / w, cy);
    }
    orrb_track r;
    r.count = 0;
    r.i_min = r.j_min = 0x7fffffff;
    r.i_max = r.j_max = -1;
    r.x = x;
    r.y = y;
    r.w = (float)w;
    r.sum_i = r.sum_j = 0;
    *t = r;
}

// Reductions over the wave by an inclusive DPP scan (shifts by 1, 2, 4, 8 inside each
// 16-lane row, then rows 0 -> 1, 2 -> 3 and 1 -> 2, 3; lanes without a source take the
// identity); the last lane holds the result, which every lane receives.
template <class Op>
ORRB_INLINE int wave_reduce(int v, int identity, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x111, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x112, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x114, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x118, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x142, 0xa, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, kWave - 1);
}
ORRB_INLINE int wave_min(int v) {
    return wave_reduce(v, 0x7fffffff, [](int x, int y) { return min(x, y); });
}
ORRB_INLINE int wave_max(int v) {
    return wave_reduce(v, -0x7fffffff - 1, [](int x, int y) { return max(x, y); });
}
ORRB_INLINE unsigned wave_sum(unsigned v) {
    return (unsigned)wave_reduce((int)v, 0, [](int x, int y) { return (int)((unsigned)x + (unsigned)y); });
}

// Two 16-bit lanes of a 32-bit value, reduced pairwise (v_pk_min_u16 / v_pk_max_u16).
typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));
ORRB_INLINE int pk_min_u16(int x, int y) {
    return __builtin_bit_cast(int, __builtin_elementwise_min(__builtin_bit_cast(ushort2v, x), __builtin_bit_cast(ushort2v, y)));
}
ORRB_INLINE int pk_max_u16(int x, int y) {
    return __builtin_bit_cast(int, __builtin_elementwise_max(__builtin_bit_cast(ushort2v, x), __builtin_bit_cast(ushort2v, y)));
}

// Add the wave's pixels to their tracker records: lane L holds pixel (i, j) of record
// `rec` (-1: none), 0 <= i, j < 65536.  Must be called with every lane of the wave
// active.  One group of global atomics per distinct record in the wave; integer min /
// max / sums, so the result does not depend on the order of waves or tiles.  The
// column and row travel packed as i | j << 16: their minima and maxima reduce as 16-bit
// pairs, and so do their sums when NARROW (i, j < 1024: 64 lanes sum below 2^16).
template <bool NARROW>
ORRB_INLINE void track_wave(orrb_track *base, int rec, int i, int j) {
    unsigned long long pend = __ballot(rec >= 0);
    const int ij = (int)((unsigned)i | ((unsigned)j << 16));
    while (pend) {
        const int first = __builtin_ctzll(pend);
        const int r0 = __builtin_amdgcn_readlane(rec, first);
        const bool mine = rec == r0;
        const unsigned long long m = __ballot(mine);
        const unsigned mn = (unsigned)wave_reduce(mine ? ij : -1, -1, pk_min_u16);
        const unsigned mx = (unsigned)wave_reduce(mine ? ij : 0, 0, pk_max_u16);
        unsigned si, sj;
        if constexpr (NARROW) {
            const unsigned s2 = wave_sum(mine ? (unsigned)ij : 0u);
            si = s2 & 0xffffu;
            sj = s2 >> 16;
        } else {
            si = wave_sum(mine ? (unsigned)i : 0u);
            sj = wave_sum(mine ? (unsigned)j : 0u);
        }
        if (lane_id() == first) {
            orrb_track *t = base + r0;
            atomicAdd(&t->count, (int)__popcll(m));
            atomicMin(&t->i_min, (int)(mn & 0xffffu));
            atomicMin(&t->j_min, (int)(mn >> 16));
            atomicMax(&t->i_max, (int)(mx & 0xffffu));
            atomicMax(&t->j_max, (int)(mx >> 16));
            atomicAdd((unsigned long long *)&t->sum_i, (unsigned long long)si);
            atomicAdd((unsigned long long *)&t->sum_j, (unsigned long long)sj);
        }
        pend &= ~m;
    }
}

// The same for a whole 64 x 4 tile of the frame path: lane L holds the four pixels
// (i0 + q, j), q < 4, with object slot s[q] of the frame's records `base` (-1: not
// covered).  One reduction and one group of atomics per object present in the tile
// rather than per 64 covered pixels.  i0 + 3 and j are below 256 (the frame path's
// frames), so a tile's column and row sums (at most 256 x 255) fit 16 bits and travel
// packed like the minima and maxima; the count (0 to 4 per lane) is summed from three
// ballots.  Must be called with every lane of the wave active.
ORRB_INLINE void track_tile(orrb_track *base, const int s[4], int i0, int j) {
    int left = (s[0] >= 0 ? 1 : 0) | (s[1] >= 0 ? 2 : 0) | (s[2] >= 0 ? 4 : 0) | (s[3] >= 0 ? 8 : 0);
    unsigned long long pend = __ballot(left != 0);
    while (pend) {
        const int first = __builtin_ctzll(pend);
        int mine = -1;  // the lane's lowest pending slot
#pragma unroll
        for (int q = 3; q >= 0; --q)
            if ((left >> q) & 1) mine = s[q];
        const int r0 = __builtin_amdgcn_readlane(mine, first);
        int cnt = 0, mn = -1, mx = 0;
        unsigned sum = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (((left >> q) & 1) && s[q] == r0) {
                const int ij = (int)((unsigned)(i0 + q) | ((unsigned)j << 16));
                ++cnt;
                mn = pk_min_u16(mn, ij);
                mx = pk_max_u16(mx, ij);
                sum += (unsigned)ij;
                left &= ~(1 << q);
            }
        }
        const unsigned MN = (unsigned)wave_reduce(mn, -1, pk_min_u16);
        const unsigned MX = (unsigned)wave_reduce(mx, 0, pk_max_u16);
        const unsigned S2 = wave_sum(sum);
        const int C = __popcll(__ballot(cnt & 1)) + 2 * __popcll(__ballot(cnt & 2)) + 4 * __popcll(__ballot(cnt & 4));
        if (lane_id() == first) {
            orrb_track *t = base + r0;
            atomicAdd(&t->count, C);
            atomicMin(&t->i_min, (int)(MN & 0xffffu));
            atomicMin(&t->j_min, (int)(MN >> 16));
            atomicMax(&t->i_max, (int)(MX & 0xffffu));
            atomicMax(&t->j_max, (int)(MX >> 16));
            atomicAdd((unsigned long long *)&t->sum_i, (unsigned long long)(S2 & 0xffffu));
            atomicAdd((unsigned long long *)&t->sum_j, (unsigned long long)(S2 >> 16));
        }
        pend = __ballot(left != 0);
    }
}

ORRB_INLINE CamF frame_camera(const RenderArgs &a, int f) {
    const float *K = a.intr + 4 * (int64_t)f;
    CamF c;
    c.cx = K[2];
    c.cy = K[3];
    c.ifx = (float)(1.0 / (double)K[0]);
    c.ify = (float)(1.0 / (double)K[1]);
    c.expo = a.exposure[f];
    return c;
}

ORRB_INLINE Material object_material(const RenderArgs &a, int o) {
    Material m;
    m.rough = a.roughness[o];
    m.ks = a.specular[o];
    m.al0 = a.albedo[3 * o + 0];
    m.al1 = a.albedo[3 * o + 1];
    m.al2 = a.albedo[3 * o + 2];
    return m;
}

}  // namespace orrb
