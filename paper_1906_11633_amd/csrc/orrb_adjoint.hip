// Adjoint of the shading over a fixed visibility buffer (HIP, gfx950).
//
// Given the visibility keys of a forward render and dL/d(rgb), computes dL/d of the
// per-object albedo (3), roughness and specular, the per-light world vector (3: the
// position of a point light, the direction vector of a directional light) and
// intensity, and the per-frame exposure.  Visibility is fixed: none of these
// parameters moves geometry.
//
//   k_grad_tile    one workgroup per (frame, 32x32 tile): per pixel, rebuild the
//                  fragment from its key (exact edge functions of the snapped vertices,
//                  perspective-correct normal, view-space position: the forward's own
//                  fp32 arithmetic) and evaluate the analytic adjoint of the shading in
//                  fp32; every sum is FP64.  Per object: each wave adds its pixels'
//                  terms per distinct object (wave reductions), then the four waves in
//                  order; lights and exposure likewise.  The tile's sums go to a
//                  per-tile FP64 partial vector.
//   k_grad_reduce  per (scene, 64 parameters): the four waves sum interleaved quarters
//                  of the scene's tile partials, then combine in order, and write the
//                  gradient.
// No floating-point atomics: repeated calls are bit-identical.
#include "orrb_primitives.h"

namespace orrb {

constexpr int kGTile = 32;
constexpr int kGPix = kGTile * kGTile;      // pixels per tile
constexpr int kGPer = kGPix / kBlock;       // pixels per thread
constexpr int kGWaves = kBlock / kWave;
constexpr int kGMaxObj = 1024;              // objects per scene supported by the adjoint
constexpr int kGPresent = 64;               // distinct objects per tile summed per wave in LDS
constexpr int kGChunk = 64;                 // parameters per reduce workgroup

struct GradLds {
    float4 light[kMaxLights];     // view space: point position / unit direction to the light; w = intensity
    float light_qn[kMaxLights];   // directional: |R_V u| before normalization
    int light_type[kMaxLights];
    int o_tbase[kGMaxObj];        // scene triangle base of each object (object lookup)
    int pix_obj[kGPix];           // local object of each pixel's fragment, -1 none
    float pix_val[5][kGPix];      // its albedo (3), roughness and specular terms
    unsigned char present[kGMaxObj];
    int slot_of[kGMaxObj];        // present objects: their compact slot
    int slot_obj[kGPresent];
    double oacc[kGWaves][kGPresent][5];               // per-wave object sums
    double wacc[kGWaves][4 * kMaxLights + 1];         // per-wave light / exposure sums
    int n_present;
};

// Shift of a double across lanes by a DPP control (both halves moved alike; lanes
// without a source get 0.0).
template <int CTRL, int ROW_MASK>
ORRB_INLINE double dpp_d(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the wave in a fixed order: an inclusive DPP scan (shifts by 1, 2, 4, 8 in
// each 16-lane row, then rows 0 -> 1, 2 -> 3 and 1 -> 2, 3), whose last lane holds the
// total, broadcast to every lane.  No LDS round trips.
ORRB_INLINE double wave_sum(double x) {
    x += dpp_d<0x111, 0xf>(x);
    x += dpp_d<0x112, 0xf>(x);
    x += dpp_d<0x114, 0xf>(x);
    x += dpp_d<0x118, 0xf>(x);
    x += dpp_d<0x142, 0xa>(x);
    x += dpp_d<0x143, 0xc>(x);
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, kWave - 1);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), kWave - 1);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(kBlock) void k_grad_tile(GradArgs g) {
    __shared__ GradLds S;
    const RenderArgs &a = g.r;
    const int2 it = g.gitems[blockIdx.x];
    const int f = it.x;
    const FrameInfo fi = a.frames[f];
    const int W = fi.width, H = fi.height;
    const int ntx = (W + kGTile - 1) / kGTile;
    const int x0 = (it.y % ntx) * kGTile, y0 = (it.y / ntx) * kGTile;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int nl = fi.n_lights, n_obj = fi.n_obj;
    const float *V = a.view + 12 * (int64_t)f;

    if (tid < nl) {
        const int l = fi.light_begin + tid;
        const float *u = a.light_vec + 3 * (int64_t)l;
        const int type = a.light_type[l];
        double q[3];
        for (int r = 0; r < 3; ++r) {
            const double d = (double)V[r * 4 + 0] * u[0] + (double)V[r * 4 + 1] * u[1] + (double)V[r * 4 + 2] * u[2];
            q[r] = type == 0 ? d + (double)V[r * 4 + 3] : -d;
        }
        double qn = 1.0;
        if (type != 0) {
            qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
            for (int r = 0; r < 3; ++r) q[r] /= qn;
        }
        // the forward's view-space light (view_light), so the fragment terms agree
        S.light[tid] = view_light(V, u, type, a.light_intensity[l]);
        S.light_qn[tid] = (float)qn;
        S.light_type[tid] = type;
    }
    for (int k = tid; k < n_obj; k += kBlock) {
        S.o_tbase[k] = a.objs[fi.obj_begin + k].scene_tbase;
        S.present[k] = 0;
    }
    for (int k = tid; k < kGWaves * (4 * kMaxLights + 1); k += kBlock) (&S.wacc[0][0])[k] = 0.0;
    for (int k = tid; k < kGWaves * kGPresent * 5; k += kBlock) (&S.oacc[0][0][0])[k] = 0.0;
    __syncthreads();

    const CamF cam = frame_camera(a, f);
    const float e = cam.expo;
    const int64_t HW = (int64_t)W * H, po = fi.pixel_offset;
    for (int q = 0; q < kGPer; ++q) {
        const int p = tid + kBlock * q;
        const int li = p & (kGTile - 1), lj = p / kGTile;
        const int i = x0 + li, j = y0 + lj;
        int obj_local = -1;
        float ov[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f;
        float3 n = f3(0.f, 0.f, 1.f), pp = f3(0.f, 0.f, -1.f), v = f3(0.f, 0.f, 1.f);
        float al0 = 0.f, al1 = 0.f, al2 = 0.f, r = 1.f, ks = 0.f, m = 0.f, G = 0.f;
        if (i < W && j < H) {
            const int64_t pix = (int64_t)j * W + i;
            const unsigned long long key = g.vis[po + pix];
            gc0 = g.grad_rgb[3 * po + pix];
            gc1 = g.grad_rgb[3 * po + HW + pix];
            gc2 = g.grad_rgb[3 * po + 2 * HW + pix];
            if (key != kEmptyKey && (gc0 != 0.f || gc1 != 0.f || gc2 != 0.f)) {
                const int tri = (int)(unsigned)(key & 0xffffffffu);
                const float z = __uint_as_float((unsigned)(key >> 32));
                obj_local = find_slot(S.o_tbase, n_obj, tri);
                const int o = fi.obj_begin + obj_local;
                const ObjInfo ob = a.objs[o];
                const int4 tv = a.mesh_tri[ob.mesh_tbegin + (tri - ob.scene_tbase)];
                const int64_t vb = fi.vbase + ob.scene_vbase;
                const int4 pa = a.vtx_pos[vb + tv.x], pb = a.vtx_pos[vb + tv.z], pc = a.vtx_pos[vb + tv.y];
                const Edges ed = edge_eval(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, (i << 8) + 128, (j << 8) + 128,
                                           extent_flag(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y));
                const float t0 = ed.e0 * __int_as_float(pa.z), t1 = ed.e1 * __int_as_float(pb.z),
                            t2 = ed.e2 * __int_as_float(pc.z);
                const float4 na = a.mesh_nrm[ob.mesh_vbegin + tv.x], nb = a.mesh_nrm[ob.mesh_vbegin + tv.z],
                             nc = a.mesh_nrm[ob.mesh_vbegin + tv.y];
                const float4 *rot = a.obj_rot + 3 * (int64_t)(fi.oi_base + obj_local);
                const float4 R0 = rot[0], R1 = rot[1], R2 = rot[2];
                const float R[9] = {R0.x, R0.y, R0.z, R1.x, R1.y, R1.z, R2.x, R2.y, R2.z};
                {
#pragma clang fp contract(off)
                    const float4 no = make_float4(fmaf(t0, na.x, fmaf(t1, nb.x, t2 * nc.x)),
                                                  fmaf(t0, na.y, fmaf(t1, nb.y, t2 * nc.y)),
                                                  fmaf(t0, na.z, fmaf(t1, nb.z, t2 * nc.z)), 0.f);
                    n = rotate_normal(R, no);
                    pp = f3(z * (((float)i + 0.5f - cam.cx) * cam.ifx), -z * (((float)j + 0.5f - cam.cy) * cam.ify), -z);
                    const float pinv = rsqrtf(dot3(pp, pp));
                    v = f3(-pp.x * pinv, -pp.y * pinv, -pp.z * pinv);
                }
                r = a.roughness[o];
                ks = a.specular[o];
                m = 2.0f * __builtin_amdgcn_rcpf(r * r) - 2.0f;
                al0 = a.albedo[3 * o + 0];
                al1 = a.albedo[3 * o + 1];
                al2 = a.albedo[3 * o + 2];
                G = gc0 + gc1 + gc2;
            }
        }
        const bool frag = obj_local >= 0;
        float U0 = 0.f, U1 = 0.f, U2 = 0.f, sAnd = 0.f, sAnds = 0.f, sAndsln = 0.f;
        for (int l = 0; l < nl; ++l) {  // wave-uniform trip count
#pragma clang fp contract(off)
            float gq0 = 0.f, gq1 = 0.f, gq2 = 0.f, gI = 0.f;
            const bool point = S.light_type[l] == 0;
            if (frag) {
                const float4 Lq = S.light[l];
                float3 ld;
                float D = 1.f, dist = 1.f, A;
                if (point) {
                    const float3 d = f3(Lq.x - pp.x, Lq.y - pp.y, Lq.z - pp.z);
                    D = dot3(d, d);
                    const float dinv = rsqrtf(D);
                    dist = D * dinv;
                    ld = f3(d.x * dinv, d.y * dinv, d.z * dinv);
                    A = Lq.w * __builtin_amdgcn_rcpf(fmaxf(D, 1e-4f));
                } else {
                    ld = f3(Lq.x, Lq.y, Lq.z);
                    A = Lq.w;
                }
                const float ndl = dot3(n, ld);
                if (ndl > 0.f) {  // max(0, n.l) inactive: no contribution, sub-gradient 0
                    const float3 hh = f3(ld.x + v.x, ld.y + v.y, ld.z + v.z);
                    const float H2 = dot3(hh, hh);
                    float s = 0.f, ndh = 0.f, lnh = 0.f, hinv = 0.f;
                    float3 h = f3(0.f, 0.f, 0.f), w = f3(0.f, 0.f, 0.f);
                    if (H2 >= 1e-12f) {
                        hinv = rsqrtf(H2);
                        h = f3(hh.x * hinv, hh.y * hinv, hh.z * hinv);
                        const float3 dd = f3(n.x - h.x, n.y - h.y, n.z - h.z);
                        const float u = 0.5f * dot3(dd, dd);  // 1 - n.h, without cancellation
                        if (u < 1.0f) {
                            ndh = 1.0f - u;
                            const float l2 = log2_one_minus(u);
                            s = m == 0.f ? 1.0f : __builtin_amdgcn_exp2f(m * l2);
                            lnh = l2 * 0.69314718055994531f;
                            // n - (n.h) h = (n - h) + u h
                            w = f3(dd.x + u * h.x, dd.y + u * h.y, dd.z + u * h.z);
                        }
                    }
                    const float c0 = fmaf(ks, s, al0), c1 = fmaf(ks, s, al1), c2 = fmaf(ks, s, al2);
                    const float An = A * ndl;
                    U0 = fmaf(An, c0, U0);
                    U1 = fmaf(An, c1, U1);
                    U2 = fmaf(An, c2, U2);
                    const float Gh = gc0 * c0 + gc1 * c1 + gc2 * c2;
                    sAnd += An;
                    sAnds += An * s;
                    if (ndh > 0.f) sAndsln += An * s * lnh;
                    // n.h^(m - 1) = s / n.h; hl = |l + v| = 1 / hinv
                    const float spec = (ndh > 0.f && m != 0.f) ? e * G * An * ks * m * (s / ndh) * hinv : 0.f;
                    if (point) {
                        const float Ainv = __builtin_amdgcn_rcpf(fmaxf(D, 1e-4f));
                        gI = e * Gh * ndl * Ainv;
                        if (D > 1e-4f) {  // d A / d q through 1 / D
                            const float kk = e * Gh * ndl * (-2.0f * Lq.w) * Ainv * Ainv;
                            gq0 = kk * (ld.x * dist);
                            gq1 = kk * (ld.y * dist);
                            gq2 = kk * (ld.z * dist);
                        }
                        const float dinv = 1.0f / dist;
                        const float kn = e * Gh * A * dinv;
                        gq0 += kn * (n.x - ndl * ld.x);
                        gq1 += kn * (n.y - ndl * ld.y);
                        gq2 += kn * (n.z - ndl * ld.z);
                        if (spec != 0.f) {
                            const float lw = dot3(ld, w), ks2 = spec * dinv;
                            gq0 += ks2 * (w.x - lw * ld.x);
                            gq1 += ks2 * (w.y - lw * ld.y);
                            gq2 += ks2 * (w.z - lw * ld.z);
                        }
                    } else {
                        // directional: l = a / |a| with a = -R_V u reaches the shade through
                        // n.l and h = (l + v) / |l + v|; dL/da = (I - l l^T) dL/dl / |a|;
                        // gq holds dL/d(R_V u) = -dL/da (rotated to world below)
                        gI = e * Gh * ndl;
                        const float kn = e * Gh * A;
                        float3 gl = f3(kn * n.x, kn * n.y, kn * n.z);
                        if (spec != 0.f) gl = f3(gl.x + spec * w.x, gl.y + spec * w.y, gl.z + spec * w.z);
                        const float lg = dot3(ld, gl), qi = 1.0f / S.light_qn[l];
                        gq0 = -(gl.x - lg * ld.x) * qi;
                        gq1 = -(gl.y - lg * ld.y) * qi;
                        gq2 = -(gl.z - lg * ld.z) * qi;
                    }
                }
            }
            const double s0 = wave_sum((double)gq0), s1 = wave_sum((double)gq1), s2 = wave_sum((double)gq2),
                         s3 = wave_sum((double)gI);
            if (lane == 0) {
                S.wacc[wave][4 * l + 0] += s0;
                S.wacc[wave][4 * l + 1] += s1;
                S.wacc[wave][4 * l + 2] += s2;
                S.wacc[wave][4 * l + 3] += s3;
            }
        }
        {
            const double se = wave_sum((double)gc0 * U0 + (double)gc1 * U1 + (double)gc2 * U2);
            if (lane == 0) S.wacc[wave][4 * kMaxLights] += se;
        }
        if (frag) {
            ov[0] = e * gc0 * sAnd;
            ov[1] = e * gc1 * sAnd;
            ov[2] = e * gc2 * sAnd;
            ov[3] = e * G * ks * sAndsln * (-4.0f / (r * r * r));
            ov[4] = e * G * sAnds;
            S.present[obj_local] = 1;
        }
        S.pix_obj[p] = obj_local;
#pragma unroll
        for (int k = 0; k < 5; ++k) S.pix_val[k][p] = ov[k];
    }
    __syncthreads();

    // compact slots of the objects present in the tile (wave 0: a scan over the flags)
    if (wave == 0) {
        int base = 0;
        for (int k0 = 0; k0 < n_obj; k0 += kWave) {
            const int k = k0 + lane;
            const bool pr = k < n_obj && S.present[k];
            const unsigned long long mk = __ballot(pr);
            if (pr) {
                const int sl = base + lanes_below(mk);
                S.slot_of[k] = sl;
                if (sl < kGPresent) S.slot_obj[sl] = k;
            }
            base += __popcll(mk);
        }
        if (lane == 0) S.n_present = base;
    }
    __syncthreads();
    const int n_present = S.n_present;
    double *part = g.partial + g.gitem_pbase[blockIdx.x];
    if (n_present <= kGPresent) {
        // each wave adds its pixels (rows of 64 in order) per distinct object
        for (int q = 0; q < kGPer; ++q) {
            const int p = wave * kWave + lane + kBlock * q;
            const int k = S.pix_obj[p];
            unsigned long long pend = __ballot(k >= 0);
            while (pend) {
                const int k0 = __builtin_amdgcn_readlane(k, __builtin_ctzll(pend));
                const bool mine = k == k0;
                pend &= ~__ballot(mine);
                const int sl = S.slot_of[k0];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const double x = wave_sum(mine ? (double)S.pix_val[c][p] : 0.0);
                    if (lane == 0) S.oacc[wave][sl][c] += x;
                }
            }
        }
        __syncthreads();
        for (int k = tid; k < 5 * n_obj; k += kBlock) {
            const int o = k / 5, c = k - 5 * o;
            double x = 0.0;
            if (S.present[o]) {
                const int sl = S.slot_of[o];
                for (int w = 0; w < kGWaves; ++w) x += S.oacc[w][sl][c];
            }
            part[k] = x;
        }
    } else {
        // many objects in one tile: each present object in turn, every wave, then in order
        for (int k = 0; k < n_obj; ++k) {
            if (!S.present[k]) {
                if (tid < 5) part[5 * k + tid] = 0.0;
                continue;
            }
            for (int q = 0; q < kGPer; ++q) {
                const int p = wave * kWave + lane + kBlock * q;
                const bool mine = S.pix_obj[p] == k;
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const double x = wave_sum(mine ? (double)S.pix_val[c][p] : 0.0);
                    if (lane == 0) S.oacc[wave][0][c] += x;
                }
            }
            __syncthreads();
            if (tid < 5) {
                double x = 0.0;
                for (int w = 0; w < kGWaves; ++w) x += S.oacc[w][0][tid];
                part[5 * k + tid] = x;
            }
            __syncthreads();
            if (tid < kGWaves * 5) (&S.oacc[0][0][0])[(tid / 5) * kGPresent * 5 + tid % 5] = 0.0;
            __syncthreads();
        }
    }
    // lights (view -> world: dL/dq_world = R_V^T dL/dq_view) and exposure: waves summed in order
    double *lp = part + 5 * n_obj;
    if (tid < nl) {
        const int l = tid;
        double gv[4] = {0, 0, 0, 0};
        for (int w = 0; w < kGWaves; ++w)
            for (int c = 0; c < 4; ++c) gv[c] += S.wacc[w][4 * l + c];
        for (int c = 0; c < 3; ++c)
            lp[4 * l + c] = (double)V[0 * 4 + c] * gv[0] + (double)V[1 * 4 + c] * gv[1] + (double)V[2 * 4 + c] * gv[2];
        lp[4 * l + 3] = gv[3];
    }
    if (tid == kBlock - 1) {
        double se = 0.0;
        for (int w = 0; w < kGWaves; ++w) se += S.wacc[w][4 * kMaxLights];
        lp[4 * nl] = se;
    }
}

// Grid: x over 64-parameter chunks, y over scenes.  A scene's parameters: 5 per object,
// 4 per light, then 1 per frame (its exposure).  Wave w sums the scene's tile partials
// t = w, w + 4, ... in order; the four results are added in order.
__global__ __launch_bounds__(kBlock) void k_grad_reduce(GradArgs g, int s_base) {
    __shared__ double red[kGWaves][kGChunk];
    const int sc = s_base + (int)blockIdx.y;
    const int ob = g.scene_obj_begin[sc], no = g.scene_obj_begin[sc + 1] - ob;
    const int lb = g.scene_light_begin[sc], nl = g.scene_light_begin[sc + 1] - lb;
    const int fb = g.scene_frame_begin[sc], nf = g.scene_frame_begin[sc + 1] - fb;
    const int n_par = 5 * no + 4 * nl + nf;
    const int p = blockIdx.x * kGChunk + lane_id(), wave = threadIdx.x / kWave;
    if (blockIdx.x * kGChunk >= n_par) return;  // whole block past the scene's parameters
    double acc = 0.0;
    if (p < n_par) {
        int off, f_only = -1;
        if (p < 5 * no) off = p;
        else if (p < 5 * no + 4 * nl) off = p;  // lights follow the objects in every tile's vector
        else f_only = g.scene_frames[fb + (p - 5 * no - 4 * nl)], off = 5 * no + 4 * nl;
        int t = 0;  // the tile's position in the scene's list
        for (int fk = 0; fk < nf; ++fk) {
            const int f = g.scene_frames[fb + fk];
            const int i0 = g.frame_item_begin[f], i1 = g.frame_item_begin[f + 1];
            if (f_only >= 0 && f != f_only) {
                t += i1 - i0;
                continue;
            }
            for (int it = i0; it < i1; ++it, ++t)
                if ((t & (kGWaves - 1)) == wave) acc += g.partial[g.gitem_pbase[it] + off];
        }
    }
    red[wave][lane_id()] = acc;
    __syncthreads();
    if (wave != 0 || p >= n_par) return;
    double x = 0.0;
    for (int w = 0; w < kGWaves; ++w) x += red[w][lane_id()];
    if (p < 5 * no) {
        const int o = ob + p / 5, k = p % 5;
        if (k < 3) g.g_albedo[3 * o + k] = (float)x;
        else if (k == 3) g.g_rough[o] = (float)x;
        else g.g_spec[o] = (float)x;
    } else if (p < 5 * no + 4 * nl) {
        const int l = lb + (p - 5 * no) / 4, k = (p - 5 * no) % 4;
        if (k < 3) g.g_lpos[3 * l + k] = (float)x;
        else g.g_lint[l] = (float)x;
    } else {
        g.g_expo[g.scene_frames[fb + (p - 5 * no - 4 * nl)]] = (float)x;
    }
}

hipError_t launch_grad(const GradArgs &g, hipStream_t stream) {
    hipError_t e = launch_vertex(g.r, stream);
    if (e != hipSuccess) return e;
    if (g.n_gitems > 0) {
        hipLaunchKernelGGL(k_grad_tile, dim3(g.n_gitems), dim3(kBlock), 0, stream, g);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int chunks = (g.max_scene_params + kGChunk - 1) / kGChunk;
    constexpr int kMaxY = 32768;  // scenes per launch (grid y)
    for (int s0 = 0; s0 < g.n_scenes && e == hipSuccess; s0 += kMaxY) {
        const int ns = g.n_scenes - s0 < kMaxY ? g.n_scenes - s0 : kMaxY;
        hipLaunchKernelGGL(k_grad_reduce, dim3(chunks > 0 ? chunks : 1, ns), dim3(kBlock), 0, stream, g, s0);
        e = hipGetLastError();
    }
    return e;
}

int grad_tile_size() { return kGTile; }
int grad_max_objects() { return kGMaxObj; }

}  // namespace orrb
