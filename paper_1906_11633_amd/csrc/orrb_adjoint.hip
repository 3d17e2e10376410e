// Adjoint of the shading over a fixed visibility buffer (HIP, gfx950).
//
// Given the visibility keys of a forward render and dL/d(rgb), computes dL/d of the
// per-object albedo (3), roughness and specular, the per-light world vector (3: the
// position of a point light, the direction vector of a directional light) and
// intensity, and the per-frame exposure.  Visibility is fixed: none of these
// parameters moves geometry.
//
//   k_grad_tile    one workgroup per (frame, 32x32 tile): per pixel, rebuild the
//                  fragment from its key (exact edge functions of the snapped
//                  vertices, perspective-correct normal, view-space position) and
//                  evaluate the analytic adjoint of the shading in FP64; reduce the
//                  tile in a fixed order (wave shuffles, then waves in order) into a
//                  per-tile FP64 partial vector.
//   k_grad_reduce  one thread per output parameter: sums the partials of the tiles
//                  that can touch it, in a fixed order, and writes the gradient.
// No floating-point atomics: the result is deterministic.
#include "orrb_primitives.h"

namespace orrb {

constexpr int kGTile = 32;
constexpr int kGPix = kGTile * kGTile;      // pixels per tile
constexpr int kGPer = kGPix / kBlock;       // pixels per thread
constexpr int kGMaxObj = 1024;              // objects per scene supported by the adjoint

struct GradLds {
    double light_q[kMaxLights][3];
    double light_qn[kMaxLights];  // directional: |R_V u| before normalization
    double light_I[kMaxLights];
    int light_type[kMaxLights];
    int pix_obj[kGPix];
    double pix_val[5][kGPix];
    unsigned char present[kGMaxObj];
    double wacc[kBlock / kWave][4 * kMaxLights + 1];  // per-wave light / exposure sums
    double red[kBlock / kWave][5];
    double out[5];
};

// Sum over the wave (fixed butterfly order).
ORRB_INLINE double wave_sum(double x) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Sum of v[0..5) over the workgroup, fixed order; every thread gets the result.
ORRB_INLINE void block_sum5(double (&v)[5], GradLds &S) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double x = wave_sum(v[k]);
        if (lane == 0) S.red[wave][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double x = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) x += S.red[w][threadIdx.x];
        S.out[threadIdx.x] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = S.out[k];
    __syncthreads();
}

ORRB_INLINE double dot3d(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__global__ __launch_bounds__(kBlock) void k_grad_tile(GradArgs g) {
    __shared__ GradLds S;
    const RenderArgs &a = g.r;
    const int2 it = g.gitems[blockIdx.x];
    const int f = it.x;
    const FrameInfo fi = a.frames[f];
    const int W = fi.width, H = fi.height;
    const int ntx = (W + kGTile - 1) / kGTile;
    const int x0 = (it.y % ntx) * kGTile, y0 = (it.y / ntx) * kGTile;
    const int tid = threadIdx.x;
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
            qn = sqrt(dot3d(q, q));
            const double inv = 1.0 / qn;
            for (int r = 0; r < 3; ++r) q[r] *= inv;
        }
        for (int r = 0; r < 3; ++r) S.light_q[tid][r] = q[r];
        S.light_qn[tid] = qn;
        S.light_I[tid] = a.light_intensity[l];
        S.light_type[tid] = type;
    }
    for (int k = tid; k < n_obj; k += kBlock) S.present[k] = 0;
    for (int k = tid; k < (kBlock / kWave) * (4 * kMaxLights + 1); k += kBlock) (&S.wacc[0][0])[k] = 0.0;
    __syncthreads();
    const int lane = lane_id(), wave = tid / kWave;

    const float *K = a.intr + 4 * (int64_t)f;
    const double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    const double e = a.exposure[f];
    const int64_t HW = (int64_t)W * H, po = fi.pixel_offset;
    for (int q = 0; q < kGPer; ++q) {
        const int p = tid + kBlock * q;
        const int li = p & (kGTile - 1), lj = p / kGTile;
        const int i = x0 + li, j = y0 + lj;
        int obj_local = -1;
        double ov[5] = {0, 0, 0, 0, 0};
        // fragment state (valid when obj_local >= 0)
        double n[3] = {0, 0, 1}, pp[3] = {0, 0, -1}, v[3] = {0, 0, 1}, al[3] = {0, 0, 0}, gc[3] = {0, 0, 0};
        double r = 1.0, ks = 0.0, m = 0.0, G = 0.0;
        if (i < W && j < H) {
            const int64_t pix = (int64_t)j * W + i;
            const unsigned long long key = g.vis[po + pix];
            gc[0] = g.grad_rgb[3 * po + pix];
            gc[1] = g.grad_rgb[3 * po + HW + pix];
            gc[2] = g.grad_rgb[3 * po + 2 * HW + pix];
            if (key != kEmptyKey && (gc[0] != 0.0 || gc[1] != 0.0 || gc[2] != 0.0)) {
                const int tri = (int)(unsigned)(key & 0xffffffffu);
                const double z = (double)__uint_as_float((unsigned)(key >> 32));
                int lo = 0, hi = n_obj;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (a.objs[fi.obj_begin + mid].scene_tbase <= tri) lo = mid; else hi = mid;
                }
                obj_local = lo;
                const int o = fi.obj_begin + lo;
                const ObjInfo ob = a.objs[o];
                const int4 tv = a.mesh_tri[ob.mesh_tbegin + (tri - ob.scene_tbase)];
                const int64_t vb = fi.vbase + ob.scene_vbase;
                const int4 pa = a.vtx_pos[vb + tv.x], pb = a.vtx_pos[vb + tv.z], pc = a.vtx_pos[vb + tv.y];
                const Edges ed = edge_eval(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, (i << 8) + 128, (j << 8) + 128,
                                           extent_flag(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y));
                const double tw[3] = {(double)ed.e0 * __int_as_float(pa.z), (double)ed.e1 * __int_as_float(pb.z),
                                      (double)ed.e2 * __int_as_float(pc.z)};
                const float4 *rot = a.obj_rot + 3 * (int64_t)(fi.oi_base + lo);
                const float4 R0 = rot[0], R1 = rot[1], R2 = rot[2];
                const int vi[3] = {tv.x, tv.z, tv.y};
                n[0] = n[1] = n[2] = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float4 nm = a.mesh_nrm[ob.mesh_vbegin + vi[k]];
                    const double rr[3] = {(double)R0.x * nm.x + (double)R0.y * nm.y + (double)R0.z * nm.z,
                                          (double)R1.x * nm.x + (double)R1.y * nm.y + (double)R1.z * nm.z,
                                          (double)R2.x * nm.x + (double)R2.y * nm.y + (double)R2.z * nm.z};
                    const double sc = tw[k] / sqrt(dot3d(rr, rr));
                    n[0] += sc * rr[0];
                    n[1] += sc * rr[1];
                    n[2] += sc * rr[2];
                }
                const double ninv = 1.0 / sqrt(dot3d(n, n));
                n[0] *= ninv;
                n[1] *= ninv;
                n[2] *= ninv;
                pp[0] = z * ((i + 0.5 - cx) / fx);
                pp[1] = z * (-(j + 0.5 - cy) / fy);
                pp[2] = -z;
                const double pinv = 1.0 / sqrt(dot3d(pp, pp));
                v[0] = -pp[0] * pinv;
                v[1] = -pp[1] * pinv;
                v[2] = -pp[2] * pinv;
                r = a.roughness[o];
                ks = a.specular[o];
                m = 2.0 / (r * r) - 2.0;
                al[0] = a.albedo[3 * o + 0];
                al[1] = a.albedo[3 * o + 1];
                al[2] = a.albedo[3 * o + 2];
                G = gc[0] + gc[1] + gc[2];
            }
        }
        const bool frag = obj_local >= 0;
        double U[3] = {0, 0, 0}, sAnd = 0, sAnds = 0, sAndsln = 0;
        for (int l = 0; l < nl; ++l) {  // wave-uniform trip count
            double gq[3] = {0, 0, 0}, gI = 0.0;
            const bool point = S.light_type[l] == 0;
            if (frag) {
                double ld[3], D = 1.0, dist = 1.0, A;
                if (point) {
                    const double d[3] = {S.light_q[l][0] - pp[0], S.light_q[l][1] - pp[1], S.light_q[l][2] - pp[2]};
                    D = dot3d(d, d);
                    dist = sqrt(D);
                    for (int k = 0; k < 3; ++k) ld[k] = d[k] / dist;
                    A = S.light_I[l] / (D > 1e-4 ? D : 1e-4);
                } else {
                    for (int k = 0; k < 3; ++k) ld[k] = S.light_q[l][k];
                    A = S.light_I[l];
                }
                const double ndl = dot3d(n, ld);
                if (ndl > 0.0) {  // max(0, n.l) inactive: no contribution, sub-gradient 0
                    const double hh[3] = {ld[0] + v[0], ld[1] + v[1], ld[2] + v[2]};
                    const double H2 = dot3d(hh, hh);
                    double s = 0.0, ndh = 0.0, hl = 0.0, h[3] = {0, 0, 0};
                    if (H2 >= 1e-12) {
                        hl = sqrt(H2);
                        for (int k = 0; k < 3; ++k) h[k] = hh[k] / hl;
                        const double c2 = dot3d(n, h);
                        ndh = c2 > 0.0 ? c2 : 0.0;
                        s = ndh > 0.0 ? pow(ndh, m) : 0.0;
                    }
                    double Gh = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        U[c] += A * ndl * (al[c] + ks * s);
                        Gh += gc[c] * (al[c] + ks * s);
                    }
                    sAnd += A * ndl;
                    sAnds += A * ndl * s;
                    if (ndh > 0.0) sAndsln += A * ndl * s * log(ndh);
                    gI = e * Gh * ndl * (point ? 1.0 / (D > 1e-4 ? D : 1e-4) : 1.0);
                    if (point) {
                        if (D > 1e-4) {
                            const double kk = -2.0 * S.light_I[l] / (D * D);
                            for (int c = 0; c < 3; ++c) gq[c] += e * Gh * ndl * kk * (ld[c] * dist);
                        }
                        for (int c = 0; c < 3; ++c) gq[c] += e * Gh * A * (n[c] - ndl * ld[c]) / dist;
                        if (H2 >= 1e-12 && ndh > 0.0 && m != 0.0) {
                            double w[3];
                            for (int c = 0; c < 3; ++c) w[c] = n[c] - ndh * h[c];
                            const double lw = dot3d(ld, w);
                            const double coef = e * G * A * ndl * ks * m * pow(ndh, m - 1.0) / (hl * dist);
                            for (int c = 0; c < 3; ++c) gq[c] += coef * (w[c] - lw * ld[c]);
                        }
                    } else {
                        // directional: l = a / |a| with a = -R_V u reaches the shade through
                        // n.l and h = (l + v) / |l + v|; dL/dl, then dL/da = (I - l l^T)
                        // dL/dl / |a|; gq holds dL/d(R_V u) = -dL/da (rotated to world below)
                        double gl[3];
                        for (int c = 0; c < 3; ++c) gl[c] = e * Gh * A * n[c];
                        if (H2 >= 1e-12 && ndh > 0.0 && m != 0.0) {
                            const double coef = e * G * A * ndl * ks * m * pow(ndh, m - 1.0) / hl;
                            for (int c = 0; c < 3; ++c) gl[c] += coef * (n[c] - ndh * h[c]);
                        }
                        const double lg = dot3d(ld, gl);
                        for (int c = 0; c < 3; ++c) gq[c] = -(gl[c] - lg * ld[c]) / S.light_qn[l];
                    }
                }
            }
            const double s0 = wave_sum(gq[0]), s1 = wave_sum(gq[1]), s2 = wave_sum(gq[2]), s3 = wave_sum(gI);
            if (lane == 0) {
                S.wacc[wave][4 * l + 0] += s0;
                S.wacc[wave][4 * l + 1] += s1;
                S.wacc[wave][4 * l + 2] += s2;
                S.wacc[wave][4 * l + 3] += s3;
            }
        }
        {
            const double se = wave_sum(gc[0] * U[0] + gc[1] * U[1] + gc[2] * U[2]);
            if (lane == 0) S.wacc[wave][4 * kMaxLights] += se;
        }
        if (frag) {
            ov[0] = e * gc[0] * sAnd;
            ov[1] = e * gc[1] * sAnd;
            ov[2] = e * gc[2] * sAnd;
            ov[3] = e * G * ks * sAndsln * (-4.0 / (r * r * r));
            ov[4] = e * G * sAnds;
        }
        S.pix_obj[p] = obj_local;
        for (int k = 0; k < 5; ++k) S.pix_val[k][p] = ov[k];
        if (obj_local >= 0) S.present[obj_local] = 1;
    }
    __syncthreads();

    double *part = g.partial + g.gitem_pbase[blockIdx.x];
    // objects present in the tile: fixed-order masked sums; absent ones get zeros
    for (int k = 0; k < n_obj; ++k) {
        if (!S.present[k]) {
            if (tid < 5) part[5 * k + tid] = 0.0;
            continue;
        }
        double v5[5] = {0, 0, 0, 0, 0};
        for (int q = 0; q < kGPer; ++q) {
            const int p = tid + kBlock * q;
            if (S.pix_obj[p] == k)
                for (int c = 0; c < 5; ++c) v5[c] += S.pix_val[c][p];
        }
        block_sum5(v5, S);
        if (tid < 5) part[5 * k + tid] = v5[tid];
    }
    // lights (view -> world: dL/dq_world = R_V^T dL/dq_view) and exposure: waves summed in order
    double *lp = part + 5 * n_obj;
    if (tid < nl) {
        const int l = tid;
        double gv[4] = {0, 0, 0, 0};
        for (int w = 0; w < kBlock / kWave; ++w)
            for (int c = 0; c < 4; ++c) gv[c] += S.wacc[w][4 * l + c];
        // dq_world = R_V^T dq_view
        for (int c = 0; c < 3; ++c)
            lp[4 * l + c] = (double)V[0 * 4 + c] * gv[0] + (double)V[1 * 4 + c] * gv[1] + (double)V[2 * 4 + c] * gv[2];
        lp[4 * l + 3] = gv[3];
    }
    if (tid == kBlock - 1) {
        double se = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) se += S.wacc[w][4 * kMaxLights];
        lp[4 * nl] = se;
    }
}

__global__ __launch_bounds__(kBlock) void k_grad_reduce(GradArgs g) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n_obj_p = 5 * (int64_t)g.n_objects, n_light_p = 4 * (int64_t)g.n_lights;
    if (idx >= n_obj_p + n_light_p + g.n_frames) return;
    int scene, slot, f_only = -1;
    if (idx < n_obj_p) {
        const int o = (int)(idx / 5), k = (int)(idx % 5);
        scene = g.obj_scene[o];
        slot = 5 * g.obj_local[o] + k;
    } else if (idx < n_obj_p + n_light_p) {
        const int l = (int)((idx - n_obj_p) / 4), k = (int)((idx - n_obj_p) % 4);
        scene = g.light_scene[l];
        slot = -1 - (4 * g.light_local[l] + k);  // relative to the light block
    } else {
        f_only = (int)(idx - n_obj_p - n_light_p);
        scene = g.r.frames[f_only].scene;
        slot = 0;
    }
    double acc = 0.0;
    for (int fk = g.scene_frame_begin[scene]; fk < g.scene_frame_begin[scene + 1]; ++fk) {
        const int f = g.scene_frames[fk];
        if (f_only >= 0 && f != f_only) continue;
        const FrameInfo fi = g.r.frames[f];
        int off;
        if (f_only >= 0) off = 5 * fi.n_obj + 4 * fi.n_lights;
        else if (slot >= 0) off = slot;
        else off = 5 * fi.n_obj + (-1 - slot);
        for (int it = g.frame_item_begin[f]; it < g.frame_item_begin[f + 1]; ++it) acc += g.partial[g.gitem_pbase[it] + off];
    }
    if (idx < n_obj_p) {
        const int o = (int)(idx / 5), k = (int)(idx % 5);
        if (k < 3) g.g_albedo[3 * o + k] = (float)acc;
        else if (k == 3) g.g_rough[o] = (float)acc;
        else g.g_spec[o] = (float)acc;
    } else if (idx < n_obj_p + n_light_p) {
        const int l = (int)((idx - n_obj_p) / 4), k = (int)((idx - n_obj_p) % 4);
        if (k < 3) g.g_lpos[3 * l + k] = (float)acc;
        else g.g_lint[l] = (float)acc;
    } else {
        g.g_expo[f_only] = (float)acc;
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
    const int64_t n = 5 * (int64_t)g.n_objects + 4 * (int64_t)g.n_lights + g.n_frames;
    if (n > 0) {
        hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream, g);
        e = hipGetLastError();
    }
    return e;
}

int grad_tile_size() { return kGTile; }
int grad_max_objects() { return kGMaxObj; }

}  // namespace orrb
