// HIP kernels of the batched randomized renderer, written for CDNA4 (gfx950, wave64).
//
// Pipeline per batch (all frames of all scenes in two launches):
//   k_vertex        one workgroup per (frame, object): FP64 transform, projection and
//                   1/256-px snapping of the object's vertices in a fixed fma order,
//                   view-space normals, and the object's covered pixel-centre range.
//   k_raster_shade  one workgroup per (frame, screen tile): cull objects by their
//                   range, set up their triangles (exact integer area, back-face and
//                   range cull) and stage the survivors in an LDS bin; rasterize the
//                   bin with exact edge functions and the top-left rule, one lane per
//                   (triangle, pixel) pair, into an LDS visibility tile of 64-bit keys
//                   (fp32 eye depth << 32 | scene-local triangle ID) resolved with
//                   ds_min_u64; then shade every pixel of the tile from its key
//                   (deferred shading) and write the planar channels.
//
// The visibility result is a 64-bit minimum, so it does not depend on the order in
// which lanes, bins, tiles or workgroups run: outputs are bit-identical for every
// tile size, bin capacity, launch shape and batch composition.
#include "orrb_device.h"

namespace orrb {

// ------------------------------------------------------------------------------------
// small wave / block helpers
// ------------------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// floor(a / 256) and ceil(a / 256) for int32 (arithmetic shift floors)
__device__ __forceinline__ int floor256(int a) { return a >> 8; }
__device__ __forceinline__ int ceil256(int a) { return -((-a) >> 8); }

// Exclusive block scan of cnt(k) for k < n (n <= 4 * kBlock); writes pre[0..n].
template <class F>
__device__ void block_scan(F cnt, int n, int *pre, int *wave_tot) {
    const int per = (n + kBlock - 1) / kBlock;
    const int t = threadIdx.x, lane = lane_id(), wave = t / kWave;
    const int start = t * per;
    int local = 0;
    for (int k = 0; k < per; ++k)
        if (start + k < n) local += cnt(start + k);
    int incl = local;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wave_tot[wave] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += wave_tot[w];
    int run = wbase + incl - local;
    for (int k = 0; k < per; ++k) {
        if (start + k < n) {
            pre[start + k] = run;
            run += cnt(start + k);
        }
    }
    if (t == kBlock - 1) pre[n] = wbase + incl;
    __syncthreads();
}

// ------------------------------------------------------------------------------------
// k_vertex
// ------------------------------------------------------------------------------------

// One entry of M = V o W (3x4 affine, row-major) in the fixed fma order the oracle
// uses; contraction is off so no other fusing can change a rounding.
__device__ double compose_entry(const float *V, const float *Wp, int e) {
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
    double w;
};

__device__ Snapped snap_vertex(const double *M, float4 p, double fx, double fy, double cx, double cy, double nearp) {
#pragma clang fp contract(off)
    const double x = p.x, y = p.y, z = p.z;
    const double e0 = fma(M[0], x, fma(M[1], y, fma(M[2], z, M[3])));
    const double e1 = fma(M[4], x, fma(M[5], y, fma(M[6], z, M[7])));
    const double e2 = fma(M[8], x, fma(M[9], y, fma(M[10], z, M[11])));
    Snapped s;
    s.w = -e2;
    s.valid = 0;
    s.X = s.Y = 0;
    if (s.w >= nearp) {
        const double qx = e0 / s.w, qy = e1 / s.w;       // IEEE division, round to nearest
        const double sx = fma(fx, qx, cx), sy = fma(-fy, qy, cy);
        const double Xd = rint(256.0 * sx), Yd = rint(256.0 * sy);  // half to even
        if (fabs(Xd) <= (double)kGuard && fabs(Yd) <= (double)kGuard) {
            s.valid = 1;
            s.X = (int)Xd;
            s.Y = (int)Yd;
        }
    }
    return s;
}

__global__ __launch_bounds__(kBlock) void k_vertex(RenderArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.queue = 0u;  // persistent raster counter
    if ((int)blockIdx.x >= a.n_vitems) return;
    __shared__ double M[12];
    __shared__ int red[4][kBlock / kWave];
    const int2 it = a.vitems[blockIdx.x];
    const int f = it.x;
    const FrameInfo fi = a.frames[f];
    const int o = fi.obj_begin + it.y;
    const int oi = fi.oi_base + it.y;
    if (!a.visible[o]) {
        if (threadIdx.x == 0) a.obj_bbox[oi] = make_int4(1, 1, 0, 0);
        return;
    }
    const ObjInfo ob = a.objs[o];
    if (threadIdx.x < 12) M[threadIdx.x] = compose_entry(a.view + 12 * (int64_t)f, a.pose + 12 * (int64_t)o, threadIdx.x);
    __syncthreads();
    const float *K = a.intr + 4 * (int64_t)f;
    const double fx = K[0], fy = K[1], cx = K[2], cy = K[3], nearp = a.near_plane[f];
    double Mr[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) Mr[k] = M[k];
    int xmin = 0x7fffffff, ymin = 0x7fffffff, xmax = -0x7fffffff, ymax = -0x7fffffff;
    const int64_t vb = fi.vbase + ob.scene_vbase;
    for (int v = threadIdx.x; v < ob.n_verts; v += kBlock) {
        const float4 p = a.mesh_pos[ob.mesh_vbegin + v];
        const float4 nn = a.mesh_nrm[ob.mesh_vbegin + v];
        const Snapped s = snap_vertex(Mr, p, fx, fy, cx, cy, nearp);
        double nx = Mr[0] * nn.x + Mr[1] * nn.y + Mr[2] * nn.z;
        double ny = Mr[4] * nn.x + Mr[5] * nn.y + Mr[6] * nn.z;
        double nz = Mr[8] * nn.x + Mr[9] * nn.y + Mr[10] * nn.z;
        const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        const float wf = (float)s.w;
        const float iw = 1.0f / wf;
        a.vtx_pos[vb + v] = make_int4(s.X, s.Y, __float_as_int(iw), s.valid);
        a.vtx_nrm[vb + v] = make_float4((float)(nx * inv), (float)(ny * inv), (float)(nz * inv), wf);
        if (s.valid) {
            xmin = min(xmin, s.X);
            xmax = max(xmax, s.X);
            ymin = min(ymin, s.Y);
            ymax = max(ymax, s.Y);
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        xmin = min(xmin, __shfl_xor(xmin, off));
        ymin = min(ymin, __shfl_xor(ymin, off));
        xmax = max(xmax, __shfl_xor(xmax, off));
        ymax = max(ymax, __shfl_xor(ymax, off));
    }
    const int wave = threadIdx.x / kWave;
    if (lane_id() == 0) {
        red[0][wave] = xmin;
        red[1][wave] = ymin;
        red[2][wave] = xmax;
        red[3][wave] = ymax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) {
            xmin = min(xmin, red[0][w]);
            ymin = min(ymin, red[1][w]);
            xmax = max(xmax, red[2][w]);
            ymax = max(ymax, red[3][w]);
        }
        int4 bb = make_int4(1, 1, 0, 0);
        if (xmin <= xmax) {
            bb.x = max(ceil256(xmin - 128), 0);
            bb.y = max(ceil256(ymin - 128), 0);
            bb.z = min(floor256(xmax - 128), fi.width - 1);
            bb.w = min(floor256(ymax - 128), fi.height - 1);
        }
        a.obj_bbox[oi] = bb;
    }
}

// ------------------------------------------------------------------------------------
// k_raster_shade
// ------------------------------------------------------------------------------------

// LDS carve-up of one raster workgroup.
struct Lds {
    unsigned long long *vis;  // tile_w * tile_h keys
    int *b_tri, *b_x0, *b_y0, *b_x1, *b_y1, *b_x2, *b_y2, *b_rng, *b_flags, *b_pre;
    float *b_iw0, *b_iw1, *b_iw2, *b_area;
    int *ol_obj, *ol_cnt, *ol_pre;
    float4 *light;
    int *light_type;
    int *misc;  // [0] bin count, [1] next item, [4..8) scan scratch
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t lds_layout(int tw, int th, int cap, char *base, Lds *L) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = align16(off + bytes);
        return p;
    };
    char *vis = take(sizeof(unsigned long long) * tw * th);
    char *bi[10];
    for (int k = 0; k < 9; ++k) bi[k] = take(sizeof(int) * cap);
    bi[9] = take(sizeof(int) * (cap + 1));
    char *bf[4];
    for (int k = 0; k < 4; ++k) bf[k] = take(sizeof(float) * cap);
    char *ol0 = take(sizeof(int) * kBlock), *ol1 = take(sizeof(int) * kBlock), *ol2 = take(sizeof(int) * (kBlock + 1));
    char *lt = take(sizeof(float4) * kMaxLights), *ltt = take(sizeof(int) * kMaxLights);
    char *misc = take(sizeof(int) * 16);
    if (L) {
        L->vis = (unsigned long long *)vis;
        L->b_tri = (int *)bi[0];
        L->b_x0 = (int *)bi[1];
        L->b_y0 = (int *)bi[2];
        L->b_x1 = (int *)bi[3];
        L->b_y1 = (int *)bi[4];
        L->b_x2 = (int *)bi[5];
        L->b_y2 = (int *)bi[6];
        L->b_rng = (int *)bi[7];
        L->b_flags = (int *)bi[8];
        L->b_pre = (int *)bi[9];
        L->b_iw0 = (float *)bf[0];
        L->b_iw1 = (float *)bf[1];
        L->b_iw2 = (float *)bf[2];
        L->b_area = (float *)bf[3];
        L->ol_obj = (int *)ol0;
        L->ol_cnt = (int *)ol1;
        L->ol_pre = (int *)ol2;
        L->light = (float4 *)lt;
        L->light_type = (int *)ltt;
        L->misc = (int *)misc;
    }
    return off;
}

size_t raster_lds_bytes(int tile_w, int tile_h, int bin_cap) { return lds_layout(tile_w, tile_h, bin_cap, nullptr, nullptr); }

// Exact edge functions of the (already swapped, positive-area) triangle a, b, c at
// pixel centre (PX, PY).  Small triangles (extent <= 2^14) use 24-bit integer
// products, larger ones FP64 products (exact below 2^53).  Returns E as floats.
struct Edges {
    float e0, e1, e2;
    bool covered;
};

__device__ __forceinline__ Edges edge_eval(int xa, int ya, int xb, int yb, int xc, int yc, int PX, int PY, int flags) {
    Edges r;
    const int b0 = (flags & 1) ? 0 : 1, b1 = (flags & 2) ? 0 : 1, b2 = (flags & 4) ? 0 : 1;
    if (!(flags & 8)) {
        const int E0 = __mul24(xc - xb, PY - yb) - __mul24(yc - yb, PX - xb);
        const int E1 = __mul24(xa - xc, PY - yc) - __mul24(ya - yc, PX - xc);
        const int E2 = __mul24(xb - xa, PY - ya) - __mul24(yb - ya, PX - xa);
        r.covered = ((E0 - b0) | (E1 - b1) | (E2 - b2)) >= 0;
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

__device__ __forceinline__ int top_left(int dX, int dY) { return dY < 0 || (dY == 0 && dX > 0); }

// Edge flags of triangle a, b, c: bit k = edge opposite vertex k is top-left, bit 3 =
// large triangle (FP64 edge path).
__device__ __forceinline__ int tri_flags(int xa, int ya, int xb, int yb, int xc, int yc, int extent) {
    return top_left(xc - xb, yc - yb) | (top_left(xa - xc, ya - yc) << 1) | (top_left(xb - xa, yb - ya) << 2) |
           ((extent > kSmallExtent) ? 8 : 0);
}

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

// Raster every staged triangle of the bin into the LDS visibility tile.
__device__ void flush_bin(const Lds &L, int n, int tx0, int ty0, int tile_w) {
    block_scan([&](int k) { const unsigned r = (unsigned)L.b_rng[k]; return (int)(((r >> 16) & 0xff) * (r >> 24)); },
               n, L.b_pre, L.misc + 4);
    const int total = L.b_pre[n];
    for (int w = threadIdx.x; w < total; w += kBlock) {
        int lo = 0, hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (L.b_pre[mid] <= w) lo = mid; else hi = mid;
        }
        const int k = lo;
        const unsigned rng = (unsigned)L.b_rng[k];
        const int nx = (rng >> 16) & 0xff;
        const int r = w - L.b_pre[k];
        const int dj = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)nx));
        const int di = r - dj * nx;
        const int li = (int)(rng & 0xff) + di, lj = (int)((rng >> 8) & 0xff) + dj;
        const int PX = ((tx0 + li) << 8) + 128, PY = ((ty0 + lj) << 8) + 128;
        const Edges e = edge_eval(L.b_x0[k], L.b_y0[k], L.b_x1[k], L.b_y1[k], L.b_x2[k], L.b_y2[k], PX, PY, L.b_flags[k]);
        if (!e.covered) continue;
        const float T = fmaf(e.e0, L.b_iw0[k], fmaf(e.e1, L.b_iw1[k], e.e2 * L.b_iw2[k]));
        const float z = L.b_area[k] / T;
        const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned)L.b_tri[k];
        atomicMin(&L.vis[lj * tile_w + li], key);
    }
    __syncthreads();
}

__device__ void raster_shade_tile(const RenderArgs &a, int item, const Lds &L) {
    const int2 it = a.titems[item];
    const int f = it.x;
    const FrameInfo fi = a.frames[f];
    const int TW = a.tile_w, TH = a.tile_h, cap = a.bin_cap;
    const int tx0 = (it.y % fi.tiles_x) * TW, ty0 = (it.y / fi.tiles_x) * TH;
    const int tw = min(TW, fi.width - tx0), th = min(TH, fi.height - ty0);
    const int tx1 = tx0 + tw - 1, ty1 = ty0 + th - 1;
    const int tid = threadIdx.x, lane = lane_id();

    for (int p = tid; p < TW * TH; p += kBlock) L.vis[p] = kEmptyKey;
    if (tid == 0) L.misc[0] = 0;
    if (tid < fi.n_lights) {
        const int l = fi.light_begin + tid;
        const float *V = a.view + 12 * (int64_t)f;
        const float *u = a.light_vec + 3 * (int64_t)l;
        const int type = a.light_type[l];
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
        L.light[tid] = make_float4((float)q[0], (float)q[1], (float)q[2], a.light_intensity[l]);
        L.light_type[tid] = type;
    }
    __syncthreads();

    // ---- visibility: object cull, triangle set-up into the LDS bin, raster ----
    const int64_t vbase = fi.vbase;
    for (int c0 = 0; c0 < fi.n_obj; c0 += kBlock) {
        const int s = c0 + tid;
        bool ov = false;
        int ntri = 0;
        if (s < fi.n_obj) {
            const int4 bb = a.obj_bbox[fi.oi_base + s];
            ov = bb.x <= bb.z && bb.y <= bb.w && bb.x <= tx1 && bb.z >= tx0 && bb.y <= ty1 && bb.w >= ty0;
            if (ov) ntri = a.objs[fi.obj_begin + s].n_tris;
        }
        {   // order-free compaction of overlapping objects
            const unsigned long long m = __ballot(ov);
            int base = 0;
            if (lane == 0 && m) base = atomicAdd(&L.misc[2], __popcll(m));
            base = __shfl(base, 0);
            if (ov) {
                const int slot = base + lanes_below(m);
                L.ol_obj[slot] = fi.obj_begin + s;
                L.ol_cnt[slot] = ntri;
            }
        }
        __syncthreads();
        const int n_ol = L.misc[2];
        block_scan([&](int k) { return L.ol_cnt[k]; }, n_ol, L.ol_pre, L.misc + 4);
        const int n_cand = L.ol_pre[n_ol];
        for (int base = 0; base < n_cand; base += kBlock) {
            const int k = base + tid;
            bool keep = false;
            int xa = 0, ya = 0, xb = 0, yb = 0, xc = 0, yc = 0, rng = 0, flags = 0, tri_id = 0;
            float iwa = 0.f, iwb = 0.f, iwc = 0.f, area = 0.f;
            if (k < n_cand) {
                int lo = 0, hi = n_ol;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (L.ol_pre[mid] <= k) lo = mid; else hi = mid;
                }
                const int o = L.ol_obj[lo];
                const int t = k - L.ol_pre[lo];
                const ObjInfo ob = a.objs[o];
                const int4 tri = a.mesh_tri[ob.mesh_tbegin + t];
                const int64_t vb = vbase + ob.scene_vbase;
                const int4 p0 = a.vtx_pos[vb + tri.x], p1 = a.vtx_pos[vb + tri.y], p2 = a.vtx_pos[vb + tri.z];
                if (p0.w & p1.w & p2.w) {
                    const long long A = (long long)(p1.x - p0.x) * (p2.y - p0.y) - (long long)(p1.y - p0.y) * (p2.x - p0.x);
                    if (A < 0) {
                        // front face: a = v0, b = v2, c = v1 gives a positive area
                        xa = p0.x; ya = p0.y; xb = p2.x; yb = p2.y; xc = p1.x; yc = p1.y;
                        const int xmin = min(xa, min(xb, xc)), xmax = max(xa, max(xb, xc));
                        const int ymin = min(ya, min(yb, yc)), ymax = max(ya, max(yb, yc));
                        const int i0 = max(ceil256(xmin - 128), tx0), i1 = min(floor256(xmax - 128), tx1);
                        const int j0 = max(ceil256(ymin - 128), ty0), j1 = min(floor256(ymax - 128), ty1);
                        if (i0 <= i1 && j0 <= j1) {
                            keep = true;
                            rng = (i0 - tx0) | ((j0 - ty0) << 8) | ((i1 - i0 + 1) << 16) | ((j1 - j0 + 1) << 24);
                            flags = tri_flags(xa, ya, xb, yb, xc, yc, max(xmax - xmin, ymax - ymin));
                            iwa = __int_as_float(p0.z);
                            iwb = __int_as_float(p2.z);
                            iwc = __int_as_float(p1.z);
                            area = (float)(-A);
                            tri_id = ob.scene_tbase + t;
                        }
                    }
                }
            }
            const unsigned long long m = __ballot(keep);
            int wb = 0;
            if (lane == 0 && m) wb = atomicAdd(&L.misc[0], __popcll(m));
            wb = __shfl(wb, 0);
            if (keep) {
                const int slot = wb + lanes_below(m);
                L.b_tri[slot] = tri_id;
                L.b_x0[slot] = xa; L.b_y0[slot] = ya;
                L.b_x1[slot] = xb; L.b_y1[slot] = yb;
                L.b_x2[slot] = xc; L.b_y2[slot] = yc;
                L.b_rng[slot] = rng;
                L.b_flags[slot] = flags;
                L.b_iw0[slot] = iwa; L.b_iw1[slot] = iwb; L.b_iw2[slot] = iwc;
                L.b_area[slot] = area;
            }
            __syncthreads();
            const int nb = L.misc[0];
            if (nb > cap - kBlock || (base + kBlock >= n_cand && c0 + kBlock >= fi.n_obj && nb > 0)) {
                flush_bin(L, nb, tx0, ty0, TW);
                if (tid == 0) L.misc[0] = 0;
                __syncthreads();
            }
        }
        if (tid == 0) L.misc[2] = 0;
        __syncthreads();
    }
    // a bin left non-empty by a chunk without candidates in its last round
    if (L.misc[0] > 0) {
        flush_bin(L, L.misc[0], tx0, ty0, TW);
    }

    // ---- deferred shading of the tile ----
    const float *K = a.intr + 4 * (int64_t)f;
    const float cx = K[2], cy = K[3];
    const float ifx = (float)(1.0 / (double)K[0]), ify = (float)(1.0 / (double)K[1]);
    const float expo = a.exposure[f];
    const int64_t HW = (int64_t)fi.width * fi.height, po = fi.pixel_offset;
    const float inv_tw = __builtin_amdgcn_rcpf((float)tw);
    const int nl = fi.n_lights;
    for (int p = tid; p < tw * th; p += kBlock) {
        const int lj = (int)(((float)p + 0.5f) * inv_tw);
        const int li = p - lj * tw;
        const int i = tx0 + li, j = ty0 + lj;
        const int64_t pix = (int64_t)j * fi.width + i;
        const unsigned long long key = L.vis[lj * TW + li];
        float r0 = 0.f, r1 = 0.f, r2 = 0.f, z = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
        int segv = -1, triv = -1;
        if (key != kEmptyKey) {
            const int tri = (int)(unsigned)(key & 0xffffffffu);
            z = __uint_as_float((unsigned)(key >> 32));
            int lo = 0, hi = fi.n_obj;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.objs[fi.obj_begin + mid].scene_tbase <= tri) lo = mid; else hi = mid;
            }
            const int o = fi.obj_begin + lo;
            const ObjInfo ob = a.objs[o];
            const int4 tv = a.mesh_tri[ob.mesh_tbegin + (tri - ob.scene_tbase)];
            const int64_t vb = vbase + ob.scene_vbase;
            // the winning triangle is front-facing: same swap as in set-up
            const int4 pa = a.vtx_pos[vb + tv.x], pb = a.vtx_pos[vb + tv.z], pc = a.vtx_pos[vb + tv.y];
            const float4 na = a.vtx_nrm[vb + tv.x], nb = a.vtx_nrm[vb + tv.z], nc = a.vtx_nrm[vb + tv.y];
            const int xmin = min(pa.x, min(pb.x, pc.x)), xmax = max(pa.x, max(pb.x, pc.x));
            const int ymin = min(pa.y, min(pb.y, pc.y)), ymax = max(pa.y, max(pb.y, pc.y));
            const int flags = (max(xmax - xmin, ymax - ymin) > kSmallExtent) ? 8 : 0;
            const Edges e = edge_eval(pa.x, pa.y, pb.x, pb.y, pc.x, pc.y, (i << 8) + 128, (j << 8) + 128, flags);
            // perspective-correct weights are proportional to E_k / w_k
            const float t0 = e.e0 * __int_as_float(pa.z), t1 = e.e1 * __int_as_float(pb.z), t2 = e.e2 * __int_as_float(pc.z);
            float3 n = f3(fmaf(t0, na.x, fmaf(t1, nb.x, t2 * nc.x)), fmaf(t0, na.y, fmaf(t1, nb.y, t2 * nc.y)),
                          fmaf(t0, na.z, fmaf(t1, nb.z, t2 * nc.z)));
            const float ninv = rsqrtf(dot3(n, n));
            n = f3(n.x * ninv, n.y * ninv, n.z * ninv);
            const float3 pp = f3(z * ((float)i + 0.5f - cx) * ifx, -z * ((float)j + 0.5f - cy) * ify, -z);
            const float pinv = rsqrtf(dot3(pp, pp));
            const float3 v = f3(-pp.x * pinv, -pp.y * pinv, -pp.z * pinv);
            const float rough = a.roughness[o], ks = a.specular[o];
            const float mexp = 2.0f / (rough * rough) - 2.0f;
            const float al0 = a.albedo[3 * o + 0], al1 = a.albedo[3 * o + 1], al2 = a.albedo[3 * o + 2];
            for (int l = 0; l < nl; ++l) {
                const float4 Lq = L.light[l];
                float3 ld;
                float A;
                if (L.light_type[l] == 0) {
                    const float3 d = f3(Lq.x - pp.x, Lq.y - pp.y, Lq.z - pp.z);
                    const float D = dot3(d, d);
                    const float dinv = rsqrtf(D);
                    ld = f3(d.x * dinv, d.y * dinv, d.z * dinv);
                    A = Lq.w / fmaxf(D, 1e-4f);
                } else {
                    ld = f3(Lq.x, Lq.y, Lq.z);
                    A = Lq.w;
                }
                const float ndl = dot3(n, ld);
                if (ndl <= 0.f) continue;
                float s = 0.f;
                const float3 hh = f3(ld.x + v.x, ld.y + v.y, ld.z + v.z);
                const float H2 = dot3(hh, hh);
                if (H2 >= 1e-12f) {
                    const float hinv = rsqrtf(H2);
                    const float3 dd = f3(n.x - hh.x * hinv, n.y - hh.y * hinv, n.z - hh.z * hinv);
                    // 1 - n.h evaluated as |n - h|^2 / 2: no cancellation near the highlight
                    const float u = 0.5f * dot3(dd, dd);
                    if (u < 1.0f) s = (mexp == 0.f) ? 1.0f : expf(mexp * log1pf(-u));
                }
                const float An = A * ndl;
                r0 = fmaf(An, fmaf(ks, s, al0), r0);
                r1 = fmaf(An, fmaf(ks, s, al1), r1);
                r2 = fmaf(An, fmaf(ks, s, al2), r2);
            }
            r0 *= expo;
            r1 *= expo;
            r2 *= expo;
            n0 = n.x;
            n1 = n.y;
            n2 = n.z;
            segv = a.seg[o];
            triv = tri;
        }
        if (a.out_rgb) {
            __builtin_nontemporal_store(r0, a.out_rgb + 3 * po + pix);
            __builtin_nontemporal_store(r1, a.out_rgb + 3 * po + HW + pix);
            __builtin_nontemporal_store(r2, a.out_rgb + 3 * po + 2 * HW + pix);
        }
        if (a.out_depth) __builtin_nontemporal_store(z, a.out_depth + po + pix);
        if (a.out_normal) {
            __builtin_nontemporal_store(n0, a.out_normal + 3 * po + pix);
            __builtin_nontemporal_store(n1, a.out_normal + 3 * po + HW + pix);
            __builtin_nontemporal_store(n2, a.out_normal + 3 * po + 2 * HW + pix);
        }
        if (a.out_seg) __builtin_nontemporal_store(segv, a.out_seg + po + pix);
        if (a.out_tri) a.out_tri[po + pix] = triv;
        if (a.out_vis) a.out_vis[po + pix] = key;
    }
}

// Work-item index of workgroup `bid` among `n`, grouping consecutive items on the same
// XCD (workgroups are dispatched to the 8 XCDs round-robin), so the tiles of one frame
// share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int q = n >> 3, r = n & 7, xcd = bid & 7, local = bid >> 3;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

__global__ __launch_bounds__(kBlock) void k_raster_shade(RenderArgs a) {
    extern __shared__ __align__(16) char smem[];
    Lds L;
    lds_layout(a.tile_w, a.tile_h, a.bin_cap, smem, &L);
    if (threadIdx.x == 0) L.misc[2] = 0;
    if (!a.persistent) {
        __syncthreads();
        raster_shade_tile(a, xcd_remap(blockIdx.x, gridDim.x), L);
        return;
    }
    int item = blockIdx.x;
    while (item < a.n_titems) {
        __syncthreads();
        raster_shade_tile(a, item, L);
        __syncthreads();
        if (threadIdx.x == 0) L.misc[1] = (int)gridDim.x + (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        item = L.misc[1];
    }
}

hipError_t launch_vertex(const RenderArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(k_vertex, dim3(a.n_vitems > 0 ? a.n_vitems : 1), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_raster(const RenderArgs &a, hipStream_t stream, int n_cu) {
    hipError_t e = hipSuccess;
    if (a.n_titems <= 0) return hipSuccess;
    const size_t lds = raster_lds_bytes(a.tile_w, a.tile_h, a.bin_cap);
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_raster_shade),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int grid = a.n_titems;
    if (a.persistent) {
        int per_cu = (int)((160 * 1024) / (lds + 1024));
        per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
        grid = n_cu * per_cu;
        if (grid > a.n_titems) grid = a.n_titems;
    }
    hipLaunchKernelGGL(k_raster_shade, dim3(grid), dim3(kBlock), lds, stream, a);
    return hipGetLastError();
}

}  // namespace orrb
