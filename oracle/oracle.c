/*
 * FP64 CPU oracle for the batched randomized renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  It shares no code, header, table or
 * helper with the HIP path, and the HIP path never calls it.
 *
 * What it computes: for every frame of a batch of scenes, the four channels ORRB
 * renders (Sec. 4.4: RGB, segmentation, depth, screen-space normal) of a scene whose
 * material, camera, light and exposure parameters were drawn by the randomizers of
 * Sec. 4.3.1.  The paper prints no projection, fill, depth, normal or shading rule;
 * the readings taken here (FP64 vertex stage with a fixed fma order, 8-bit sub-pixel
 * snapping, top-left fill rule, nearest-depth-then-lowest-triangle-ID visibility,
 * eye depth, view-space normal, Lambert plus Blinn-Phong with point and directional
 * lights, linear exposure) are the definitions this file writes out in the plainest
 * form: loop over frames, objects, triangles, then the pixel centres in each
 * triangle's bounding box, keep the two nearest fragments of every pixel, then shade
 * the nearest.  Everything is FP64 except the integer snapping.
 *
 * The shading adjoint (oracle_shade_grad) is the analytic derivative of the per-pixel
 * shading function over the fixed visibility, accumulated in FP64 in a fixed order.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC oracle.c -lm
 * (contraction must stay off so every rounding is the one written here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GUARD_SUBPX 16777216LL /* 2^24 sub-pixel units = 65536 px */
#define LIGHT_EPS 1e-4         /* clamp of the squared light distance, m^2 */
#define SHADOW_BIAS 0.02       /* spot-light shadow test: lit if (1 - bias) w <= map depth */
#define SHADOW_AMB_DEPTH 1e-4  /* relative band of a depth comparison reported as ambiguous */
#define SHADOW_AMB_TEXEL 1e-3  /* texels: band of a texel-boundary decision reported as ambiguous */
#define HALF_EPS 1e-12         /* |l+v|^2 below this: no specular term */

/* ------------------------------------------------------------------------------ */
/* inputs, bundled once so the per-frame routines stay readable                     */
/* ------------------------------------------------------------------------------ */
typedef struct {
    const int64_t *mesh_vbegin, *mesh_tbegin;
    const double *mesh_pos, *mesh_nrm;
    const int32_t *mesh_idx;
    const int32_t *scene_object_begin, *object_mesh, *object_seg;
    const double *object_pose;
    const uint8_t *object_visible;
    const double *albedo, *roughness, *specular;
    const int32_t *scene_light_begin, *light_type;
    const double *light_vec, *light_intensity;
    const int32_t *frame_scene, *width, *height;
    const double *view, *intr, *near_, *exposure;
    const int64_t *pixel_offset;
    /* spot lights (type 2): axis, cone, shadow camera and shadow map (may be NULL when
     * the batch has no spot light) */
    const double *light_dir, *light_cone, *shadow_view, *shadow_intr, *shadow_maps;
    const int32_t *shadow_slot;
    int32_t shadow_res;
    /* materials with pattern textures and emission (NULL when unused): per-vertex UVs
     * of the mesh pool, the textures (RGB texels, row-major, tex_info[3k] = first texel,
     * width, height), each object's texture (-1 none) and UV transform (su, sv, ou, ov),
     * and its emissive power */
    const double *mesh_uv, *tex_texels;
    const int64_t *tex_info;
    const int32_t *obj_tex;
    const double *obj_txf, *emission;
    /* normal (bump) textures: each object's normal texture (-1 none; NULL when the batch
     * has none), sampled at the same transformed UV as the pattern texture */
    const int32_t *obj_ntex;
} Inputs;

/* per-vertex results of the vertex stage for one (frame, object) */
typedef struct {
    int valid;       /* w >= near and inside the guard band */
    int64_t X, Y;    /* snapped position, 1/256 px */
    double w;        /* eye depth */
    double n[3];     /* unit view-space normal */
    double uv[2];    /* texture coordinates (0 without UVs) */
} Vert;

/* per-pixel visibility record */
typedef struct {
    double d1, d2; /* nearest and second-nearest fragment depth (d2 = +inf if none) */
    int32_t tri;   /* scene-local triangle ID of the nearest, -1 = none */
    int32_t obj;   /* object of the nearest */
    int32_t local; /* triangle index inside that object's mesh */
    int32_t count; /* number of covering fragments */
} Pix;

/* ------------------------------------------------------------------------------ */
/* vertex stage                                                                     */
/* ------------------------------------------------------------------------------ */

/* M = V o W for 3x4 affine matrices (rows), in the fixed fma order. */
static void compose(const double *V, const double *W, double *M) {
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) {
            double t = V[i * 4 + 2] * W[2 * 4 + j];
            t = fma(V[i * 4 + 1], W[1 * 4 + j], t);
            M[i * 4 + j] = fma(V[i * 4 + 0], W[0 * 4 + j], t);
        }
        M[i * 4 + 3] = fma(V[i * 4 + 0], W[0 * 4 + 3],
                           fma(V[i * 4 + 1], W[1 * 4 + 3], fma(V[i * 4 + 2], W[2 * 4 + 3], V[i * 4 + 3])));
    }
}

static void normalize3(double *v) {
    double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= l;
    v[1] /= l;
    v[2] /= l;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Transform, project and snap every vertex of one object for one frame. */
static void vertex_stage(const Inputs *in, int f, int o, Vert *out) {
    int m = in->object_mesh[o];
    double M[12];
    compose(in->view + 12 * (int64_t)f, in->object_pose + 12 * (int64_t)o, M);
    const double *K = in->intr + 4 * (int64_t)f;
    double fx = K[0], fy = K[1], cx = K[2], cy = K[3], nearp = in->near_[f];
    int64_t v0 = in->mesh_vbegin[m], nv = in->mesh_vbegin[m + 1] - v0;
    for (int64_t v = 0; v < nv; v++) {
        const double *p = in->mesh_pos + 3 * (v0 + v);
        const double *nn = in->mesh_nrm + 3 * (v0 + v);
        double e[3];
        for (int i = 0; i < 3; i++)
            e[i] = fma(M[i * 4 + 0], p[0], fma(M[i * 4 + 1], p[1], fma(M[i * 4 + 2], p[2], M[i * 4 + 3])));
        Vert *q = out + v;
        q->w = -e[2];
        q->valid = 0;
        q->X = q->Y = 0;
        if (q->w >= nearp) {
            double qx = e[0] / q->w, qy = e[1] / q->w;
            double sx = fma(fx, qx, cx), sy = fma(-fy, qy, cy);
            double Xd = rint(256.0 * sx), Yd = rint(256.0 * sy);
            if (fabs(Xd) <= (double)GUARD_SUBPX && fabs(Yd) <= (double)GUARD_SUBPX) {
                q->valid = 1;
                q->X = (int64_t)Xd;
                q->Y = (int64_t)Yd;
            }
        }
        for (int i = 0; i < 3; i++) q->n[i] = M[i * 4 + 0] * nn[0] + M[i * 4 + 1] * nn[1] + M[i * 4 + 2] * nn[2];
        normalize3(q->n);
        q->uv[0] = in->mesh_uv ? in->mesh_uv[2 * (v0 + v)] : 0.0;
        q->uv[1] = in->mesh_uv ? in->mesh_uv[2 * (v0 + v) + 1] : 0.0;
    }
}

/* ------------------------------------------------------------------------------ */
/* triangle set-up, fill rule, fragment depth                                       */
/* ------------------------------------------------------------------------------ */

static int64_t floor_div(int64_t a, int64_t b) { /* b > 0 */
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}

static int64_t edge_fn(int64_t Xa, int64_t Ya, int64_t Xb, int64_t Yb, int64_t PX, int64_t PY) {
    return (Xb - Xa) * (PY - Ya) - (Yb - Ya) * (PX - Xa);
}

static int top_left(int64_t Xa, int64_t Ya, int64_t Xb, int64_t Yb) {
    int64_t dX = Xb - Xa, dY = Yb - Ya;
    return dY < 0 || (dY == 0 && dX > 0);
}

static int covered(int64_t E, int tl) { return E > 0 || (E == 0 && tl); }

/* The three vertices of a front-facing triangle after the v1 <-> v2 swap that makes
 * its area positive; returns 0 if the triangle is culled (invalid vertex, back-facing
 * or degenerate). */
static int setup(const Vert *vt, const int32_t *idx, const Vert **a, const Vert **b, const Vert **c, int64_t *area) {
    const Vert *p0 = vt + idx[0], *p1 = vt + idx[1], *p2 = vt + idx[2];
    if (!p0->valid || !p1->valid || !p2->valid) return 0;
    int64_t A = (p1->X - p0->X) * (p2->Y - p0->Y) - (p1->Y - p0->Y) * (p2->X - p0->X);
    if (A >= 0) return 0;
    *a = p0;
    *b = p2;
    *c = p1;
    *area = -A;
    return 1;
}

/* ------------------------------------------------------------------------------ */
/* visibility of one frame                                                          */
/* ------------------------------------------------------------------------------ */

/* Rasterize every visible object of frame f into pix[W*H].  vt_of[o - ob] points at
 * that object's vertex-stage results. */
static void visibility(const Inputs *in, int f, Vert **vt_of, Pix *pix) {
    int s = in->frame_scene[f], W = in->width[f], H = in->height[f];
    int ob = in->scene_object_begin[s], oe = in->scene_object_begin[s + 1];
    for (int64_t p = 0; p < (int64_t)W * H; p++) {
        pix[p].d1 = pix[p].d2 = INFINITY;
        pix[p].tri = pix[p].obj = pix[p].local = -1;
        pix[p].count = 0;
    }
    int32_t tri_base = 0;
    for (int o = ob; o < oe; o++) {
        int m = in->object_mesh[o];
        int64_t t0 = in->mesh_tbegin[m], nt = in->mesh_tbegin[m + 1] - t0;
        if (in->object_visible[o]) {
            const Vert *vt = vt_of[o - ob];
            for (int64_t t = 0; t < nt; t++) {
                const Vert *a, *b, *c;
                int64_t A;
                if (!setup(vt, in->mesh_idx + 3 * (t0 + t), &a, &b, &c, &A)) continue;
                int64_t xmin = a->X < b->X ? a->X : b->X, xmax = a->X > b->X ? a->X : b->X;
                int64_t ymin = a->Y < b->Y ? a->Y : b->Y, ymax = a->Y > b->Y ? a->Y : b->Y;
                if (c->X < xmin) xmin = c->X;
                if (c->X > xmax) xmax = c->X;
                if (c->Y < ymin) ymin = c->Y;
                if (c->Y > ymax) ymax = c->Y;
                /* pixel centres 256 i + 128 inside [xmin, xmax] */
                int64_t i0 = -floor_div(-(xmin - 128), 256), i1 = floor_div(xmax - 128, 256);
                int64_t j0 = -floor_div(-(ymin - 128), 256), j1 = floor_div(ymax - 128, 256);
                if (i0 < 0) i0 = 0;
                if (j0 < 0) j0 = 0;
                if (i1 > W - 1) i1 = W - 1;
                if (j1 > H - 1) j1 = H - 1;
                int tl0 = top_left(b->X, b->Y, c->X, c->Y); /* edge opposite a */
                int tl1 = top_left(c->X, c->Y, a->X, a->Y); /* edge opposite b */
                int tl2 = top_left(a->X, a->Y, b->X, b->Y); /* edge opposite c */
                for (int64_t j = j0; j <= j1; j++) {
                    for (int64_t i = i0; i <= i1; i++) {
                        int64_t PX = 256 * i + 128, PY = 256 * j + 128;
                        int64_t E0 = edge_fn(b->X, b->Y, c->X, c->Y, PX, PY);
                        int64_t E1 = edge_fn(c->X, c->Y, a->X, a->Y, PX, PY);
                        int64_t E2 = edge_fn(a->X, a->Y, b->X, b->Y, PX, PY);
                        if (!(covered(E0, tl0) && covered(E1, tl1) && covered(E2, tl2))) continue;
                        double b0 = (double)E0 / (double)A, b1 = (double)E1 / (double)A, b2 = (double)E2 / (double)A;
                        double z = 1.0 / (b0 / a->w + b1 / b->w + b2 / c->w);
                        int32_t id = tri_base + (int32_t)t;
                        Pix *q = pix + j * W + i;
                        q->count++;
                        if (z < q->d1 || (z == q->d1 && id < q->tri)) {
                            q->d2 = q->d1;
                            q->d1 = z;
                            q->tri = id;
                            q->obj = o;
                            q->local = (int32_t)t;
                        } else if (z < q->d2) {
                            q->d2 = z;
                        }
                    }
                }
            }
        }
        tri_base += (int32_t)nt;
    }
}

/* ------------------------------------------------------------------------------ */
/* shading                                                                          */
/* ------------------------------------------------------------------------------ */

/* Everything the shading function and its adjoint need at one covered pixel. */
typedef struct {
    double z;       /* eye depth */
    double n[3];    /* unit view-space normal */
    double p[3];    /* view-space position */
    double v[3];    /* unit direction to the eye */
    double uv[2];   /* perspective-correct texture coordinates */
} Frag;

static void fragment(const Inputs *in, int f, Vert **vt_of, const Pix *q, int i, int j, Frag *fr) {
    int s = in->frame_scene[f];
    int ob = in->scene_object_begin[s];
    int m = in->object_mesh[q->obj];
    const Vert *vt = vt_of[q->obj - ob];
    const Vert *a, *b, *c;
    int64_t A;
    setup(vt, in->mesh_idx + 3 * (in->mesh_tbegin[m] + q->local), &a, &b, &c, &A);
    int64_t PX = 256 * (int64_t)i + 128, PY = 256 * (int64_t)j + 128;
    double b0 = (double)edge_fn(b->X, b->Y, c->X, c->Y, PX, PY) / (double)A;
    double b1 = (double)edge_fn(c->X, c->Y, a->X, a->Y, PX, PY) / (double)A;
    double b2 = (double)edge_fn(a->X, a->Y, b->X, b->Y, PX, PY) / (double)A;
    double z = 1.0 / (b0 / a->w + b1 / b->w + b2 / c->w);
    double be0 = z * b0 / a->w, be1 = z * b1 / b->w, be2 = z * b2 / c->w;
    for (int k = 0; k < 3; k++) fr->n[k] = be0 * a->n[k] + be1 * b->n[k] + be2 * c->n[k];
    normalize3(fr->n);
    for (int k = 0; k < 2; k++) fr->uv[k] = be0 * a->uv[k] + be1 * b->uv[k] + be2 * c->uv[k];
    const double *K = in->intr + 4 * (int64_t)f;
    fr->z = z;
    fr->p[0] = z * ((i + 0.5 - K[2]) / K[0]);
    fr->p[1] = z * (-(j + 0.5 - K[3]) / K[1]);
    fr->p[2] = -z;
    double pl = sqrt(dot3(fr->p, fr->p));
    for (int k = 0; k < 3; k++) fr->v[k] = -fr->p[k] / pl;
}

/* Bilinear sample of texture t at (u, v) with repeat addressing: texel (i, j) is
 * centred at ((i + 1/2) / W, (j + 1/2) / H), row j = 0 first. */
static void tex_sample(const Inputs *in, int t, double u, double v, double *rgb) {
    int64_t off = in->tex_info[3 * (int64_t)t], W = in->tex_info[3 * (int64_t)t + 1], H = in->tex_info[3 * (int64_t)t + 2];
    double x = u * (double)W - 0.5, y = v * (double)H - 0.5;
    double fx = floor(x), fy = floor(y), ax = x - fx, ay = y - fy;
    int64_t i0 = (int64_t)fmod(fx, (double)W), j0 = (int64_t)fmod(fy, (double)H);
    if (i0 < 0) i0 += W;
    if (j0 < 0) j0 += H;
    int64_t i1 = (i0 + 1) % W, j1 = (j0 + 1) % H;
    const double *T = in->tex_texels + 3 * off;
    for (int c = 0; c < 3; c++)
        rgb[c] = (1 - ay) * ((1 - ax) * T[3 * (j0 * W + i0) + c] + ax * T[3 * (j0 * W + i1) + c]) +
                 ay * ((1 - ax) * T[3 * (j1 * W + i0) + c] + ax * T[3 * (j1 * W + i1) + c]);
}

/* Object o's textures are sampled at the transformed UV (u su + ou, v sv + ov). */
static void object_uv(const Inputs *in, int o, const Frag *fr, double *uv) {
    const double *x = in->obj_txf + 4 * (int64_t)o;
    uv[0] = fr->uv[0] * x[0] + x[2];
    uv[1] = fr->uv[1] * x[1] + x[3];
}

/* The albedo at a fragment of object o: the tint times its pattern texture, if it has
 * one. */
static void fragment_albedo(const Inputs *in, int o, const Frag *fr, double *alb) {
    for (int c = 0; c < 3; c++) alb[c] = in->albedo[3 * (int64_t)o + c];
    int t = in->obj_tex ? in->obj_tex[o] : -1;
    if (t < 0) return;
    double uv[2], rgb[3];
    object_uv(in, o, fr, uv);
    tex_sample(in, t, uv[0], uv[1], rgb);
    for (int c = 0; c < 3; c++) alb[c] *= rgb[c];
}

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* The shading normal at a fragment of object o (frame f, mesh triangle `local`): the
 * interpolated normal n, perturbed by the object's normal texture if it has one.  The
 * texture sampled (bilinear, repeat) at the pattern texture's transformed UV encodes a
 * tangent-space direction t = 2 rgb - 1 (normalized).  The tangent frame is the
 * triangle's: T and B solve e1 = du1 T + dv1 B, e2 = du2 T + dv2 B for the object-space
 * edges e_k = p_k - p_0 and UV differences (du_k, dv_k), taken to view space by the
 * composed matrix; T is made orthogonal to n (Gram-Schmidt), B' = h n x T' with h the
 * sign of (n x T') . B (the UV mapping's handedness), and the shading normal is
 * normalize(t_x T' + t_y B' + t_z n).  A triangle whose UVs are degenerate (zero UV
 * area), a tangent parallel to n or t = 0 leaves n unchanged. */
static void shading_normal(const Inputs *in, int f, int o, int local, const Frag *fr, double *ns) {
    for (int k = 0; k < 3; k++) ns[k] = fr->n[k];
    int t = in->obj_ntex ? in->obj_ntex[o] : -1;
    if (t < 0) return;
    double uv[2], rgb[3];
    object_uv(in, o, fr, uv);
    tex_sample(in, t, uv[0], uv[1], rgb);
    double tn[3] = {2 * rgb[0] - 1, 2 * rgb[1] - 1, 2 * rgb[2] - 1};
    double tl = sqrt(dot3(tn, tn));
    if (tl == 0) return;
    for (int k = 0; k < 3; k++) tn[k] /= tl;
    int m = in->object_mesh[o];
    const int32_t *tri = in->mesh_idx + 3 * (in->mesh_tbegin[m] + local);
    int64_t v0 = in->mesh_vbegin[m];
    const double *p0 = in->mesh_pos + 3 * (v0 + tri[0]), *p1 = in->mesh_pos + 3 * (v0 + tri[1]),
                 *p2 = in->mesh_pos + 3 * (v0 + tri[2]);
    const double *u0 = in->mesh_uv + 2 * (v0 + tri[0]), *u1 = in->mesh_uv + 2 * (v0 + tri[1]),
                 *u2 = in->mesh_uv + 2 * (v0 + tri[2]);
    double du1 = u1[0] - u0[0], dv1 = u1[1] - u0[1], du2 = u2[0] - u0[0], dv2 = u2[1] - u0[1];
    double det = du1 * dv2 - du2 * dv1;
    if (det == 0) return;
    double To[3], Bo[3];
    for (int k = 0; k < 3; k++) {
        double e1 = p1[k] - p0[k], e2 = p2[k] - p0[k];
        To[k] = (e1 * dv2 - e2 * dv1) / det;
        Bo[k] = (e2 * du1 - e1 * du2) / det;
    }
    double M[12], T[3], B[3];
    compose(in->view + 12 * (int64_t)f, in->object_pose + 12 * (int64_t)o, M);
    for (int r = 0; r < 3; r++) {
        T[r] = M[r * 4 + 0] * To[0] + M[r * 4 + 1] * To[1] + M[r * 4 + 2] * To[2];
        B[r] = M[r * 4 + 0] * Bo[0] + M[r * 4 + 1] * Bo[1] + M[r * 4 + 2] * Bo[2];
    }
    const double *n = fr->n;
    double nt = dot3(n, T);
    double Tp[3] = {T[0] - nt * n[0], T[1] - nt * n[1], T[2] - nt * n[2]};
    double tpl = sqrt(dot3(Tp, Tp));
    if (tpl == 0) return;
    for (int k = 0; k < 3; k++) Tp[k] /= tpl;
    double Bp[3];
    cross3(n, Tp, Bp);
    if (dot3(Bp, B) < 0)
        for (int k = 0; k < 3; k++) Bp[k] = -Bp[k];
    for (int k = 0; k < 3; k++) ns[k] = tn[0] * Tp[k] + tn[1] * Bp[k] + tn[2] * n[k];
    normalize3(ns);
}

/* A light expressed in the frame's view space. */
typedef struct {
    int type;      /* 0 point, 1 directional, 2 spot (with a shadow map) */
    double q[3];   /* point, spot: view-space position; directional: unit direction to the light */
    double qn;     /* directional: |R_V u| before normalization (1 for point lights) */
    double I;
    /* spot: unit view-space axis, cosines of the inner and outer half-angles, the map
     * (N x N depths) and T = shadow view o V^-1 (view space -> shadow camera space) */
    double axis[3], cos_in, cos_out;
    const double *map;
    double T[12], sK[4];
} VLight;

static void view_lights(const Inputs *in, int f, VLight *L, int *nL) {
    int s = in->frame_scene[f];
    const double *V = in->view + 12 * (int64_t)f;
    int lb = in->scene_light_begin[s], le = in->scene_light_begin[s + 1];
    *nL = le - lb;
    for (int l = lb; l < le; l++) {
        VLight *x = L + (l - lb);
        const double *u = in->light_vec + 3 * (int64_t)l;
        x->type = in->light_type[l];
        x->I = in->light_intensity[l];
        x->qn = 1.0;
        if (x->type == 0 || x->type == 2) {
            for (int r = 0; r < 3; r++) x->q[r] = V[r * 4 + 0] * u[0] + V[r * 4 + 1] * u[1] + V[r * 4 + 2] * u[2] + V[r * 4 + 3];
        }
        if (x->type == 2) {
            const double *d = in->light_dir + 3 * (int64_t)l;
            for (int r = 0; r < 3; r++) x->axis[r] = V[r * 4 + 0] * d[0] + V[r * 4 + 1] * d[1] + V[r * 4 + 2] * d[2];
            normalize3(x->axis);
            x->cos_in = in->light_cone[2 * (int64_t)l];
            x->cos_out = in->light_cone[2 * (int64_t)l + 1];
            int slot = in->shadow_slot[l];
            int64_t N = in->shadow_res;
            x->map = in->shadow_maps + (int64_t)slot * N * N;
            /* V^-1 of the rigid view [R | t] is [R^T | -R^T t]; T = S o V^-1 */
            const double *Sv = in->shadow_view + 12 * (int64_t)l;
            double Vi[12];
            for (int r = 0; r < 3; r++) {
                for (int c = 0; c < 3; c++) Vi[r * 4 + c] = V[c * 4 + r];
                Vi[r * 4 + 3] = -(V[0 * 4 + r] * V[3] + V[1 * 4 + r] * V[7] + V[2 * 4 + r] * V[11]);
            }
            for (int r = 0; r < 3; r++) {
                for (int c = 0; c < 4; c++)
                    x->T[r * 4 + c] = Sv[r * 4 + 0] * Vi[0 * 4 + c] + Sv[r * 4 + 1] * Vi[1 * 4 + c] + Sv[r * 4 + 2] * Vi[2 * 4 + c];
                x->T[r * 4 + 3] += Sv[r * 4 + 3];
            }
            for (int k = 0; k < 4; k++) x->sK[k] = in->shadow_intr[4 * (int64_t)l + k];
        } else if (x->type == 1) {
            for (int r = 0; r < 3; r++) x->q[r] = -(V[r * 4 + 0] * u[0] + V[r * 4 + 1] * u[1] + V[r * 4 + 2] * u[2]);
            x->qn = sqrt(dot3(x->q, x->q));
            normalize3(x->q);
        }
    }
}

/* Per-light terms of the shading function at one fragment. */
typedef struct {
    double l[3], dist, D, A, ndl, h[3], hl, ndh, s;
    int has_h;     /* |l+v|^2 >= HALF_EPS */
    double cone;   /* spot: smoothstep cone factor (1 otherwise) */
    double vis;    /* spot: fraction of the 3 x 3 shadow-map texels that see the point (1 otherwise) */
    int amb;       /* spot: a texel choice or depth comparison lies within the reporting band */
} LTerm;

/* Spot-light shadow visibility by 3 x 3 percentage-closer filtering: the point p (view
 * space) goes to the shadow camera (T), projects to continuous map coordinates (u, v)
 * (pixel units, origin top-left, y down); the 3 x 3 texels around the texel holding
 * (u, v) each count as lit when (1 - bias) w <= their depth (an empty texel, depth 0,
 * and a texel outside the map count as lit).  A point not in front of the shadow
 * camera is lit.  *amb reports decisions within the bands. */
static double shadow_visibility(const VLight *L, int64_t N, const double *p, int *amb) {
    double q[3];
    for (int r = 0; r < 3; r++) q[r] = L->T[r * 4 + 0] * p[0] + L->T[r * 4 + 1] * p[1] + L->T[r * 4 + 2] * p[2] + L->T[r * 4 + 3];
    double w = -q[2];
    *amb = 0;
    if (w <= 0) return 1.0;
    double u = L->sK[0] * (q[0] / w) + L->sK[2], v = -L->sK[1] * (q[1] / w) + L->sK[3];
    double fu = floor(u), fv = floor(v);
    if (u - fu < SHADOW_AMB_TEXEL || fu + 1 - u < SHADOW_AMB_TEXEL || v - fv < SHADOW_AMB_TEXEL ||
        fv + 1 - v < SHADOW_AMB_TEXEL)
        *amb = 1;
    double wb = (1.0 - SHADOW_BIAS) * w;
    int lit = 0;
    for (int dj = -1; dj <= 1; dj++) {
        for (int di = -1; di <= 1; di++) {
            double ti = fu + di, tj = fv + dj;
            if (ti < 0 || tj < 0 || ti >= (double)N || tj >= (double)N) {
                lit++;
                continue;
            }
            double z = L->map[(int64_t)tj * N + (int64_t)ti];
            if (z == 0 || wb <= z) lit++;
            if (z != 0 && fabs(wb - z) < SHADOW_AMB_DEPTH * w) *amb = 1;
        }
    }
    return lit / 9.0;
}

/* Spot cone: smoothstep of cos(angle to the axis) from the outer to the inner cosine. */
static double spot_cone(const VLight *L, const double *l) {
    double c = -dot3(l, L->axis);
    double t = (c - L->cos_out) / (L->cos_in - L->cos_out);
    t = t < 0 ? 0 : (t > 1 ? 1 : t);
    return t * t * (3 - 2 * t);
}

static void light_term(const VLight *L, const Frag *fr, double m, LTerm *t, int64_t shadow_res) {
    t->cone = t->vis = 1.0;
    t->amb = 0;
    if (L->type == 0 || L->type == 2) {
        double d[3] = {L->q[0] - fr->p[0], L->q[1] - fr->p[1], L->q[2] - fr->p[2]};
        t->D = dot3(d, d);
        t->dist = sqrt(t->D);
        for (int k = 0; k < 3; k++) t->l[k] = d[k] / t->dist;
        t->A = L->I / (t->D > LIGHT_EPS ? t->D : LIGHT_EPS);
        if (L->type == 2) {
            t->cone = spot_cone(L, t->l);
            t->vis = shadow_visibility(L, shadow_res, fr->p, &t->amb);
            t->A *= t->cone * t->vis;
        }
    } else {
        for (int k = 0; k < 3; k++) t->l[k] = L->q[k];
        t->D = t->dist = 1.0;
        t->A = L->I;
    }
    double c = dot3(fr->n, t->l);
    t->ndl = c > 0 ? c : 0;
    double hh[3] = {t->l[0] + fr->v[0], t->l[1] + fr->v[1], t->l[2] + fr->v[2]};
    double H2 = dot3(hh, hh);
    t->has_h = H2 >= HALF_EPS;
    t->s = 0;
    t->ndh = 0;
    t->hl = 0;
    if (t->has_h) {
        t->hl = sqrt(H2);
        for (int k = 0; k < 3; k++) t->h[k] = hh[k] / t->hl;
        double e = dot3(fr->n, t->h);
        t->ndh = e > 0 ? e : 0;
        t->s = t->ndh > 0 ? pow(t->ndh, m) : 0;
    }
}

/* ------------------------------------------------------------------------------ */
/* per-frame driver shared by render and gradient                                   */
/* ------------------------------------------------------------------------------ */

typedef struct {
    Vert **vt_of;
    Vert *vbuf;
    Pix *pix;
} FrameWork;

static int frame_begin(const Inputs *in, int f, FrameWork *fw) {
    int s = in->frame_scene[f];
    int ob = in->scene_object_begin[s], oe = in->scene_object_begin[s + 1];
    int64_t nv = 0;
    for (int o = ob; o < oe; o++) {
        int m = in->object_mesh[o];
        nv += in->mesh_vbegin[m + 1] - in->mesh_vbegin[m];
    }
    fw->vt_of = (Vert **)malloc(sizeof(Vert *) * (size_t)(oe - ob + 1));
    fw->vbuf = (Vert *)malloc(sizeof(Vert) * (size_t)(nv + 1));
    fw->pix = (Pix *)malloc(sizeof(Pix) * (size_t)((int64_t)in->width[f] * in->height[f] + 1));
    if (!fw->vt_of || !fw->vbuf || !fw->pix) return -1;
    int64_t off = 0;
    for (int o = ob; o < oe; o++) {
        int m = in->object_mesh[o];
        fw->vt_of[o - ob] = fw->vbuf + off;
        vertex_stage(in, f, o, fw->vbuf + off);
        off += in->mesh_vbegin[m + 1] - in->mesh_vbegin[m];
    }
    visibility(in, f, fw->vt_of, fw->pix);
    return 0;
}

static void frame_end(FrameWork *fw) {
    free(fw->vt_of);
    free(fw->vbuf);
    free(fw->pix);
}

static void render_frame(const Inputs *in, int f, double *rgb, double *depth, double *normal, int32_t *seg,
                         int32_t *tri_id, double *depth2, int32_t *frag_count, int32_t *obj_id, uint8_t *shadow_amb,
                         int *err) {
    FrameWork fw;
    if (frame_begin(in, f, &fw)) {
        *err = 1;
        frame_end(&fw);
        return;
    }
    int W = in->width[f], H = in->height[f];
    int64_t HW = (int64_t)W * H, po = in->pixel_offset[f];
    VLight L[64];
    int nL;
    view_lights(in, f, L, &nL);
    for (int j = 0; j < H; j++) {
        for (int i = 0; i < W; i++) {
            int64_t p = (int64_t)j * W + i;
            const Pix *q = fw.pix + p;
            if (depth2) depth2[po + p] = q->tri >= 0 ? q->d2 : INFINITY;
            if (frag_count) frag_count[po + p] = q->count;
            if (obj_id) obj_id[po + p] = q->tri >= 0 ? q->obj : -1;
            if (shadow_amb) shadow_amb[po + p] = 0;
            if (q->tri < 0) {
                for (int c = 0; c < 3; c++) {
                    rgb[3 * po + c * HW + p] = 0;
                    normal[3 * po + c * HW + p] = 0;
                }
                depth[po + p] = 0;
                seg[po + p] = -1;
                if (tri_id) tri_id[po + p] = -1;
                continue;
            }
            Frag fr;
            fragment(in, f, fw.vt_of, q, i, j, &fr);
            int o = q->obj;
            double r = in->roughness[o], ks = in->specular[o], mexp = 2.0 / (r * r) - 2.0;
            double alb[3];
            fragment_albedo(in, o, &fr, alb);
            Frag fs = fr;  /* lights see the normal-mapped normal; the normal channel keeps n */
            shading_normal(in, f, o, q->local, &fr, fs.n);
            double E = in->emission ? in->emission[o] : 0.0;
            double U[3] = {E * alb[0], E * alb[1], E * alb[2]};
            for (int l = 0; l < nL; l++) {
                LTerm t;
                light_term(L + l, &fs, mexp, &t, in->shadow_res);
                for (int c = 0; c < 3; c++) U[c] += t.A * t.ndl * (alb[c] + ks * t.s);
                if (shadow_amb && t.amb && t.ndl > 0 && t.cone > 0) shadow_amb[po + p] = 1;
            }
            double e = in->exposure[f];
            for (int c = 0; c < 3; c++) {
                rgb[3 * po + c * HW + p] = e * U[c];
                normal[3 * po + c * HW + p] = fr.n[c];
            }
            depth[po + p] = q->d1;
            seg[po + p] = in->object_seg[o];
            if (tri_id) tri_id[po + p] = q->tri;
        }
    }
    frame_end(&fw);
}

/* ------------------------------------------------------------------------------ */
/* exported entry points                                                            */
/* ------------------------------------------------------------------------------ */

#define INPUT_ARGS                                                                                            \
    const int64_t *mesh_vbegin, const int64_t *mesh_tbegin, const double *mesh_pos, const double *mesh_nrm,   \
        const int32_t *mesh_idx, const int32_t *scene_object_begin, const int32_t *object_mesh,               \
        const double *object_pose, const int32_t *object_seg, const uint8_t *object_visible,                  \
        const double *albedo, const double *roughness, const double *specular,                                \
        const int32_t *scene_light_begin, const int32_t *light_type, const double *light_vec,                 \
        const double *light_intensity, int32_t n_frames, const int32_t *frame_scene, const double *view,      \
        const double *intr, const double *near_, const double *exposure, const int32_t *width,                \
        const int32_t *height, const int64_t *pixel_offset, const double *light_dir, const double *light_cone,      \
        const double *shadow_view, const double *shadow_intr, const double *shadow_maps,                        \
        const int32_t *shadow_slot, int32_t shadow_res, const double *mesh_uv, const double *tex_texels,        \
        const int64_t *tex_info, const int32_t *obj_tex, const double *obj_txf, const double *emission,         \
        const int32_t *obj_ntex

#define FILL_INPUTS(in)                                                                                         \
    Inputs in = {mesh_vbegin, mesh_tbegin, mesh_pos, mesh_nrm, mesh_idx, scene_object_begin, object_mesh,      \
                 object_seg, object_pose, object_visible, albedo, roughness, specular, scene_light_begin,      \
                 light_type, light_vec, light_intensity, frame_scene, width, height, view, intr, near_,        \
                 exposure, pixel_offset, light_dir, light_cone, shadow_view, shadow_intr, shadow_maps,         \
                 shadow_slot, shadow_res, mesh_uv, tex_texels, tex_info, obj_tex, obj_txf, emission, obj_ntex}

static void set_threads(int n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
}

/* Render all frames.  Outputs use the planar layout: rgb and normal planes of frame f
 * at 3*pixel_offset[f] + c*H*W, depth/seg/tri_id/depth2/frag_count at
 * pixel_offset[f].  obj_id receives the (global) object index of each pixel's nearest
 * fragment, -1 for background.  tri_id, depth2, frag_count and obj_id may be NULL.
 * Returns 0 on success. */
int oracle_render(INPUT_ARGS, double *rgb, double *depth, double *normal, int32_t *seg, int32_t *tri_id,
                  double *depth2, int32_t *frag_count, int32_t *obj_id, uint8_t *shadow_amb, int32_t n_threads) {
    FILL_INPUTS(in);
    int err = 0;
    set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int f = 0; f < n_frames; f++) {
        int e = 0;
        render_frame(&in, f, rgb, depth, normal, seg, tri_id, depth2, frag_count, obj_id, shadow_amb, &e);
        err |= e;
    }
    return err;
}

/* Loss L = sum over frames, pixels and channels of w_px (rgb - target)^2, and its
 * analytic gradient over the fixed visibility with respect to per-object albedo (3),
 * roughness and specular, per-light vector (world, 3: the position of a point light,
 * the direction of a directional light) and intensity, and per-frame exposure.  w_px is pixel_weight[px] (0/1, NULL = all 1).  Gradients are overwritten.
 * When dl_drgb is not NULL the loss is linear instead, L = sum w_px dl_drgb . rgb
 * (planar like rgb, target ignored): the adjoint is then that of a fixed upstream
 * gradient, which is what a backward pass receives from the layers above it.
 * Scenes are processed in parallel; within a scene, frames and pixels are summed in
 * order, so the result is deterministic. */
int oracle_shade_grad(INPUT_ARGS, int32_t n_scenes, const double *target, const uint8_t *pixel_weight,
                      const double *dl_drgb, double *loss_out, double *g_albedo, double *g_rough, double *g_spec, double *g_lightvec,
                      double *g_intensity, double *g_exposure, int32_t n_threads) {
    FILL_INPUTS(in);
    for (int64_t l = 0; l < scene_light_begin[n_scenes]; l++)
        if (light_type[l] == 2) return 2; /* spot lights: no adjoint (shadow visibility is not differentiated) */
    if (obj_tex || emission || obj_ntex) return 2;   /* textured or emissive materials: no adjoint */
    int err = 0;
    double *scene_loss = (double *)calloc((size_t)n_scenes + 1, sizeof(double));
    if (!scene_loss) return 1;
    int64_t n_obj = scene_object_begin[n_scenes], n_light = scene_light_begin[n_scenes];
    memset(g_albedo, 0, sizeof(double) * 3 * (size_t)n_obj);
    memset(g_rough, 0, sizeof(double) * (size_t)n_obj);
    memset(g_spec, 0, sizeof(double) * (size_t)n_obj);
    memset(g_lightvec, 0, sizeof(double) * 3 * (size_t)n_light);
    memset(g_intensity, 0, sizeof(double) * (size_t)n_light);
    memset(g_exposure, 0, sizeof(double) * (size_t)n_frames);
    set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int s = 0; s < n_scenes; s++) {
        int lb = scene_light_begin[s];
        for (int f = 0; f < n_frames; f++) {
            if (frame_scene[f] != s) continue;
            FrameWork fw;
            if (frame_begin(&in, f, &fw)) {
                err |= 1;
                frame_end(&fw);
                continue;
            }
            int W = width[f], H = height[f];
            int64_t HW = (int64_t)W * H, po = pixel_offset[f];
            VLight L[64];
            int nL;
            view_lights(&in, f, L, &nL);
            const double *V = view + 12 * (int64_t)f;
            double e = exposure[f];
            for (int j = 0; j < H; j++) {
                for (int i = 0; i < W; i++) {
                    int64_t p = (int64_t)j * W + i;
                    const Pix *q = fw.pix + p;
                    if (pixel_weight && !pixel_weight[po + p]) continue;
                    if (q->tri < 0) { /* background renders 0: constant loss, no gradient */
                        if (!dl_drgb)
                            for (int c = 0; c < 3; c++) scene_loss[s] += target[3 * po + c * HW + p] * target[3 * po + c * HW + p];
                        continue;
                    }
                    Frag fr;
                    fragment(&in, f, fw.vt_of, q, i, j, &fr);
                    int o = q->obj;
                    double r = roughness[o], ks = specular[o], mexp = 2.0 / (r * r) - 2.0;
                    const double *alb = albedo + 3 * (int64_t)o;
                    LTerm t[64];
                    double U[3] = {0, 0, 0};
                    for (int l = 0; l < nL; l++) {
                        light_term(L + l, &fr, mexp, t + l, in.shadow_res);
                        for (int c = 0; c < 3; c++) U[c] += t[l].A * t[l].ndl * (alb[c] + ks * t[l].s);
                    }
                    double g[3], G = 0;
                    for (int c = 0; c < 3; c++) {
                        double rgbc = e * U[c];
                        if (dl_drgb) {
                            g[c] = dl_drgb[3 * po + c * HW + p];
                            scene_loss[s] += g[c] * rgbc;
                        } else {
                            double d = rgbc - target[3 * po + c * HW + p];
                            scene_loss[s] += d * d;
                            g[c] = 2.0 * d;
                        }
                        G += g[c];
                    }
                    /* exposure */
                    g_exposure[f] += g[0] * U[0] + g[1] * U[1] + g[2] * U[2];
                    double sum_And = 0, sum_Ands = 0, sum_Ands_ln = 0;
                    for (int l = 0; l < nL; l++) {
                        const LTerm *x = t + l;
                        sum_And += x->A * x->ndl;
                        sum_Ands += x->A * x->ndl * x->s;
                        if (x->ndh > 0) sum_Ands_ln += x->A * x->ndl * x->s * log(x->ndh);
                        /* intensity: A = I / max(D, eps) (point) or I (directional) */
                        double Gh = 0;
                        for (int c = 0; c < 3; c++) Gh += g[c] * (alb[c] + ks * x->s);
                        double dA_dI = L[l].type == 0 ? 1.0 / (x->D > LIGHT_EPS ? x->D : LIGHT_EPS) : 1.0;
                        g_intensity[lb + l] += e * Gh * x->ndl * dA_dI;
                        if (L[l].type != 0) {
                            /* directional light: l = a / |a| with a = -R_V u.  The shade
                             * depends on l through n.l and through h = (l + v) / |l + v|:
                             * dL/dl = e [Gh A n + G A ndl k_s m ndh^(m-1) (n - ndh h) / |l+v|],
                             * then dL/da = (I - l l^T) dL/dl / |a| and dL/du = -R_V^T dL/da */
                            if (x->ndl <= 0) continue;
                            double gl[3];
                            for (int c = 0; c < 3; c++) gl[c] = e * Gh * x->A * fr.n[c];
                            if (x->has_h && x->ndh > 0 && mexp != 0) {
                                double coef = e * G * x->A * x->ndl * ks * mexp * pow(x->ndh, mexp - 1.0) / x->hl;
                                for (int c = 0; c < 3; c++) gl[c] += coef * (fr.n[c] - x->ndh * x->h[c]);
                            }
                            double lg = dot3(x->l, gl), ga[3];
                            for (int c = 0; c < 3; c++) ga[c] = (gl[c] - lg * x->l[c]) / L[l].qn;
                            for (int c = 0; c < 3; c++)
                                g_lightvec[3 * (int64_t)(lb + l) + c] -= V[0 * 4 + c] * ga[0] + V[1 * 4 + c] * ga[1] + V[2 * 4 + c] * ga[2];
                            continue;
                        }
                        /* point-light position, view space, then rotated to world */
                        double gq[3] = {0, 0, 0};
                        if (x->D > LIGHT_EPS) {
                            double k = -2.0 * L[l].I / (x->D * x->D);
                            double d[3] = {x->l[0] * x->dist, x->l[1] * x->dist, x->l[2] * x->dist};
                            for (int c = 0; c < 3; c++) gq[c] += e * Gh * x->ndl * k * d[c];
                        }
                        if (x->ndl > 0) {
                            for (int c = 0; c < 3; c++) gq[c] += e * Gh * x->A * (fr.n[c] - x->ndl * x->l[c]) / x->dist;
                            if (x->has_h && x->ndh > 0 && mexp != 0) {
                                /* d(n.h)/dd = (I - l l^T)(n - (n.h) h) / (|l+v| |d|) */
                                double w[3], lw;
                                for (int c = 0; c < 3; c++) w[c] = fr.n[c] - x->ndh * x->h[c];
                                lw = dot3(x->l, w);
                                double coef = e * G * x->A * x->ndl * ks * mexp * pow(x->ndh, mexp - 1.0) / (x->hl * x->dist);
                                for (int c = 0; c < 3; c++) gq[c] += coef * (w[c] - lw * x->l[c]);
                            }
                        }
                        for (int c = 0; c < 3; c++)
                            g_lightvec[3 * (int64_t)(lb + l) + c] += V[0 * 4 + c] * gq[0] + V[1 * 4 + c] * gq[1] + V[2 * 4 + c] * gq[2];
                    }
                    for (int c = 0; c < 3; c++) g_albedo[3 * (int64_t)o + c] += e * g[c] * sum_And;
                    g_spec[o] += e * G * sum_Ands;
                    g_rough[o] += e * G * ks * sum_Ands_ln * (-4.0 / (r * r * r));
                }
            }
            frame_end(&fw);
        }
    }
    double loss = 0;
    for (int s = 0; s < n_scenes; s++) loss += scene_loss[s];
    *loss_out = loss;
    free(scene_loss);
    return err;
}
