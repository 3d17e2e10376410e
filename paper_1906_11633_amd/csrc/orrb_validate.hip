// Checks of the per-call state that the render kernels take as preconditions without
// testing them (testing them on the host would need a device-to-host copy of the
// state).  One thread per object, light and frame index counts the elements that
// break a precondition into the call's stats buffer; nothing is rendered and nothing is
// changed.  The conventions checked are those of the library (the paper prints none):
// poses and views are rotations times a positive uniform scale (views unscaled),
// materials and lights are finite with non-negative colours and intensities and
// positive roughness, cameras have positive focal lengths and near planes.
#include "orrb_primitives.h"

namespace orrb {

namespace {

constexpr int kValidateBlock = 256;
constexpr double kSimilarityTol = 1e-3;  // relative, for fp32 matrices

ORRB_INLINE bool finite(float x) { return __builtin_isfinite(x); }

ORRB_INLINE bool all_finite(const float *p, int n) {
    bool ok = true;
    for (int k = 0; k < n; ++k) ok = ok && finite(p[k]);
    return ok;
}

// The 3 x 3 part M of a row-major 3 x 4 matrix is a rotation times a uniform scale
// s > 0 (s = 1 when unit): M^T M = s^2 I and det M > 0, within kSimilarityTol.
ORRB_INLINE bool similarity(const float *P, bool unit) {
    if (!all_finite(P, 12)) return false;
    double g[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += (double)P[4 * r + i] * (double)P[4 * r + j];
            g[i][j] = s;
        }
    const double s2 = (g[0][0] + g[1][1] + g[2][2]) / 3.0;
    if (!(s2 > 0.0)) return false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (fabs(g[i][j] - (i == j ? s2 : 0.0)) > kSimilarityTol * s2) return false;
    if (unit && fabs(s2 - 1.0) > kSimilarityTol) return false;
    const double det = (double)P[0] * ((double)P[5] * P[10] - (double)P[6] * P[9]) -
                       (double)P[1] * ((double)P[4] * P[10] - (double)P[6] * P[8]) +
                       (double)P[2] * ((double)P[4] * P[9] - (double)P[5] * P[8]);
    return det > 0.0;
}

struct ValidateArgs {
    RenderArgs a;
    const float *post;
    int32_t n_obj, n_lights, n_frames;
    uint32_t *stats;
};

__global__ __launch_bounds__(kValidateBlock) void k_validate(ValidateArgs v) {
    const RenderArgs &a = v.a;
    const int i = (int)(blockIdx.x * kValidateBlock + threadIdx.x);
    unsigned bad = 0;
    if (i < v.n_obj) {  // object i
        bool ok = similarity(a.pose + 12 * (int64_t)i, false);
        const float *al = a.albedo + 3 * (int64_t)i;
        ok = ok && all_finite(al, 3) && al[0] >= 0.f && al[1] >= 0.f && al[2] >= 0.f;
        ok = ok && finite(a.roughness[i]) && a.roughness[i] > 0.f;
        ok = ok && finite(a.specular[i]) && a.specular[i] >= 0.f;
        if (a.emission) ok = ok && finite(a.emission[i]) && a.emission[i] >= 0.f;
        const bool textured = (a.obj_tex && a.obj_tex[i] >= 0) || (a.obj_ntex && a.obj_ntex[i] >= 0);
        if (textured && a.tex_xform) ok = ok && all_finite(a.tex_xform + 4 * (int64_t)i, 4);
        bad += !ok;
    }
    if (i < v.n_lights) {  // light i
        const int t = a.light_type[i];
        const float *u = a.light_vec + 3 * (int64_t)i;
        bool ok = all_finite(u, 3) && finite(a.light_intensity[i]) && a.light_intensity[i] >= 0.f;
        if (t == 1) ok = ok && (u[0] != 0.f || u[1] != 0.f || u[2] != 0.f);
        if (t == 2) {
            const float *d = a.light_dir + 3 * (int64_t)i, *c = a.light_cone + 2 * (int64_t)i;
            const float *K = a.shadow_intr + 4 * (int64_t)i;
            ok = ok && all_finite(d, 3) && (d[0] != 0.f || d[1] != 0.f || d[2] != 0.f);
            ok = ok && all_finite(c, 2) && c[0] > c[1] && c[0] <= 1.f && c[1] >= -1.f;
            ok = ok && similarity(a.shadow_view + 12 * (int64_t)i, true);
            ok = ok && all_finite(K, 4) && K[0] > 0.f && K[1] > 0.f;
        }
        bad += !ok;
    }
    if (i < v.n_frames) {  // frame i
        const float *K = a.intr + 4 * (int64_t)i;
        bool ok = similarity(a.view + 12 * (int64_t)i, true);
        ok = ok && all_finite(K, 4) && K[0] > 0.f && K[1] > 0.f;
        ok = ok && finite(a.near_plane[i]) && a.near_plane[i] > 0.f;
        ok = ok && finite(a.exposure[i]) && a.exposure[i] >= 0.f;
        if (v.post) ok = ok && all_finite(v.post + (int64_t)ORRB_POST_WORDS * i, ORRB_POST_WORDS);
        bad += !ok;
    }
    if (bad) atomicAdd(v.stats + ORRB_STAT_INVALID_STATE, bad);
}

}  // namespace

hipError_t launch_validate(const RenderArgs &a, const float *post, int n_obj, int n_lights, int n_frames,
                           uint32_t *stats, hipStream_t stream) {
    const int n = max(n_obj, max(n_lights, n_frames));
    if (n <= 0) return hipSuccess;
    ValidateArgs v;
    v.a = a;
    v.post = post;
    v.n_obj = n_obj;
    v.n_lights = n_lights;
    v.n_frames = n_frames;
    v.stats = stats;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((n + kValidateBlock - 1) / kValidateBlock)), dim3(kValidateBlock), 0,
                       stream, v);
    return hipGetLastError();
}

}  // namespace orrb
