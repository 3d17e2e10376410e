"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of oracle.c (a dropped term, a wrong
sign, index or constant, a transposed rotation), compiles it, swaps it in for the
real oracle and runs the pins that should notice: at least one of them must fail.
The real oracle is restored afterwards; nothing here touches the GPU path.  A case
whose planted text no longer appears exactly once in oracle.c fails too, so the list
follows the source.
"""
from __future__ import annotations

import functools
import subprocess

import pytest

import oracle
from tests import test_oracle_edge_cases as E
from tests import test_oracle_geometry as G
from tests import test_oracle_grad as D
from tests import test_oracle_materials as MA
from tests import test_oracle_normal_maps as NM
from tests import test_oracle_shading as SH
from tests import test_oracle_shadows as SD


def pin(fn, *args):
    p = functools.partial(fn, *args)
    p.__name__ = fn.__name__ + (str(args) if args else "")
    return p


GUARD_PINS = [pin(E.test_guard_band_discards_triangles_beyond_65536_px, *c) for c in E.GUARD_CASES]
TIE_PINS = [pin(E.test_second_nearest_depth_and_near_ties, o, g) for o in ((1, 2, 0), (1, 0, 2)) for g in (3e-6, 3e-5)]
FD_PINS = [pin(D.test_adjoint_matches_central_differences)]

# (name, text in oracle.c, replacement, pins expected to notice)
MUTANTS = [
    ("near_cull_at_zero", "if (q->w >= nearp) {", "if (q->w > 0) {", [pin(G.test_near_plane_cull)]),
    ("no_guard_band", "if (fabs(Xd) <= (double)GUARD_SUBPX && fabs(Yd) <= (double)GUARD_SUBPX) {", "if (1) {", GUARD_PINS),
    ("guard_strict", "if (fabs(Xd) <= (double)GUARD_SUBPX && fabs(Yd) <= (double)GUARD_SUBPX) {",
     "if (fabs(Xd) < (double)GUARD_SUBPX && fabs(Yd) < (double)GUARD_SUBPX) {", GUARD_PINS),
    ("guard_one_sided", "if (fabs(Xd) <= (double)GUARD_SUBPX && fabs(Yd) <= (double)GUARD_SUBPX) {",
     "if (Xd <= (double)GUARD_SUBPX && Yd <= (double)GUARD_SUBPX) {", GUARD_PINS),
    ("guard_x_only", "if (fabs(Xd) <= (double)GUARD_SUBPX && fabs(Yd) <= (double)GUARD_SUBPX) {",
     "if (fabs(Xd) <= (double)GUARD_SUBPX) {", GUARD_PINS),
    ("guard_in_pixels", "#define GUARD_SUBPX 16777216LL", "#define GUARD_SUBPX 65536LL", GUARD_PINS),
    ("snap_half_up", "double Xd = rint(256.0 * sx), Yd = rint(256.0 * sy);",
     "double Xd = floor(256.0 * sx + 0.5), Yd = floor(256.0 * sy + 0.5);",
     [pin(G.test_snap_round_half_even, 0.5, True), pin(G.test_snap_round_half_even, 1.5, False)]),
    ("fill_rule_bottom_right", "return dY < 0 || (dY == 0 && dX > 0);", "return dY > 0 || (dY == 0 && dX < 0);",
     [pin(G.test_top_left_fill_rule_on_exact_edges)]),
    ("fill_rule_inclusive", "static int covered(int64_t E, int tl) { return E > 0 || (E == 0 && tl); }",
     "static int covered(int64_t E, int tl) { return E >= 0; }",
     [pin(G.test_top_left_fill_rule_on_exact_edges), pin(G.test_watertight_plane_each_pixel_covered_once, False)]),
    ("cull_front_faces", "if (A >= 0) return 0;", "if (A <= 0) return 0;", [pin(G.test_back_faces_culled)]),
    ("depth_not_perspective", "double z = 1.0 / (b0 / a->w + b1 / b->w + b2 / c->w);\n                        int32_t id",
     "double z = b0 * a->w + b1 * b->w + b2 * c->w;\n                        int32_t id",
     [pin(G.test_tilted_plane_depth_closed_form)]),
    ("tie_to_higher_id", "(z == q->d1 && id < q->tri)", "(z == q->d1 && id > q->tri)",
     [pin(G.test_exact_depth_tie_goes_to_lower_triangle_id)]),
    ("d2_keeps_old_second", "q->d2 = q->d1;\n", "", TIE_PINS),
    ("d2_overwritten_by_farther", "} else if (z < q->d2) {", "} else {", TIE_PINS),
    ("normal_affine_weights", "double be0 = z * b0 / a->w, be1 = z * b1 / b->w, be2 = z * b2 / c->w;",
     "double be0 = b0, be1 = b1, be2 = b2;", [pin(G.test_normals_match_brute_force_interpolation)]),
    ("normal_transposed_rotation",
     "q->n[i] = M[i * 4 + 0] * nn[0] + M[i * 4 + 1] * nn[1] + M[i * 4 + 2] * nn[2];",
     "q->n[i] = M[0 * 4 + i] * nn[0] + M[1 * 4 + i] * nn[1] + M[2 * 4 + i] * nn[2];",
     [pin(G.test_rotated_cube_normals_are_rotated_axes)]),
    ("position_y_up", "fr->p[1] = z * (-(j + 0.5 - K[3]) / K[1]);", "fr->p[1] = z * ((j + 0.5 - K[3]) / K[1]);",
     [pin(SH.test_lambert_plane_point_light_closed_form)]),
    ("point_light_transposed_view",
     "x->q[r] = V[r * 4 + 0] * u[0] + V[r * 4 + 1] * u[1] + V[r * 4 + 2] * u[2] + V[r * 4 + 3];",
     "x->q[r] = V[0 * 4 + r] * u[0] + V[1 * 4 + r] * u[1] + V[2 * 4 + r] * u[2] + V[r * 4 + 3];",
     [pin(SH.test_lambert_plane_point_light_closed_form)]),
    ("directional_transposed_view",
     "x->q[r] = -(V[r * 4 + 0] * u[0] + V[r * 4 + 1] * u[1] + V[r * 4 + 2] * u[2]);",
     "x->q[r] = -(V[0 * 4 + r] * u[0] + V[1 * 4 + r] * u[1] + V[2 * 4 + r] * u[2]);",
     [pin(E.test_directional_light_rotated_camera_lambert)]),
    ("directional_sign",
     "x->q[r] = -(V[r * 4 + 0] * u[0] + V[r * 4 + 1] * u[1] + V[r * 4 + 2] * u[2]);",
     "x->q[r] = (V[r * 4 + 0] * u[0] + V[r * 4 + 1] * u[1] + V[r * 4 + 2] * u[2]);",
     [pin(SH.test_lambert_plane_directional_light_is_constant), pin(E.test_directional_light_rotated_camera_lambert)]),
    ("no_distance_clamp", "t->A = L->I / (t->D > LIGHT_EPS ? t->D : LIGHT_EPS);", "t->A = L->I / t->D;",
     [pin(E.test_point_light_distance_clamp_closed_form)]),
    ("clamp_epsilon", "#define LIGHT_EPS 1e-4 ", "#define LIGHT_EPS 1e-5 ", [pin(E.test_point_light_distance_clamp_closed_form)]),
    ("phong_exponent", "double r = in->roughness[o], ks = in->specular[o], mexp = 2.0 / (r * r) - 2.0;\n            double alb[3];",
     "double r = in->roughness[o], ks = in->specular[o], mexp = 2.0 / r - 2.0;\n            double alb[3];",
     [pin(SH.test_off_mirror_highlight_half_angle, 0.5, 0.4)]),
    ("half_vector_difference", "double hh[3] = {t->l[0] + fr->v[0], t->l[1] + fr->v[1], t->l[2] + fr->v[2]};",
     "double hh[3] = {t->l[0] - fr->v[0], t->l[1] - fr->v[1], t->l[2] - fr->v[2]};",
     [pin(SH.test_mirror_highlight_independent_of_roughness), pin(E.test_directional_light_rotated_camera_specular)]),
    ("no_ndl_clamp", "t->ndl = c > 0 ? c : 0;", "t->ndl = c;", [pin(SH.test_light_behind_surface_gives_black)]),
    ("no_exposure", "rgb[3 * po + c * HW + p] = e * U[c];", "rgb[3 * po + c * HW + p] = U[c];",
     [pin(SH.test_linearity_in_exposure_intensity_albedo), pin(SH.test_lambert_plane_directional_light_is_constant)]),
    ("adjoint_roughness_factor", "(-4.0 / (r * r * r))", "(-2.0 / (r * r * r))", FD_PINS),
    ("adjoint_clamp_dA_dd", "if (x->D > LIGHT_EPS) {\n                            double k", "if (1) {\n                            double k",
     [pin(E.test_point_light_clamp_gradient_matches_differences, 0.0)]),
    ("adjoint_clamp_dA_dI", "double dA_dI = L[l].type == 0 ? 1.0 / (x->D > LIGHT_EPS ? x->D : LIGHT_EPS) : 1.0;",
     "double dA_dI = L[l].type == 0 ? 1.0 / x->D : 1.0;", [pin(E.test_point_light_clamp_gradient_matches_differences, 0.0)]),
    ("adjoint_point_rotation",
     "g_lightvec[3 * (int64_t)(lb + l) + c] += V[0 * 4 + c] * gq[0] + V[1 * 4 + c] * gq[1] + V[2 * 4 + c] * gq[2];",
     "g_lightvec[3 * (int64_t)(lb + l) + c] += V[c * 4 + 0] * gq[0] + V[c * 4 + 1] * gq[1] + V[c * 4 + 2] * gq[2];",
     FD_PINS),
    ("adjoint_ndh_projection", "for (int c = 0; c < 3; c++) w[c] = fr.n[c] - x->ndh * x->h[c];",
     "for (int c = 0; c < 3; c++) w[c] = fr.n[c];", FD_PINS),
    ("adjoint_directional_no_projection", "ga[c] = (gl[c] - lg * x->l[c]) / L[l].qn;", "ga[c] = gl[c] / L[l].qn;",
     [pin(E.test_directional_and_point_gradients_rotated_camera)]),
    ("adjoint_directional_no_norm", "ga[c] = (gl[c] - lg * x->l[c]) / L[l].qn;", "ga[c] = (gl[c] - lg * x->l[c]);",
     [pin(E.test_directional_and_point_gradients_rotated_camera)]),
    ("adjoint_directional_sign",
     "g_lightvec[3 * (int64_t)(lb + l) + c] -= V[0 * 4 + c] * ga[0]",
     "g_lightvec[3 * (int64_t)(lb + l) + c] += V[0 * 4 + c] * ga[0]",
     [pin(E.test_directional_and_point_gradients_rotated_camera)]),
    ("adjoint_exposure_term", "g_exposure[f] += g[0] * U[0] + g[1] * U[1] + g[2] * U[2];",
     "g_exposure[f] += g[0] * U[0] + g[1] * U[1] + g[1] * U[2];", FD_PINS),
    # spot lights and shadow maps
    ("shadow_bias_sign", "double wb = (1.0 - SHADOW_BIAS) * w;", "double wb = (1.0 + SHADOW_BIAS) * w;",
     [pin(SD.test_occluder_shadow_is_its_central_projection)]),
    ("shadow_v_flip", "double u = L->sK[0] * (q[0] / w) + L->sK[2], v = -L->sK[1] * (q[1] / w) + L->sK[3];",
     "double u = L->sK[0] * (q[0] / w) + L->sK[2], v = L->sK[1] * (q[1] / w) + L->sK[3];",
     [pin(SD.test_light_behind_a_ground_point_and_ambiguity_report)]),
    ("shadow_empty_texel_dark", "if (z == 0 || wb <= z) lit++;", "if (wb <= z) lit++;",
     [pin(SD.test_lone_plane_is_fully_lit_and_cone_is_smoothstep)]),
    ("spot_cone_no_smoothstep", "return t * t * (3 - 2 * t);", "return t;",
     [pin(SD.test_lone_plane_is_fully_lit_and_cone_is_smoothstep)]),
    ("shadow_pcf_one_texel", "for (int dj = -1; dj <= 1; dj++) {", "for (int dj = 0; dj <= 0; dj++) {",
     [pin(SD.test_lone_plane_is_fully_lit_and_cone_is_smoothstep)]),
    # pattern textures and emission
    ("tex_bilinear_weights_swapped", "rgb[c] = (1 - ay) * ((1 - ax) * T[3 * (j0 * W + i0) + c] + ax * T[3 * (j0 * W + i1) + c]) +",
     "rgb[c] = (1 - ay) * (ax * T[3 * (j0 * W + i0) + c] + (1 - ax) * T[3 * (j0 * W + i1) + c]) +",
     [pin(MA.test_bilinear_weights_quarter_texel)]),
    ("tex_no_half_texel", "double x = u * (double)W - 0.5, y = v * (double)H - 0.5;", "double x = u * (double)W, y = v * (double)H;",
     [pin(MA.test_pixel_centres_on_texel_centres_show_the_texels)]),
    ("tex_offset_tiling_order", "uv[0] = fr->uv[0] * x[0] + x[2];", "uv[0] = (fr->uv[0] + x[2]) * x[0];",
     [pin(MA.test_tiling_and_offset_are_periodic_shifts)]),
    ("uv_wrong_weight", "for (int k = 0; k < 2; k++) fr->uv[k] = be0 * a->uv[k] + be1 * b->uv[k] + be2 * c->uv[k];",
     "for (int k = 0; k < 2; k++) fr->uv[k] = be0 * a->uv[k] + be2 * b->uv[k] + be1 * c->uv[k];",
     [pin(MA.test_pixel_centres_on_texel_centres_show_the_texels)]),
    ("emission_dropped", "double U[3] = {E * alb[0], E * alb[1], E * alb[2]};", "double U[3] = {0, 0, 0};",
     [pin(MA.test_emission_adds_power_times_albedo)]),
    # normal textures
    ("normal_map_no_handedness", "if (dot3(Bp, B) < 0)", "if (0)",
     [pin(NM.test_tilt_along_v_follows_the_bitangent_and_mirrored_uvs_flip_it)]),
    ("normal_map_tangent_bitangent_swapped", "for (int k = 0; k < 3; k++) ns[k] = tn[0] * Tp[k] + tn[1] * Bp[k] + tn[2] * n[k];",
     "for (int k = 0; k < 3; k++) ns[k] = tn[1] * Tp[k] + tn[0] * Bp[k] + tn[2] * n[k];",
     [pin(NM.test_tilt_along_u_follows_the_tangent)]),
    ("normal_map_not_decoded", "double tn[3] = {2 * rgb[0] - 1, 2 * rgb[1] - 1, 2 * rgb[2] - 1};",
     "double tn[3] = {rgb[0], rgb[1], rgb[2]};", [pin(NM.test_flat_map_changes_nothing)]),
    ("normal_map_tangent_sign", "To[k] = (e1 * dv2 - e2 * dv1) / det;", "To[k] = (e2 * dv1 - e1 * dv2) / det;",
     [pin(NM.test_tilt_along_u_follows_the_tangent)]),
    ("normal_map_tangent_object_space", "T[r] = M[r * 4 + 0] * To[0] + M[r * 4 + 1] * To[1] + M[r * 4 + 2] * To[2];",
     "T[r] = To[r];", [pin(NM.test_tangent_turns_with_the_pose)]),
    ("normal_map_ignored_by_lights", "light_term(L + l, &fs, mexp, &t, in->shadow_res);",
     "light_term(L + l, &fr, mexp, &t, in->shadow_res);", [pin(NM.test_bump_texture_pixel_by_pixel)]),
]


def _compile(src: str, tmp_path) -> str:
    c = tmp_path / "mutant.c"
    c.write_text(src)
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-o", str(so),
                    str(c), "-lm"], check=True)
    return str(so)


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(name, old, new, pins, tmp_path):
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"{name}: the planted text must appear exactly once in oracle.c"
    lib = oracle.open_library(_compile(src.replace(old, new), tmp_path))
    real = oracle._load()
    caught = []
    oracle._lib = lib
    try:
        for p in pins:
            try:
                p()
            except AssertionError:
                caught.append(p.__name__)
                break
    finally:
        oracle._lib = real
    assert caught, f"mutant {name}: every pin passed ({[p.__name__ for p in pins]})"


def test_real_oracle_passes_the_same_pins():
    """The pins the mutants are run against pass on the real oracle (so a mutant's
    failure is the planted mistake's doing)."""
    seen = set()
    for _, _, _, pins in MUTANTS:
        for p in pins:
            if p.__name__ not in seen:
                seen.add(p.__name__)
                p()
