"""Mutation check of the oracle's pins: each plausible mistake below (a flipped sign, a wrong
index, a dropped term, a transposed operand, the Mesh-Splatting min-opacity rule instead of
the paper's mean) is compiled into a copy of the oracle, and the pin suite must reject every
copy.  A mutation that survives means the pins have a blind spot."""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O
from tests import test_oracle_face_sigma as FSIG
from tests import test_oracle_fd as FD
from tests import test_oracle_pins as PINS
from tests import test_oracle_perspective as PERSP
from tests import test_oracle_tight_bins as TIGHT

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "tsr_oracle.c")

MUTATIONS = {
    "window_sign": ("double rho = -L[ks] / f->r;", "double rho = L[ks] / f->r;"),
    "barycentric_index": ("lam[0] = -L[1] * f->len[1] / f->area2;", "lam[0] = -L[2] * f->len[1] / f->area2;"),
    "transmittance_assign": ("T *= 1.0 - h[j].alpha;", "T = 1.0 - h[j].alpha;"),
    "min_opacity_rule": (": (s->opa[f->v[0]] + s->opa[f->v[1]] + s->opa[f->v[2]]) / 3.0;",
                         ": fmin(s->opa[f->v[0]], fmin(s->opa[f->v[1]], s->opa[f->v[2]]));"),
    "depth_order_reversed": ("if (x->zkey < y->zkey) return -1;\n    if (x->zkey > y->zkey) return 1;",
                             "if (x->zkey < y->zkey) return 1;\n    if (x->zkey > y->zkey) return -1;"),
    "fx_fy_transposed": ("c->fx * f->vc[k][0] / f->vc[k][2] + c->cx", "c->fy * f->vc[k][0] / f->vc[k][2] + c->cx"),
    "pose_theta_sign": ("pg[3] += vc[1] * gc[2] - vc[2] * gc[1];", "pg[3] += vc[2] * gc[1] - vc[1] * gc[2];"),
    "rotation_not_transposed": ("R[0][a] * gc[0] + R[1][a] * gc[1] + R[2][a] * gc[2]",
                                "R[a][0] * gc[0] + R[a][1] * gc[1] + R[a][2] * gc[2]"),
    "behind_colour_no_decay": ("B[ch] = e->c[ch] * e->alpha + (1.0 - e->alpha) * B[ch];",
                               "B[ch] = e->c[ch] * e->alpha + B[ch];"),
    "dropped_depth_term": ("+ gd * (e->zf - BD)", "+ gd * e->zf"),
    "dual_division_sign": ("(a.d[i] * b.v - a.v * b.d[i])", "(a.d[i] * b.v + a.v * b.d[i])"),
    "wrong_depth_key": ("f->zkey = (float)f->zf;", "f->zkey = (float)f->vc[0][2];"),
    "binning_off_by_one": ("double lo_u = ceil(fmax(f->umin, -1.0))", "double lo_u = 1.0 + ceil(fmax(f->umin, -1.0))"),
    "transmittance_grad_sign": ("- gt * (1.0 - BA)", "- gt * (1.0 + BA)"),
    "inradius_from_area": ("f->r = f->area2 / f->perim;", "f->r = 0.5 * f->area2 / f->perim;"),
    "normal_ignores_winding": ("f->n[k][0] = so * ey / f->len[k];\n        f->n[k][1] = -so * ex / f->len[k];",
                               "f->n[k][0] = ey / f->len[k];\n        f->n[k][1] = -ex / f->len[k];"),
    "dual_barycentric_index": ("lam[1] = dn_scale(dn_div(dn_mul(L[2], len[2]), area), -1.0);",
                               "lam[1] = dn_scale(dn_div(dn_mul(L[0], len[2]), area), -1.0);"),
    "dual_depth_weight": ("*zf_out = dn_scale(zf, 1.0 / 3.0);", "*zf_out = dn_scale(zf, 1.0 / 2.0);"),
    "face_sigma_ignored": ("f->sig = s->face_sigma ? s->face_sigma[m] : p->sigma;", "f->sig = p->sigma;"),
    "sigma_grad_log2": ("double gs = galpha * f->of * e->I * log(e->rho);",
                        "double gs = galpha * f->of * e->I * log2(e->rho);"),
    "sigma_grad_no_opacity": ("double gs = galpha * f->of * e->I * log(e->rho);",
                              "double gs = galpha * e->I * log(e->rho);"),
    "tight_tiles_far_corner": ("double u = f->n[k][0] > 0 ? ulo : uhi, v = f->n[k][1] > 0 ? vlo : vhi;",
                               "double u = f->n[k][0] > 0 ? uhi : ulo, v = f->n[k][1] > 0 ? vhi : vlo;"),
    "persp_weight_times_depth": ("for (int i = 0; i < 3; i++) { w[i] = lam[i] / f->vc[i][2]; W += w[i]; }",
                                 "for (int i = 0; i < 3; i++) { w[i] = lam[i] * f->vc[i][2]; W += w[i]; }"),
    "persp_depth_not_inverted": ("e->zf = 1.0 / W;", "e->zf = W;"),
    "persp_dual_depth_constant": ("w[i] = dn_div(lam[i], dn_var(f->vc[i][2], 3 * i + 2));",
                                  "w[i] = dn_div(lam[i], dn_const(f->vc[i][2]));"),
    "tight_tiles_box_unclipped": ("double ulo = fmax(16.0 * x, r[0]), uhi = fmin(16.0 * x + 15.0, r[1]);",
                                  "double ulo = 16.0 * x, uhi = 16.0 * x + 15.0;"),
}


def _pin_checks():
    """The pin suite as plain callables (parametrised tests expanded)."""
    out = []
    for s in (0.5, 1.0, 2.0):
        out.append(lambda s=s: PINS.test_window_closed_forms_right_triangle(s))
        out.append(lambda s=s: PINS.test_window_invariances(s))
    out += [PINS.test_window_incentre_and_inradius_equilateral, PINS.test_barycentric_partition_and_linear_precision,
            PINS.test_partition_of_unity_and_constant_depth, PINS.test_two_faces_closed_form_and_order,
            PINS.test_empty_scene, PINS.test_full_occlusion, PINS.test_single_frontal_opaque_face,
            PINS.test_face_order_in_arrays_is_irrelevant, PINS.test_projection_pinhole,
            PINS.test_near_plane_and_degenerate_cull, PINS.test_binner_against_brute_force,
            PINS.test_binner_multi_view_numbering, PINS.test_l1_seeds_by_finite_differences,
            PINS.test_depth_order_uses_the_centroid_depth, PINS.test_three_layer_compositing,
            lambda: FD.test_gradients_with_deep_overlap(1.0),
            lambda: FD.test_pose_gradient_identities(7), FD.test_opacity_mean_rule]
    for sigma, seed in [(1.0, 1), (0.5, 2), (2.0, 3)]:
        out.append(lambda sigma=sigma, seed=seed: FD.test_gradients_match_finite_differences(sigma, seed))
    out += [lambda: FSIG.test_golden_right_triangle_with_its_own_exponent(0.7),
            FSIG.test_two_faces_use_their_own_exponents,
            lambda: FSIG.test_gradients_under_face_sigma_match_finite_differences(41),
            TIGHT.test_right_triangle_closed_form, TIGHT.test_box_is_clipped_to_the_pixel_rectangle, lambda: TIGHT.test_between_exact_and_bounding_box(1),
            TIGHT.test_thin_slanted_faces_drop_pairs,
            PERSP.test_ray_meets_the_face_plane, lambda: PERSP.test_gradients_match_finite_differences(11)]
    return out


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory() as d:
        yield d


def test_unmutated_oracle_passes_every_pin():
    for chk in _pin_checks():
        chk()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutation(name, workdir):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    c_path = os.path.join(workdir, f"{name}.c")
    so_path = os.path.join(workdir, f"lib{name}.so")
    with open(c_path, "w") as f:
        f.write(mutated)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11", c_path, "-o",
                    so_path, "-lm"], check=True)
    caught = None
    with O.use_library(so_path):
        for chk in _pin_checks():
            try:
                chk()
            except Exception as e:          # AssertionError or a failed call: the pin fired
                caught = type(e).__name__
                break
    assert caught is not None, f"mutation {name} survived every pin"
