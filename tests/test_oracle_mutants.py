"""The pins are strong enough: each plausible mistake planted in a copy of
the oracle's source (a dropped term, a wrong sign or index, a transposed
operand, a wrong exponent or normalisation) makes at least one pin fail.

Every mutant is compiled with gcc into a temporary library and the pin
functions of the other oracle test modules are run against it through
`oracle.use_library`; the planted mistakes never touch the real oracle."""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O

import test_oracle_bin as TB
import test_oracle_composite as TC
import test_oracle_grad as TG
import test_oracle_prune as TP
import test_oracle_sh as TS
import test_oracle_window as TW
import test_oracle_window_variants as TV

SRC = os.path.join(os.path.dirname(O.__file__), "ts_oracle.c")

# cheap pins first: the run stops at the first one that fails
PINS = [
    ("window worked example", TW.test_worked_example_window),
    ("render worked example", TW.test_worked_example_render_3d),
    ("setup worked example", TW.test_worked_example_setup_and_tight_box),
    ("two triangles", TC.test_two_triangle_worked_example),
    ("projection", TW.test_projection_pinhole),
    ("culls", TC.test_culls),
    ("background", TC.test_background_term),
    ("depth tie", TC.test_depth_tie_lower_index_first),
    ("termination", TC.test_early_termination_rule),
    ("sh scipy", TS.test_matches_scipy_complex_harmonics),
    ("sh quadrature", TS.test_orthonormal_by_quadrature),
    ("sh gradient", TS.test_gradient_on_sphere),
    ("colour dir", TC.test_view_dependent_colour_direction),
    ("colour posed", TC.test_colour_direction_from_posed_camera),
    ("closed form", lambda: TC.test_single_triangle_closed_form(0.97, 1.7)),
    ("closed form clamp", lambda: TC.test_single_triangle_closed_form(1.0, 0.05)),
    ("window props", lambda: TW.test_window_properties(0)),
    ("barycentric", lambda: TW.test_sdf_equals_barycentric_form(3)),
    ("binning", TB.test_binning_matches_brute_force),
    ("partition", lambda: TC.test_partition_of_unity(1)),
    ("fd v", lambda: TG.test_fd_state_stable_pixels("v", (1.0, 1.5))),
    ("fd o", lambda: TG.test_fd_state_stable_pixels("o", (1.0, 1.5))),
    ("fd sigma", lambda: TG.test_fd_state_stable_pixels("sigma", (1.0, 1.5))),
    ("fd sh", lambda: TG.test_fd_state_stable_pixels("sh", (1.0, 1.5))),
    ("fd posed", TG.test_fd_posed_camera_and_clamped_colour),
    ("fd clamp", TG.test_fd_clamped_and_terminated),
    ("homogeneity", TG.test_opacity_gradient_homogeneity),
    ("tight box", lambda: TW.test_tight_box_brute_force(0)),
    ("over", lambda: TC.test_textbook_over_operator(3)),
    ("prune single", TP.test_single_triangle),
    ("prune stack", TP.test_stack_with_termination),
    ("prune order", TP.test_front_back_order_and_sample),
    ("sigmoid points", TV.test_sigmoid_at_incentre_boundary_and_outside),
    ("lse small", TV.test_lse_small_triangle_has_no_inside),
    ("lse points", TV.test_lse_pointwise_and_bounds),
    ("sigmoid box", lambda: TV.test_variant_tight_box_brute_force(1, 0)),
    ("lse box", lambda: TV.test_variant_tight_box_brute_force(2, 0)),
    ("sigmoid render", lambda: TV.test_variant_single_triangle_closed_form(1)),
    ("lse render", lambda: TV.test_variant_single_triangle_closed_form(2)),
    ("sigmoid fd v", lambda: TV.test_variant_fd_gradients(1, "v")),
    ("sigmoid fd sigma", lambda: TV.test_variant_fd_gradients(1, "sigma")),
    ("lse fd v", lambda: TV.test_variant_fd_gradients(2, "v")),
    ("lse fd sigma", lambda: TV.test_variant_fd_gradients(2, "sigma")),
]

# (label, exact source text, replacement)
MUTANTS = [
    ("normal sign", "T->n[k][0] = T->sgn * T->e[k][1] / T->len[k];",
     "T->n[k][0] = -T->sgn * T->e[k][1] / T->len[k];"),
    ("incentre weights", "T->s[0] = (T->len[1] * T->q[0][0] + T->len[2] * T->q[1][0]",
     "T->s[0] = (T->len[0] * T->q[0][0] + T->len[2] * T->q[1][0]"),
    ("no perspective divide", "T->q[i][0] = cam->fx * T->xc[i][0] / T->xc[i][2] + cam->cx;",
     "T->q[i][0] = cam->fx * T->xc[i][0] + cam->cx;"),
    ("transposed R", "T->xc[i][a] = cam->R[3 * a + 0] * v[3 * i + 0] + cam->R[3 * a + 1] * v[3 * i + 1]\n"
     "                        + cam->R[3 * a + 2] * v[3 * i + 2] + cam->t[a];",
     "T->xc[i][a] = cam->R[a + 0] * v[3 * i + 0] + cam->R[a + 3] * v[3 * i + 1]\n"
     "                        + cam->R[a + 6] * v[3 * i + 2] + cam->t[a];"),
    ("weight without T", "double w = a * T;\n        for (int c = 0; c < 3; ++c) C[c] += w * tr->rgb[c];",
     "double w = a;\n        for (int c = 0; c < 3; ++c) C[c] += w * tr->rgb[c];"),
    ("background dropped", "out->C[c] = C[c] + cfg->bg[c] * T;", "out->C[c] = C[c];"),
    ("termination test on old T", "int stop = Tn < cfg->T_min;", "int stop = T < cfg->T_min;"),
    ("no cut-off skip", "int skip = a < cfg->alpha_min;", "int skip = a <= 0.0;"),
    ("no clamp", "if (a > cfg->alpha_max) { a = cfg->alpha_max; clamped = 1; }",
     "if (a > cfg->alpha_max) { clamped = 1; }"),
    ("sh normalisation", "sqrt((2.0 * l + 1.0) / (4.0 * M_PI)", "sqrt((2.0 * l + 1.0) / (2.0 * M_PI)"),
    ("sh sin/cos swap", "Y[k] = a * re * Pm;", "Y[k] = a * im * Pm;"),
    ("colour offset dropped", "T->rgb_raw[c] = acc + 0.5;", "T->rgb_raw[c] = acc;"),
    ("view direction reversed", "double dv[3] = {cen[0] - cc[0], cen[1] - cc[1], cen[2] - cc[2]};",
     "double dv[3] = {cc[0] - cen[0], cc[1] - cen[1], cc[2] - cen[2]};"),
    ("camera centre R not transposed",
     "cc[a] = -(cam->R[0 + a] * cam->t[0] + cam->R[3 + a] * cam->t[1] + cam->R[6 + a] * cam->t[2]);",
     "cc[a] = -(cam->R[3 * a + 0] * cam->t[0] + cam->R[3 * a + 1] * cam->t[1] + cam->R[3 * a + 2] * cam->t[2]);"),
    ("tight box exponent", "dist = -T->phis * pow(cfg->alpha_min / o, 1.0 / sigma);",
     "dist = -T->phis * pow(cfg->alpha_min / o, sigma);"),
    ("rect rounding", "double fx0 = ceil(xmin - 0.5), fx1 = floor(xmax - 0.5);",
     "double fx0 = floor(xmin - 0.5), fx1 = floor(xmax - 0.5);"),
    ("back-to-front order", "if (ki < kj) return -1;\n    if (ki > kj) return 1;",
     "if (ki < kj) return 1;\n    if (ki > kj) return -1;"),
    ("tie order reversed", "return (i > j) - (i < j);", "return (i < j) - (i > j);"),
    ("window exponent", "I = pow(u, tr->sigma);", "I = pow(u, 1.0 / tr->sigma);"),
    ("near plane one vertex", "if (!(T->xc[i][2] > cfg->z_near)) T->visible = 0;",
     "if (i == 0 && !(T->xc[i][2] > cfg->z_near)) T->visible = 0;"),
    ("depth weight", "D += w * tr->zc;\n        T = Tn;", "D += a * tr->zc;\n        T = Tn;"),
    ("grad: later-sum term dropped", "ga += gC[c] * (tr->rgb[c] * Ti - SC[c] / om);",
     "ga += gC[c] * (tr->rgb[c] * Ti);"),
    ("grad: inradius sign", "double du = (gL[i][c] + F->u * gr[i][c]) / phis;",
     "double du = (gL[i][c] - F->u * gr[i][c]) / phis;"),
    ("grad: log base", "atomic_add(&A->gsig, gI * F->I * log(F->u));",
     "atomic_add(&A->gsig, gI * F->I * log2(F->u));"),
    ("grad: camera jacobian", "gx[2] = -cam.fx * x / (z * z) * A->gq[j][0]",
     "gx[2] = -cam.fx * x / z * A->gq[j][0]"),
    ("grad: R not transposed",
     "gvi[3 * j + b] += cam.R[0 + b] * gx[0] + cam.R[3 + b] * gx[1] + cam.R[6 + b] * gx[2];",
     "gvi[3 * j + b] += cam.R[3 * b + 0] * gx[0] + cam.R[3 * b + 1] * gx[1] + cam.R[3 * b + 2] * gx[2];"),
    ("grad: colour clamp ignored", "geff[c] = tr->rgb_raw[c] > 0.0 ? A->grgb[c] : 0.0;",
     "geff[c] = A->grgb[c];"),
    ("grad: background term dropped", "ga += (gA - gbg) * Tf / om;", "ga += gA * Tf / om;"),
    ("grad: clamp ignored", "if (F->clamped) continue;", "if (0) continue;"),
    ("grad: opacity factor", "atomic_add(&A->go, ga * F->I);", "atomic_add(&A->go, ga);"),
    ("grad: normal jacobian sign", "const double jx = T->sgn * (-wy / l - ex * Re_w / (l * l * l));",
     "const double jx = T->sgn * (wy / l - ex * Re_w / (l * l * l));"),
    ("grad: area derivative", "{q1[1] - q2[1], q2[0] - q1[0]},", "{q2[1] - q1[1], q2[0] - q1[0]},"),
    ("prune weight after blending", "const double wt = fr[f].T * S.tri[i].o;",
     "const double wt = fr[f].T * (1.0 - fr[f].a) * S.tri[i].o;"),
    ("prune weight alpha for o", "const double wt = fr[f].T * S.tri[i].o;",
     "const double wt = fr[f].T * fr[f].a;"),
    ("prune sum for max", "if (lw[i] > maxw[i]) maxw[i] = lw[i];",
     "maxw[i] += lw[i];"),
    ("sigmoid sign", "I = 1.0 / (1.0 + exp(phi / tr->sigma));",
     "I = 1.0 / (1.0 + exp(-phi / tr->sigma));"),
    ("sigmoid box outward sign", "dist = -sigma * log(o / cfg->alpha_min - 1.0);",
     "dist = sigma * log(o / cfg->alpha_min - 1.0);"),
    ("sigmoid grad sigma sign", "atomic_add(&A->gsig, g * F->u / (s * s));",
     "atomic_add(&A->gsig, -g * F->u / (s * s));"),
    ("lse normalised by max phi(s)", "u = phi / (cfg->window == WIN_LSE ? tr->phis_lse : tr->phis);",
     "u = phi / tr->phis;"),
    ("lse box from max phi(s)", "dist = -T->phis_lse * pow(", "dist = -T->phis * pow("),
    ("lse softmax unnormalised", "w[k] = exp(L[k] - m) / sum;", "w[k] = exp(L[k] - m);"),
    ("lse grad through one edge", "gL[i][c] += w[k] * gk[i][c];",
     "gL[i][c] += (k == F->kmax) * gk[i][c];"),
]


def _build(src_text, out_dir, name):
    cpath = os.path.join(out_dir, name + ".c")
    spath = os.path.join(out_dir, name + ".so")
    with open(cpath, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                           "-ffp-contract=off", cpath, "-o", spath, "-lm"])
    return spath


def _first_failing_pin(path):
    with O.use_library(path):
        for label, fn in PINS:
            try:
                fn()
            except Exception:          # AssertionError or a numerical blow-up
                return label
    return None


def test_unmutated_copy_passes_every_pin():
    with tempfile.TemporaryDirectory() as d:
        src = open(SRC).read()
        assert _first_failing_pin(_build(src, d, "clean")) is None


@pytest.mark.parametrize("label,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(label, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {label}"
    with tempfile.TemporaryDirectory() as d:
        caught = _first_failing_pin(_build(src.replace(old, new), d, "mutant"))
    assert caught is not None, f"no pin catches the planted mistake: {label}"
