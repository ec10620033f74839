"""Mutation check of the oracle's pins: plausible mistakes are planted in a copy of the
oracle's C source (on the CPU, in a temporary directory), and every such mutant must
fail at least one pin of ``test_oracle_pins``.  This shows the pins constrain each
term of the oracle (Eq. 5, 7, 8 and the gradient), not just its overall shape.
"""
import inspect
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "wn_oracle.c")

# (name, original text, replacement); each original must occur in the source.
MUTANTS = [
    ("no_half_angle_factor", "nsum_add(&s, 2.0 * wno_atan2_eq8(a, b));", "nsum_add(&s, wno_atan2_eq8(a, b));"),
    ("no_half_angle_factor_single", "return 2.0 * wno_atan2_eq8(a, b);", "return wno_atan2_eq8(a, b);"),
    ("plain_arctan", "nsum_add(&s, 2.0 * wno_atan2_eq8(a, b));", "nsum_add(&s, 2.0 * atan(a / b));"),
    ("beta_sign", "+ dot3(e[2], e[0]);\n}", "- dot3(e[2], e[0]);\n}"),
    ("beta_missing_one", "*beta = 1.0 + dot3", "*beta = dot3"),
    ("transposed_cross", "cross3(e[1], e[2], x12);\n    *alpha", "cross3(e[2], e[1], x12);\n    *alpha"),
    ("wrong_vertex_index", "V + 3 * F[3 * f + 1], V + 3 * F[3 * f + 2], q, &a, &b);",
     "V + 3 * F[3 * f + 1], V + 3 * F[3 * f + 1], q, &a, &b);"),
    ("eq8_branch_sign", "if (y >= 0) return atan(y / x) + M_PI;", "if (y >= 0) return atan(y / x) - M_PI;"),
    ("eq8_zero_case", "if (y < 0) return -M_PI / 2;\n    return 0.0;", "if (y < 0) return -M_PI / 2;\n    return M_PI;"),
    ("eq8_strict_y", "if (y >= 0) return atan(y / x) + M_PI;", "if (y > 0) return atan(y / x) + M_PI;"),
    ("zero_vertex_direction", "e[j][c] = len > 0 ? r[c] / len : 0.0;\n    }\n    double x12[3];\n    cross3(e[1], e[2], x12);\n    *alpha",
     "e[j][c] = len > 0 ? r[c] / len : 0.57735;\n    }\n    double x12[3];\n    cross3(e[1], e[2], x12);\n    *alpha"),
    ("wrong_normaliser", "W[i] = nsum_get(&s) / (4.0 * M_PI);", "W[i] = nsum_get(&s) / (2.0 * M_PI);"),
    ("grad_no_projection", "out[3 * j + c] = (g[c] - ge * e[j][c]) / len[j];", "out[3 * j + c] = g[c] / len[j];"),
    ("grad_sign", "(beta * u[c] - alpha * (e[k][c] + e[l][c]))", "(beta * u[c] + alpha * (e[k][c] + e[l][c]))"),
    ("grad_cyclic_order", "int k = (j + 1) % 3, l = (j + 2) % 3;", "int k = (j + 2) % 3, l = (j + 1) % 3;"),
    ("grad_no_radius", "out[3 * j + c] = (g[c] - ge * e[j][c]) / len[j];", "out[3 * j + c] = (g[c] - ge * e[j][c]);"),
    ("grad_scale", "T[9 * f + c] = nsum_get(&s[c]) / (4.0 * M_PI);", "T[9 * f + c] = nsum_get(&s[c]);"),
    ("grad_gather_index", "nsum_add(&acc[3 * F[3 * f + j] + c]", "nsum_add(&acc[3 * F[3 * f] + c]"),
    ("grid_half_offset", "((double)ijk[d] + 0.5)", "((double)ijk[d])"),
    ("dist_plane", "return fabs(t) * sqrt(nn);", "return fabs(t) * nn;"),
    ("naive_centroid", "r[d] = (a[d] + b[d] + c[d]) / 3.0 - q[d];", "r[d] = (a[d] + b[d] + c[d]) / 2.0 - q[d];"),
    ("naive_power", "return dot3(N, r) / (r2 * sqrt(r2));", "return dot3(N, r) / r2;"),
    ("naive_scale", "W[i] = nsum_get(&s) / (8.0 * M_PI);", "W[i] = nsum_get(&s) / (4.0 * M_PI);"),
    ("naive_grad_third", "* ir3 / r2) / 3.0 + x[d];", "* ir3 / r2) + x[d];"),
    ("naive_grad_three", "- 3.0 * nr * r[d] * ir3 / r2", "- 2.0 * nr * r[d] * ir3 / r2"),
    ("naive_grad_cross", "cross3(e, a, x);", "cross3(a, e, x);"),
    ("naive_grad_scale", "T[9 * f + c] = nsum_get(&s[c]) / (8.0 * M_PI);\n    }\n    if (dLdV) {\n        nsum *acc = (nsum *)calloc((size_t)(nV > 0 ? nV : 1) * 3, sizeof(nsum));\n        if (!acc) { free(own); return -2; }\n        for (int64_t f = 0; f < nF; ++f)\n            for (int j = 0; j < 3; ++j)\n                for (int c = 0; c < 3; ++c) nsum_add(&acc[3 * F[3 * f + j] + c], T[9 * f + 3 * j + c]);\n        for (int64_t x = 0; x < 3 * nV; ++x) dLdV[x] = nsum_get(&acc[x]);\n        free(acc);\n    }\n    free(own);\n    return 0;\n}\n\n/* ----",
     "T[9 * f + c] = nsum_get(&s[c]) / (4.0 * M_PI);\n    }\n    if (dLdV) {\n        nsum *acc = (nsum *)calloc((size_t)(nV > 0 ? nV : 1) * 3, sizeof(nsum));\n        if (!acc) { free(own); return -2; }\n        for (int64_t f = 0; f < nF; ++f)\n            for (int j = 0; j < 3; ++j)\n                for (int c = 0; c < 3; ++c) nsum_add(&acc[3 * F[3 * f + j] + c], T[9 * f + 3 * j + c]);\n        for (int64_t x = 0; x < 3 * nV; ++x) dLdV[x] = nsum_get(&acc[x]);\n        free(acc);\n    }\n    free(own);\n    return 0;\n}\n\n/* ----"),
]

PIN_TESTS = [fn for name, fn in inspect.getmembers(pins, inspect.isfunction)
             if name.startswith("test_") and "orc" in inspect.signature(fn).parameters]


def run_pin(fn, orc):
    """Run one pin with every parametrisation it has (the morphing pins take the integral)."""
    if "integral" in inspect.signature(fn).parameters:
        for integral in ("naive", "gwn"):
            fn(orc, integral)
    else:
        fn(orc)


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutant {name}: pattern not found"
    mutated = src.replace(old, new, 1)
    assert mutated != src
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(c), "-lm"],
                   check=True)
    return str(so)


def test_pins_pass_on_unmodified_oracle(orc):
    for fn in PIN_TESTS:
        run_pin(fn, orc)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_every_mutant_is_caught(tmp_path, orc, name, old, new):
    so = _build(tmp_path, name, old, new)
    failed = []
    with oracle.use_library(so):
        for fn in PIN_TESTS:
            try:
                run_pin(fn, oracle)
            except Exception:  # an assertion, or a numerical error a pin provokes
                failed.append(fn.__name__)
    assert failed, f"mutant {name} passed every pin"


# Mistakes planted in the numpy parts of the oracle (Adam and the morphing loop): the
# function's source is edited and re-executed in the oracle module's namespace.
PY_MUTANTS = [
    ("adam", "adam_no_bias_correction", "m_hat = m / (1.0 - beta1 ** t)", "m_hat = m"),
    ("adam", "adam_v_no_bias_correction", "v_hat = v / (1.0 - beta2 ** t)", "v_hat = v"),
    ("adam", "adam_bias_power", "m_hat = m / (1.0 - beta1 ** t)", "m_hat = m / (1.0 - beta1 ** (t + 1))"),
    ("adam", "adam_eps_under_root", "np.sqrt(v_hat) + eps", "np.sqrt(v_hat + eps)"),
    ("adam", "adam_v_linear", "(1.0 - beta2) * g * g", "(1.0 - beta2) * np.abs(g)"),
    ("adam", "adam_m_weights", "beta1 * m + (1.0 - beta1) * g", "(1.0 - beta1) * m + beta1 * g"),
    ("adam", "adam_ascent", "return x - lr", "return x + lr"),
    ("morph", "morph_no_chain_rule", "_, dLdV = bwd(V, F, Q, dLdW, threads=threads)",
     "_, dLdV = bwd(V, F, Q, np.ones_like(dLdW), threads=threads)"),
    ("morph", "morph_step_number", "t0 + 1 + i", "t0 + i + 2"),
    ("morph", "morph_loss_after_update", "        V, m, v = adam(V, dLdV, m, v, t0 + 1 + i, lr, beta1, beta2, eps)\n        losses.append(L)",
     "        V, m, v = adam(V, dLdV, m, v, t0 + 1 + i, lr, beta1, beta2, eps)\n        losses.append(sigmoid_mse(fwd(V, F, Q, threads=threads), target, tau, k)[0])"),
    ("_quad_corners", "cubify_inward_faces", "tris = [(out[0], out[2], out[1]), (out[0], out[3], out[2])]",
     "tris = [(out[0], out[1], out[2]), (out[0], out[2], out[3])]"),
    ("_quad_corners", "cubify_wrong_side", "base[axis] += side", "base[axis] += 1 - side"),
    ("cubify", "cubify_interior_faces", "bnd = ~pad[", "bnd = pad["),
    ("laplacian_smooth", "smooth_full_step", "V + lam * (mean - V)", "V + lam * mean"),
    ("laplacian_smooth", "smooth_unnormalised", "S[has] / deg[has, None]", "S[has] / 6.0"),
    ("laplacian_smooth", "smooth_volume_no_cube_root", "V = V * np.cbrt(ratio)", "V = V * ratio"),
    ("laplacian_smooth", "smooth_volume_about_centroid", "V = V * np.cbrt(ratio)",
     "V = V.mean(0) + (V - V.mean(0)) * np.cbrt(ratio)"),
    ("laplacian_smooth", "smooth_volume_never_kept", "if ratio > 0.0 and np.isfinite(ratio):", "if False:"),
    ("enclosed_volume", "volume_factor", "))) / 6.0", "))) / 3.0"),
    ("enclosed_volume", "volume_cross_order", "np.cross(b, c)", "np.cross(c, b)"),
    ("vertex_normals", "normals_uniform_weights", "acc[f[j]] += n", "acc[f[j]] += n / np.linalg.norm(n)"),
    ("vertex_normals", "normals_reversed", "n = np.cross(V[f[1]] - V[f[0]], V[f[2]] - V[f[0]])",
     "n = np.cross(V[f[2]] - V[f[0]], V[f[1]] - V[f[0]])"),
    ("vertex_normals", "normals_first_corner_only", "for j in range(3):\n            acc[f[j]] += n",
     "for j in range(1):\n            acc[f[j]] += n"),
    ("flip_duplicate", "flip_copy_not_reversed", "F[:, [0, 2, 1]] + len(V)", "F[:, [0, 1, 2]] + len(V)"),
    ("flip_duplicate", "flip_moved_outward", "V - eps * N", "V + eps * N"),
    ("flip_duplicate", "flip_copy_offset", "+ len(V)\n", "+ len(V) - 1\n"),
    ("vertex_neighbours", "smooth_duplicate_edges", "e = np.unique(e, axis=0)", "e = e[np.argsort(e[:, 0], kind='stable')]"),
    ("sample_surface", "sample_cdf_side", 'side="right"', 'side="left"'),
    ("sample_surface", "sample_no_reflection", "r1[flip], r2[flip] = 1.0 - r1[flip], 1.0 - r2[flip]",
     "r1[flip], r2[flip] = r2[flip], r1[flip]"),
    ("face_area_weights", "sample_area_squared", "0.5 * np.sqrt((cx * cx + cy * cy) + cz * cz)",
     "0.25 * ((cx * cx + cy * cy) + cz * cz)"),
    ("chamfer_hausdorff", "chamfer_one_way", "dab.mean() + dba.mean()", "dab.mean()"),
    ("chamfer_hausdorff", "hausdorff_one_way", "max(dab.max(), dba.max())", "dab.max()"),
    ("_mc_loops", "mc_join_inside_corners", "for s in range(1, len(walk) + 1)", "for s in range(len(walk) - 1, 0, -1)"),
    ("_mc_fan", "mc_fan_from_first_vertex", "        if all(not (on[s] & on[j])", "        if s == 0 or all(not (on[s] & on[j])"),
    ("_mc_case", "mc_inward_faces", "if _MC_FLIP else tris", "if not _MC_FLIP else tris"),
    ("marching_cubes", "mc_interpolation_sign", "t = (iso - fa) / (fb - fa)", "t = (fa - iso) / (fb - fa)"),
    ("marching_cubes", "mc_level_inclusive", "ins = f > iso", "ins = f >= iso"),
    ("marching_cubes", "mc_padding_inside", "reshape(n), 1)", "reshape(n), 1, constant_values=1.0)"),
    ("marching_cubes", "mc_vertex_numbering", "vid = np.cumsum(flags.reshape(-1)) - 1", "vid = np.cumsum(flags.reshape(-1))"),
]

PY_PIN_TESTS = [fn for fn in PIN_TESTS
                if any(k in fn.__name__ for k in ("adam", "morph", "cubify", "laplacian", "sampling", "nn_dist",
                                                  "marching", "volume", "normals", "flip"))]


@pytest.mark.parametrize("func,name,old,new", PY_MUTANTS, ids=[m[1] for m in PY_MUTANTS])
def test_every_python_mutant_is_caught(monkeypatch, orc, func, name, old, new):
    import textwrap
    src = textwrap.dedent(inspect.getsource(getattr(oracle, func)))
    assert src.count(old) >= 1, f"mutant {name}: pattern not found"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new, 1), f"<{name}>", "exec"), ns)
    monkeypatch.setattr(oracle, func, ns[func])
    failed = []
    for fn in PY_PIN_TESTS:
        try:
            run_pin(fn, oracle)
        except Exception:
            failed.append(fn.__name__)
    assert failed, f"mutant {name} passed every pin"
