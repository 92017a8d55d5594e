"""Plants plausible mistakes in a copy of the oracle's source and checks that
the pins catch each one. The copy lives only in this process; the oracle
itself is untouched. CPU only."""
import pathlib
import sys
import types

import pytest

import tests.test_oracle_pins as pins

SRC = (pathlib.Path(__file__).resolve().parents[1] / "oracle" / "adr_oracle.py").read_text()

# (name, text in the oracle, replacement, pins expected to notice)
MUTATIONS = [
    ("conic off-diagonal sign", "conic = np.stack([c / det, -b / det, a / det], axis=1)",
     "conic = np.stack([c / det, b / det, a / det], axis=1)",
     ["test_rotated_gaussian_on_axis_closed_form"]),
    ("low-pass dropped", "a = cov2[:, 0, 0] + params.lowpass", "a = cov2[:, 0, 0]",
     ["test_ewa_isotropic_on_axis_closed_form"]),
    ("Jacobian third column sign", "jac[:, 0, 2] = -fx * xt / (zs * zs)", "jac[:, 0, 2] = fx * xt / (zs * zs)",
     ["test_ewa_matches_numerical_jacobian_off_axis"]),
    ("rotation transposed", "r[..., 0, 1] = 2 * (x * y - w * z)", "r[..., 0, 1] = 2 * (x * y + w * z)",
     ["test_quaternion_matches_scipy"]),
    ("blend without transmittance", "cacc[bl] += col[g[k]][None, :] * wgt[:, None]",
     "cacc[bl] += col[g[k]][None, :] * a[bl][:, None]",
     ["test_two_gaussians_over_closed_form"]),
    ("stop tested before blending", "                    stop = bl & (tt < params.t_min)",
     "                    stop = bl & (tt * (1.0 - a) < params.t_min)",
     ["test_termination_after_three_blends"]),
    ("AABB uses the wrong diagonal", "rx = np.minimum(np.sqrt(2.0 * pre[\"cov2\"][:, 0] * lnr), r_o)",
     "rx = np.minimum(np.sqrt(2.0 * pre[\"cov2\"][:, 2] * lnr), r_o)",
     ["test_adaptive_radius_and_aabb_equal_brute_force_extents"]),
    ("adaptive radius without the factor 2", "r = np.minimum(np.sqrt(2.0 * pre[\"lam_max\"] * lnr), r_o)",
     "r = np.minimum(np.sqrt(pre[\"lam_max\"] * lnr), r_o)",
     ["test_adaptive_radius_and_aabb_equal_brute_force_extents"]),
    ("tile id transposed", "tile = (ty * tx_n + tx).astype(np.uint64)", "tile = (tx * tx_n + ty).astype(np.uint64)",
     ["test_integer_stage_matches_brute_force"]),
    ("rect rounds the wrong way", "i_lo = np.clip(np.maximum(np.ceil(x - rx), 0.0), 0, w)",
     "i_lo = np.clip(np.maximum(np.floor(x - rx), 0.0), 0, w)",
     ["test_integer_stage_matches_brute_force"]),
    ("SH m<0 sign", "v = math.sqrt(2.0) * n_lm * p[(l, am)] * np.sin(am * ph)",
     "v = -math.sqrt(2.0) * n_lm * p[(l, am)] * np.sin(am * ph)",
     ["test_sh_basis_matches_scipy_complex_harmonics"]),
    ("load std as sample std", "var = (n * s2 - s1 * s1) / (n * n)", "var = (n * s2 - s1 * s1) / (n * (n - 1))",
     ["test_load_stats_closed_form"]),
    ("camera centre +R^T t", "return -r.T @ t", "return r.T @ t",
     ["test_camera_position_is_the_eye_of_a_rotated_camera",
      "test_sh_degree_one_colour_follows_the_direction_from_the_camera"]),
    ("SH direction from the Gaussian to the camera", "v = mu - camera_position(cam)[None, :]",
     "v = camera_position(cam)[None, :] - mu",
     ["test_sh_degree_one_colour_follows_the_direction_from_the_camera"]),
    ("EWA clamp of x uses the height", "lim_x = params.ewa_clamp * (cam.width / 2.0) / fx",
     "lim_x = params.ewa_clamp * (cam.height / 2.0) / fx",
     ["test_ewa_jacobian_is_clamped_off_screen"]),
    ("EWA clamp removed", "xt = zs * np.clip(p[:, 0] / zs, -lim_x, lim_x)", "xt = p[:, 0]",
     ["test_ewa_jacobian_is_clamped_off_screen"]),
]


def _mutated_oracle(monkeypatch, old, new):
    assert SRC.count(old) == 1, old
    mod = types.ModuleType("oracle_mutant")
    monkeypatch.setitem(sys.modules, "oracle_mutant", mod)
    exec(compile(SRC.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    return mod


def _call(fn):
    import inspect
    sig = inspect.signature(fn)
    kwargs = {}
    marks = getattr(fn, "pytestmark", [])
    param_sets = [m.args for m in marks if m.name == "parametrize"]
    if param_sets:
        # run every parametrisation; any failure counts
        import itertools
        names = [p[0] for p in param_sets]
        values = [p[1] for p in param_sets]
        for combo in itertools.product(*values):
            fn(**dict(zip(names, combo)))
        return
    for name in sig.parameters:
        if name == "small_scene":
            from synth import scene_small
            kwargs[name] = scene_small(2000, 0)
        elif name == "small_camera":
            from synth import camera_small
            kwargs[name] = camera_small()
    fn(**kwargs)


@pytest.mark.parametrize("name,old,new,catchers", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(monkeypatch, name, old, new, catchers):
    mutant = _mutated_oracle(monkeypatch, old, new)
    monkeypatch.setattr(pins, "O", mutant)
    caught = False
    for c in catchers:
        try:
            _call(getattr(pins, c))
        except (AssertionError, ValueError, IndexError):
            caught = True
    assert caught, f"no pin noticed: {name}"
