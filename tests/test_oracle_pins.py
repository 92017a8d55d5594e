"""Pins of the FP64 oracle to facts fixed outside it: closed forms, library
routines for special cases, brute force on tiny inputs and the invariants the
paper states (lossless culling, nested extents). CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy import special

import oracle as O
from synth import Scene, Camera, scene_small, camera_small

ALOW = 1.0 / 255.0


def one_scene(means, log_scales, quats, logits, rgb=None, sh=None, degree=0):
    means = np.asarray(means, dtype=np.float32).reshape(-1, 3)
    n = means.shape[0]
    if sh is None:
        rgb = np.asarray(rgb if rgb is not None else [[0.5, 0.5, 0.5]] * n, dtype=np.float64).reshape(n, 3)
        sh = ((rgb - 0.5) * 2.0 * math.sqrt(math.pi)).reshape(n, 1, 3)
    return Scene(means, np.asarray(log_scales, np.float32).reshape(n, 3),
                 np.asarray(quats, np.float32).reshape(n, 4),
                 np.asarray(logits, np.float32).reshape(n),
                 np.asarray(sh, np.float32), degree)


def axis_camera(w=33, h=33, f=40.0, z=4.0):
    """Camera at (0, 0, -z) looking along +z with cx = W/2 so that the world
    origin projects onto the centre of pixel ((W-1)/2, (H-1)/2)."""
    w2c = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 1.0, z]])
    return Camera(w2c, f, f, w / 2.0, h / 2.0, w, h, 0.2)


def logit(p):
    return math.log(p / (1.0 - p))


# ---------------------------------------------------------------- rotation / SH

def test_quaternion_matches_scipy():
    rng = np.random.default_rng(1)
    q = rng.normal(size=(200, 4))
    ours = O.quat_to_rotmat(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy wants (x, y, z, w)
    np.testing.assert_allclose(ours, ref, atol=1e-12)


def test_quaternion_quarter_turn_about_z_maps_x_to_y():
    h = math.sqrt(0.5)
    r = O.quat_to_rotmat(np.array([[h, 0.0, 0.0, h]]))[0]
    np.testing.assert_allclose(r @ [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], atol=1e-15)


def test_covariance_of_rotated_axis_scales():
    h = math.sqrt(0.5)
    ls = np.log([[0.1, 0.3, 0.7]])
    sig = O.covariance_3d(ls, [[h, 0, 0, h]])[0]
    np.testing.assert_allclose(sig, np.diag([0.09, 0.01, 0.49]), atol=1e-15)


def _real_from_complex(l, m, theta, phi):
    # scipy's complex SH carry the Condon-Shortley phase; the real basis is
    # sqrt(2) Re / sqrt(2) Im of the m >= 0 member.
    y = special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * y.real
    if m < 0:
        return math.sqrt(2.0) * y.imag
    return y.real


def test_sh_basis_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(2)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    ours = O.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(ours[:, l * l + l + m], _real_from_complex(l, m, theta, phi),
                                       atol=1e-12, err_msg=f"l={l} m={m}")


def test_sh_basis_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(24)  # exact for the polynomial part in cos(theta)
    nphi = 48
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).ravel()
    y = O.sh_basis(3, d)
    gram = (y * w[:, None]).T @ y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_degree_one_closed_form():
    d = np.array([[0.48, -0.6, 0.64]])
    y = O.sh_basis(1, d)[0]
    k = math.sqrt(3.0 / (4.0 * math.pi))
    np.testing.assert_allclose(y, [0.5 / math.sqrt(math.pi), -k * -0.6, k * 0.64, -k * 0.48], atol=1e-15)


def test_sh_degree0_colour_is_dc_times_y00_plus_half():
    s = one_scene([[0, 0, 0]], [[-2, -2, -2]], [[1, 0, 0, 0]], [0.0], rgb=[[0.2, 0.7, 1.0]])
    pre = O.preprocess(s, axis_camera(), O.Params())
    np.testing.assert_allclose(pre["color"][0], [0.2, 0.7, 1.0], atol=1e-6)


# ---------------------------------------------------------------- projection

def test_projected_centre_and_pixel_convention():
    cam = axis_camera(w=33, h=33, f=40.0, z=4.0)
    s = one_scene([[0.5, -0.25, 1.0]], [[-3, -3, -3]], [[1, 0, 0, 0]], [0.0])
    pre = O.preprocess(s, cam, O.Params())
    # u = f X / Z + cx in continuous coordinates; pixel centres at integers => -1/2
    assert pre["x"][0] == pytest.approx(40.0 * 0.5 / 5.0 + 16.5 - 0.5, abs=1e-12)
    assert pre["y"][0] == pytest.approx(40.0 * -0.25 / 5.0 + 16.5 - 0.5, abs=1e-12)
    assert pre["depth32"][0] == np.float32(5.0)


def test_ewa_isotropic_on_axis_closed_form():
    f, z, s_ = 40.0, 4.0, 0.3
    cam = axis_camera(f=f, z=z)
    s = one_scene([[0, 0, 0]], [[math.log(s_)] * 3], [[0.3, -0.2, 0.5, 0.1]], [0.0])
    pre = O.preprocess(s, cam, O.Params())
    s_ = math.exp(float(np.float32(math.log(s_))))  # the scale the float32 scene holds
    v = (f * s_ / z) ** 2 + 0.3
    np.testing.assert_allclose(pre["cov2"][0], [v, 0.0, v], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(pre["lam_max"][0], v, rtol=1e-13)
    np.testing.assert_allclose(pre["r_o"][0], 3 * math.sqrt(v), rtol=1e-12)


def test_ewa_matches_numerical_jacobian_off_axis():
    """Sigma' = J Sigma J^T + 0.3 I with J the derivative of the pixel
    projection, taken here by central differences (inside the clamp)."""
    rng = np.random.default_rng(3)
    cam = camera_small(128, 96)
    s = one_scene(rng.uniform(-0.8, 0.8, size=(20, 3)), rng.normal(-2.5, 0.4, size=(20, 3)),
                  rng.normal(size=(20, 4)), np.zeros(20))
    pre = O.preprocess(s, cam, O.Params())
    w2c = cam.world_to_cam
    sig3 = O.covariance_3d(s.log_scales, s.quats)

    def proj(pw):
        pc = w2c[:, :3] @ pw + w2c[:, 3]
        return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    for g in range(20):
        mu = s.means[g].astype(np.float64)
        jac = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-5
            jac[:, k] = (proj(mu + e) - proj(mu - e)) / 2e-5
        cov = jac @ sig3[g] @ jac.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(pre["cov2"][g], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-6, atol=1e-9)


def _rotated_camera(eye, seed, w=128, h=96, f=60.0):
    """A camera with a random orientation R whose centre is at `eye`:
    p_cam = R p + t with t = -R eye, so that p = eye maps to the origin."""
    r = Rotation.random(random_state=seed).as_matrix()
    t = -r @ np.asarray(eye, dtype=np.float64)
    return Camera(np.concatenate([r, t[:, None]], axis=1), f, f, w / 2.0, h / 2.0, w, h, 0.2)


def test_camera_position_is_the_eye_of_a_rotated_camera():
    for seed, eye in enumerate(([2.0, -1.0, -5.0], [0.0, 0.0, 7.5], [-3.0, 4.0, 0.25])):
        cam = _rotated_camera(eye, seed)
        np.testing.assert_allclose(O.camera_position(cam), eye, atol=1e-12)


def test_sh_degree_one_colour_follows_the_direction_from_the_camera():
    """Degree-1 colour in closed form, with the viewing direction written
    out from the camera's eye (not from its [R | t]): channel 0 carries only
    the m = 1 coefficient (Y = -k x), channel 1 only m = 0 (Y = k z), channel 2
    only m = -1 (Y = -k y), k = sqrt(3 / (4 pi)); colour = 1/2 + coef Y."""
    k = math.sqrt(3.0 / (4.0 * math.pi))
    rng = np.random.default_rng(21)
    for seed, eye in enumerate(([2.0, -1.0, -5.0], [-4.0, 3.0, 1.0])):
        cam = _rotated_camera(eye, 10 + seed)
        means = rng.uniform(-1.5, 1.5, size=(6, 3))
        sh = np.zeros((6, 4, 3))
        sh[:, 3, 0] = 0.7   # m = +1 -> red
        sh[:, 2, 1] = -0.6  # m = 0  -> green
        sh[:, 1, 2] = 0.5   # m = -1 -> blue
        scene = one_scene(means, [[-2.0] * 3] * 6, [[1, 0, 0, 0]] * 6, [0.0] * 6, sh=sh, degree=1)
        col = O.preprocess(scene, cam, O.Params())["color"]
        v = scene.means.astype(np.float64) - np.asarray(eye)[None, :]
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        sh32 = scene.sh.astype(np.float64)
        expect = np.stack([0.5 + sh32[:, 3, 0] * (-k * v[:, 0]),
                           0.5 + sh32[:, 2, 1] * (k * v[:, 2]),
                           0.5 + sh32[:, 1, 2] * (-k * v[:, 1])], axis=1)
        np.testing.assert_allclose(col, np.maximum(expect, 0.0), atol=1e-12)


def test_ewa_jacobian_is_clamped_off_screen():
    """Centres beyond the EWA clamp: the Jacobian is taken at x/z (or y/z)
    clamped to +-1.3 (W/2)/fx (or (H/2)/fy), written out here by hand, on a
    camera with W != H so that the two limits differ. Camera at the origin,
    no rotation, isotropic Sigma = s^2 I, so Sigma' = s^2 J J^T + 0.3 I."""
    w, h, f = 128, 64, 40.0
    cam = Camera(np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 1.0, 0]]), f, f, w / 2.0, h / 2.0, w, h, 0.2)
    lim_x, lim_y = 1.3 * (w / 2) / f, 1.3 * (h / 2) / f  # 2.08 and 1.04
    # beyond the x limit; beyond the -y limit; inside both
    pts = np.array([[5.0, 0.5, 2.0], [0.5, -3.0, 2.0], [0.8, 0.4, 2.0]])
    scene = one_scene(pts, [[-1.0] * 3] * 3, [[1, 0, 0, 0]] * 3, [0.0] * 3)
    cov = O.preprocess(scene, cam, O.Params())["cov2"]
    s2 = math.exp(-1.0) ** 2
    m = scene.means.astype(np.float64)  # the float32 centres the scene holds
    xt = [2.0 * lim_x, m[1, 0], m[2, 0]]  # clamped x/z times z (first point only)
    yt = [m[0, 1], -2.0 * lim_y, m[2, 1]]  # clamped y/z times z (second point only)
    for g in range(3):
        z = 2.0
        jx = np.array([f / z, 0.0, -f * xt[g] / z ** 2])
        jy = np.array([0.0, f / z, -f * yt[g] / z ** 2])
        a = s2 * jx @ jx + 0.3
        b = s2 * jx @ jy
        c = s2 * jy @ jy + 0.3
        np.testing.assert_allclose(cov[g], [a, b, c], rtol=1e-13, atol=1e-13, err_msg=f"point {g}")


def test_tiny_gaussian_projects_to_lowpass_only():
    s = one_scene([[0.1, 0.1, 0.0]], [[-30, -30, -30]], [[1, 0, 0, 0]], [0.0])
    pre = O.preprocess(s, axis_camera(), O.Params())
    np.testing.assert_allclose(pre["cov2"][0], [0.3, 0.0, 0.3], atol=1e-12)


def test_behind_near_plane_is_invisible():
    s = one_scene([[0, 0, -3.9], [0, 0, -3.7]], [[-3] * 3] * 2, [[1, 0, 0, 0]] * 2, [3.0, 3.0])
    pre = O.preprocess(s, axis_camera(), O.Params())
    assert list(pre["valid"]) == [False, True]
    r = O.tile_rects(pre, axis_camera(), O.Params(cull=O.CULL_3SIGMA))
    assert r["tiles_touched"][0] == 0 and r["tiles_touched"][1] > 0


# ---------------------------------------------------------------- blending closed forms

def _frame(scene, cam, **kw):
    return O.render_frame(scene, cam, O.Params(**kw))


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_single_gaussian_image_closed_form(mode):
    f, z = 40.0, 4.0
    sx, sy, sig = 0.35, 0.15, 0.8
    h = math.sqrt(0.5)  # quarter turn about z swaps the x and y scales
    cam = axis_camera(f=f, z=z)
    s = one_scene([[0, 0, 0]], [[math.log(sx), math.log(sy), -3.0]], [[h, 0, 0, h]], [logit(sig)],
                  rgb=[[0.9, 0.4, 0.1]])
    out = _frame(s, cam, cull=mode, background=(0.1, 0.2, 0.3))
    sx, sy = (math.exp(float(v)) for v in s.log_scales[0, :2])  # float32-held values
    sig = 1.0 / (1.0 + math.exp(-float(s.opacity_logits[0])))
    vx = (f * sy / z) ** 2 + 0.3
    vy = (f * sx / z) ** 2 + 0.3
    jj, ii = np.mgrid[0:33, 0:33]
    a = sig * np.exp(-0.5 * ((ii - 16.0) ** 2 / vx + (jj - 16.0) ** 2 / vy))
    a = np.where(a >= ALOW, np.minimum(a, 0.99), 0.0)
    for ch, (c, b) in enumerate(zip((0.9, 0.4, 0.1), (0.1, 0.2, 0.3))):
        np.testing.assert_allclose(out["image"][ch], c * a + (1 - a) * b, atol=1e-6)
    np.testing.assert_array_equal(out["l_blend"], (a > 0).astype(np.uint32))


def test_rotated_gaussian_on_axis_closed_form():
    """Off-diagonal Sigma': a Gaussian turned 30 degrees about the optical axis;
    Sigma' = (f/z)^2 R diag(sx^2, sy^2) R^T + 0.3 I, inverted by numpy."""
    f, z, th = 40.0, 4.0, math.radians(30.0)
    cam = axis_camera(f=f, z=z)
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    s = one_scene([[0, 0, 0]], [[math.log(0.4), math.log(0.1), -3.0]], [q], [logit(0.9)], rgb=[[1, 1, 1]])
    out = _frame(s, cam)
    sx, sy = (math.exp(float(v)) for v in s.log_scales[0, :2])
    sig = 1.0 / (1.0 + math.exp(-float(s.opacity_logits[0])))
    c = float(s.sh[0, 0, 0]) * 0.5 / math.sqrt(math.pi) + 0.5
    qn = np.asarray(s.quats[0], np.float64)
    qn /= np.linalg.norm(qn)
    th = 2 * math.atan2(qn[3], qn[0])
    r2 = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    cov = (f / z) ** 2 * r2 @ np.diag([sx * sx, sy * sy]) @ r2.T + 0.3 * np.eye(2)
    inv = np.linalg.inv(cov)
    jj, ii = np.mgrid[0:33, 0:33]
    d = np.stack([ii - 16.0, jj - 16.0], axis=-1)
    a = sig * np.exp(-0.5 * np.einsum("...i,ij,...j->...", d, inv, d))
    a = np.where(a >= ALOW, np.minimum(a, 0.99), 0.0)
    np.testing.assert_allclose(out["image"][0], c * a, atol=1e-9)


def test_two_gaussians_over_closed_form():
    cam = axis_camera()
    s = one_scene([[0, 0, 0.5], [0, 0, 0]], [[-2.5] * 3] * 2, [[1, 0, 0, 0]] * 2,
                  [logit(0.3), logit(0.6)], rgb=[[1, 0, 0], [0, 0, 1]])
    out = _frame(s, cam)
    # the second row is nearer (depth 4 < 4.5), so it is blended first
    px = out["image"][:, 16, 16]
    a_near, a_far = 0.6, 0.3
    np.testing.assert_allclose(px, [a_far * (1 - a_near), 0.0, a_near], atol=1e-6)
    assert out["l_blend"][16, 16] == 2


def test_termination_after_three_blends():
    cam = axis_camera()
    n = 6
    s = one_scene([[0, 0, 0.01 * k] for k in range(n)], [[-2.0] * 3] * n, [[1, 0, 0, 0]] * n,
                  [logit(0.98)] * n, rgb=[[1, 1, 1]] * n)
    out = _frame(s, cam)
    a = 1.0 / (1.0 + math.exp(-float(s.opacity_logits[0])))  # 0.98 as the float32 logit holds it
    # T: 0.02, 4e-4, 8e-6 -> stops after the third blend
    assert out["l_blend"][16, 16] == 3
    assert out["l_iter"][16, 16] == 3
    assert out["final_t"][16, 16] == pytest.approx((1 - a) ** 3, rel=1e-9)
    c = float(s.sh[0, 0, 0]) * 0.5 / math.sqrt(math.pi) + 0.5  # 1 as the float32 DC holds it
    assert out["image"][0, 16, 16] == pytest.approx(c * (1 - (1 - a) ** 3), abs=1e-12)


def test_load_balancing_cap_stops_after_k_blends():
    cam = axis_camera()
    n = 6
    s = one_scene([[0, 0, 0.01 * k] for k in range(n)], [[-2.0] * 3] * n, [[1, 0, 0, 0]] * n,
                  [logit(0.5)] * n, rgb=[[1, 1, 1]] * n)
    out = _frame(s, cam, lb_cap=2)
    a = 1.0 / (1.0 + math.exp(-float(s.opacity_logits[0])))
    c = float(s.sh[0, 0, 0]) * 0.5 / math.sqrt(math.pi) + 0.5
    assert out["l_blend"][16, 16] == 2
    assert out["final_t"][16, 16] == pytest.approx((1 - a) ** 2, rel=1e-12)
    assert out["image"][0, 16, 16] == pytest.approx(c * (1 - (1 - a) ** 2), rel=1e-12)
    full = _frame(s, cam)
    assert full["l_blend"][16, 16] == 6


# ---------------------------------------------------------------- radii (Eqs. 5-11)

def _bisect_extent(inv, sig, angles, alow=ALOW):
    """For each direction, the largest rho with sig exp(-1/2 rho^2 u^T inv u)
    >= alow, found by bisection on the opacity itself (Eq. 2); returns the
    boundary points (n, 2)."""
    u = np.stack([np.cos(angles), np.sin(angles)], axis=1)
    q = np.einsum("ni,ij,nj->n", u, inv, u)
    def ok(r):
        return sig * np.exp(-0.5 * r * r * q) >= alow
    lo = np.zeros(len(angles))
    hi = np.ones(len(angles))
    while not np.all(~ok(hi)):
        hi = np.where(ok(hi), 2 * hi, hi)
    for _ in range(70):
        mid = 0.5 * (lo + hi)
        good = ok(mid)
        lo = np.where(good, mid, lo)
        hi = np.where(good, hi, mid)
    return lo[:, None] * u


def _max_over_angles(inv, sig, f):
    """max over the boundary of f(points), on a coarse grid then refined twice
    around the best angle."""
    ang = np.linspace(0, 2 * math.pi, 4001)
    best = None
    width = math.pi
    for _ in range(3):
        v = f(_bisect_extent(inv, sig, ang))
        k = int(np.argmax(v))
        best, centre = v[k], ang[k]
        width = (ang[1] - ang[0]) * 2
        ang = np.linspace(centre - width, centre + width, 4001)
    return best


def _random_pre(rng, n):
    a = rng.uniform(0.3, 40, n)
    c = rng.uniform(0.3, 40, n)
    b = rng.uniform(-0.95, 0.95, n) * np.sqrt(a * c)
    det = a * c - b * b
    mid = 0.5 * (a + c)
    lam = mid + np.sqrt(np.maximum(mid * mid - det, 0))
    return dict(valid=np.ones(n, bool), cov2=np.stack([a, b, c], 1), lam_max=lam,
                r_o=3 * np.sqrt(lam), opacity=rng.uniform(ALOW, 0.35, n))


def test_adaptive_radius_and_aabb_equal_brute_force_extents():
    rng = np.random.default_rng(4)
    pre = _random_pre(rng, 40)
    _, r_ad, _ = O.cull_radii(pre, O.Params(cull=O.CULL_ADAPTIVE))
    _, x_max, y_max = O.cull_radii(pre, O.Params(cull=O.CULL_AABB))
    for g in range(40):
        a, b, c = pre["cov2"][g]
        inv = np.linalg.inv(np.array([[a, b], [b, c]]))
        sig = pre["opacity"][g]
        assert r_ad[g] == pytest.approx(_max_over_angles(inv, sig, lambda p: np.hypot(p[:, 0], p[:, 1])), rel=1e-9)
        assert x_max[g] == pytest.approx(_max_over_angles(inv, sig, lambda p: p[:, 0]), rel=1e-9)
        assert y_max[g] == pytest.approx(_max_over_angles(inv, sig, lambda p: p[:, 1]), rel=1e-9)


def test_conic_coefficient_form_of_adaptive_radius():
    """The A..D expression of the semi-major axis (Sec. 4.2) equals Eq. 7."""
    rng = np.random.default_rng(5)
    pre = _random_pre(rng, 500)
    _, r_ad, _ = O.cull_radii(pre, O.Params(cull=O.CULL_ADAPTIVE))
    a, b, c = pre["cov2"].T
    lnr = np.log(pre["opacity"] / ALOW)
    A, B, C, D = c, a, -2 * b, -2 * (a * c - b * b) * lnr
    r_abcd = np.sqrt(2 * D / (-(A + B) + np.sqrt((A - B) ** 2 + C ** 2)))
    np.testing.assert_allclose(np.minimum(r_abcd, pre["r_o"]), r_ad, rtol=1e-9)


def test_radius_cap_crossover_at_alpha_low_e_to_4_5():
    star = ALOW * math.exp(4.5)
    assert star == pytest.approx(0.353, abs=1e-3)
    pre = dict(valid=np.ones(2, bool), cov2=np.array([[4.0, 0, 4.0]] * 2), lam_max=np.array([4.0, 4.0]),
               r_o=np.array([6.0, 6.0]), opacity=np.array([star * 0.999, star * 1.001]))
    _, r, _ = O.cull_radii(pre, O.Params(cull=O.CULL_ADAPTIVE))
    assert r[0] < 6.0 and r[1] == 6.0


def test_opacity_below_alpha_low_has_no_pairs_in_culling_modes():
    pre = dict(valid=np.ones(1, bool), cov2=np.array([[4.0, 0, 4.0]]), lam_max=np.array([4.0]),
               r_o=np.array([6.0]), opacity=np.array([ALOW * 0.99]))
    for m in (O.CULL_ADAPTIVE, O.CULL_AABB):
        keep, _, _ = O.cull_radii(pre, O.Params(cull=m))
        assert not keep[0]
    keep, _, _ = O.cull_radii(pre, O.Params(cull=O.CULL_3SIGMA))
    assert keep[0]


# ---------------------------------------------------------------- integer stage, brute force

def _tiny_scene(seed, n=24):
    rng = np.random.default_rng(seed)
    return one_scene(rng.uniform(-1, 1, (n, 3)), rng.normal(-2.2, 0.6, (n, 3)), rng.normal(size=(n, 4)),
                     rng.normal(0, 2.0, n), rgb=rng.uniform(0, 1, (n, 3)))


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1])
def test_integer_stage_matches_brute_force(mode, seed):
    cam = camera_small(40, 37)  # ragged: 3 x 3 tiles, partial last row/column
    s = _tiny_scene(seed)
    params = O.Params(cull=mode)
    out = O.render_frame(s, cam, params)
    pre, rects = out["pre"], out["rects"]
    tx_n = 3
    expected_pairs = []
    for g in range(s.n):
        tiles = set()
        if rects["keep"][g]:
            x, y, rx, ry = pre["x"][g], pre["y"][g], rects["r_x"][g], rects["r_y"][g]
            for j in range(cam.height):
                for i in range(cam.width):
                    if x - rx <= i <= x + rx and y - ry <= j <= y + ry:
                        tiles.add((j // 16) * tx_n + (i // 16))
        assert out["tiles_touched"][g] == len(tiles)
        dbits = int(pre["depth32"][g:g + 1].view(np.uint32)[0])
        expected_pairs += [((t << 32) | dbits, g) for t in tiles]
    expected_pairs.sort()
    assert out["keys"].tolist() == [k for k, _ in expected_pairs]
    assert out["values"].tolist() == [g for _, g in expected_pairs]
    ranges = np.zeros((9, 2), dtype=np.uint32)
    for p, (k, _) in enumerate(expected_pairs):
        t = k >> 32
        if ranges[t, 1] == 0:
            ranges[t, 0] = p
        ranges[t, 1] = p + 1
    np.testing.assert_array_equal(out["ranges"], ranges)


def test_depth_key_bits_order_like_depths():
    d = np.sort(np.random.default_rng(6).uniform(0.2, 100, 1000)).astype(np.float32)
    bits = d.view(np.uint32)
    assert np.all(np.diff(bits.astype(np.int64)) >= 0)


def test_tiled_lists_equal_brute_force_per_pixel():
    cam = camera_small(48, 48)
    s = scene_small(300, seed=7)
    params = O.Params(cull=O.CULL_3SIGMA)
    out = O.render_frame(s, cam, params)
    jj, ii = np.mgrid[0:48, 0:48]
    bf = O.brute_force_render(out["pre"], out["rects"], cam, params, ii.ravel(), jj.ravel())
    np.testing.assert_allclose(bf["image"].T.reshape(3, 48, 48), out["image"], atol=1e-13)
    np.testing.assert_array_equal(bf["l_iter"].reshape(48, 48), out["l_iter"])


def test_vectorised_renderer_equals_per_pixel_loop(small_scene, small_camera):
    out = O.render_frame(small_scene, small_camera, O.Params())
    rng = np.random.default_rng(8)
    ii = rng.integers(0, 128, 400)
    jj = rng.integers(0, 128, 400)
    pp = O.render_pixels(out["pre"], out["values"], out["ranges"], small_camera, O.Params(), ii, jj)
    np.testing.assert_allclose(pp["image"].T, out["image"][:, jj, ii], atol=1e-13)
    np.testing.assert_array_equal(pp["l_iter"], out["l_iter"][jj, ii])
    np.testing.assert_array_equal(pp["l_blend"], out["l_blend"][jj, ii])


# ---------------------------------------------------------------- the paper's invariants

def test_culling_is_lossless_and_nested(small_scene, small_camera):
    outs = [O.render_frame(small_scene, small_camera, O.Params(cull=m)) for m in (0, 1, 2)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o["image"], outs[0]["image"])
        np.testing.assert_array_equal(o["l_blend"], outs[0]["l_blend"])
    assert np.all(outs[0]["l_iter"] >= outs[1]["l_iter"])
    assert np.all(outs[1]["l_iter"] >= outs[2]["l_iter"])
    assert outs[0]["n_pairs"] > outs[1]["n_pairs"] > outs[2]["n_pairs"]
    r3, ra, rb = (o["rects"] for o in outs)
    vis = rb["nonempty"]
    for key, cmp in (("i_lo", np.greater_equal), ("j_lo", np.greater_equal),
                     ("i_hi", np.less_equal), ("j_hi", np.less_equal)):
        assert np.all(cmp(rb[key][vis], ra[key][vis]))
        assert np.all(cmp(ra[key][ra["nonempty"]], r3[key][ra["nonempty"]]))


def test_every_visible_pair_lies_in_every_modes_tiles(small_scene, small_camera):
    """Brute force over all Gaussian-pixel pairs of the 3-sigma support: a pair
    with alpha >= alpha_low has its pixel inside the AABB and adaptive
    rectangles whenever the radius came from the alpha_low ellipse."""
    cam = small_camera
    p = O.Params(cull=O.CULL_3SIGMA)
    pre = O.preprocess(small_scene, cam, p)
    r3 = O.tile_rects(pre, cam, p)
    ra = O.tile_rects(pre, cam, O.Params(cull=O.CULL_ADAPTIVE))
    rb = O.tile_rects(pre, cam, O.Params(cull=O.CULL_AABB))
    jj, ii = np.mgrid[0:cam.height, 0:cam.width]
    bad = 0
    for g in np.nonzero(r3["nonempty"])[0]:
        x0, x1 = r3["tx_lo"][g] * 16, (r3["tx_hi"][g] + 1) * 16
        y0, y1 = r3["ty_lo"][g] * 16, (r3["ty_hi"][g] + 1) * 16
        si, sj = ii[y0:y1, x0:x1], jj[y0:y1, x0:x1]
        dx, dy = pre["x"][g] - si, pre["y"][g] - sj
        ca, cb, cc = pre["conic"][g]
        a = pre["opacity"][g] * np.exp(-0.5 * (ca * dx * dx + 2 * cb * dx * dy + cc * dy * dy))
        hit = a >= ALOW
        if not hit.any():
            continue
        ti, tj = si[hit] // 16, sj[hit] // 16
        for r in (ra, rb):
            inside = (r["nonempty"][g] & (ti >= r["tx_lo"][g]) & (ti <= r["tx_hi"][g])
                      & (tj >= r["ty_lo"][g]) & (tj <= r["ty_hi"][g]))
            bad += int((~inside).sum())
    assert bad == 0


def test_everything_below_alpha_low_renders_background():
    s = scene_small(200, seed=9)
    s.opacity_logits[:] = np.float32(logit(ALOW * 0.9))
    cam = camera_small(64, 64)
    bg = (0.25, 0.5, 0.75)
    for m in (0, 1, 2):
        out = O.render_frame(s, cam, O.Params(cull=m, background=bg))
        if m == 0:
            assert out["n_pairs"] > 0
        else:
            assert out["n_pairs"] == 0
        for ch in range(3):
            np.testing.assert_array_equal(out["image"][ch], np.full((64, 64), bg[ch]))
        assert out["l_blend"].max() == 0


def test_empty_scene():
    s = scene_small(0, seed=0)
    out = O.render_frame(s, camera_small(32, 32), O.Params())
    assert out["n_pairs"] == 0
    assert np.all(out["image"] == 0) and np.all(out["final_t"] == 1)


# ---------------------------------------------------------------- Eq. 13 and PSNR

def test_load_stats_closed_form():
    m, s = O.load_stats(np.array([[0, 0], [2, 2]]))
    assert m == 1.0 and s == 1.0
    rng = np.random.default_rng(10)
    l = rng.integers(0, 500, size=(37, 41))
    m, s = O.load_stats(l)
    assert m == pytest.approx(l.mean(), rel=1e-15)
    assert s == pytest.approx(l.std(ddof=0), rel=1e-12)


def test_psnr_known_mse():
    a = np.zeros((3, 4, 4))
    b = np.full((3, 4, 4), 0.1)
    assert O.psnr(a, b) == pytest.approx(20.0, abs=1e-12)
    assert O.psnr(a, a) == math.inf
