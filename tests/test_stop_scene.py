"""Preconditions of the stopped-pixel scene (tests/stop_scene.py), checked on
the oracle so that the GPU test built on it exercises what it claims: pixels
that stop (T < t_min, Eq. 3) at the last wall while the rest of their 8 x 8
quadrant keeps blending, a next list entry whose FP32 exponent has no usable
error bound (so the blend decides it in FP64 only), and a Gaussian 0 that
would blend at the stopped pixels if they went on."""
import math

import numpy as np
import pytest

import oracle as O
from tests.stop_scene import stop_scene
from tests.test_fp32_exponent_bound import H, bound, principal_axes


@pytest.mark.parametrize("n_weak", [0, 1])
@pytest.mark.parametrize("mode", [O.CULL_3SIGMA, O.CULL_AABB])
def test_stop_scene_preconditions(n_weak, mode):
    scene, cam, n_walls = stop_scene(n_weak)
    prm = O.Params(cull=mode)
    fr = O.render_frame(scene, cam, prm)
    pre = fr["pre"]
    needle = scene.n - 1
    s, e = (int(v) for v in fr["ranges"][0])
    tile0 = [int(v) for v in fr["values"][s:e]]
    # front to back: the walls, the needle, then Gaussian 0
    assert tile0 == list(range(1, n_walls + 1)) + [needle, 0]
    quad = (slice(0, 8), slice(0, 8))
    stopped = (fr["final_t"][quad] < prm.t_min) & (fr["l_iter"][quad] == n_walls)
    assert stopped.sum() >= 4
    assert (fr["l_blend"][quad][stopped] == n_walls).all()
    assert (fr["l_iter"][quad] == e - s).sum() >= 32  # most of the quadrant goes to the end of the list
    # the needle: the FP32 exponent bound fails (decided in FP64 only)
    ca, cb, cc = pre["conic"][needle]
    _, _, a1, a2 = principal_axes(np.float64(H * ca), np.float64(H * cb), np.float64(H * cc))
    _, ok = bound(np.float64(a1), np.float64(a2), math.log2(pre["opacity"][needle]))
    assert not bool(ok)
    # Gaussian 0 reaches every stopped pixel
    jj, ii = np.nonzero(stopped)
    dx, dy = pre["x"][0] - ii, pre["y"][0] - jj
    c0 = pre["conic"][0]
    a0 = pre["opacity"][0] * np.exp(-0.5 * (c0[0] * dx * dx + 2 * c0[1] * dx * dy + c0[2] * dy * dy))
    assert (a0 >= prm.alpha_low).all()
    assert min(fr["t_margin"].min(), fr["alpha_margin"].min()) > 1e-6


def test_empty_box_meets_no_sub_block():
    """The blend kernels give list positions past a list's end the box
    lo = 65535, hi = 0 on both axes (packed lo | hi << 16), and test a box
    against the four 4 x 4 sub-blocks of the quadrant at (qx0, qy0) as
    lo <= q0 + 3 + 4 c and hi >= q0 + 4 c per axis. Over every quadrant origin
    an image of up to 65535 pixels has, that box meets none; the box
    lo = 1, hi = 0 meets sub-block 0 of the first quadrant, which is what sent
    the top-left pixels phantom copies of a tile's last entry."""
    q0 = np.arange(0, 65536, 8, dtype=np.int64)

    def meets(lo, hi):
        return np.stack([(lo <= q0 + 3 + 4 * c) & (hi >= q0 + 4 * c) for c in (0, 1)])

    assert not meets(0xffff, 0).any()
    hit = meets(1, 0)
    assert hit[0, 0] and hit.sum() == 1
