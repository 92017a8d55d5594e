"""FP64 CPU oracle of the AdR-Gaussian forward rasterizer (arXiv 2409.08669).

TEST INFRASTRUCTURE. Only the tests, the smoke check of the entry module and the
CPU-baseline leg of the benchmark may import this module. It shares no code,
constants or helpers with the HIP library; the two meet only in the seeded
inputs of the ``synth`` package.

What it computes, in the paper's order (Sec. 3.2, the six-stage pipeline):

1. Preprocess, one Gaussian at a time (Sec. 3.1, Eq. 1; Sec. 4.2-4.3, Eqs. 5-11):
   3D covariance from scale and rotation, EWA projection to the screen-space
   covariance Sigma', its inverse (the conic), its larger eigenvalue, the
   "99% confidence" radius r_o = 3 sqrt(lambda'_max), and per cull mode the
   radii that bound the pixels a Gaussian may touch:
     3-sigma : r_x = r_y = r_o                                   (baseline)
     adaptive: r = min(sqrt(2 lambda'_max ln(sigma/alpha_low)), r_o)  (Eqs. 7-8)
     AABB    : r_x = min(sqrt(2 Sigma'_X ln(sigma/alpha_low)), r_o),
               r_y = min(sqrt(2 Sigma'_Y ln(sigma/alpha_low)), r_o) (Eqs. 10-11)
   then the pixel rectangle, the 16x16 tile rectangle and tiles_touched.
2. InclusiveSum + DuplicateWithKeys: one (tile|depth) key per Gaussian-tile
   pair, Gaussian id as value.
3. SortPairs: ascending (key, Gaussian id).
4. IdentifyTileRanges: [first, last+1) per tile, (0, 0) when empty.
5. Render, one pixel at a time (Eqs. 2-3): front-to-back over the tile's list,
   alpha = min(alpha_max, sigma exp(-1/2 d^T Sigma'^-1 d)), skip below
   alpha_low, blend, stop once T < T_min (and, in the load-balancing mode, once
   the pixel has blended K Gaussians); per-pixel load counters (Eq. 12).
6. Load statistics: the population standard deviation of the per-pixel load
   over the H x W pixels (Eq. 13), computed exactly from integer sums.

Readings of the paper where it is silent (EWA Jacobian, low-pass, pixel
centres, SH basis, termination semantics, key layout) are listed next to the
code that takes them. Everything is float64; inputs are the float32 scene
arrays upcast exactly.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CULL_3SIGMA = 0
CULL_ADAPTIVE = 1
CULL_AABB = 2

TILE = 16  # 16 x 16 pixel tiles (Sec. 3.2)


@dataclasses.dataclass
class Params:
    cull: int = CULL_AABB
    alpha_low: float = 1.0 / 255.0   # minimum splatting opacity (Sec. 5.1.2)
    alpha_max: float = 0.99          # upper clamp of alpha (reading; not in the paper)
    t_min: float = 1e-4              # transmittance stop threshold (reading)
    lowpass: float = 0.3             # screen-space dilation added to Sigma' (reading)
    ewa_clamp: float = 1.3           # off-screen clamp of the EWA Jacobian, x tan(fov/2)
    background: tuple = (0.0, 0.0, 0.0)
    lb_cap: int = 0                  # load-balancing mode: stop after K blends (0 = off)


# ----------------------------------------------------------------------------
# Sec. 3.1: covariance from a scaling and a rotation
# ----------------------------------------------------------------------------

def quat_to_rotmat(q) -> np.ndarray:
    """Rotation matrices of quaternions (w, x, y, z), normalised first.

    Reading: the paper only says Sigma is decomposed into a scaling and a
    rotation (Sec. 3.1); the rotation is the usual active rotation of a unit
    quaternion, R v = q v q*.
    """
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def covariance_3d(log_scales, quats) -> np.ndarray:
    """Sigma = R S S^T R^T with S = diag(exp(log_scale)) (Sec. 3.1, Eq. 1)."""
    s = np.exp(np.asarray(log_scales, dtype=np.float64))
    r = quat_to_rotmat(quats)
    m = r * s[..., None, :]  # R @ diag(s)
    return m @ np.swapaxes(m, -1, -2)


# ----------------------------------------------------------------------------
# SH colour (Sec. 3.1 names SH as the colour representation; basis is a reading)
# ----------------------------------------------------------------------------

def _assoc_legendre(lmax: int, x: np.ndarray) -> dict:
    """P_l^m(x), 0 <= m <= l <= lmax, with the Condon-Shortley phase (-1)^m,
    by the standard three-term recurrence in l."""
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    out = {}
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = -(2 * m - 1) * s * pmm
        out[(m, m)] = pmm
        if m + 1 <= lmax:
            out[(m + 1, m)] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            out[(l, m)] = ((2 * l - 1) * x * out[(l - 1, m)] - (l + m - 1) * out[(l - 2, m)]) / (l - m)
    return out


def sh_basis(degree: int, dirs) -> np.ndarray:
    """Real orthonormal spherical harmonics at unit directions, (N, (d+1)^2).

    Reading (the paper does not give the basis): coefficient index l*l + l + m;
    Y_l^m = sqrt(2) N_lm P_l^m(cos th) cos(m ph) for m > 0, N_l0 P_l(cos th) for
    m = 0 and sqrt(2) N_l|m| P_l^|m|(cos th) sin(|m| ph) for m < 0, where
    N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m carries the Condon-Shortley
    phase, th is the polar angle from +z and ph = atan2(y, x).
    """
    d = np.asarray(dirs, dtype=np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    ph = np.arctan2(y, x)
    p = _assoc_legendre(degree, z)
    out = np.empty((d.shape[0], (degree + 1) ** 2))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            n_lm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m > 0:
                v = math.sqrt(2.0) * n_lm * p[(l, am)] * np.cos(am * ph)
            elif m == 0:
                v = n_lm * p[(l, 0)]
            else:
                v = math.sqrt(2.0) * n_lm * p[(l, am)] * np.sin(am * ph)
            out[:, l * l + l + m] = v
    return out


def camera_position(cam) -> np.ndarray:
    r = np.asarray(cam.world_to_cam, dtype=np.float64)[:, :3]
    t = np.asarray(cam.world_to_cam, dtype=np.float64)[:, 3]
    return -r.T @ t


def sh_to_rgb(sh, degree: int, means, cam) -> np.ndarray:
    """c = max(0, sum_lm k_lm Y_lm(v) + 1/2) per channel, v the unit direction
    from the camera centre to the Gaussian centre (reading)."""
    mu = np.asarray(means, dtype=np.float64)
    v = mu - camera_position(cam)[None, :]
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    y = sh_basis(degree, v)
    k = np.asarray(sh, dtype=np.float64)[:, : (degree + 1) ** 2, :]
    return np.maximum(0.0, np.einsum("nk,nkc->nc", y, k) + 0.5)


# ----------------------------------------------------------------------------
# Stage 1: Preprocess (Sec. 3.2 stage 1; Sec. 4.2 and 4.3)
# ----------------------------------------------------------------------------

def preprocess(scene, cam, params: Params) -> dict:
    """Per-Gaussian projection, conic, eigenvalue, 3-sigma radius and colour.

    EWA (Sec. 3.1 cites EWA without the formula) is read as the local affine
    approximation of the perspective map at the camera-space centre p:
      J = [[fx/z, 0, -fx x~/z^2], [0, fy/z, -fy y~/z^2]],
    with x~ = z clamp(p_x/z, +-ewa_clamp (W/2)/fx) and likewise y~, and
      Sigma' = J W Sigma W^T J^T + lowpass I  (W = world-to-camera rotation).
    Pixel (i, j) covers [i, i+1) x [j, j+1); centres are moved to integers, so
    the projected centre is x = fx p_x/z + cx - 1/2, y = fy p_y/z + cy - 1/2.
    A Gaussian with z <= near is invisible.
    """
    mu = np.asarray(scene.means, dtype=np.float64)
    w2c = np.asarray(cam.world_to_cam, dtype=np.float64)
    rot, trans = w2c[:, :3], w2c[:, 3]
    p = mu @ rot.T + trans[None, :]
    z = p[:, 2]
    valid = z > cam.near
    zs = np.where(valid, z, 1.0)  # keep the arithmetic finite for invisible rows

    sigma3 = covariance_3d(scene.log_scales, scene.quats)

    fx, fy = float(cam.fx), float(cam.fy)
    lim_x = params.ewa_clamp * (cam.width / 2.0) / fx
    lim_y = params.ewa_clamp * (cam.height / 2.0) / fy
    xt = zs * np.clip(p[:, 0] / zs, -lim_x, lim_x)
    yt = zs * np.clip(p[:, 1] / zs, -lim_y, lim_y)
    jac = np.zeros((mu.shape[0], 2, 3))
    jac[:, 0, 0] = fx / zs
    jac[:, 0, 2] = -fx * xt / (zs * zs)
    jac[:, 1, 1] = fy / zs
    jac[:, 1, 2] = -fy * yt / (zs * zs)
    tm = jac @ rot  # (N, 2, 3)
    cov2 = tm @ sigma3 @ np.swapaxes(tm, -1, -2)
    a = cov2[:, 0, 0] + params.lowpass
    b = cov2[:, 0, 1]
    c = cov2[:, 1, 1] + params.lowpass

    det = a * c - b * b
    # Reading: a degenerate projected covariance (det <= 0, possible only with
    # lowpass = 0) is not drawn.
    valid = valid & (det > 0)
    det = np.where(det > 0, det, 1.0)
    conic = np.stack([c / det, -b / det, a / det], axis=1)
    # Larger eigenvalue of Sigma' (the paper defers its formula to supplementary
    # material). mid + sqrt(mid^2 - det) equals mid + sqrt(((a - c)/2)^2 + b^2);
    # the second form has no cancellation, so it is accurate to a few ulp even
    # for nearly isotropic Sigma', where the first loses half the digits.
    mid = 0.5 * (a + c)
    lam_max = mid + np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    r_o = 3.0 * np.sqrt(lam_max)

    x = fx * p[:, 0] / zs + cam.cx - 0.5
    y = fy * p[:, 1] / zs + cam.cy - 0.5
    opacity = 1.0 / (1.0 + np.exp(-np.asarray(scene.opacity_logits, dtype=np.float64)))
    color = sh_to_rgb(scene.sh, scene.sh_degree, mu, cam)

    return dict(valid=valid, p=p, depth32=z.astype(np.float32), x=x, y=y,
                cov2=np.stack([a, b, c], axis=1), conic=conic, lam_max=lam_max,
                r_o=r_o, opacity=opacity, color=color)


def cull_radii(pre: dict, params: Params):
    """(keep, r_x, r_y) per cull mode (Eqs. 7-8 and 10-11).

    Reading: with opacity < alpha_low the logarithm is negative and the
    Gaussian can reach no pixel (alpha <= opacity < alpha_low), so the adaptive
    and AABB modes give it no pairs; the 3-sigma baseline keeps it.
    """
    valid = pre["valid"]
    r_o = pre["r_o"]
    if params.cull == CULL_3SIGMA:
        return valid.copy(), r_o.copy(), r_o.copy()
    keep = valid & (pre["opacity"] >= params.alpha_low)
    lnr = np.log(np.where(keep, pre["opacity"], 1.0) / params.alpha_low)
    lnr = np.where(keep, lnr, 0.0)
    if params.cull == CULL_ADAPTIVE:
        r = np.minimum(np.sqrt(2.0 * pre["lam_max"] * lnr), r_o)
        return keep, r, r.copy()
    if params.cull == CULL_AABB:
        rx = np.minimum(np.sqrt(2.0 * pre["cov2"][:, 0] * lnr), r_o)
        ry = np.minimum(np.sqrt(2.0 * pre["cov2"][:, 2] * lnr), r_o)
        return keep, rx, ry
    raise ValueError("unknown cull mode")


def tile_rects(pre: dict, cam, params: Params) -> dict:
    """Pixel and tile rectangles and tiles_touched.

    Reading of "the circumscribed square" (Sec. 4.2): the pixels whose centres
    lie in [x - r_x, x + r_x] x [y - r_y, y + r_y], clipped to the image, i.e.
    i in [max(ceil(x - r_x), 0), min(floor(x + r_x), W - 1)]; a tile is touched
    when it holds one of those pixels.
    """
    keep, rx, ry = cull_radii(pre, params)
    w, h = cam.width, cam.height
    x, y = pre["x"], pre["y"]
    with np.errstate(invalid="ignore"):
        i_lo = np.clip(np.maximum(np.ceil(x - rx), 0.0), 0, w)
        i_hi = np.clip(np.minimum(np.floor(x + rx), w - 1.0), -1, w - 1)
        j_lo = np.clip(np.maximum(np.ceil(y - ry), 0.0), 0, h)
        j_hi = np.clip(np.minimum(np.floor(y + ry), h - 1.0), -1, h - 1)
    i_lo, i_hi = i_lo.astype(np.int64), i_hi.astype(np.int64)
    j_lo, j_hi = j_lo.astype(np.int64), j_hi.astype(np.int64)
    nonempty = keep & (i_lo <= i_hi) & (j_lo <= j_hi)
    tx_lo, tx_hi = i_lo // TILE, np.maximum(i_hi, 0) // TILE
    ty_lo, ty_hi = j_lo // TILE, np.maximum(j_hi, 0) // TILE
    touched = np.where(nonempty, (tx_hi - tx_lo + 1) * (ty_hi - ty_lo + 1), 0).astype(np.uint32)
    return dict(keep=keep, r_x=rx, r_y=ry, i_lo=i_lo, i_hi=i_hi, j_lo=j_lo, j_hi=j_hi,
                tx_lo=tx_lo, tx_hi=tx_hi, ty_lo=ty_lo, ty_hi=ty_hi,
                nonempty=nonempty, tiles_touched=touched)


def n_tiles(cam):
    tx = (cam.width + TILE - 1) // TILE
    ty = (cam.height + TILE - 1) // TILE
    return tx, ty


# ----------------------------------------------------------------------------
# Stages 2-5: InclusiveSum, DuplicateWithKeys, SortPairs, IdentifyTileRanges
# ----------------------------------------------------------------------------

def duplicate_and_sort(pre: dict, rects: dict, cam):
    """Keys and values in sorted order.

    key = (tile_id << 32) | bits(depth32), tile_id = ty * TX + tx (reading: the
    paper gives no key layout); the value is the Gaussian id. Pairs are emitted
    Gaussian by Gaussian, row-major over the tile rectangle, at the offsets of
    the inclusive sum of tiles_touched, and sorted ascending by (key, id).
    """
    tx_n, _ = n_tiles(cam)
    touched = rects["tiles_touched"].astype(np.int64)
    offsets = np.cumsum(touched)  # InclusiveSum
    n_pairs = int(offsets[-1]) if offsets.size else 0
    gids = np.repeat(np.arange(touched.size, dtype=np.int64), touched)
    start = offsets - touched
    k = np.arange(n_pairs, dtype=np.int64) - start[gids]
    width = (rects["tx_hi"] - rects["tx_lo"] + 1)[gids]
    tx = rects["tx_lo"][gids] + k % width
    ty = rects["ty_lo"][gids] + k // width
    tile = (ty * tx_n + tx).astype(np.uint64)
    dbits = pre["depth32"].view(np.uint32)[gids].astype(np.uint64)
    keys = (tile << np.uint64(32)) | dbits
    order = np.lexsort((gids, keys))
    return keys[order], gids[order].astype(np.uint32), offsets.astype(np.uint64)


def tile_ranges(keys_sorted, cam) -> np.ndarray:
    """ranges[t] = [first, last + 1) of the pairs of tile t; (0, 0) if none."""
    tx_n, ty_n = n_tiles(cam)
    t_all = np.arange(tx_n * ty_n, dtype=np.uint64)
    tiles = (np.asarray(keys_sorted, dtype=np.uint64) >> np.uint64(32))
    lo = np.searchsorted(tiles, t_all, side="left")
    hi = np.searchsorted(tiles, t_all, side="right")
    empty = lo == hi
    lo[empty] = 0
    hi[empty] = 0
    return np.stack([lo, hi], axis=1).astype(np.uint32)


# ----------------------------------------------------------------------------
# Stage 6: Render (Eqs. 2-3) and the per-pixel load (Eq. 12)
# ----------------------------------------------------------------------------

def _alpha(pre, g, dx, dy, params):
    ca, cb, cc = pre["conic"][g, 0], pre["conic"][g, 1], pre["conic"][g, 2]
    power = -0.5 * (ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy)
    return np.minimum(params.alpha_max, pre["opacity"][g] * np.exp(power))


def render_pixels(pre: dict, values, ranges, cam, params: Params, pix_i, pix_j) -> dict:
    """The per-pixel definition, one pixel at a time (pure Python loops; for
    sampled pixels and small images).

    For the pixel's tile, in list order: l_iter counts every entry examined;
    an entry with alpha < alpha_low is skipped; otherwise C += c alpha T,
    T *= 1 - alpha, l_blend += 1, and the pixel stops once T < t_min (reading:
    blend, then test) or, with lb_cap = K > 0, once l_blend = K.
    Also returns, per pixel, the smallest relative distance of any examined
    alpha to alpha_low and of any post-blend T to t_min (decision margins).
    """
    tx_n, _ = n_tiles(cam)
    bg = np.asarray(params.background, dtype=np.float64)
    pix_i = np.asarray(pix_i, dtype=np.int64)
    pix_j = np.asarray(pix_j, dtype=np.int64)
    n = pix_i.size
    img = np.zeros((n, 3))
    tf = np.ones(n)
    li = np.zeros(n, dtype=np.uint32)
    lb = np.zeros(n, dtype=np.uint32)
    am = np.full(n, np.inf)
    tm = np.full(n, np.inf)
    x, y, op, col, con = pre["x"], pre["y"], pre["opacity"], pre["color"], pre["conic"]
    for q in range(n):
        i, j = int(pix_i[q]), int(pix_j[q])
        t = (j // TILE) * tx_n + (i // TILE)
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        tt, cr, cg, cbl = 1.0, 0.0, 0.0, 0.0
        n_it = n_bl = 0
        amarg = tmarg = math.inf
        for k in range(s, e):
            g = int(values[k])
            n_it += 1
            dx, dy = x[g] - i, y[g] - j
            power = -0.5 * (con[g, 0] * dx * dx + 2.0 * con[g, 1] * dx * dy + con[g, 2] * dy * dy)
            a = min(params.alpha_max, op[g] * math.exp(power))
            amarg = min(amarg, abs(a / params.alpha_low - 1.0))
            if a < params.alpha_low:
                continue
            cr += col[g, 0] * a * tt
            cg += col[g, 1] * a * tt
            cbl += col[g, 2] * a * tt
            tt = tt * (1.0 - a)
            n_bl += 1
            tmarg = min(tmarg, abs(tt / params.t_min - 1.0))
            if tt < params.t_min:
                break
            if params.lb_cap > 0 and n_bl == params.lb_cap:
                break
        img[q] = (cr + tt * bg[0], cg + tt * bg[1], cbl + tt * bg[2])
        tf[q], li[q], lb[q], am[q], tm[q] = tt, n_it, n_bl, amarg, tmarg
    return dict(image=img, final_t=tf, l_iter=li, l_blend=lb, alpha_margin=am, t_margin=tm)


def render_image(pre: dict, values, ranges, cam, params: Params, tiles=None) -> dict:
    """The same per-pixel definition as render_pixels, evaluated for all the
    pixels of a tile at once (vectorised over pixels, sequential over the
    tile's list). ``tiles`` restricts the work to a subset of tile ids; pixels
    of other tiles are left at their initial values and flagged in ``done``."""
    w, h = cam.width, cam.height
    tx_n, ty_n = n_tiles(cam)
    bg = np.asarray(params.background, dtype=np.float64)
    img = np.zeros((3, h, w))
    tf = np.ones((h, w))
    li = np.zeros((h, w), dtype=np.uint32)
    lb = np.zeros((h, w), dtype=np.uint32)
    am = np.full((h, w), np.inf)
    tm = np.full((h, w), np.inf)
    done = np.zeros((h, w), dtype=bool)
    x, y, op, col, con = pre["x"], pre["y"], pre["opacity"], pre["color"], pre["conic"]
    tile_list = range(tx_n * ty_n) if tiles is None else tiles
    for t in tile_list:
        t = int(t)
        tx, ty = t % tx_n, t // tx_n
        xs = np.arange(tx * TILE, min(tx * TILE + TILE, w))
        ys = np.arange(ty * TILE, min(ty * TILE + TILE, h))
        jj, ii = np.meshgrid(ys, xs, indexing="ij")
        ii, jj = ii.ravel(), jj.ravel()
        npx = ii.size
        cacc = np.zeros((npx, 3))
        tt = np.ones(npx)
        n_it = np.zeros(npx, dtype=np.uint32)
        n_bl = np.zeros(npx, dtype=np.uint32)
        amarg = np.full(npx, np.inf)
        tmarg = np.full(npx, np.inf)
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        if e > s:
            g = np.asarray(values[s:e], dtype=np.int64)
            dx = x[g][None, :] - ii[:, None]
            dy = y[g][None, :] - jj[:, None]
            power = -0.5 * (con[g, 0] * dx * dx + 2.0 * con[g, 1] * dx * dy + con[g, 2] * dy * dy)
            alpha = np.minimum(params.alpha_max, op[g][None, :] * np.exp(power))
            active = np.ones(npx, dtype=bool)
            for k in range(g.size):
                a = alpha[:, k]
                n_it[active] += 1
                amarg[active] = np.minimum(amarg[active], np.abs(a[active] / params.alpha_low - 1.0))
                bl = active & (a >= params.alpha_low)
                if bl.any():
                    wgt = a[bl] * tt[bl]
                    cacc[bl] += col[g[k]][None, :] * wgt[:, None]
                    tt[bl] = tt[bl] * (1.0 - a[bl])
                    n_bl[bl] += 1
                    tmarg[bl] = np.minimum(tmarg[bl], np.abs(tt[bl] / params.t_min - 1.0))
                    stop = bl & (tt < params.t_min)
                    if params.lb_cap > 0:
                        stop |= bl & (n_bl == params.lb_cap)
                    active &= ~stop
                    if not active.any():
                        break
        out = cacc + tt[:, None] * bg[None, :]
        img[:, jj, ii] = out.T
        tf[jj, ii] = tt
        li[jj, ii] = n_it
        lb[jj, ii] = n_bl
        am[jj, ii] = amarg
        tm[jj, ii] = tmarg
        done[jj, ii] = True
    return dict(image=img, final_t=tf, l_iter=li, l_blend=lb, alpha_margin=am,
                t_margin=tm, done=done)


def render_frame(scene, cam, params: Params, tiles=None) -> dict:
    """All stages for one frame; returns every intermediate the HIP path can
    expose, plus the image and counters."""
    pre = preprocess(scene, cam, params)
    rects = tile_rects(pre, cam, params)
    keys, values, offsets = duplicate_and_sort(pre, rects, cam)
    ranges = tile_ranges(keys, cam)
    out = render_image(pre, values, ranges, cam, params, tiles=tiles)
    out.update(pre=pre, rects=rects, keys=keys, values=values, offsets=offsets,
               ranges=ranges, tiles_touched=rects["tiles_touched"], n_pairs=int(keys.size))
    return out


# ----------------------------------------------------------------------------
# Eq. 13 and image quality
# ----------------------------------------------------------------------------

def load_stats(load) -> tuple:
    """(mean, population std) of per-pixel loads over all H x W pixels (Eq. 13,
    reading: population std, pixels with zero load included). Exact: the sums
    are Python integers and the variance is (n S2 - S1^2) / n^2."""
    l = np.asarray(load).astype(np.int64).ravel()
    n = l.size
    s1 = int(l.sum())
    s2 = int((l * l).sum())
    mean = s1 / n
    var = (n * s2 - s1 * s1) / (n * n)
    return mean, math.sqrt(var)


def psnr(img, ref) -> float:
    """10 log10(1 / MSE) after clipping both images to [0, 1]."""
    a = np.clip(np.asarray(img, dtype=np.float64), 0.0, 1.0)
    b = np.clip(np.asarray(ref, dtype=np.float64), 0.0, 1.0)
    mse = float(np.mean((a - b) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(1.0 / mse)


# ----------------------------------------------------------------------------
# Independent cross-check of stages 2-5: no tiles lists, no radix keys
# ----------------------------------------------------------------------------

def brute_force_render(pre: dict, rects: dict, cam, params: Params, pix_i, pix_j) -> dict:
    """Each pixel blends, in ascending (depth32, id) order, every Gaussian whose
    tile rectangle contains the pixel's tile; the ordering uses Python's sorted
    on tuples and the per-pixel steps are those of render_pixels."""
    tx_n, _ = n_tiles(cam)
    nz = np.nonzero(rects["nonempty"])[0]
    depth = pre["depth32"]
    order = sorted(nz.tolist(), key=lambda g: (float(depth[g]), g))
    pix_i = np.asarray(pix_i, dtype=np.int64)
    pix_j = np.asarray(pix_j, dtype=np.int64)
    per_tile = {}
    for g in order:
        for ty in range(int(rects["ty_lo"][g]), int(rects["ty_hi"][g]) + 1):
            for tx in range(int(rects["tx_lo"][g]), int(rects["tx_hi"][g]) + 1):
                per_tile.setdefault(ty * tx_n + tx, []).append(g)
    # Build a flat list/range table from per-tile lists and reuse the pixel loop.
    tiles_total = n_tiles(cam)[0] * n_tiles(cam)[1]
    vals, rng = [], np.zeros((tiles_total, 2), dtype=np.uint32)
    for t in range(tiles_total):
        lst = per_tile.get(t, [])
        if lst:
            rng[t] = (len(vals), len(vals) + len(lst))
            vals.extend(lst)
    return render_pixels(pre, np.asarray(vals, dtype=np.uint32), rng, cam, params, pix_i, pix_j)
