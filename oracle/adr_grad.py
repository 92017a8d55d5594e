"""FP64 CPU oracle of the gradient of the AdR-Gaussian forward rasterizer.

TEST INFRASTRUCTURE. Only the tests may import this module. It shares no code
with the HIP library.

What it computes: for a scalar loss L = sum over channels and pixels of
w[c, j, i] * image[c, j, i], the derivative of L with respect to every scene
input (means, log-scales, quaternions, opacity logits, SH coefficients).

How: the image is a piecewise smooth function of the inputs. Its pieces are
fixed by discrete decisions (which list entries each pixel blends, where it
stops), which the forward oracle takes in FP64. This module re-evaluates the
same definition on one piece with PyTorch FP64 tensors and differentiates it
by reverse-mode automatic differentiation:

* per Gaussian (Sec. 3.1, Eq. 1 and the readings of the forward oracle):
  Sigma = R S S^T R^T, the EWA projection Sigma' = J W Sigma W^T J^T + lowpass I
  with the clamped Jacobian, the conic Sigma'^-1, the projected centre, the
  opacity sigmoid and the SH colour max(0, sum k Y(v) + 1/2);
* per pixel (Eqs. 2-3): alpha_k = min(alpha_max, sigma exp(-1/2 d^T conic d))
  over the entries the forward examined, the blended ones (alpha >= alpha_low,
  decided by the forward oracle) composited front to back,
  C = sum_k c_k alpha_k T_k + T_final bg.

The clamps are part of the definition: a clamped alpha (at alpha_max), a
clamped colour channel (at 0) or a clamped EWA slope pass no derivative to
their argument. The derivative is exact up to FP64 rounding wherever no
decision lies on its threshold; the tests pin it against central finite
differences of the forward oracle.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import adr_oracle as O


def _rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrices of quaternions (w, x, y, z), normalised first."""
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    r = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                     2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                     2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], dim=1)
    return r.reshape(-1, 3, 3)


def _sh_basis(degree: int, d: torch.Tensor) -> torch.Tensor:
    """Real orthonormal SH at unit directions d (N, 3): the basis of the
    forward oracle (index l*l + l + m, Condon-Shortley phase, polar angle from
    +z, azimuth atan2(y, x)), built from the associated Legendre recurrence."""
    x, y, z = d.unbind(1)
    ph = torch.atan2(y, x)
    s = torch.sqrt(torch.clamp(1.0 - z * z, min=0.0))
    p = {}
    pmm = torch.ones_like(z)
    for m in range(degree + 1):
        if m > 0:
            pmm = -(2 * m - 1) * s * pmm
        p[(m, m)] = pmm
        if m + 1 <= degree:
            p[(m + 1, m)] = z * (2 * m + 1) * pmm
        for l in range(m + 2, degree + 1):
            p[(l, m)] = ((2 * l - 1) * z * p[(l - 1, m)] - (l + m - 1) * p[(l - 2, m)]) / (l - m)
    cols = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            n_lm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m > 0:
                cols.append(math.sqrt(2.0) * n_lm * p[(l, am)] * torch.cos(am * ph))
            elif m == 0:
                cols.append(n_lm * p[(l, 0)])
            else:
                cols.append(math.sqrt(2.0) * n_lm * p[(l, am)] * torch.sin(am * ph))
    return torch.stack(cols, dim=1)


def _preprocess(means, log_scales, quats, logits, sh, degree, cam, params: O.Params):
    """Per-Gaussian projected centre, conic, opacity and colour (the forward
    oracle's preprocess, as differentiable tensors)."""
    w2c = torch.as_tensor(np.asarray(cam.world_to_cam, dtype=np.float64))
    rot, trans = w2c[:, :3], w2c[:, 3]
    p = means @ rot.T + trans[None, :]
    z = p[:, 2]
    zs = torch.where(z > cam.near, z, torch.ones_like(z))
    scale = torch.exp(log_scales)
    m = _rotmat(quats) * scale[:, None, :]
    sigma3 = m @ m.transpose(1, 2)
    fx, fy = float(cam.fx), float(cam.fy)
    lim_x = params.ewa_clamp * (cam.width / 2.0) / fx
    lim_y = params.ewa_clamp * (cam.height / 2.0) / fy
    xt = zs * torch.clamp(p[:, 0] / zs, -lim_x, lim_x)
    yt = zs * torch.clamp(p[:, 1] / zs, -lim_y, lim_y)
    zero = torch.zeros_like(zs)
    jac = torch.stack([torch.stack([fx / zs, zero, -fx * xt / (zs * zs)], 1),
                       torch.stack([zero, fy / zs, -fy * yt / (zs * zs)], 1)], 1)
    tm = jac @ rot
    cov2 = tm @ sigma3 @ tm.transpose(1, 2)
    a = cov2[:, 0, 0] + params.lowpass
    b = cov2[:, 0, 1]
    c = cov2[:, 1, 1] + params.lowpass
    det = a * c - b * b
    det = torch.where(det > 0, det, torch.ones_like(det))
    conic = torch.stack([c / det, -b / det, a / det], 1)
    x = fx * p[:, 0] / zs + cam.cx - 0.5
    y = fy * p[:, 1] / zs + cam.cy - 0.5
    opacity = torch.sigmoid(logits)
    cam_pos = torch.as_tensor(O.camera_position(cam))
    v = means - cam_pos[None, :]
    v = v / v.norm(dim=1, keepdim=True)
    k = (degree + 1) ** 2
    ybasis = _sh_basis(degree, v)
    color = torch.clamp(torch.einsum("nk,nkc->nc", ybasis, sh[:, :k, :]) + 0.5, min=0.0)
    return x, y, conic, opacity, color


def render_grad(scene, cam, params: O.Params, dl_dimage, fwd: dict | None = None, dl_dload=None,
                tiles=None) -> dict:
    """Gradient of L = sum(dl_dimage * image) + sum(dl_dload * l_blend) with
    respect to the scene inputs, where the per-pixel load l_blend (Eq. 12) is
    taken through the surrogate sum of the blended alphas (slope 1 per blended
    entry; the paper does not say how the integer load is differentiated).

    dl_dimage: (3, H, W). fwd: the forward oracle's render_frame result for the
    same inputs (computed here when absent); its sorted lists, tile ranges and
    per-pixel l_iter fix the piece. tiles: when given, only these tiles' terms
    of L are formed; the weights must vanish on every other tile (their terms
    are then exactly zero, so the gradient is the same), and fwd needs l_iter
    only there. Returns float64 arrays shaped like the scene arrays, plus the
    loss value.
    """
    if fwd is None:
        fwd = O.render_frame(scene, cam, params)
    leaf = {k: torch.tensor(np.asarray(getattr(scene, k), dtype=np.float64), requires_grad=True)
            for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    x, y, conic, opacity, color = _preprocess(leaf["means"], leaf["log_scales"], leaf["quats"],
                                              leaf["opacity_logits"], leaf["sh"], scene.sh_degree, cam, params)
    w = torch.as_tensor(np.asarray(dl_dimage, dtype=np.float64))
    wl = None if dl_dload is None else torch.as_tensor(np.asarray(dl_dload, dtype=np.float64))
    bg = torch.as_tensor(np.asarray(params.background, dtype=np.float64))
    values = np.asarray(fwd["values"], dtype=np.int64)
    ranges = np.asarray(fwd["ranges"], dtype=np.int64)
    l_iter = np.asarray(fwd["l_iter"], dtype=np.int64)
    tx_n, ty_n = O.n_tiles(cam)
    tile_list = range(tx_n * ty_n) if tiles is None else [int(t) for t in tiles]
    if tiles is not None:
        keep = np.zeros((ty_n * O.TILE, tx_n * O.TILE), dtype=bool)
        for t in tile_list:
            keep[(t // tx_n) * O.TILE:(t // tx_n + 1) * O.TILE, (t % tx_n) * O.TILE:(t % tx_n + 1) * O.TILE] = True
        keep = keep[:cam.height, :cam.width]
        assert not np.any(np.asarray(dl_dimage)[:, ~keep]), "weights outside the given tiles"
        assert dl_dload is None or not np.any(np.asarray(dl_dload)[~keep]), "load weights outside the given tiles"
    loss = torch.zeros((), dtype=torch.float64)
    for t in tile_list:
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        tx, ty = t % tx_n, t // tx_n
        xs = np.arange(tx * O.TILE, min((tx + 1) * O.TILE, cam.width))
        ys = np.arange(ty * O.TILE, min((ty + 1) * O.TILE, cam.height))
        jj, ii = np.meshgrid(ys, xs, indexing="ij")
        ii, jj = ii.ravel(), jj.ravel()
        wt = w[:, jj, ii].T  # (npx, 3)
        if e <= s:
            loss = loss + (wt * bg[None, :]).sum()  # T = 1: the background alone
            continue
        g = torch.as_tensor(values[s:e])
        n_ex = torch.as_tensor(l_iter[jj, ii])  # entries each pixel examined
        dx = x[g][None, :] - torch.as_tensor(ii, dtype=torch.float64)[:, None]
        dy = y[g][None, :] - torch.as_tensor(jj, dtype=torch.float64)[:, None]
        cg = conic[g]
        power = -0.5 * (cg[:, 0] * dx * dx + 2.0 * cg[:, 1] * dx * dy + cg[:, 2] * dy * dy)
        alpha = torch.minimum(torch.full_like(power, params.alpha_max), opacity[g][None, :] * torch.exp(power))
        pos = torch.arange(e - s)[None, :]
        blend = (pos < n_ex[:, None]) & (alpha.detach() >= params.alpha_low)
        a = torch.where(blend, alpha, torch.zeros_like(alpha))
        one_minus = 1.0 - a
        t_after = torch.cumprod(one_minus, dim=1)
        t_before = torch.cat([torch.ones_like(t_after[:, :1]), t_after[:, :-1]], dim=1)
        wgt = a * t_before  # (npx, L)
        c_pix = wgt @ color[g]  # (npx, 3)
        t_fin = t_after[:, -1]
        out = c_pix + t_fin[:, None] * bg[None, :]
        loss = loss + (wt * out).sum()
        if wl is not None:
            loss = loss + (wl[jj, ii] * a.sum(dim=1)).sum()  # sum of blended alphas per pixel
    grads = torch.autograd.grad(loss, [leaf[k] for k in ("means", "log_scales", "quats", "opacity_logits", "sh")],
                                allow_unused=True)
    res = {}
    for k, gval in zip(("means", "log_scales", "quats", "opacity_logits", "sh"), grads):
        res[k] = np.zeros(leaf[k].shape) if gval is None else gval.detach().numpy()
    res["loss"] = float(loss.detach())
    return res


def blended_alpha_sum(scene, cam, params: O.Params) -> np.ndarray:
    """Per-pixel sum of the alphas of the entries each pixel blends (the load
    surrogate), from the forward oracle's decisions, in NumPy FP64."""
    fr = O.render_frame(scene, cam, params)
    pre = fr["pre"]
    out = np.zeros((cam.height, cam.width))
    tx_n, ty_n = O.n_tiles(cam)
    for t in range(tx_n * ty_n):
        s, e = int(fr["ranges"][t, 0]), int(fr["ranges"][t, 1])
        if e <= s:
            continue
        tx, ty = t % tx_n, t // tx_n
        for j in range(ty * O.TILE, min((ty + 1) * O.TILE, cam.height)):
            for i in range(tx * O.TILE, min((tx + 1) * O.TILE, cam.width)):
                n_ex = int(fr["l_iter"][j, i])
                g = np.asarray(fr["values"][s:s + n_ex], dtype=np.int64)
                dx, dy = pre["x"][g] - i, pre["y"][g] - j
                con = pre["conic"][g]
                power = -0.5 * (con[:, 0] * dx * dx + 2.0 * con[:, 1] * dx * dy + con[:, 2] * dy * dy)
                a = np.minimum(params.alpha_max, pre["opacity"][g] * np.exp(power))
                out[j, i] = float(a[a >= params.alpha_low].sum())
    return out


def loss_of(scene, cam, params: O.Params, dl_dimage) -> float:
    """L = sum(dl_dimage * image) from the forward oracle (FP64)."""
    img = O.render_frame(scene, cam, params)["image"]
    return float(np.sum(np.asarray(dl_dimage, dtype=np.float64) * img))
