"""FP64 CPU oracle of the 4D Gaussian rendering routine.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow, obviously correct
definition that the GPU path is checked against. Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never calls it. It shares no code with the HIP implementation.

Everything is written with plain PyTorch CPU ops in float64 so that the
gradient is torch autograd's exact derivative of this forward definition with
every discrete decision (culls, tile rectangle, alpha floor, early stop, sort
order) held fixed. The clamps (alpha <= 0.99, colour >= 0, the Jacobian's
off-screen clamp) are written with torch.clamp, so their derivative is zero on
the clamped side, as the definition requires.

Paper passages followed (Yang et al., "Real-time Photorealistic Dynamic Scene
Representation and Rendering with 4D Gaussian Splatting", ICLR 2024):
  * Sec. 3.1 Eq. (1): unnormalised Gaussian; Eqs. (3)-(4): EWA mean and
    covariance splatting; Eq. (2) alpha blending.
  * Sec. 3.2 Eqs. (5)-(6): time-conditioned blending, p_i(t) p_i(u,v|t).
  * Sec. 3.2 "Representation of 4D Gaussian": Sigma = R S S^T R^T with
    R = L(q_l) R(q_r) from the two printed 4x4 matrices.
  * Sec. 3.2: conditional mean/covariance of the slice at t, and the
    marginal p(t) = N(t; mu_4, Sigma_44).
  * Sec. 3.2 "4D spherindrical harmonics": Z_nl^m = cos(2 pi n t / T) Y_l^m.
  * Sec. 4.2: the temporal filter drops primitives with p(t) < 0.05.
Readings where the paper is silent are listed in CONVENTIONS below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

F64 = torch.float64
TILE = 16
# FP32 reach used by the parity margin policy: decisions closer than these to
# their threshold may be taken either way by a float32 implementation.
MARGIN_REL = 1e-5   # relative, for p(t), z, alpha floor, stop threshold
MARGIN_PX = 2e-3    # pixels, for footprint radius and tile-edge decisions
IMG_TOL = 1e-4      # image tolerance the flags are sized for

# Readings of points the paper leaves open (the same constants are restated,
# not shared, by the GPU path):
CONVENTIONS = dict(
    t_cull=0.05,          # Sec. 4.2: keep iff unnormalised p(t) >= 0.05
    near=0.2,             # camera-space z must exceed this
    lowpass=0.3,          # EWA screen-space dilation (px^2) added to Sigma_2d
    frustum_slack=1.3,    # Jacobian evaluated at x/z clamped to 1.3 x half-fov
    sigma_extent=3.0,     # footprint radius = ceil(3 sqrt(lambda_max))
    alpha_min=1.0 / 255.0,  # fragments with alpha below this are skipped
    alpha_max=0.99,       # alpha is clamped from above
    t_stop=1e-4,          # stop before a fragment that would drop T below this
    color_offset=0.5,     # colour = max(0, 0.5 + 4DSH sum)
)


# ---------------------------------------------------------------------------
# 4D covariance (Sec. 3.2, "Representation of 4D Gaussian")
# ---------------------------------------------------------------------------
def left_isoclinic(q: torch.Tensor) -> torch.Tensor:
    """The paper's L(q_l) for q_l = (a, b, c, d), entry by entry."""
    a, b, c, d = q.unbind(-1)
    rows = [[a, -b, -c, -d],
            [b, a, -d, c],
            [c, d, a, -b],
            [d, -c, b, a]]
    return torch.stack([torch.stack(r, -1) for r in rows], -2)


def right_isoclinic(q: torch.Tensor) -> torch.Tensor:
    """The paper's R(q_r) for q_r = (p, q, r, s), entry by entry."""
    p, q_, r, s = q.unbind(-1)
    rows = [[p, -q_, -r, -s],
            [q_, p, s, -r],
            [r, -s, p, q_],
            [s, r, -q_, p]]
    return torch.stack([torch.stack(r_, -1) for r_ in rows], -2)


def rotation_4d(q_left: torch.Tensor, q_right: torch.Tensor) -> torch.Tensor:
    """R = L(q_l) R(q_r) with both quaternions normalised first."""
    ql = q_left / q_left.norm(dim=-1, keepdim=True)
    qr = q_right / q_right.norm(dim=-1, keepdim=True)
    return left_isoclinic(ql) @ right_isoclinic(qr)


def covariance_4d(log_scales4: torch.Tensor, q_left: torch.Tensor,
                  q_right: torch.Tensor) -> torch.Tensor:
    """Sigma = R S S^T R^T, S = diag(exp(log_scales))."""
    rot = rotation_4d(q_left, q_right)
    s = torch.exp(log_scales4)
    m = rot * s.unsqueeze(-2)          # R S
    return m @ m.transpose(-1, -2)


# ---------------------------------------------------------------------------
# Slicing at time t (Sec. 3.2, conditional 3D Gaussian and marginal p(t))
# ---------------------------------------------------------------------------
def temporal_marginal(mu_t: torch.Tensor, sigma_tt: torch.Tensor, t: float) -> torch.Tensor:
    """Unnormalised marginal exp(-(t - mu_t)^2 / (2 Sigma_44)), peak 1.

    Eq. (1)'s unnormalised Gaussian; the paper does not distinguish it from
    the normalised density (Sec. 3.1), and the filter threshold of Sec. 4.2 is
    applied to this quantity."""
    return torch.exp(-0.5 * (t - mu_t) ** 2 / sigma_tt)


def slice_at(mean4: torch.Tensor, cov4: torch.Tensor, t: float):
    """Conditional mean and covariance of (x,y,z) given t."""
    s13_4 = cov4[..., :3, 3]
    s44 = cov4[..., 3, 3]
    mu_c = mean4[..., :3] + s13_4 / s44.unsqueeze(-1) * (t - mean4[..., 3]).unsqueeze(-1)
    cov_c = cov4[..., :3, :3] - s13_4.unsqueeze(-1) * s13_4.unsqueeze(-2) / s44[..., None, None]
    return mu_c, cov_c


# ---------------------------------------------------------------------------
# 4D spherindrical harmonics (Sec. 3.2)
# ---------------------------------------------------------------------------
def real_sh(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Orthonormal real spherical harmonics up to `degree`, Condon-Shortley
    phase kept, index l*l + l + m. Built from the associated-Legendre
    recurrence written as polynomials in the unit vector (x, y, z):

      Y_l^0      = K_l^0 Q_l^0(z)
      Y_l^{+m}   = sqrt(2) K_l^m Q_l^m(z) Re((x + i y)^m)
      Y_l^{-m}   = sqrt(2) K_l^m Q_l^m(z) Im((x + i y)^m)

    with Q_l^m = P_l^m / (1 - z^2)^{m/2} (P including (-1)^m) and
    K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)."""
    x, y, z = dirs.unbind(-1)
    nb = (degree + 1) ** 2
    out = [None] * nb
    # Re/Im of (x + i y)^m
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    for m in range(0, degree + 1):
        # Q_m^m = (-1)^m (2m-1)!!
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        q_prev2 = None
        q_prev = torch.full_like(z, ((-1.0) ** m) * dfact)
        for l in range(m, degree + 1):
            if l == m:
                q_l = q_prev
            elif l == m + 1:
                q_l = z * (2 * m + 1) * q_prev
                q_prev2, q_prev = q_prev, q_l
            else:
                q_l = ((2 * l - 1) * z * q_prev - (l + m - 1) * q_prev2) / (l - m)
                q_prev2, q_prev = q_prev, q_l
            kf = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[l * l + l] = kf * q_l
            else:
                out[l * l + l + m] = math.sqrt(2.0) * kf * q_l * re[m]
                out[l * l + l - m] = math.sqrt(2.0) * kf * q_l * im[m]
    return torch.stack(out, -1)


def fourier_cos(dt: torch.Tensor, order: int, period: float) -> torch.Tensor:
    """cos(2 pi n dt / T) for n = 0..order."""
    n = torch.arange(order + 1, dtype=dt.dtype)
    return torch.cos(2.0 * math.pi * n * dt.unsqueeze(-1) / period)


def color_4dsh(coeffs: torch.Tensor, dirs: torch.Tensor, dt: torch.Tensor,
               sh_degree: int, t_order: int, period: float):
    """c = max(0, 0.5 + sum_n cos(2 pi n dt/T) sum_lm k[n,lm] Y_lm(d)).

    coeffs: [G, K, 3] with K = (t_order+1)(sh_degree+1)^2, k index
    n*(sh_degree+1)^2 + lm. Returns (clamped colour, raw colour)."""
    nb = (sh_degree + 1) ** 2
    y = real_sh(dirs, sh_degree)                    # [G, nb]
    f = fourier_cos(dt, t_order, period)            # [G, Nt+1]
    basis = (f.unsqueeze(-1) * y.unsqueeze(-2)).reshape(y.shape[0], (t_order + 1) * nb)
    raw = CONVENTIONS["color_offset"] + (basis.unsqueeze(-1) * coeffs).sum(-2)
    return torch.clamp(raw, min=0.0), raw


# ---------------------------------------------------------------------------
# Per-view preprocessing: slice, project (Eqs. 3-4), footprint, colour
# ---------------------------------------------------------------------------
@dataclass
class OCamera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    rot: torch.Tensor     # [3,3] world -> camera
    trans: torch.Tensor   # [3]
    center: torch.Tensor  # [3]

    @property
    def tiles_x(self):
        return (self.width + TILE - 1) // TILE

    @property
    def tiles_y(self):
        return (self.height + TILE - 1) // TILE


def to_ocamera(cam) -> OCamera:
    w2c = torch.as_tensor(np.asarray(cam.world_to_cam, dtype=np.float64))
    return OCamera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy),
                   float(cam.cx), float(cam.cy), w2c[:, :3], w2c[:, 3],
                   torch.as_tensor(np.asarray(cam.center, dtype=np.float64)))


def params_from_scene(scene, requires_grad: bool = False) -> Dict[str, torch.Tensor]:
    p = {
        "means4": torch.as_tensor(np.asarray(scene.means4, np.float64)),
        "log_scales4": torch.as_tensor(np.asarray(scene.log_scales4, np.float64)),
        "q_left": torch.as_tensor(np.asarray(scene.q_left, np.float64)),
        "q_right": torch.as_tensor(np.asarray(scene.q_right, np.float64)),
        "opacity_logit": torch.as_tensor(np.asarray(scene.opacity_logit, np.float64)),
        "coeffs": torch.as_tensor(np.asarray(scene.coeffs, np.float64)),
    }
    if requires_grad:
        for v in p.values():
            v.requires_grad_(True)
    return p


def preprocess(params: Dict[str, torch.Tensor], cam: OCamera, t: float,
               sh_degree: int, t_order: int, period: float = 1.0) -> Dict[str, torch.Tensor]:
    """All per-primitive quantities of one view at time t (differentiable),
    plus the FP64 margin of every discrete decision."""
    C = CONVENTIONS
    cov4 = covariance_4d(params["log_scales4"], params["q_left"], params["q_right"])
    mean4 = params["means4"]
    s44 = cov4[:, 3, 3]
    pt = temporal_marginal(mean4[:, 3], s44, t)
    mu_c, cov_c = slice_at(mean4, cov4, t)

    p_cam = mu_c @ cam.rot.T + cam.trans
    x, y, z = p_cam.unbind(-1)
    u = cam.fx * x / z + cam.cx
    v = cam.fy * y / z + cam.cy
    lim_x = C["frustum_slack"] * (cam.width / 2.0) / cam.fx
    lim_y = C["frustum_slack"] * (cam.height / 2.0) / cam.fy
    xi = torch.clamp(x / z, -lim_x, lim_x)
    eta = torch.clamp(y / z, -lim_y, lim_y)
    zero = torch.zeros_like(z)
    jac = torch.stack([torch.stack([cam.fx / z, zero, -cam.fx * xi / z], -1),
                       torch.stack([zero, cam.fy / z, -cam.fy * eta / z], -1)], -2)
    cov_cam = cam.rot @ cov_c @ cam.rot.T
    cov2 = jac @ cov_cam @ jac.transpose(-1, -2)
    a2 = cov2[:, 0, 0] + C["lowpass"]
    b2 = cov2[:, 0, 1]
    c2 = cov2[:, 1, 1] + C["lowpass"]
    det = a2 * c2 - b2 * b2
    conic = torch.stack([c2 / det, -b2 / det, a2 / det], -1)

    # footprint: integer radius and half-open tile rectangle (no gradient)
    with torch.no_grad():
        mid = 0.5 * (a2 + c2)
        lam = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
        ext = C["sigma_extent"] * torch.sqrt(lam)
        rad = torch.ceil(ext)
        x0 = torch.clamp(torch.floor((u - rad) / TILE), 0, cam.tiles_x)
        x1 = torch.clamp(torch.floor((u + rad) / TILE) + 1, 0, cam.tiles_x)
        y0 = torch.clamp(torch.floor((v - rad) / TILE), 0, cam.tiles_y)
        y1 = torch.clamp(torch.floor((v + rad) / TILE) + 1, 0, cam.tiles_y)
        keep_t = pt >= C["t_cull"]
        keep_z = z > C["near"]
        keep_r = (x1 > x0) & (y1 > y0)
        active = keep_t & keep_z & keep_r
        # decision margins (FP64): small values flag decisions that FP32 may flip
        m_t = (pt - C["t_cull"]).abs() / C["t_cull"]
        m_z = (z - C["near"]).abs() / C["near"]
        frac = ext - torch.floor(ext)
        m_rad = torch.minimum(frac, 1.0 - frac)          # px, distance of 3 sqrt(lam) to an integer
        m_jac = torch.minimum((x.abs() / z - lim_x).abs() / lim_x, (y.abs() / z - lim_y).abs() / lim_y)
        # The rectangle FP32 may legitimately produce lies between a "sure"
        # rectangle (every marginal decision taken the narrow way) and a
        # "maybe" rectangle (taken the wide way); tiles between the two are
        # uncertain for this primitive.
        mpx = MARGIN_PX
        near_int = (ext - torch.round(ext)).abs() < mpx
        rad_lo = torch.where(near_int, torch.round(ext), rad)
        rad_hi = torch.where(near_int, torch.round(ext) + 1.0, rad)

        def rect_of(rr, grow):
            e = mpx if grow else -mpx
            ax0 = torch.clamp(torch.floor((u - e - rr) / TILE), 0, cam.tiles_x)
            ax1 = torch.clamp(torch.floor((u + e + rr) / TILE) + 1, 0, cam.tiles_x)
            ay0 = torch.clamp(torch.floor((v - e - rr) / TILE), 0, cam.tiles_y)
            ay1 = torch.clamp(torch.floor((v + e + rr) / TILE) + 1, 0, cam.tiles_y)
            return torch.stack([ax0, ay0, ax1, ay1], -1).long()
        rect_maybe = rect_of(rad_hi, True)
        rect_sure = rect_of(rad_lo, False)
        sure_alive = (pt >= C["t_cull"] * (1 + MARGIN_REL)) & (z > C["near"] * (1 + MARGIN_REL))
        maybe_alive = (pt >= C["t_cull"] * (1 - MARGIN_REL)) & (z > C["near"] * (1 - MARGIN_REL))
        rect_sure = torch.where(sure_alive[:, None], rect_sure, torch.zeros_like(rect_sure))
        rect_maybe = torch.where(maybe_alive[:, None], rect_maybe, torch.zeros_like(rect_maybe))

    dirs = mu_c - cam.center
    dirs = dirs / dirs.norm(dim=-1, keepdim=True)
    color, color_raw = color_4dsh(params["coeffs"], dirs, t - mean4[:, 3], sh_degree, t_order, period)
    opac = torch.sigmoid(params["opacity_logit"]) * pt
    return dict(u=u, v=v, z=z, conic=conic, opac=opac, color=color, color_raw=color_raw,
                pt=pt, mu_c=mu_c, cov_c=cov_c, cov4=cov4, cov2=torch.stack([a2, b2, c2], -1),
                radius=rad, rect=torch.stack([x0, y0, x1, y1], -1).long(), active=active,
                rect_sure=rect_sure, rect_maybe=rect_maybe,
                m_t=m_t, m_z=m_z, m_rad=m_rad, m_jac=m_jac)


# ---------------------------------------------------------------------------
# Compositing (Eqs. 5-6 with p_j inside the product)
# ---------------------------------------------------------------------------
@dataclass
class Margins:
    """Relative/absolute thresholds below which a decision counts as one that
    FP32 arithmetic may legitimately take the other way."""
    rel: float = 3e-5        # alpha vs the 1/255 floor (FP32 error of alpha is ~1e-6 |power|)
    stop_rel: float = 3e-4   # T(1-a) vs the stop threshold: FP32 T after hundreds of fragments,
                             # with (1-a) of alphas near the clamp, drifts up to ~1e-4 relative
    depth_rel: float = 5e-7  # relative depth gap within which FP32 may order two primitives either way
    clamp_rel: float = 1e-4  # alpha clamp / colour clamp / Jacobian clamp (gradients only)


def _order(pre, ids: torch.Tensor) -> torch.Tensor:
    """Sort primitive ids by (depth, index)."""
    z = pre["z"].detach()[ids].numpy()
    perm = np.lexsort((ids.numpy(), z))
    return ids[torch.as_tensor(perm)]


def composite_tile(pre, cam: OCamera, tile_id: int, bg: Sequence[float],
                   margins: Optional[Margins] = None, with_flags: bool = True):
    """Render the pixels of one 16x16 tile by the plain per-pixel definition.

    A primitive takes part at a pixel iff it is active and the pixel's tile
    lies in its tile rectangle; primitives are taken front to back by
    (camera z, index); a fragment with alpha < 1/255 is skipped; blending stops
    before a fragment that would bring the transmittance below 1e-4.
    Returns dict with rgb [3,h,w], depth, alpha, T, n_contrib, last (list
    position of the last contributor + 1), uncertain masks."""
    C = CONVENTIONS
    mg = margins or Margins()
    tx, ty = tile_id % cam.tiles_x, tile_id // cam.tiles_x
    px0, py0 = tx * TILE, ty * TILE
    w = min(TILE, cam.width - px0)
    h = min(TILE, cam.height - py0)
    ys, xs = torch.meshgrid(torch.arange(py0, py0 + h, dtype=F64),
                            torch.arange(px0, px0 + w, dtype=F64), indexing="ij")
    pxc = (xs + 0.5).reshape(-1)
    pyc = (ys + 0.5).reshape(-1)
    rect = pre["rect"]
    inr = pre["active"] & (rect[:, 0] <= tx) & (tx < rect[:, 2]) & (rect[:, 1] <= ty) & (ty < rect[:, 3])
    ids = _order(pre, torch.nonzero(inr).reshape(-1))
    P, G = pxc.shape[0], ids.shape[0]
    bgt = torch.as_tensor(bg, dtype=F64)
    if G == 0:
        rgb = bgt[:, None].expand(3, P)
        zeros = torch.zeros(P, dtype=F64)
        out = dict(rgb=rgb.reshape(3, h, w), depth=zeros.reshape(h, w), alpha=zeros.reshape(h, w),
                   T=torch.ones(P, dtype=F64).reshape(h, w), last=torch.zeros(P, dtype=torch.long).reshape(h, w),
                   n_list=0, ids=ids, blended=torch.zeros(0, dtype=torch.bool))
    else:
        u, v = pre["u"][ids], pre["v"][ids]
        conic = pre["conic"][ids]
        dx = pxc[:, None] - u[None, :]
        dy = pyc[:, None] - v[None, :]
        power = -0.5 * (conic[None, :, 0] * dx * dx + conic[None, :, 2] * dy * dy) - conic[None, :, 1] * dx * dy
        gval = pre["opac"][ids][None, :] * torch.exp(power)
        alpha = torch.clamp(gval, max=C["alpha_max"])
        with torch.no_grad():
            valid = gval >= C["alpha_min"]
            a_v = torch.where(valid, alpha, torch.zeros_like(alpha))
            t_incl = torch.cumprod(1.0 - a_v, dim=1)
            alive = t_incl >= C["t_stop"]
            contrib = valid & alive
        a_m = torch.where(contrib, alpha, torch.zeros_like(alpha))
        one_m = 1.0 - a_m
        t_excl = torch.cat([torch.ones(P, 1, dtype=F64), torch.cumprod(one_m, dim=1)[:, :-1]], 1)
        wgt = a_m * t_excl
        col = pre["color"][ids]
        rgb = wgt @ col                                    # [P,3]
        depth = wgt @ pre["z"][ids]
        t_fin = torch.prod(one_m, dim=1)
        rgb = rgb + t_fin[:, None] * bgt[None, :]
        with torch.no_grad():
            pos = torch.arange(1, G + 1).expand(P, G)
            last = torch.where(contrib, pos, torch.zeros_like(pos)).max(1).values
        out = dict(rgb=rgb.T.reshape(3, h, w), depth=depth.reshape(h, w), alpha=(1.0 - t_fin).reshape(h, w),
                   T=t_fin.reshape(h, w), last=last.reshape(h, w), n_list=G, ids=ids,
                   blended=contrib.any(0))
    if with_flags:
        out.update(_tile_flags(pre, cam, tx, ty, pxc, pyc, ids, mg, h, w))
    return out


def _tile_flags(pre, cam, tx, ty, pxc, pyc, ids, mg: Margins, h, w):
    """Pixels whose result depends on a decision within FP32 reach of its
    threshold. A value flag is raised when taking such a decision the other
    way can move an output (rgb, depth or alpha) by more than a tenth of the
    image tolerance; a gradient flag whenever the decision touches a fragment
    that contributes (the tests zero dL/dI there on both sides)."""
    C = CONVENTIONS
    P = pxc.shape[0]
    tol_v = 0.1 * IMG_TOL
    with torch.no_grad():
        rs, rm = pre["rect_sure"], pre["rect_maybe"]
        in_maybe = (rm[:, 0] <= tx) & (tx < rm[:, 2]) & (rm[:, 1] <= ty) & (ty < rm[:, 3])
        in_sure = (rs[:, 0] <= tx) & (tx < rs[:, 2]) & (rs[:, 1] <= ty) & (ty < rs[:, 3])
        cand = torch.nonzero(in_maybe & ~in_sure).reshape(-1)
        flag_v = torch.zeros(P, dtype=torch.bool)
        flag_g = torch.zeros(P, dtype=torch.bool)
        flag_o = torch.zeros(P, dtype=torch.bool)   # some valid pair may be ordered either way
        if cand.numel() > 0:
            gv = _gval(pre, cand, pxc, pyc)
            flag_v |= (gv >= C["alpha_min"] * (1 - mg.rel)).any(1)
        if ids.numel() > 0:
            gv = _gval(pre, ids, pxc, pyc)
            z = pre["z"].detach()[ids]
            col = pre["color"].detach()[ids]
            # largest change one fragment can make to any output, per unit weight a*T
            reach = (col.abs().amax(-1) + z.abs() + 1.0)[None, :]
            valid = gv >= C["alpha_min"]
            a = torch.clamp(gv, max=C["alpha_max"])
            a_v = torch.where(valid, a, torch.zeros_like(a))
            t_incl = torch.cumprod(1.0 - a_v, dim=1)
            t_ex_v = torch.cat([torch.ones_like(t_incl[:, :1]), t_incl[:, :-1]], 1)
            alive = t_incl >= C["t_stop"] * (1 - mg.stop_rel)
            # alpha floor: a fragment within reach of 1/255 may be skipped or not
            near_floor = (gv - C["alpha_min"]).abs() < mg.rel * C["alpha_min"]
            nf = near_floor & (t_ex_v >= C["t_stop"] * (1 - mg.stop_rel))
            flag_v |= (nf & (C["alpha_min"] * t_ex_v * reach > tol_v)).any(1)
            flag_g |= nf.any(1)
            # stop threshold: fragments whose T after them lies in the FP32 band
            # around the threshold may or may not be blended
            maybe = valid & (t_incl >= C["t_stop"] * (1 - mg.stop_rel)) & (t_incl < C["t_stop"] * (1 + mg.stop_rel))
            eff = torch.where(maybe, (t_ex_v - t_incl) * reach, torch.zeros_like(t_incl)).sum(1)
            flag_v |= eff > tol_v
            flag_g |= maybe.any(1)
            contrib = valid & alive
            # Depth near-ties: two consecutive fragments of a pixel whose depths
            # are within FP32 reach may be blended in either order.
            if ids.numel() > 1:
                nxt_z, nxt_i = _next_of(valid, z)
                tie = valid & ((nxt_z - z[None, :]) < mg.depth_rel * z[None, :])
                flag_o |= tie.any(1)
                if tie.any():
                    # (a) the stop can fall inside the pair in one order and not
                    # the other: T before the pair >= stop > T after both;
                    # either fragment may then be blended or not
                    a_nv = torch.gather(a_v, 1, nxt_i)
                    t_after = t_ex_v * (1.0 - a_v) * (1.0 - a_nv)
                    straddle = tie & (t_ex_v >= C["t_stop"] * (1 - mg.stop_rel)) & \
                        (t_after < C["t_stop"] * (1 + mg.stop_rel))
                    eff_s = (a_v + a_nv) * t_ex_v * torch.maximum(reach, torch.gather(reach.expand_as(a_v), 1, nxt_i))
                    flag_v |= (straddle & (eff_s > tol_v)).any(1)
                    flag_g |= straddle.any(1)
                    # (b) both blended: swapping adjacent contributors i, j changes
                    # the pixel by exactly a_i a_j T_i (c_i - c_j); flag the value
                    # when that can exceed a tenth of the image tolerance, the
                    # gradient when a_i a_j T_i does
                    nxt_zc, nxt_ic = _next_of(contrib, z)
                    tie_c = contrib & ((nxt_zc - z[None, :]) < mg.depth_rel * z[None, :])
                    a_c = torch.where(contrib, a, torch.zeros_like(a))
                    t_ex = torch.cat([torch.ones_like(a_c[:, :1]), torch.cumprod(1.0 - a_c, 1)[:, :-1]], 1)
                    a_n = torch.gather(a_c, 1, nxt_ic)
                    dc = (col[None, :, :] - col[nxt_ic]).abs().amax(-1)
                    w2 = a_c * a_n * t_ex
                    flag_v |= (tie_c & (w2 * dc > tol_v)).any(1)
                    flag_g |= (tie_c & (w2 > 0.1 * tol_v)).any(1)
            # gradient-only: alpha clamp, colour clamp, Jacobian clamp
            near_clamp = ((gv - C["alpha_max"]).abs() < mg.clamp_rel) & contrib
            col_m = (pre["color_raw"][ids].abs() < mg.clamp_rel).any(1)
            jac_m = pre["m_jac"][ids] < mg.clamp_rel
            flag_g |= near_clamp.any(1) | (contrib & (col_m | jac_m)[None, :]).any(1)
        flag_g |= flag_v
    return dict(uncertain=flag_v.reshape(h, w), uncertain_grad=flag_g.reshape(h, w),
                uncertain_order=(flag_o | flag_v).reshape(h, w))


def _next_of(mask: torch.Tensor, z: torch.Tensor):
    """Per pixel and list position k: depth and position of the next masked
    entry after k (inf / 0 when none). z is ascending along the list."""
    zm = torch.where(mask, z[None, :], torch.full(mask.shape, float("inf"), dtype=z.dtype))
    nz, nidx = torch.cummin(torch.flip(zm, [1]), dim=1)
    nz, nidx = torch.flip(nz, [1]), (zm.shape[1] - 1) - torch.flip(nidx, [1])
    nxt_z = torch.cat([nz[:, 1:], torch.full_like(nz[:, :1], float("inf"))], 1)
    nxt_i = torch.cat([nidx[:, 1:], torch.zeros_like(nidx[:, :1])], 1)
    return nxt_z, nxt_i


def _gval(pre, ids, pxc, pyc):
    u, v = pre["u"].detach()[ids], pre["v"].detach()[ids]
    conic = pre["conic"].detach()[ids]
    dx = pxc[:, None] - u[None, :]
    dy = pyc[:, None] - v[None, :]
    power = -0.5 * (conic[None, :, 0] * dx * dx + conic[None, :, 2] * dy * dy) - conic[None, :, 1] * dx * dy
    return pre["opac"].detach()[ids][None, :] * torch.exp(power)


def render_view(params, cam, t: float, sh_degree: int, t_order: int, period: float = 1.0,
                bg=(0.0, 0.0, 0.0), tiles: Optional[Sequence[int]] = None,
                margins: Optional[Margins] = None, with_flags: bool = True):
    """Render one view (all tiles, or only `tiles`). Returns full-size planes;
    pixels of tiles not rendered are NaN."""
    ocam = cam if isinstance(cam, OCamera) else to_ocamera(cam)
    pre = preprocess(params, ocam, float(t), sh_degree, t_order, period)
    H, W = ocam.height, ocam.width
    tile_list = range(ocam.tiles_x * ocam.tiles_y) if tiles is None else tiles
    rgb_rows, parts = [], []
    out = dict(pre=pre, tiles=list(tile_list), parts={})
    for tid in tile_list:
        out["parts"][int(tid)] = composite_tile(pre, ocam, int(tid), bg, margins, with_flags)
    return out


def assemble(out, cam, key: str, channels: int = 0) -> torch.Tensor:
    """Stitch per-tile results into a full image (NaN where not rendered)."""
    ocam = cam if isinstance(cam, OCamera) else to_ocamera(cam)
    H, W = ocam.height, ocam.width
    shape = (channels, H, W) if channels else (H, W)
    img = torch.full(shape, float("nan"), dtype=F64)
    if key in ("uncertain", "uncertain_grad", "uncertain_order"):
        img = torch.zeros(shape, dtype=torch.bool)
    if key == "last":
        img = torch.zeros(shape, dtype=torch.long)
    for tid, part in out["parts"].items():
        tx, ty = tid % ocam.tiles_x, tid // ocam.tiles_x
        val = part[key]
        h, w = val.shape[-2:]
        img[..., ty * TILE: ty * TILE + h, tx * TILE: tx * TILE + w] = val.detach() if key not in ("rgb", "depth", "alpha") else val
    return img


def tile_linear_loss(out, dl_rgb=None, dl_depth=None, dl_alpha=None, cam=None) -> torch.Tensor:
    """sum over rendered pixels of <dL/dI, I>: its gradient with respect to
    the parameters is the vector-Jacobian product the backward pass computes."""
    ocam = cam if isinstance(cam, OCamera) else to_ocamera(cam)
    total = torch.zeros((), dtype=F64)
    for tid, part in out["parts"].items():
        tx, ty = tid % ocam.tiles_x, tid // ocam.tiles_x
        h, w = part["depth"].shape
        sl = (slice(ty * TILE, ty * TILE + h), slice(tx * TILE, tx * TILE + w))
        if dl_rgb is not None:
            total = total + (part["rgb"] * dl_rgb[:, sl[0], sl[1]]).sum()
        if dl_depth is not None:
            total = total + (part["depth"] * dl_depth[sl[0], sl[1]]).sum()
        if dl_alpha is not None:
            total = total + (part["alpha"] * dl_alpha[sl[0], sl[1]]).sum()
    return total


def densify_stats(scene, cams, times, dl_rgb, dl_depth=None, dl_alpha=None, bg=(0.0, 0.0, 0.0)):
    """Densification statistics of Sec. 3.3 ("Densification in spacetime"):
    the view-space position gradient magnitude and the mu_t gradient
    magnitude, accumulated per primitive over the views in which it blended
    at least one pixel, with the number of such views.

    For view v with loss L_v = <dL/dI_v, I_v> (the vector-Jacobian product the
    backward computes): uv[i] += |(dL_v/du_i, dL_v/dv_i)| (pixel units),
    t[i] += |dL_v/dmu_t,i|, count[i] += 1, for every primitive i that has a
    blended fragment (alpha >= 1/255 before the stop) in view v.
    Returns float64 uv [N], t [N] and int64 count [N]."""
    n = scene.means4.shape[0]
    uv = torch.zeros(n, dtype=F64)
    tg = torch.zeros(n, dtype=F64)
    cnt = torch.zeros(n, dtype=torch.long)
    for v, (cam, t) in enumerate(zip(cams, times)):
        params = params_from_scene(scene, requires_grad=True)
        out = render_view(params, cam, float(t), scene.sh_degree, scene.t_order, scene.t_period, bg,
                          with_flags=False)
        pre = out["pre"]
        blended = torch.zeros(n, dtype=torch.bool)
        for part in out["parts"].values():
            if part["n_list"]:
                blended[part["ids"][part["blended"]]] = True
        loss = tile_linear_loss(out, torch.as_tensor(dl_rgb[v]),
                                None if dl_depth is None else torch.as_tensor(dl_depth[v]),
                                None if dl_alpha is None else torch.as_tensor(dl_alpha[v]), cam)
        gu, gv, gm = torch.autograd.grad(loss, [pre["u"], pre["v"], params["means4"]], allow_unused=True)
        gu = torch.zeros(n, dtype=F64) if gu is None else gu
        gv = torch.zeros(n, dtype=F64) if gv is None else gv
        gm = torch.zeros(n, 4, dtype=F64) if gm is None else gm
        uv = uv + torch.where(blended, torch.sqrt(gu * gu + gv * gv), torch.zeros_like(uv))
        tg = tg + torch.where(blended, gm[:, 3].abs(), torch.zeros_like(tg))
        cnt = cnt + blended.long()
    return uv.detach(), tg.detach(), cnt


def flow_displacement(params: Dict[str, torch.Tensor], cam: OCamera, t: float, dt: float) -> torch.Tensor:
    """Sec. 4.3 ("Render Flow"): the image-plane displacement of each
    primitive's conditional mean mu_xyz|t between t and t + dt, both points
    projected by the view's pinhole camera; zero when the later point is not in
    front of the near plane. Returns [N, 2] (du, dv) in pixels."""
    cov4 = covariance_4d(params["log_scales4"], params["q_left"], params["q_right"])
    mean4 = params["means4"]
    mu0, _ = slice_at(mean4, cov4, t)
    mu1, _ = slice_at(mean4, cov4, t + dt)

    def project(mu):
        p = mu @ cam.rot.T + cam.trans
        return cam.fx * p[:, 0] / p[:, 2] + cam.cx, cam.fy * p[:, 1] / p[:, 2] + cam.cy, p[:, 2]
    u0, v0, _ = project(mu0)
    u1, v1, z1 = project(mu1)
    ok = z1 > CONVENTIONS["near"]
    zero = torch.zeros_like(u0)
    return torch.stack([torch.where(ok, u1 - u0, zero), torch.where(ok, v1 - v0, zero)], -1)


def render_flow(scene, cam, t: float, dt: float, tiles=None, margins=None, with_flags=True):
    """Optical flow of one view (Sec. 4.3): each primitive's displacement
    (flow_displacement) blended with the render's weights of Eq. (6) over a
    zero background. Same primitives, footprints and order as the render.
    Returns render_view's structure whose "rgb" planes 0-1 hold the flow."""
    ocam = cam if isinstance(cam, OCamera) else to_ocamera(cam)
    params = params_from_scene(scene)
    pre = preprocess(params, ocam, float(t), scene.sh_degree, scene.t_order, scene.t_period)
    f = flow_displacement(params, ocam, float(t), float(dt))
    pre = dict(pre, color=torch.cat([f, torch.zeros_like(f[:, :1])], -1))
    tile_list = range(ocam.tiles_x * ocam.tiles_y) if tiles is None else tiles
    out = dict(pre=pre, tiles=list(tile_list), parts={})
    for tid in tile_list:
        out["parts"][int(tid)] = composite_tile(pre, ocam, int(tid), (0.0, 0.0, 0.0), margins, with_flags)
    return out


def render_full(scene, cam, t, bg=(0.0, 0.0, 0.0), requires_grad=False, with_flags=True,
                tiles=None, margins=None):
    """Convenience: render a whole view from a scenegen Scene."""
    params = params_from_scene(scene, requires_grad)
    out = render_view(params, cam, t, scene.sh_degree, scene.t_order, scene.t_period, bg,
                      tiles=tiles, margins=margins, with_flags=with_flags)
    out["params"] = params
    return out
