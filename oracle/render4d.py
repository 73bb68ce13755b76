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
U32 = 2.0 ** -24    # unit roundoff of float32
# Margins of the parity policy for the per-primitive decisions. An
# implementation that evaluates these formulas in FP64 may still decide the
# other way within: the thresholds it receives as float32 options (0.05f and
# 0.2f differ from 0.05 and 0.2 by 1.5e-8, relative), and the last bits of
# FP64 arithmetic in another order.
MARGIN_REL = 1e-7   # relative: p(t) vs t_cull, z vs near, x/z vs the Jacobian limit
MARGIN_PX = 1e-6    # pixels: 3 sqrt(lambda_max) vs an integer, rectangle edges vs tile edges
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
    out = dict(u=u, v=v, z=z, conic=conic, opac=opac, color=color, color_raw=color_raw,
               pt=pt, mu_c=mu_c, cov_c=cov_c, cov4=cov4, cov2=torch.stack([a2, b2, c2], -1),
               radius=rad, rect=torch.stack([x0, y0, x1, y1], -1).long(), active=active,
               rect_sure=rect_sure, rect_maybe=rect_maybe,
               m_t=m_t, m_z=m_z, m_rad=m_rad, m_jac=m_jac)
    out.update(record_as_float32(out))
    return out


def _f32(x: torch.Tensor) -> torch.Tensor:
    """The float32 value nearest to x (round to nearest even), as float64."""
    return x.detach().to(torch.float32).to(F64)


def _rounding_in_doubt(x: torch.Tensor, rel: float = 1e-12) -> torch.Tensor:
    """x within rel of a float32 rounding midpoint: an FP64 evaluation in
    another order (about 1e-15 relative here, 1e-12 leaves room for the
    conditioning of the conic's inverse) may round it to the other
    neighbour."""
    x = x.detach()
    x32 = x.to(torch.float32)
    inf = torch.tensor(float("inf"), dtype=torch.float32)
    up = torch.nextafter(x32, inf).to(F64)
    dn = torch.nextafter(x32, -inf).to(F64)
    c = x32.to(F64)
    d = torch.minimum((x - 0.5 * (c + up)).abs(), (x - 0.5 * (c + dn)).abs())
    return d <= rel * x.abs()


def record_as_float32(pre) -> Dict[str, torch.Tensor]:
    """The per-primitive values a GPU record holds when it evaluates the
    geometry in FP64 and rounds each value to float32 once: u, v, z, the
    conic and opacity * p(t), and whether any of them sits so close to a
    rounding midpoint that the stored neighbour is in doubt."""
    con = pre["conic"].detach()
    doubt = _rounding_in_doubt(pre["u"]) | _rounding_in_doubt(pre["v"]) | _rounding_in_doubt(pre["z"])
    doubt = doubt | _rounding_in_doubt(pre["opac"]) | _rounding_in_doubt(con).any(-1)
    return dict(u32=_f32(pre["u"]), v32=_f32(pre["v"]), z32=_f32(pre["z"]), conic32=_f32(con),
                opac32=_f32(pre["opac"]), rec_doubt=doubt)


# ---------------------------------------------------------------------------
# Compositing (Eqs. 5-6 with p_j inside the product)
# ---------------------------------------------------------------------------
@dataclass
class Margins:
    """How far an FP32 implementation may legitimately take each decision the
    other way (see alpha_reach and stop_band), and which of the resulting
    differences count as value flags."""
    frag_ulps: float = 6.0   # float32 ulps of |Q|/2 + |ln opacity| lost in the fragment's exponent
    value_frac: float = 0.3  # a decision raises a value flag when the other way moves an output by more
                             # than this fraction of the image tolerance
    clamp_rel: float = 1e-4  # colour at its clamp at 0 (a float32 4DSH sum; gradients only)

    def alpha_fp32(self, pre, ids, pxc, pyc):
        """Per (pixel, list entry): the definition's unclamped alpha
        opacity * exp(power) in FP64, the same alpha evaluated (in FP64) from
        the record rounded to float32 (record_as_float32), which is what an
        FP32 implementation evaluates, and the relative reach of its float32
        evaluation of the fragment. With A, B, C the staged conic terms and L
        the log2 opacity, the exponent A dx^2 + B dx dy + C dy^2 + L is formed
        from the offsets dx = px + 0.5 - u (1 rounding each), the three staged
        products (1 each), B dy and C dy (1 each) and three FMAs (1 each):
        at most 4 ulps of |A dx^2|, 5 of |B dx dy| and 5 of |C dy^2|, 2 of |L|
        (one rounding, log2) and 1 of the result, i.e. frag_ulps = 6 ulps of
        |Q|/2 + |ln opacity| in natural units; then the float32 constants
        log2(e) (relative 1.3e-8) and log2(1/255), and exp2 (2 ulps), 4 ulps
        of alpha in all. A record whose rounding is in doubt also takes one
        ulp of each of its values."""
        det = lambda k: pre[k].detach()[ids]
        u, v, con, op = det("u"), det("v"), det("conic"), det("opac")
        dx, dy = pxc[:, None] - u[None, :], pyc[:, None] - v[None, :]
        q = con[None, :, 0] * dx * dx + 2 * con[None, :, 1] * dx * dy + con[None, :, 2] * dy * dy
        gv = op[None, :] * torch.exp(-0.5 * q)
        u32, v32, c32, o32 = det("u32"), det("v32"), det("conic32"), det("opac32")
        dx, dy = pxc[:, None] - u32[None, :], pyc[:, None] - v32[None, :]
        q32 = c32[None, :, 0] * dx * dx + 2 * c32[None, :, 1] * dx * dy + c32[None, :, 2] * dy * dy
        gv32 = o32[None, :] * torch.exp(-0.5 * q32)
        tabs = 0.5 * (c32[None, :, 0].abs() * dx * dx + 2 * (c32[None, :, 1] * dx * dy).abs() +
                      c32[None, :, 2].abs() * dy * dy)
        eps = self.frag_ulps * U32 * (tabs + o32.log().abs()[None, :]) + 1.3e-8 * (0.5 * q32.abs() + 8.0) + 4 * U32
        doubt = det("rec_doubt")
        if bool(doubt.any()):
            gu = (c32[None, :, 0] * dx + c32[None, :, 1] * dy).abs()
            gw = (c32[None, :, 1] * dx + c32[None, :, 2] * dy).abs()
            one_ulp = 2 * U32 * (gu * u32.abs()[None, :] + gw * v32.abs()[None, :] + tabs + 1.0)
            eps = eps + torch.where(doubt[None, :], one_ulp, torch.zeros_like(eps))
        return gv, gv32, eps

    def alpha_reach(self, pre, ids, pxc, pyc):
        """The definition's unclamped alpha (FP64) and how far an FP32
        implementation's value of it may lie from it, absolute."""
        gv, gv32, eps = self.alpha_fp32(pre, ids, pxc, pyc)
        return gv, (gv32 - gv).abs() + gv32 * eps

    @staticmethod
    def stop_band(a_v: torch.Tensor, reach: torch.Tensor, clamped: torch.Tensor) -> torch.Tensor:
        """FP32 reach of the transmittance after each list entry, relative,
        for the stop decision T (1 - a) vs 1e-4 (Eq. 6 taken front to back).

        T_k is the product of the factors (1 - a_i), i <= k. A factor whose
        alpha may be off by `reach` is off by reach / (1 - a), relative; its
        product is rounded once more (1 ulp). A surely clamped alpha is the
        constant 0.99 on both sides, whose float32 representation moves
        (1 - a) by 9.5e-7, relative. Summed over the entries up to k, the
        bound grows with the list position."""
        term = torch.where(clamped, torch.full_like(a_v, 9.6e-7), reach / (1.0 - a_v))
        term = torch.where(a_v > 0, term + 2 * U32, torch.zeros_like(a_v))
        return torch.cumsum(term, dim=1)


def _order(pre, ids: torch.Tensor) -> torch.Tensor:
    """Sort primitive ids by (depth, index)."""
    z = pre["z"].detach()[ids].numpy()
    perm = np.lexsort((ids.numpy(), z))
    return ids[torch.as_tensor(perm)]


def composite_tile(pre, cam: OCamera, tile_id: int, bg: Sequence[float],
                   margins: Optional[Margins] = None, with_flags: bool = True, gval_fn=None):
    """Render the pixels of one 16x16 tile by the plain per-pixel definition.

    A primitive takes part at a pixel iff it is active and the pixel's tile
    lies in its tile rectangle; primitives are taken front to back by
    (camera z, index); a fragment with alpha < 1/255 is skipped; blending stops
    before a fragment that would bring the transmittance below 1e-4.
    Returns dict with rgb [3,h,w], depth, alpha, T, n_contrib, last (list
    position of the last contributor + 1), uncertain masks. gval_fn (tests of
    the margin policy only) replaces the unclamped alphas: gval_fn(ids, px, py)
    -> [pixels, list]."""
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
        if gval_fn is not None:
            gval = gval_fn(ids, pxc, pyc)
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
    """Pixels whose result depends on a decision that an FP32 implementation
    may take the other way (Margins: the float32 record and fragment
    arithmetic for alpha decisions, MARGIN_REL / MARGIN_PX for the
    per-primitive ones, float32 depth keys for the order). A value flag is
    raised when taking such a decision the other way can move an output (rgb,
    depth or alpha) by more than value_frac of the image tolerance; a gradient
    flag whenever the decision touches a fragment that contributes (the tests
    zero dL/dI there on both sides). Value flags are also returned per cause:
    "rect" (a primitive whose rectangle edge is in doubt reaches the floor),
    "floor" (alpha at the 1/255 floor), "stop" (the transmittance crosses the
    stop threshold within its reach), "tie" (two depths that float32 keys may
    order the other way, blended in either order)."""
    C = CONVENTIONS
    P = pxc.shape[0]
    tol_v = mg.value_frac * IMG_TOL
    thr = C["alpha_min"]
    with torch.no_grad():
        rs, rm = pre["rect_sure"], pre["rect_maybe"]
        in_maybe = (rm[:, 0] <= tx) & (tx < rm[:, 2]) & (rm[:, 1] <= ty) & (ty < rm[:, 3])
        in_sure = (rs[:, 0] <= tx) & (tx < rs[:, 2]) & (rs[:, 1] <= ty) & (ty < rs[:, 3])
        cand = torch.nonzero(in_maybe & ~in_sure).reshape(-1)
        zeros = lambda: torch.zeros(P, dtype=torch.bool)
        f_rect, f_floor, f_stop, f_tie = zeros(), zeros(), zeros(), zeros()
        flag_g = zeros()
        flag_o = zeros()   # some valid pair may be ordered either way
        # primitives that surely blend some pixel of the tile, and that may
        # (an FP32 implementation may blend them here or not when in maybe only)
        sure_ids, maybe_ids = [torch.zeros(0, dtype=torch.long)], [torch.zeros(0, dtype=torch.long)]
        if cand.numel() > 0:
            gv, reach = mg.alpha_reach(pre, cand, pxc, pyc)
            above = gv + reach >= thr
            f_rect |= above.any(1)
            maybe_ids.append(cand[above.any(0)])
        if ids.numel() > 0:
            gv, reach = mg.alpha_reach(pre, ids, pxc, pyc)
            z = pre["z"].detach()[ids]
            z32 = pre["z32"][ids]
            col = pre["color"].detach()[ids]
            # largest change one fragment can make to any output, per unit weight a*T
            reach_out = (col.abs().amax(-1) + z.abs() + 1.0)[None, :]
            valid = gv >= thr
            a = torch.clamp(gv, max=C["alpha_max"])
            a_v = torch.where(valid, a, torch.zeros_like(a))
            clamped = gv - reach >= C["alpha_max"]
            t_incl = torch.cumprod(1.0 - a_v, dim=1)
            t_ex_v = torch.cat([torch.ones_like(t_incl[:, :1]), t_incl[:, :-1]], 1)
            band = mg.stop_band(a_v, torch.where(valid, reach, torch.zeros_like(reach)), clamped)
            band_ex = torch.cat([torch.zeros_like(band[:, :1]), band[:, :-1]], 1)
            lo, hi = C["t_stop"] * (1 - band), C["t_stop"] * (1 + band)
            alive = t_incl >= lo
            # alpha floor: a fragment within reach of 1/255 may be skipped or not
            near_floor = (gv - thr).abs() <= reach
            nf = near_floor & (t_ex_v >= C["t_stop"] * (1 - band_ex))
            f_floor |= (nf & (thr * t_ex_v * reach_out > tol_v)).any(1)
            flag_g |= nf.any(1)
            # stop threshold: fragments whose T after them lies in the FP32 band
            # around the threshold may or may not be blended
            maybe = valid & (t_incl >= lo) & (t_incl < hi)
            eff = torch.where(maybe, (t_ex_v - t_incl) * reach_out, torch.zeros_like(t_incl)).sum(1)
            f_stop |= eff > tol_v
            flag_g |= maybe.any(1)
            # blended surely: above the floor and still alive after it, both
            # beyond reach (T is monotone, so no earlier stop is within reach);
            # blended maybe: above the floor and alive within reach
            sure_e = (gv - reach >= thr) & (t_incl >= hi)
            maybe_e = (gv + reach >= thr) & alive
            # Depth order: float32 keys that are equal are ordered by primitive
            # index, which may reverse two consecutive fragments of a pixel
            # (or FP64 evaluations in another order may, within 1e-12).
            if ids.numel() > 1:
                nxt_z, nxt_i = _next_of(valid, z)
                nz32 = z32[nxt_i]
                nid = ids[nxt_i]
                swap = ((nz32 == z32[None, :]) & (nid < ids[None, :])) | ((nxt_z - z[None, :]) < 1e-12 * z[None, :])
                tie = valid & torch.isfinite(nxt_z) & swap
                flag_o |= tie.any(1)
                tie_any = tie | (torch.zeros_like(nxt_i).scatter_add_(1, nxt_i, tie.long()) > 0)
                sure_e &= ~tie_any
                if tie.any():
                    # (a) the stop can fall inside the pair in one order and not
                    # the other: T before the pair >= stop > T after both;
                    # either fragment may then be blended or not
                    a_nv = torch.gather(a_v, 1, nxt_i)
                    t_after = t_ex_v * (1.0 - a_v) * (1.0 - a_nv)
                    straddle = tie & (t_ex_v >= C["t_stop"] * (1 - band_ex)) & (t_after < hi)
                    eff_s = (a_v + a_nv) * t_ex_v * torch.maximum(reach_out,
                                                                  torch.gather(reach_out.expand_as(a_v), 1, nxt_i))
                    f_tie |= (straddle & (eff_s > tol_v)).any(1)
                    flag_g |= straddle.any(1)
                    # (b) both blended: swapping adjacent contributors i, j changes
                    # the pixel by exactly a_i a_j T_i (c_i - c_j); flag the value
                    # when that can exceed value_frac of the image tolerance, the
                    # gradient when a_i a_j T_i exceeds 1 % of the tolerance
                    contrib = valid & alive
                    a_c = torch.where(contrib, a, torch.zeros_like(a))
                    t_ex = torch.cat([torch.ones_like(a_c[:, :1]), torch.cumprod(1.0 - a_c, 1)[:, :-1]], 1)
                    a_n = torch.gather(a_c, 1, nxt_i)
                    dc = (col[None, :, :] - col[nxt_i]).abs().amax(-1)
                    dz = (z[None, :] - z[nxt_i]).abs()
                    w2 = a_c * a_n * t_ex
                    tie_c = tie & contrib
                    f_tie |= (tie_c & (w2 * torch.maximum(dc, dz) > tol_v)).any(1)
                    flag_g |= (tie_c & (w2 > 0.01 * IMG_TOL)).any(1)
            contrib = valid & alive
            # gradient-only: alpha clamp, colour clamp, Jacobian clamp
            near_clamp = ((gv - C["alpha_max"]).abs() <= reach) & contrib
            col_m = (pre["color_raw"][ids].abs() < mg.clamp_rel).any(1)
            jac_m = pre["m_jac"][ids] < MARGIN_REL
            flag_g |= near_clamp.any(1) | (contrib & (col_m | jac_m)[None, :]).any(1)
            sure_ids.append(ids[sure_e.any(0) & in_sure[ids]])
            maybe_ids.append(ids[maybe_e.any(0)])
        flag_v = f_rect | f_floor | f_stop | f_tie
        flag_g |= flag_v
    shp = lambda m: m.reshape(h, w)
    return dict(uncertain=shp(flag_v), uncertain_grad=shp(flag_g), uncertain_order=shp(flag_o | flag_v),
                cause_rect=shp(f_rect), cause_floor=shp(f_floor), cause_stop=shp(f_stop), cause_tie=shp(f_tie),
                sure_ids=torch.unique(torch.cat(sure_ids)), maybe_ids=torch.unique(torch.cat(maybe_ids)))


def _next_of(mask: torch.Tensor, z: torch.Tensor):
    """Per pixel and list position k: depth and position of the next masked
    entry after k (inf / 0 when none). z is ascending along the list."""
    zm = torch.where(mask, z[None, :], torch.full(mask.shape, float("inf"), dtype=z.dtype))
    nz, nidx = torch.cummin(torch.flip(zm, [1]), dim=1)
    nz, nidx = torch.flip(nz, [1]), (zm.shape[1] - 1) - torch.flip(nidx, [1])
    nxt_z = torch.cat([nz[:, 1:], torch.full_like(nz[:, :1], float("inf"))], 1)
    nxt_i = torch.cat([nidx[:, 1:], torch.zeros_like(nidx[:, :1])], 1)
    return nxt_z, nxt_i


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
    if key in ("uncertain", "uncertain_grad", "uncertain_order") or key.startswith("cause_"):
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


def densify_stats(scene, cams, times, dl_rgb, dl_depth=None, dl_alpha=None, bg=(0.0, 0.0, 0.0),
                  margins: Optional[Margins] = None):
    """Densification statistics of Sec. 3.3 ("Densification in spacetime"):
    the view-space position gradient magnitude and the mu_t gradient
    magnitude, accumulated per primitive over the views in which it blended
    at least one pixel, with the number of such views.

    For view v with loss L_v = <dL/dI_v, I_v> (the vector-Jacobian product the
    backward computes): uv[i] += |(dL_v/du_i, dL_v/dv_i)| (pixel units),
    t[i] += |dL_v/dmu_t,i|, count[i] += 1, for every primitive i that has a
    blended fragment (alpha >= 1/255 before the stop) in view v.
    Returns float64 uv [N], t [N], int64 count [N] and int64 unsure [N]: the
    number of views in which primitive i's blended-or-not decision rests on a
    decision within FP32 reach of its threshold (the margin policy), so that
    an FP32 implementation may count that view or not."""
    n = scene.means4.shape[0]
    uv = torch.zeros(n, dtype=F64)
    tg = torch.zeros(n, dtype=F64)
    cnt = torch.zeros(n, dtype=torch.long)
    unsure = torch.zeros(n, dtype=torch.long)
    for v, (cam, t) in enumerate(zip(cams, times)):
        params = params_from_scene(scene, requires_grad=True)
        out = render_view(params, cam, float(t), scene.sh_degree, scene.t_order, scene.t_period, bg,
                          margins=margins, with_flags=True)
        pre = out["pre"]
        blended = torch.zeros(n, dtype=torch.bool)
        sure = torch.zeros(n, dtype=torch.bool)
        maybe = torch.zeros(n, dtype=torch.bool)
        for part in out["parts"].values():
            if part["n_list"]:
                blended[part["ids"][part["blended"]]] = True
            sure[part["sure_ids"]] = True
            maybe[part["maybe_ids"]] = True
        doubt = maybe & ~sure
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
        unsure = unsure + doubt.long()
    return uv.detach(), tg.detach(), cnt, unsure


def flow_displacement(params: Dict[str, torch.Tensor], cam: OCamera, t: float, dt: float) -> torch.Tensor:
    """Sec. 4.4 (rendered flow, "Ablation and analysis"): the image-plane displacement of each
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
    """Optical flow of one view (Sec. 4.4): each primitive's displacement
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
