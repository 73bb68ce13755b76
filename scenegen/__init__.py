"""Seeded synthetic 4D Gaussian scenes and pinhole cameras.

This module only draws inputs: primitive parameters, camera poses, render times
and loss targets. It holds none of the rendering arithmetic, so both the FP64
oracle and the GPU path can read the exact same float32 arrays from it.

Workload shapes follow the paper's experiments: multi-view captures at
1352x1014 (the Plenoptic Video resolution, Section 4.1), 800x800 monocular
views (the D-NeRF setting, Table 2 caption), and long sequences whose per-frame
active set is kept small by the temporal filter (Appendix, temporal
statistics). The datasets themselves are not used; these seeded draws stand in
for them.

Draw order for a scene (all draws FP64, cast once to float32):
  xyz ~ U[-1,1]^(N,3) -> mu_t ~ U[0,1]^N -> log-scale xyz ~ N(-3,0.5)^(N,3)
  -> log-scale t ~ N(mu_lt,0.5)^N -> q_left ~ N(0,I4) normalised
  -> q_right ~ N(0,I4) normalised -> opacity logit ~ N(0,1)
  -> 4DSH coefficients ~ N(0,0.3)^(N,K,3) -> per view: ring angle, time
  -> loss targets ~ U[0,1].
N(a, b) means mean a and standard deviation b.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

TILE = 16


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # float32 [3, 4], row-major [R | t]
    center: np.ndarray        # float32 [3], camera position in world frame


@dataclass
class Scene:
    means4: np.ndarray         # float32 [N, 4]  (x, y, z, t)
    log_scales4: np.ndarray    # float32 [N, 4]
    q_left: np.ndarray         # float32 [N, 4]  (a, b, c, d)
    q_right: np.ndarray        # float32 [N, 4]  (p, q, r, s)
    opacity_logit: np.ndarray  # float32 [N]
    coeffs: np.ndarray         # float32 [N, K, 3], K = (t_order+1)*(sh_degree+1)^2
    sh_degree: int
    t_order: int
    t_period: float = 1.0

    @property
    def n(self) -> int:
        return int(self.means4.shape[0])


@dataclass
class Workload:
    name: str
    scene: Scene
    cameras: List[Camera]
    times: np.ndarray                      # float32 [V]
    loss: Optional[str] = None             # None, "l1" or "l2"
    targets: Optional[List[np.ndarray]] = None  # per view float32 [3, H, W]
    notes: dict = field(default_factory=dict)


def look_at_camera(eye, width: int, height: int, fov_x_deg: float = 60.0) -> Camera:
    """Camera at `eye` looking at the origin with world up +y, OpenCV axes."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = -eye / np.linalg.norm(eye)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    rot = np.stack([right, down, fwd], 0)          # rows: camera axes in world frame
    trans = -rot @ eye
    w2c = np.concatenate([rot, trans[:, None]], 1)
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(width, height, float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0,
                  w2c.astype(np.float32), eye.astype(np.float32))


def ring_camera(theta: float, width: int, height: int, radius: float = 4.0) -> Camera:
    return look_at_camera((radius * math.sin(theta), 0.0, radius * math.cos(theta)), width, height)


def draw_scene(rng: np.random.Generator, n: int, sh_degree: int, t_order: int,
               mu_log_t: float = -3.0) -> Scene:
    xyz = rng.uniform(-1.0, 1.0, size=(n, 3))
    mu_t = rng.uniform(0.0, 1.0, size=(n,))
    ls_xyz = rng.normal(-3.0, 0.5, size=(n, 3))
    ls_t = rng.normal(mu_log_t, 0.5, size=(n,))
    ql = rng.normal(0.0, 1.0, size=(n, 4))
    ql /= np.linalg.norm(ql, axis=1, keepdims=True)
    qr = rng.normal(0.0, 1.0, size=(n, 4))
    qr /= np.linalg.norm(qr, axis=1, keepdims=True)
    logit = rng.normal(0.0, 1.0, size=(n,))
    k = (t_order + 1) * (sh_degree + 1) ** 2
    coeffs = rng.normal(0.0, 0.3, size=(n, k, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(
        means4=f32(np.concatenate([xyz, mu_t[:, None]], 1)),
        log_scales4=f32(np.concatenate([ls_xyz, ls_t[:, None]], 1)),
        q_left=f32(ql), q_right=f32(qr), opacity_logit=f32(logit),
        coeffs=f32(coeffs), sh_degree=sh_degree, t_order=t_order)


def _targets(rng, cams):
    return [rng.uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]


def make_workload(config: int, n_override: Optional[int] = None) -> Workload:
    """The five seeded workloads. `n_override` shrinks N for quick tests only."""
    rng = np.random.default_rng(config)
    if config == 0:
        sc = draw_scene(rng, n_override or 1000, 1, 1)
        cams = [look_at_camera((0.0, 0.0, 4.0), 64, 64)]
        return Workload("plain_fwd_1k_64x64", sc, cams, np.array([0.5], np.float32))
    if config == 1:
        sc = draw_scene(rng, n_override or 300_000, 3, 2)
        theta = rng.uniform(0.0, 2 * math.pi)
        t = rng.uniform(0.0, 1.0)
        cams = [ring_camera(theta, 1352, 1014)]
        return Workload("fwd_bwd_300k_1352x1014_l1", sc, cams, np.array([t], np.float32),
                        loss="l1", targets=_targets(rng, cams))
    if config == 2:
        sc = draw_scene(rng, n_override or 1_000_000, 3, 2, mu_log_t=-4.0)
        cams, ts = [], []
        for v in range(16):
            theta = rng.uniform(0.0, 2 * math.pi)
            ts.append(rng.uniform(0.0, 1.0))
            w, h = (800, 800) if v % 2 == 0 else (1352, 1014)
            cams.append(ring_camera(theta, w, h))
        return Workload("batched_fwd_1m_16views_mixed", sc, cams, np.array(ts, np.float32))
    if config == 3:
        sc = draw_scene(rng, n_override or 500_000, 3, 2)
        cams, ts = [], []
        for _ in range(8):
            cams.append(ring_camera(rng.uniform(0.0, 2 * math.pi), 1352, 1014))
            ts.append(rng.uniform(0.0, 1.0))
        return Workload("batched_fwd_bwd_500k_8views_l2", sc, cams, np.array(ts, np.float32),
                        loss="l2", targets=_targets(rng, cams))
    if config == 4:
        sc = draw_scene(rng, n_override or 3_000_000, 3, 2, mu_log_t=-5.0)
        cams, ts = [], []
        for f in range(120, 180):
            for q in range(4):
                cams.append(ring_camera(q * math.pi / 2.0, 1920, 1080))
                ts.append(f / 299.0)
        return Workload("long_seq_3m_240views_1080p", sc, cams, np.array(ts, np.float32))
    raise ValueError(f"unknown config {config}")


def bench_workload(n_views: int = 8) -> Workload:
    """The 300k-primitive scene of the training-step workload seen from
    `n_views` ring cameras at distinct times, 1352x1014, L1 loss."""
    base = make_workload(1)
    rng = np.random.default_rng(101)
    cams, ts = [], []
    for _ in range(n_views):
        cams.append(ring_camera(rng.uniform(0.0, 2 * math.pi), 1352, 1014))
        ts.append(rng.uniform(0.0, 1.0))
    return Workload(f"fwd_bwd_300k_{n_views}views_1352x1014_l1", base.scene, cams,
                    np.array(ts, np.float32), loss="l1", targets=_targets(rng, cams))


def random_scene(seed: int, n: int, sh_degree: int = 1, t_order: int = 1,
                 mu_log_t: float = -3.0, spread: float = 1.0) -> Scene:
    """Small ad-hoc scene for unit tests (same distributions, custom size)."""
    rng = np.random.default_rng(seed)
    sc = draw_scene(rng, n, sh_degree, t_order, mu_log_t)
    sc.means4[:, :3] *= np.float32(spread)
    return sc


def sample_pixels_dlddi(seed: int, cams: List[Camera], tiles_per_view: int):
    """Pick random 16x16 tiles per view (for sampled parity at full size)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in cams:
        tx, ty = (c.width + TILE - 1) // TILE, (c.height + TILE - 1) // TILE
        ids = rng.choice(tx * ty, size=min(tiles_per_view, tx * ty), replace=False)
        out.append(np.sort(ids).astype(np.int64))
    return out
