"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, invariants stated in the paper, a library routine, an independent
sequential loop, or finite differences.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.special
import torch

import scenegen
from oracle import render4d as O

F64 = torch.float64


def rand_quats(rng, n):
    q = rng.normal(size=(n, 4))
    return torch.as_tensor(q / np.linalg.norm(q, axis=1, keepdims=True))


def hamilton(p, q):
    """Quaternion product in scalar/vector form: (s1,v1)(s2,v2) =
    (s1 s2 - v1.v2, s1 v2 + s2 v1 + v1 x v2)."""
    s1, v1 = p[..., 0], p[..., 1:]
    s2, v2 = q[..., 0], q[..., 1:]
    s = s1 * s2 - (v1 * v2).sum(-1)
    v = s1[..., None] * v2 + s2[..., None] * v1 + torch.cross(v1, v2, dim=-1)
    return torch.cat([s[..., None], v], -1)


# --- Sec. 3.2: 4D rotation from a left and a right isoclinic rotation --------
def test_rotation_orthonormal_det_one():
    rng = np.random.default_rng(0)
    ql, qr = rand_quats(rng, 256), rand_quats(rng, 256)
    R = O.rotation_4d(ql, qr)
    eye = torch.eye(4, dtype=F64).expand(256, 4, 4)
    assert torch.allclose(R.transpose(-1, -2) @ R, eye, atol=1e-14)
    assert torch.allclose(torch.linalg.det(R), torch.ones(256, dtype=F64), atol=1e-13)


def test_left_right_commute_and_hamilton_form():
    rng = np.random.default_rng(1)
    ql, qr = rand_quats(rng, 64), rand_quats(rng, 64)
    L, Rr = O.left_isoclinic(ql), O.right_isoclinic(qr)
    assert torch.allclose(L @ Rr, Rr @ L, atol=1e-14)
    v = torch.as_tensor(rng.normal(size=(64, 4)))
    rv = (O.rotation_4d(ql, qr) @ v[..., None])[..., 0]
    ref = hamilton(hamilton(ql, v), qr)        # R v = q_l * v * q_r
    assert torch.allclose(rv, ref, atol=1e-14)


def test_identity_quaternions_give_identity():
    one = torch.tensor([[1.0, 0.0, 0.0, 0.0]], dtype=F64)
    assert torch.equal(O.rotation_4d(one, one)[0], torch.eye(4, dtype=F64))


def test_unnormalised_quaternions_are_normalised():
    rng = np.random.default_rng(2)
    ql, qr = rand_quats(rng, 8), rand_quats(rng, 8)
    a = O.rotation_4d(ql, qr)
    b = O.rotation_4d(3.7 * ql, 0.2 * qr)
    assert torch.allclose(a, b, atol=1e-14)


# --- Sec. 3.2: Sigma = R S S^T R^T -----------------------------------------------
def test_covariance_eigenvalues_are_squared_scales():
    rng = np.random.default_rng(3)
    ls = torch.as_tensor(rng.normal(-1.0, 0.5, size=(32, 4)))
    cov = O.covariance_4d(ls, rand_quats(rng, 32), rand_quats(rng, 32))
    assert torch.allclose(cov, cov.transpose(-1, -2), atol=1e-15)
    ev = np.linalg.eigvalsh(cov.numpy())
    ref = np.sort(np.exp(2 * ls.numpy()), axis=1)
    assert np.allclose(ev, ref, rtol=1e-12)


# --- Sec. 3.2 conditional Gaussian; Appendix B factorisation --------------------
def _random_gauss(seed, n=64):
    rng = np.random.default_rng(seed)
    ls = torch.as_tensor(rng.normal(-1.0, 0.6, size=(n, 4)))
    ql, qr = rand_quats(rng, n), rand_quats(rng, n)
    cov = O.covariance_4d(ls, ql, qr)
    mean = torch.as_tensor(rng.normal(size=(n, 4)))
    return rng, ls, ql, qr, cov, mean


def test_conditional_covariance_is_precision_block_inverse():
    """Sigma_xyz|t equals the inverse of the xyz block of the precision
    R diag(s^-2) R^T (an independent route to the Schur complement)."""
    rng, ls, ql, qr, cov, mean = _random_gauss(4)
    _, cov_c = O.slice_at(mean, cov, 0.3)
    R = O.rotation_4d(ql, qr)
    prec = R @ torch.diag_embed(torch.exp(-2 * ls)) @ R.transpose(-1, -2)
    ref = torch.linalg.inv(prec[:, :3, :3])
    assert torch.allclose(cov_c, ref, rtol=1e-10, atol=1e-13)
    assert (torch.linalg.eigvalsh(cov_c) > 0).all()


def test_determinant_factorisation():
    """det Sigma = Sigma_44 det Sigma_xyz|t = prod s_k^2 (Appendix B)."""
    rng, ls, ql, qr, cov, mean = _random_gauss(5)
    _, cov_c = O.slice_at(mean, cov, -0.7)
    lhs = torch.linalg.det(cov)
    mid = cov[:, 3, 3] * torch.linalg.det(cov_c)
    ref = torch.exp(2 * ls.sum(-1))
    assert torch.allclose(lhs, ref, rtol=1e-10)
    assert torch.allclose(mid, ref, rtol=1e-10)


def test_exponent_factorisation():
    """p(x,t) = p(t) p(x|t) for the unnormalised Gaussian (Appendix B)."""
    rng, ls, ql, qr, cov, mean = _random_gauss(6)
    t = torch.as_tensor(rng.normal(size=64))
    xyz = torch.as_tensor(rng.normal(size=(64, 3)))
    lhs_vec = torch.cat([xyz, t[:, None]], 1) - mean
    lhs = (lhs_vec[:, None, :] @ torch.linalg.inv(cov) @ lhs_vec[:, :, None])[:, 0, 0]
    rhs = torch.empty(64, dtype=F64)
    for i in range(64):
        mu_c, cov_c = O.slice_at(mean[i:i + 1], cov[i:i + 1], float(t[i]))
        d = xyz[i] - mu_c[0]
        rhs[i] = (t[i] - mean[i, 3]) ** 2 / cov[i, 3, 3] + d @ torch.linalg.inv(cov_c[0]) @ d
    assert torch.allclose(lhs, rhs, rtol=1e-10)


def test_conditional_mean_linear_in_t():
    rng, ls, ql, qr, cov, mean = _random_gauss(7)
    mu0, _ = O.slice_at(mean, cov, 0.0)
    mu1, _ = O.slice_at(mean, cov, 1.0)
    mu_half, c_half = O.slice_at(mean, cov, 0.5)
    assert torch.allclose(mu_half, 0.5 * (mu0 + mu1), atol=1e-13)
    at_mean = torch.stack([O.slice_at(mean[i:i + 1], cov[i:i + 1], float(mean[i, 3]))[0][0] for i in range(8)])
    assert torch.allclose(at_mean, mean[:8, :3], atol=1e-14)
    vel = cov[:, :3, 3] / cov[:, 3, 3:4]
    assert torch.allclose(mu1 - mu0, vel, atol=1e-13)


def test_block_diagonal_case_is_static_3d():
    """With identity rotations space and time decouple: the slice is the
    static 3D Gaussian at every t and only p(t) varies (the independent
    space-time baseline of Sec. 3.2)."""
    one = torch.tensor([[1.0, 0.0, 0.0, 0.0]], dtype=F64)
    ls = torch.tensor([[-1.0, -0.5, -2.0, -1.5]], dtype=F64)
    cov = O.covariance_4d(ls, one, one)
    mean = torch.tensor([[0.1, 0.2, 0.3, 0.4]], dtype=F64)
    for t in (-1.0, 0.4, 2.0):
        mu_c, cov_c = O.slice_at(mean, cov, t)
        assert torch.allclose(mu_c, mean[:, :3], atol=0)
        assert torch.allclose(cov_c[0], torch.diag(torch.exp(2 * ls[0, :3])), atol=1e-15)
        pt = O.temporal_marginal(mean[:, 3], cov[:, 3, 3], t)
        assert torch.allclose(pt, torch.exp(-0.5 * (t - 0.4) ** 2 / torch.exp(2 * ls[:, 3])), rtol=1e-14)


def test_time_axis_fixing_pair_gives_block_rotation():
    """q_r = -k conj(q_l) k gives R = diag(R3, 1): S_xt = 0 for any scales."""
    rng = np.random.default_rng(8)
    ql = rand_quats(rng, 16)
    k = torch.tensor([0.0, 0.0, 0.0, 1.0], dtype=F64).expand(16, 4)
    conj = ql * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)
    qr = -hamilton(hamilton(k, conj), k)
    R = O.rotation_4d(ql, qr)
    assert torch.allclose(R[:, 3, :3], torch.zeros(16, 3, dtype=F64), atol=1e-14)
    assert torch.allclose(R[:, :3, 3], torch.zeros(16, 3, dtype=F64), atol=1e-14)
    assert torch.allclose(R[:, 3, 3], torch.ones(16, dtype=F64), atol=1e-14)
    ls = torch.as_tensor(rng.normal(-1, 0.5, size=(16, 4)))
    cov = O.covariance_4d(ls, ql, qr)
    assert torch.allclose(cov[:, :3, 3], torch.zeros(16, 3, dtype=F64), atol=1e-15)


# --- Sec. 3.2 marginal p(t); Sec. 4.2 temporal filter ------------------------------
def test_marginal_integrates_to_one_when_normalised():
    mu, var = 0.3, 0.02 ** 2
    t = np.linspace(mu - 1, mu + 1, 200001)
    pt = O.temporal_marginal(torch.tensor(mu, dtype=F64), torch.tensor(var, dtype=F64),
                             torch.as_tensor(t)).numpy()
    integral = np.trapezoid(pt, t) / math.sqrt(2 * math.pi * var)
    assert abs(integral - 1.0) < 1e-9
    assert float(O.temporal_marginal(torch.tensor(mu, dtype=F64), torch.tensor(var, dtype=F64), mu)) == 1.0


def test_temporal_filter_threshold_closed_form():
    """Kept iff |t - mu_t| <= sigma_t sqrt(2 ln 20)."""
    sc = scenegen.random_scene(9, 1)
    sc.q_left[:] = [1, 0, 0, 0]
    sc.q_right[:] = [1, 0, 0, 0]
    sc.means4[0] = [0.0, 0.0, 0.0, 0.5]
    sc.log_scales4[0] = [-2.0, -2.0, -2.0, math.log(0.1)]
    cam = scenegen.look_at_camera((0.0, 0.0, 4.0), 32, 32)
    lim = 0.1 * math.sqrt(2 * math.log(20.0))
    for dt, keep in ((lim * 0.999, True), (lim * 1.001, False), (-lim * 0.999, True), (-lim * 1.001, False)):
        pre = O.preprocess(O.params_from_scene(sc), O.to_ocamera(cam), 0.5 + dt, 1, 1)
        assert bool(pre["active"][0]) == keep


# --- Sec. 3.2 4D spherindrical harmonics ------------------------------------------
def test_real_sh_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(10)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    ours = O.real_sh(torch.as_tensor(d), 3).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            ylm = scipy.special.sph_harm_y(l, abs(m), theta, phi)   # Condon-Shortley phase included
            if m == 0:
                ref = ylm.real
            elif m > 0:
                ref = math.sqrt(2) * ylm.real
            else:
                ref = math.sqrt(2) * ylm.imag
            assert np.allclose(ours[:, l * l + l + m], ref, atol=1e-13), (l, m)


def test_real_sh_low_degree_closed_forms():
    d = torch.tensor([[0.48, -0.6, 0.64]], dtype=F64)
    y = O.real_sh(d, 1)[0]
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3.0 / (4 * math.pi))
    ref = torch.tensor([c0, -c1 * -0.6, c1 * 0.64, -c1 * 0.48], dtype=F64)
    assert torch.allclose(y, ref, atol=1e-15)


def test_real_sh_orthonormal_by_quadrature():
    """Gauss-Legendre in cos(theta) x uniform in phi integrates degree <= 6
    products exactly."""
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = 2 * np.pi * np.arange(nphi) / nphi
    z = np.repeat(xg, nphi)
    w = np.repeat(wg, nphi) * (2 * np.pi / nphi)
    ph = np.tile(phi, len(xg))
    s = np.sqrt(1 - z * z)
    d = np.stack([s * np.cos(ph), s * np.sin(ph), z], 1)
    Y = O.real_sh(torch.as_tensor(d), 3).numpy()
    gram = (Y * w[:, None]).T @ Y
    assert np.allclose(gram, np.eye(16), atol=1e-12)


def test_fourier_terms_orthogonal_over_period():
    T = 1.0
    t = (np.arange(4096) + 0.5) / 4096 * T
    f = O.fourier_cos(torch.as_tensor(t), 2, T).numpy()
    gram = f.T @ f / len(t)
    assert np.allclose(gram, np.diag([1.0, 0.5, 0.5]), atol=1e-12)


def test_color_order_zero_reduces_to_sh_and_is_even_in_dt():
    rng = np.random.default_rng(11)
    d = rng.normal(size=(10, 3))
    d = torch.as_tensor(d / np.linalg.norm(d, axis=1, keepdims=True))
    k1 = torch.as_tensor(rng.normal(0, 0.3, size=(10, 4 * 2, 3)))
    dt = torch.as_tensor(rng.uniform(-1, 1, size=10))
    c_pos, _ = O.color_4dsh(k1, d, dt, 1, 1, 1.0)
    c_neg, _ = O.color_4dsh(k1, d, -dt, 1, 1, 1.0)
    assert torch.allclose(c_pos, c_neg, atol=1e-15)
    k0 = k1[:, :4]
    c0, raw0 = O.color_4dsh(k0, d, dt, 1, 0, 1.0)
    Y = O.real_sh(d, 1)
    ref = 0.5 + (Y[:, :, None] * k0).sum(1)
    assert torch.allclose(raw0, ref, atol=1e-15)
    # the n = 1 term at dt = T/2 flips sign: cos(pi) = -1
    half = torch.full((10,), 0.5, dtype=F64)
    _, raw_h = O.color_4dsh(k1, d, half, 1, 1, 1.0)
    ref_h = 0.5 + (Y[:, :, None] * k1[:, :4]).sum(1) - (Y[:, :, None] * k1[:, 4:]).sum(1)
    assert torch.allclose(raw_h, ref_h, atol=1e-14)


# --- Eqs. (3)-(4): EWA projection ------------------------------------------------
def test_centred_isotropic_gaussian_projects_to_circle():
    """A centred isotropic Gaussian at distance D projects to the principal
    point with sigma_2d^2 = f^2 s^2 / D^2 + 0.3 (low-pass)."""
    sc = scenegen.random_scene(12, 1)
    s = 0.05
    sc.means4[0] = [0, 0, 0, 0.5]
    sc.log_scales4[0] = [math.log(s)] * 3 + [0.0]
    sc.q_left[0] = [1, 0, 0, 0]
    sc.q_right[0] = [1, 0, 0, 0]
    cam = scenegen.look_at_camera((0.0, 0.0, 4.0), 64, 48)
    pre = O.preprocess(O.params_from_scene(sc), O.to_ocamera(cam), 0.5, 1, 1)
    f = cam.fx
    s = math.exp(float(sc.log_scales4[0, 0]))          # the float32-stored scale
    var = f * f * s * s / 16.0 + 0.3
    assert abs(float(pre["u"][0]) - 32.0) < 1e-12 and abs(float(pre["v"][0]) - 24.0) < 1e-12
    assert torch.allclose(pre["cov2"][0], torch.tensor([var, 0.0, var], dtype=F64), rtol=1e-12, atol=1e-14)
    assert torch.allclose(pre["conic"][0], torch.tensor([1 / var, 0.0, 1 / var], dtype=F64), rtol=1e-12, atol=1e-14)
    assert float(pre["radius"][0]) == math.ceil(3 * math.sqrt(var))
    assert abs(float(pre["z"][0]) - 4.0) < 1e-12


def _rot4_hamilton(ql, qr):
    """4x4 rotation v -> ql (x) v (x) qr built column by column from the
    scalar/vector quaternion product (independent of the oracle's matrices)."""
    qln = ql / ql.norm(dim=-1, keepdim=True)
    qrn = qr / qr.norm(dim=-1, keepdim=True)
    cols = []
    for j in range(4):
        e = torch.zeros(qln.shape[0], 4, dtype=F64)
        e[:, j] = 1.0
        cols.append(hamilton(hamilton(qln, e), qrn))
    return torch.stack(cols, -1)


def _sliced_cov_independent(sc, t):
    """Conditional mean and covariance of (x, y, z) at t, by an independent
    route: Sigma from the Hamilton-product rotation, the conditional
    covariance as the inverse of the precision's xyz block, the conditional
    mean by solving the precision's xyz block against its t column."""
    ls = torch.as_tensor(sc.log_scales4.astype(np.float64))
    R = _rot4_hamilton(torch.as_tensor(sc.q_left.astype(np.float64)), torch.as_tensor(sc.q_right.astype(np.float64)))
    prec = R @ torch.diag_embed(torch.exp(-2 * ls)) @ R.transpose(-1, -2)
    cov_c = torch.linalg.inv(prec[:, :3, :3])
    mu = torch.as_tensor(sc.means4.astype(np.float64))
    # the conditional mean minimises the quadratic form over xyz at fixed t
    mu_c = mu[:, :3] - (cov_c @ prec[:, :3, 3:4])[..., 0] * (t - mu[:, 3])[:, None]
    return mu_c, cov_c


def _pinhole(cam, p_world):
    pc = p_world @ cam.rot.T + cam.trans
    return torch.stack([cam.fx * pc[..., 0] / pc[..., 2] + cam.cx, cam.fy * pc[..., 1] / pc[..., 2] + cam.cy], -1)


def _fd_jacobian(fn, p, h=1e-5):
    """Central-difference Jacobian [N, 2, 3] of fn: [N, 3] -> [N, 2]."""
    cols = []
    for k in range(3):
        d = torch.zeros_like(p)
        d[:, k] = h
        cols.append((fn(p + d) - fn(p - d)) / (2 * h))
    return torch.stack(cols, -1)


def _offaxis_scene(seed, n, spread, aniso=1.0):
    sc = scenegen.random_scene(seed, n, sh_degree=1, t_order=1, mu_log_t=-0.5, spread=spread)
    rng = np.random.default_rng(seed + 100)
    sc.log_scales4[:, :3] = (rng.normal(-2.5, aniso, size=(n, 3))).astype(np.float32)
    return sc


def test_offaxis_ewa_is_pinhole_jacobian_sandwich():
    """Eqs. (3)-(4) off the axis: for rotated anisotropic primitives at time t
    away from their temporal mean, Sigma_2d - 0.3 I = J (Sigma_c) J^T with J the
    central-difference Jacobian of the world-to-pixel pinhole map at the
    conditional mean (which holds W Sigma W^T, the -f x / z^2 column and
    its sign), and (u, v) is the pinhole image of the conditional mean. Only
    primitives inside the 1.3x Jacobian limit are checked here."""
    sc = _offaxis_scene(21, 200, 1.6)
    cam = O.to_ocamera(scenegen.look_at_camera((1.3, -0.8, 3.6), 160, 120))
    t = 0.37
    pre = O.preprocess(O.params_from_scene(sc), cam, t, 1, 1)
    mu_c, cov_c = _sliced_cov_independent(sc, t)
    pc = mu_c @ cam.rot.T + cam.trans
    lim_x, lim_y = 1.3 * 80.0 / cam.fx, 1.3 * 60.0 / cam.fy
    ok = (pc[:, 2] > 0.5) & ((pc[:, 0] / pc[:, 2]).abs() < 0.98 * lim_x) & ((pc[:, 1] / pc[:, 2]).abs() < 0.98 * lim_y)
    assert int(ok.sum()) > 100
    off = ((pc[:, 0] / pc[:, 2]).abs() > 0.3 * lim_x) & ok
    assert int(off.sum()) > 20                       # genuinely off-axis
    J = _fd_jacobian(lambda p: _pinhole(cam, p), mu_c)
    ref = J @ cov_c @ J.transpose(-1, -2)
    cov2 = pre["cov2"]
    got = torch.stack([torch.stack([cov2[:, 0] - 0.3, cov2[:, 1]], -1), torch.stack([cov2[:, 1], cov2[:, 2] - 0.3], -1)], -2)
    scale = ref.abs().amax((-1, -2), keepdim=True)
    assert torch.allclose(got[ok] / scale[ok], ref[ok] / scale[ok], atol=1e-8, rtol=0)
    uv = _pinhole(cam, mu_c)
    assert torch.allclose(torch.stack([pre["u"], pre["v"]], -1)[ok], uv[ok], atol=1e-9, rtol=0)
    # a dropped depth column or a transposed camera rotation (W^T Sigma W)
    # would fail the sandwich on these primitives: check that both differ
    bad = J.clone()
    bad[..., 2] = 0.0
    dropped = bad @ cov_c @ bad.transpose(-1, -2)
    assert not torch.allclose(got[off] / scale[off], dropped[off] / scale[off], atol=1e-3, rtol=0)
    Wc = torch.as_tensor(cam.rot)
    J_cam = _fd_jacobian(lambda q: torch.stack([cam.fx * q[:, 0] / q[:, 2] + cam.cx,
                                                 cam.fy * q[:, 1] / q[:, 2] + cam.cy], -1), pc)
    transposed = J_cam @ Wc.T @ cov_c @ Wc @ J_cam.transpose(-1, -2)
    assert not torch.allclose(got[off] / scale[off], transposed[off] / scale[off], atol=1e-3, rtol=0)


def test_ewa_jacobian_clamp_beyond_the_limit():
    """Beyond 1.3x the half field of view the Jacobian is the pinhole
    Jacobian at the camera-space point moved onto the limit, x/z -> xi =
    clamp(x/z), y/z -> eta = clamp(y/z), at the same depth:
    Sigma_2d - 0.3 I = J(xi z, eta z, z) W Sigma_c W^T J(...)^T."""
    sc = _offaxis_scene(22, 400, 3.0)
    cam = O.to_ocamera(scenegen.look_at_camera((0.2, 0.1, 3.0), 96, 64))
    t = 0.61
    pre = O.preprocess(O.params_from_scene(sc), cam, t, 1, 1)
    mu_c, cov_c = _sliced_cov_independent(sc, t)
    pc = mu_c @ cam.rot.T + cam.trans
    lim_x, lim_y = 1.3 * 48.0 / cam.fx, 1.3 * 32.0 / cam.fy
    z = pc[:, 2]
    xr, yr = pc[:, 0] / z, pc[:, 1] / z
    front = z > 0.5
    clx = front & (xr.abs() > 1.02 * lim_x)
    cly = front & (yr.abs() > 1.02 * lim_y)
    assert int(clx.sum()) > 20 and int(cly.sum()) > 20 and int((clx & cly).sum()) > 5
    q = torch.stack([xr.clamp(-lim_x, lim_x) * z, yr.clamp(-lim_y, lim_y) * z, z], -1)
    J = _fd_jacobian(lambda p: torch.stack([cam.fx * p[:, 0] / p[:, 2] + cam.cx, cam.fy * p[:, 1] / p[:, 2] + cam.cy], -1), q)
    Wc = torch.as_tensor(cam.rot)
    ref = J @ (Wc @ cov_c @ Wc.T) @ J.transpose(-1, -2)
    cov2 = pre["cov2"]
    got = torch.stack([torch.stack([cov2[:, 0] - 0.3, cov2[:, 1]], -1), torch.stack([cov2[:, 1], cov2[:, 2] - 0.3], -1)], -2)
    sel = clx | cly
    scale = ref.abs().amax((-1, -2), keepdim=True)
    assert torch.allclose(got[sel] / scale[sel], ref[sel] / scale[sel], atol=1e-8, rtol=0)
    # unclamped, the sandwich would differ for these primitives
    J_raw = _fd_jacobian(lambda p: torch.stack([cam.fx * p[:, 0] / p[:, 2] + cam.cx, cam.fy * p[:, 1] / p[:, 2] + cam.cy], -1), pc)
    raw = J_raw @ (Wc @ cov_c @ Wc.T) @ J_raw.transpose(-1, -2)
    assert not torch.allclose(got[sel] / scale[sel], raw[sel] / scale[sel], atol=1e-3, rtol=0)


def _rotate_scene_and_camera(sc, cam, a):
    """The scene and the camera turned together by the 3D rotation that the
    unit quaternion a induces on (x, y, z) with t fixed: as a 4D rotation it
    is v -> a (x) v (x) b with b = -k conj(a) k, so each primitive's pair
    becomes (a (x) q_l, q_r (x) b), its mean Q mu, and the camera
    W' = W Q^T, centre Q c."""
    a = a / a.norm()
    k = torch.tensor([0.0, 0.0, 0.0, 1.0], dtype=F64)
    ac = a * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)
    b = -hamilton(hamilton(k[None], ac[None]), k[None])[0]
    M = _rot4_hamilton(a[None], b[None])[0]
    assert torch.allclose(M[3], torch.tensor([0.0, 0.0, 0.0, 1.0], dtype=F64), atol=1e-14)
    Q = M[:3, :3]
    n = sc.n
    ql = hamilton(a[None].expand(n, 4), torch.as_tensor(sc.q_left.astype(np.float64)))
    qr = hamilton(torch.as_tensor(sc.q_right.astype(np.float64)), b[None].expand(n, 4))
    params = O.params_from_scene(sc)
    params["q_left"], params["q_right"] = ql, qr
    params["means4"] = torch.cat([params["means4"][:, :3] @ Q.T, params["means4"][:, 3:]], 1)
    cam2 = dataclasses.replace(cam, rot=cam.rot @ Q.T, center=Q @ cam.center)
    return params, cam2


def test_projection_invariant_under_joint_rotation():
    """Turning the scene and the camera together by one rotation changes
    nothing the camera sees: u, v, z, Sigma_2d and the view direction
    relative to the camera are unchanged (Eqs. 3-4 with the view transform
    applied as W Sigma W^T; W^T Sigma W would not be invariant)."""
    sc = _offaxis_scene(23, 300, 1.5)
    cam = O.to_ocamera(scenegen.look_at_camera((1.0, 0.7, 3.4), 120, 90))
    t = 0.45
    pre = O.preprocess(O.params_from_scene(sc), cam, t, 1, 1)
    for seed in range(3):
        a = torch.as_tensor(np.random.default_rng(seed).normal(size=4))
        params2, cam2 = _rotate_scene_and_camera(sc, cam, a)
        pre2 = O.preprocess(params2, cam2, t, 1, 1)
        keep = pre["z"] > 0.3
        for key in ("u", "v", "z", "cov2", "conic", "pt"):
            assert torch.allclose(pre2[key][keep], pre[key][keep], rtol=1e-9, atol=1e-9), key
        assert torch.equal(pre2["active"], pre["active"])


# --- Eqs. (5)-(6): compositing ----------------------------------------------------
def sequential_pixel(px, py, gauss, bg):
    """Independent front-to-back loop for one pixel over a list of
    (z, idx, u, v, conic, opac, color, rect) already restricted to the pixel's
    tile; pure Python scalars."""
    T, C, D, last = 1.0, [0.0, 0.0, 0.0], 0.0, 0
    for pos, g in enumerate(sorted(gauss, key=lambda g: (g["z"], g["idx"])), start=1):
        dx, dy = px - g["u"], py - g["v"]
        a_, b_, c_ = g["conic"]
        power = -0.5 * (a_ * dx * dx + c_ * dy * dy) - b_ * dx * dy
        G = g["opac"] * math.exp(power)
        alpha = min(0.99, G)
        if G < 1.0 / 255.0:
            continue
        if T * (1.0 - alpha) < 1e-4:
            break
        for k in range(3):
            C[k] += alpha * T * g["color"][k]
        D += alpha * T * g["z"]
        T *= 1.0 - alpha
        last = pos
    return [C[k] + T * bg[k] for k in range(3)], D, 1.0 - T, T, last


@pytest.mark.parametrize("seed,n,spread,grow", [(20, 12, 0.3, 1.0), (21, 40, 1.0, 1.0), (22, 80, 0.3, 1.5)])
def test_tile_composite_equals_sequential_loop(seed, n, spread, grow):
    sc = scenegen.random_scene(seed, n, spread=spread, mu_log_t=-1.0)
    sc.log_scales4[:, :3] += grow         # large splats: overlaps and early stops
    sc.opacity_logit[:] += 2.0
    cam = scenegen.look_at_camera((0.0, 0.0, 4.0), 32, 32)
    bg = (0.1, 0.2, 0.3)
    out = O.render_full(sc, cam, 0.5, bg=bg, with_flags=False)
    pre = out["pre"]
    ocam = O.to_ocamera(cam)
    rgb = O.assemble(out, cam, "rgb", 3).detach()
    depth = O.assemble(out, cam, "depth").detach()
    last = O.assemble(out, cam, "last")
    stopped = 0
    for py in range(0, 32, 2):
        for px in range(0, 32, 2):
            tx, ty = px // 16, py // 16
            gauss = []
            for i in range(n):
                r = pre["rect"][i]
                if bool(pre["active"][i]) and r[0] <= tx < r[2] and r[1] <= ty < r[3]:
                    gauss.append(dict(z=float(pre["z"][i]), idx=i, u=float(pre["u"][i]), v=float(pre["v"][i]),
                                      conic=[float(c) for c in pre["conic"][i]], opac=float(pre["opac"][i]),
                                      color=[float(c) for c in pre["color"][i]]))
            c, d, a, T, lst = sequential_pixel(px + 0.5, py + 0.5, gauss, bg)
            stopped += T < 1e-3
            assert np.allclose(rgb[:, py, px].numpy(), c, atol=1e-12)
            assert abs(float(depth[py, px]) - d) < 1e-12
            assert int(last[py, px]) == lst
    if seed == 22:
        assert stopped > 0     # the early-stop rule was exercised


def test_two_gaussian_pixel_by_hand():
    """Two coincident-axis isotropic Gaussians in front of the camera; the
    centre pixel's colour follows Eq. (6) written out by hand."""
    sc = scenegen.random_scene(30, 2, sh_degree=0, t_order=0)
    sc.q_left[:] = [1, 0, 0, 0]
    sc.q_right[:] = [1, 0, 0, 0]
    sc.means4[:] = [[0, 0, 0.5, 0.5], [0, 0, -0.5, 0.7]]   # front one at z_cam = 3.5
    sc.log_scales4[:] = [[math.log(0.2)] * 3 + [math.log(0.3)]] * 2
    sc.opacity_logit[:] = [0.0, 1.0]
    sc.coeffs[:] = 0.0
    sc.coeffs[0, 0] = [0.4, 0.0, -0.2]
    sc.coeffs[1, 0] = [0.0, 0.6, 0.2]
    cam = scenegen.look_at_camera((0.0, 0.0, 4.0), 32, 32)
    t = 0.5
    out = O.render_full(sc, cam, t, with_flags=False, tiles=[0, 1, 2, 3])
    rgb = O.assemble(out, cam, "rgb", 3).detach()
    f = cam.fx
    y00 = 0.5 / math.sqrt(math.pi)
    s2 = math.exp(2 * float(sc.log_scales4[0, 0]))
    st2 = math.exp(2 * float(sc.log_scales4[0, 3]))
    def contrib(zc, logit, mu_t, k):
        var = f * f * s2 / zc ** 2 + 0.3
        power = -0.5 * (0.5 * 0.5 + 0.5 * 0.5) / var          # pixel (16,16) centre is 0.5 px off
        pt = math.exp(-0.5 * (t - float(np.float32(mu_t))) ** 2 / st2)
        a = min(0.99, 1 / (1 + math.exp(-logit)) * pt * math.exp(power))
        col = [max(0.0, 0.5 + kk * y00) for kk in k]
        return a, col
    a1, c1 = contrib(3.5, 0.0, 0.5, [0.4, 0.0, -0.2])
    a2, c2 = contrib(4.5, 1.0, 0.7, [0.0, 0.6, 0.2])
    ref = [a1 * c1[i] + a2 * (1 - a1) * c2[i] for i in range(3)]
    assert np.allclose(rgb[:, 16, 16].numpy(), ref, atol=1e-13)


# --- gradients: autograd of the definition vs central finite differences ------------
def test_gradient_matches_finite_differences():
    sc = scenegen.random_scene(40, 24, sh_degree=2, t_order=2, spread=0.4, mu_log_t=-1.5)
    sc.log_scales4[:, :3] += 1.0
    cam = scenegen.look_at_camera((0.3, 0.2, 3.0), 32, 32)
    t = 0.45
    rng = np.random.default_rng(41)
    dl = torch.as_tensor(rng.normal(size=(3, 32, 32)))
    dd = torch.as_tensor(rng.normal(size=(32, 32))) * 0.1
    da = torch.as_tensor(rng.normal(size=(32, 32)))

    def loss_of(params, flags=False):
        out = O.render_view(params, cam, t, 2, 2, 1.0, with_flags=flags)
        return O.tile_linear_loss(out, dl, dd, da, cam), out

    params = O.params_from_scene(sc, requires_grad=True)
    L, out = loss_of(params, flags=True)
    assert not bool(O.assemble(out, cam, "uncertain_grad").any())
    L.backward()
    base = {k: v.detach().clone() for k, v in params.items()}
    h = 1e-6
    checked = 0
    for name in ["means4", "log_scales4", "q_left", "q_right", "opacity_logit", "coeffs"]:
        flat_idx = rng.choice(base[name].numel(), size=8, replace=False)
        for fi in flat_idx:
            vals = []
            for sgn in (1.0, -1.0):
                p2 = {k: v.clone() for k, v in base.items()}
                p2[name].view(-1)[fi] += sgn * h
                vals.append(float(loss_of(p2)[0]))
            fd = (vals[0] - vals[1]) / (2 * h)
            g = float(params[name].grad.view(-1)[fi])
            assert abs(fd - g) <= 1e-5 * (1 + abs(g)), (name, fi, fd, g)
            checked += 1
    assert checked == 48


def test_config0_renders_with_no_uncertain_pixels():
    wl = scenegen.make_workload(0)
    out = O.render_full(wl.scene, wl.cameras[0], float(wl.times[0]))
    assert int(out["pre"]["active"].sum()) > 0
    assert not bool(O.assemble(out, wl.cameras[0], "uncertain").any())


# --- Sec. 3.3 "Densification in spacetime": statistics --------------------------------
def _blend_sets_by_sequential_loop(sc, cam, t):
    """Primitives blended at some pixel of the view, from the independent
    per-pixel loop (which pixel decides nothing beyond alpha >= 1/255 before
    the stop)."""
    out = O.render_full(sc, cam, t, with_flags=False)
    pre = out["pre"]
    n = sc.means4.shape[0]
    blended = set()
    for py in range(cam.height):
        for px in range(cam.width):
            tx, ty = px // 16, py // 16
            T = 1.0
            cand = []
            for i in range(n):
                r = pre["rect"][i]
                if bool(pre["active"][i]) and r[0] <= tx < r[2] and r[1] <= ty < r[3]:
                    cand.append((float(pre["z"][i]), i))
            for _, i in sorted(cand):
                dx, dy = px + 0.5 - float(pre["u"][i]), py + 0.5 - float(pre["v"][i])
                a_, b_, c_ = [float(c) for c in pre["conic"][i]]
                G = float(pre["opac"][i]) * math.exp(-0.5 * (a_ * dx * dx + c_ * dy * dy) - b_ * dx * dy)
                if G < 1.0 / 255.0:
                    continue
                alpha = min(0.99, G)
                if T * (1.0 - alpha) < 1e-4:
                    break
                blended.add(i)
                T *= 1.0 - alpha
    return blended


def test_densify_count_matches_sequential_loop():
    sc = scenegen.random_scene(23, 30, spread=0.4, mu_log_t=-1.0)
    sc.log_scales4[:, :3] += 1.2
    sc.opacity_logit[:] += 2.0
    sc.means4[:3, 3] = 0.95                    # three short-lived primitives, culled at both times
    sc.log_scales4[:3, 3] = math.log(0.02)
    cams = [scenegen.look_at_camera((0.0, 0.0, 3.5), 32, 32), scenegen.look_at_camera((1.5, 0.3, 3.0), 32, 32)]
    times = [0.35, 0.6]
    rng = np.random.default_rng(24)
    dl = [rng.normal(size=(3, 32, 32)) for _ in cams]
    _, _, cnt, _ = O.densify_stats(sc, cams, times, dl)
    ref = np.zeros(sc.means4.shape[0], np.int64)
    for cam, t in zip(cams, times):
        for i in _blend_sets_by_sequential_loop(sc, cam, t):
            ref[i] += 1
    assert np.array_equal(cnt.numpy(), ref)
    assert ref.max() == 2 and (ref == 0).any()   # seen in both views by some, in none by others


def test_densify_uv_gradient_is_principal_point_derivative():
    """With one primitive, moving the principal point by h moves its projected
    mean by h and nothing else, so dL/du = dL/dc_x and dL/dv = dL/dc_y."""
    sc = scenegen.random_scene(25, 1, sh_degree=1, t_order=1)
    sc.means4[:] = [[0.1, -0.05, 0.0, 0.5]]
    sc.log_scales4[:] = [[math.log(0.25), math.log(0.15), math.log(0.2), math.log(0.3)]]
    sc.opacity_logit[:] = [1.5]
    cam = scenegen.look_at_camera((0.0, 0.0, 3.0), 32, 32)
    t = 0.5
    dl = np.random.default_rng(26).normal(size=(3, 32, 32))
    uv, _, cnt, _ = O.densify_stats(sc, [cam], [t], [dl])
    assert int(cnt[0]) == 1

    def loss(c):
        out = O.render_full(sc, c, t, with_flags=False)
        return float(O.tile_linear_loss(out, torch.as_tensor(dl), cam=c))
    h = 1e-6
    du = (loss(dataclasses.replace(cam, cx=cam.cx + h)) - loss(dataclasses.replace(cam, cx=cam.cx - h))) / (2 * h)
    dv = (loss(dataclasses.replace(cam, cy=cam.cy + h)) - loss(dataclasses.replace(cam, cy=cam.cy - h))) / (2 * h)
    assert abs(float(uv[0]) - math.hypot(du, dv)) <= 1e-6 * (1 + math.hypot(du, dv))


def test_densify_t_gradient_sums_per_view_magnitudes():
    """|dL_v/dmu_t| is taken per view before summing: with two views whose
    time derivatives differ in sign the statistic is the sum of magnitudes."""
    sc = scenegen.random_scene(27, 1, sh_degree=1, t_order=2)
    sc.means4[:] = [[0.0, 0.05, 0.0, 0.5]]
    sc.log_scales4[:] = [[math.log(0.3), math.log(0.2), math.log(0.25), math.log(0.2)]]
    sc.opacity_logit[:] = [1.0]
    cam = scenegen.look_at_camera((0.0, 0.0, 3.0), 32, 32)
    times = [0.4, 0.62]
    ones = np.ones((3, 32, 32))
    _, tg, cnt, _ = O.densify_stats(sc, [cam, cam], times, [ones, ones])
    assert int(cnt[0]) == 2
    h = 1e-6
    fd = []
    for t in times:
        vals = []
        for sgn in (1.0, -1.0):
            params = O.params_from_scene(sc)          # float64: the step is not rounded away
            params["means4"][0, 3] += sgn * h
            out = O.render_view(params, cam, t, sc.sh_degree, sc.t_order, sc.t_period, with_flags=False)
            vals.append(float(O.tile_linear_loss(out, torch.as_tensor(ones), cam=cam)))
        fd.append((vals[0] - vals[1]) / (2 * h))
    assert fd[0] * fd[1] < 0                    # the two views pull mu_t in opposite directions
    ref = abs(fd[0]) + abs(fd[1])
    assert abs(float(tg[0]) - ref) <= 1e-5 * (1 + ref)


# --- Sec. 4.4: rendered optical flow -------------------------------------------------
def _xt_rotation_scene(theta, sx=0.3, st=0.1):
    """One primitive at the origin rotated by theta in the (x, t) plane:
    q_l = q_r = (cos theta/2, 0, 0, sin theta/2) (x <-> 1, t <-> k)."""
    sc = scenegen.random_scene(28, 1, sh_degree=0, t_order=0)
    q = [math.cos(theta / 2), 0.0, 0.0, math.sin(theta / 2)]
    sc.q_left[:] = q
    sc.q_right[:] = q
    sc.means4[:] = [[0.0, 0.0, 0.0, 0.5]]
    sc.log_scales4[:] = [[math.log(sx), math.log(0.3), math.log(0.3), math.log(st)]]
    sc.opacity_logit[:] = [2.0]
    return sc


def test_static_primitives_have_no_flow():
    """q_l = (cos a, 0, 0, sin a), q_r = (cos a, 0, 0, -sin a) fixes the x and t
    axes and rotates the (y, z) plane: Sigma_xyz,t = 0, the slice mean does
    not move and no primitive has flow."""
    sc = scenegen.random_scene(29, 40, spread=0.6)
    ang = np.random.default_rng(30).uniform(0, math.pi, 40)
    sc.q_left[:] = np.stack([np.cos(ang), 0 * ang, 0 * ang, np.sin(ang)], 1)
    sc.q_right[:] = np.stack([np.cos(ang), 0 * ang, 0 * ang, -np.sin(ang)], 1)
    cam = scenegen.look_at_camera((0.4, 0.2, 3.5), 32, 32)
    out = O.render_flow(sc, cam, 0.5, 0.05, with_flags=False)
    flow = O.assemble(out, cam, "rgb", 3)
    assert float(flow.abs().max()) < 1e-12
    alpha = O.assemble(O.render_full(sc, cam, 0.5, with_flags=False), cam, "alpha")
    assert float(alpha.max()) > 0.5               # the primitives are on screen


def test_flow_of_xt_rotated_primitive_closed_form():
    """A rotation by theta in the (x, t) plane gives the slice mean the velocity
    Sigma_xt / Sigma_tt = (s_x^2 - s_t^2) sin cos / (s_x^2 sin^2 + s_t^2 cos^2)
    along world x (sign aside), which the camera on the z axis sees as a
    horizontal image velocity f_x v / z; the centre pixel holds its alpha times
    the displacement."""
    cam = scenegen.look_at_camera((0.0, 0.0, 4.0), 32, 32)
    sx, st, dt = 0.3, 0.1, 0.02
    flows = []
    for theta in (0.4, -0.4):
        sc = _xt_rotation_scene(theta, sx, st)
        out = O.render_flow(sc, cam, 0.5, dt, with_flags=False)
        flow = O.assemble(out, cam, "rgb", 3)
        alpha = O.assemble(O.render_full(sc, cam, 0.5, with_flags=False), cam, "alpha").detach()
        # the stored (float32) parameters, exactly
        qs = [float(x) for x in sc.q_left[0]]
        th = 2.0 * math.atan2(qs[3], qs[0])
        ax, at = math.exp(float(sc.log_scales4[0, 0])), math.exp(float(sc.log_scales4[0, 3]))
        vel = (ax * ax - at * at) * math.sin(th) * math.cos(th) / (
            ax * ax * math.sin(th) ** 2 + at * at * math.cos(th) ** 2)
        expect = float(alpha[15, 15]) * cam.fx * abs(vel) * dt / 4.0
        assert abs(abs(float(flow[0, 15, 15])) - expect) <= 1e-9 * (1 + expect)
        assert abs(float(flow[1, 15, 15])) < 1e-12 and float(flow[2].abs().max()) == 0.0
        flows.append(float(flow[0, 15, 15]))
    assert flows[0] != 0.0 and abs(flows[0] + flows[1]) <= 1e-12   # opposite rotations, opposite ways


# --- the parity margin policy ----------------------------------------------------
def _dense_scene(seed, n, grow, spread, sh, to):
    sc = scenegen.random_scene(seed, n, sh_degree=sh, t_order=to, spread=spread, mu_log_t=-1.5)
    sc.log_scales4[:, :3] += np.float32(grow)
    return sc


@pytest.mark.parametrize("seed,n,grow,spread,eye,w,h,t", [
    (6, 2500, 1.5, 0.5, (0.0, -0.3, 3.0), 48, 40, 0.6),
    (5, 3000, 0.8, 1.0, (1.0, 0.5, 3.5), 100, 70, 0.37),
])
def test_flags_cover_every_decision_within_fp32_reach(seed, n, grow, spread, eye, w, h, t):
    """The value flags are what the parity tests exclude, so they must hold
    every pixel whose value an FP32 implementation may move beyond the image
    tolerance by taking a decision the other way. Simulated here: the records
    rounded to float32 (depth order by the float32 depth, ties by index, as
    the GPU sorts), every fragment's alpha moved by a random amount within
    the float32 evaluation reach the margins assume. No unflagged pixel may
    change by more than the 1e-4 image tolerance. With the alphas moved 30x
    beyond that reach some unflagged pixel does (the check has teeth)."""
    sc = _dense_scene(seed, n, grow, spread, 3, 1)
    cam = O.to_ocamera(scenegen.look_at_camera(eye, w, h))
    params = O.params_from_scene(sc)
    pre = O.preprocess(params, cam, t, sc.sh_degree, sc.t_order)
    mg = O.Margins()
    tiles = range(cam.tiles_x * cam.tiles_y)
    base = {tid: O.composite_tile(pre, cam, tid, (0.0, 0.0, 0.0), mg) for tid in tiles}
    n_flagged = sum(int(b["uncertain"].sum()) for b in base.values())
    # the FP32 record: float32 u, v, conic, opacity and depth key
    p32 = dict(pre)
    p32["z"] = pre["z32"]
    p32["color"] = pre["color"].detach().to(torch.float32).to(F64)

    def worst(scale, trials, rng):
        w_unf = 0.0
        for _ in range(trials):
            def gval32(ids, pxc, pyc):
                _, gv32, eps = mg.alpha_fp32(pre, ids, pxc, pyc)
                k = torch.as_tensor(rng.uniform(-1.0, 1.0, size=tuple(gv32.shape)))
                return gv32 * (1.0 + scale * eps * k)
            for tid in tiles:
                a = base[tid]
                b = O.composite_tile(p32, cam, tid, (0.0, 0.0, 0.0), with_flags=False, gval_fn=gval32)
                d = torch.maximum((a["rgb"].detach() - b["rgb"].detach()).abs().amax(0),
                                  torch.maximum((a["depth"].detach() - b["depth"].detach()).abs(),
                                                (a["alpha"].detach() - b["alpha"].detach()).abs()))
                unf = ~a["uncertain"]
                if bool(unf.any()):
                    w_unf = max(w_unf, float(d[unf].max()))
        return w_unf

    rng = np.random.default_rng(seed)
    w1 = worst(1.0, 6, rng)
    assert w1 <= O.IMG_TOL, (w1, n_flagged)
    assert worst(30.0, 3, rng) > O.IMG_TOL
