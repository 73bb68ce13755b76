"""Python binding of libg4d (ctypes) and its torch.autograd wrapper.

Argument marshalling only: every step of the render and its backward runs in
the library's HIP kernels. PyTorch supplies device memory and the stream.
The binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime first, so libg4d binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libg4d.so")

G4D_OK, G4D_EINVAL, G4D_ENOMEM, G4D_EHIP, G4D_ESTATE, G4D_ECAPACITY = 0, -1, -2, -3, -4, -5
G4D_TUNE_SORT_BLOCKS, G4D_TUNE_STAGE_TIMING = 1, 2
G4D_TUNE_ROUND_PAIRS, G4D_TUNE_ROUND_INSTANCES = 3, 4
G4D_TUNE_SYNC_FREE, G4D_TUNE_ARENA_INSTANCES, G4D_TUNE_TILE_ORDER, G4D_TUNE_AUTOTUNE = 5, 6, 7, 8
G4D_TUNE_ELLIPSE_CULL, G4D_TUNE_PERSISTENT_BLOCKS, G4D_TUNE_LDS_BATCH = 9, 10, 11
G4D_GRAD_ACCUMULATE = 1
G4D_LOSS_L1, G4D_LOSS_L2 = 1, 2
STAGES = ["preprocess", "binning", "raster_fwd", "raster_bwd", "preprocess_bwd", "loss", "colour"]
DBG = dict(records=1, ids=2, tile_keys=3, tile_vals=4, ranges=5, pix_t=6, pix_last=7, grad2d=8, tile_order=9)

EXPORTED = ["g4d_default_options", "g4d_create", "g4d_destroy", "g4d_set_stream", "g4d_set_primitives",
            "g4d_render", "g4d_render_noalloc", "g4d_render_flow", "g4d_render_backward", "g4d_render_backward_loss", "g4d_image_loss", "g4d_get_stats", "g4d_set_tuning",
            "g4d_get_tuning", "g4d_set_densify_stats", "g4d_adam_step", "g4d_split_sample", "g4d_stage_times", "g4d_last_error", "g4d_debug_size", "g4d_debug_copy"]


class G4DOptions(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("t_order", ctypes.c_int32), ("t_period", ctypes.c_float),
                ("t_cull", ctypes.c_float), ("near_plane", ctypes.c_float), ("bg", ctypes.c_float * 3)]


class G4DCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("world_to_cam", ctypes.c_float * 12), ("center", ctypes.c_float * 3)]


class G4DStats(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int64), ("active_total", ctypes.c_int64), ("instances", ctypes.c_int64),
                ("tiles", ctypes.c_int64), ("max_tile_list", ctypes.c_int64), ("fragments", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("culled_nonfinite", ctypes.c_int64)]


class G4DError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"g4d error {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libg4d.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libg4d.so not found at {path}; build it with paper_2310_10642_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i32, i64, fp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.g4d_default_options.argtypes = [ctypes.POINTER(G4DOptions)]
    lib.g4d_default_options.restype = None
    lib.g4d_create.argtypes = [ctypes.POINTER(G4DOptions), vp, ctypes.POINTER(vp)]
    lib.g4d_destroy.argtypes = [vp]
    lib.g4d_set_stream.argtypes = [vp, vp]
    lib.g4d_set_primitives.argtypes = [vp, i64, fp, fp, fp, fp, fp, fp]
    lib.g4d_render.argtypes = [vp, i32, ctypes.POINTER(G4DCamera), ctypes.POINTER(ctypes.c_float), fp, fp, fp]
    lib.g4d_render_noalloc.argtypes = [vp, i32, ctypes.POINTER(G4DCamera), ctypes.POINTER(ctypes.c_float), fp, fp,
                                       fp]
    lib.g4d_render_flow.argtypes = [vp, i32, ctypes.POINTER(G4DCamera), ctypes.POINTER(ctypes.c_float), ctypes.c_float,
                                    fp]
    lib.g4d_render_backward.argtypes = [vp, fp, fp, fp, fp, fp, fp, fp, fp, fp, i32]
    lib.g4d_render_backward_loss.argtypes = [vp, i32, fp, fp, ctypes.c_float, fp, fp, fp, fp, fp, fp, fp, fp, fp,
                                             i32]
    lib.g4d_image_loss.argtypes = [vp, i32, i64, fp, fp, ctypes.c_float, fp, fp]
    lib.g4d_get_stats.argtypes = [vp, ctypes.POINTER(G4DStats), ctypes.POINTER(ctypes.c_int64)]
    lib.g4d_set_tuning.argtypes = [vp, i32, i32]
    lib.g4d_get_tuning.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.g4d_set_densify_stats.argtypes = [vp, fp, fp, vp]
    lib.g4d_adam_step.argtypes = [vp, i64, ctypes.POINTER(G4DAdamOptions), i64, ctypes.POINTER(vp),
                                  ctypes.POINTER(vp), fp, fp]
    lib.g4d_split_sample.argtypes = [vp, i64, vp, fp, fp]
    lib.g4d_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.g4d_last_error.argtypes = [vp]
    lib.g4d_last_error.restype = ctypes.c_char_p
    lib.g4d_debug_size.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.g4d_debug_copy.argtypes = [vp, i32, vp, i64]
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in ("g4d_default_options", "g4d_last_error"):
            fn.restype = ctypes.c_int32
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def to_camera(cam) -> G4DCamera:
    """From any object with width, height, fx, fy, cx, cy, world_to_cam[3,4], center[3]."""
    c = G4DCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w2c = np.asarray(cam.world_to_cam, dtype=np.float32).reshape(12)
    for i in range(12):
        c.world_to_cam[i] = float(w2c[i])
    ctr = np.asarray(cam.center, dtype=np.float32).reshape(3)
    for i in range(3):
        c.center[i] = float(ctr[i])
    return c


class G4DAdamOptions(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 6), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class Renderer:
    """One library context: options, borrowed primitives, last-render state."""

    def __init__(self, sh_degree: int = 3, t_order: int = 2, t_period: float = 1.0, t_cull: float = 0.05,
                 near_plane: float = 0.2, bg: Sequence[float] = (0.0, 0.0, 0.0)):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("g4d needs a HIP device")
        o = G4DOptions()
        self.lib.g4d_default_options(ctypes.byref(o))
        o.sh_degree, o.t_order, o.t_period, o.t_cull, o.near_plane = sh_degree, t_order, t_period, t_cull, near_plane
        for i in range(3):
            o.bg[i] = float(bg[i])
        self.opts = o
        self.sh_degree, self.t_order = sh_degree, t_order
        self.n_coeffs = (t_order + 1) * (sh_degree + 1) ** 2
        h = ctypes.c_void_p()
        self._check(self.lib.g4d_create(ctypes.byref(o), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                        ctypes.byref(h)), ctx=None)
        self.ctx = h
        self.generation = 0
        self._prims = None
        self._views = None
        self._densify = None
        self.n = -1

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.g4d_destroy(ctx)
            self.ctx = None

    def _check(self, status: int, ctx="self"):
        if status != G4D_OK:
            c = self.ctx if ctx == "self" else None
            msg = self.lib.g4d_last_error(c).decode() if c is not None else "invalid arguments"
            raise G4DError(status, msg)

    def _stream(self):
        self._check(self.lib.g4d_set_stream(self.ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def set_tuning(self, key: int, value: int):
        self._check(self.lib.g4d_set_tuning(self.ctx, key, value))

    def get_tuning(self, key: int) -> int:
        v = ctypes.c_int32()
        self._check(self.lib.g4d_get_tuning(self.ctx, key, ctypes.byref(v)))
        return int(v.value)

    def set_primitives(self, means4, log_scales4, q_left, q_right, opacity_logit, coeffs):
        ts = [means4, log_scales4, q_left, q_right, opacity_logit, coeffs]
        n = int(means4.shape[0])
        for t in ts:
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("primitive tensors must be contiguous float32 on the GPU")
            if int(t.shape[0]) != n:
                raise ValueError("primitive tensors disagree on n")
        if coeffs.numel() != n * self.n_coeffs * 3:
            raise ValueError(f"coeffs must hold n x {self.n_coeffs} x 3 values")
        if self._densify is not None and n != self.n:
            # the registered accumulators have the old primitive count
            self.set_densify_stats(None, None, None)
            raise ValueError(f"densification accumulators were registered for {self.n} primitives, not {n}; "
                             "register accumulators of the new size after set_primitives")
        self._prims = ts  # keep alive
        self._check(self.lib.g4d_set_primitives(self.ctx, n, *[_ptr(t) for t in ts]))
        self.n = n
        if self._densify is not None:
            # the library drops the accumulators on set_primitives; the same
            # primitive count keeps them registered (e.g. the autograd path,
            # which sets the primitives on every forward)
            self._check(self.lib.g4d_set_densify_stats(self.ctx, *[_ptr(t) for t in self._densify]))

    def render(self, cameras: Sequence, times: Sequence[float], depth: bool = True, alpha: bool = True,
               out: Optional[Sequence[Optional[torch.Tensor]]] = None):
        """Returns flat (rgb, depth, alpha) tensors over the concatenated views,
        written into `out` = (rgb, depth or None, alpha or None) when given."""
        self._stream()
        V = len(cameras)
        cams = (G4DCamera * V)(*[to_camera(c) for c in cameras])
        tarr = (ctypes.c_float * V)(*[float(t) for t in times])
        npix = sum(int(c.width) * int(c.height) for c in cameras)
        dev = torch.device("cuda", torch.cuda.current_device())
        if out is not None:
            rgb, dep, alp = out
            for t, k in ((rgb, 3), (dep, 1), (alp, 1)):
                if t is not None and not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                                          and t.numel() == k * npix):
                    raise ValueError("render outputs must be contiguous float32 GPU tensors of the batch's size")
        else:
            rgb = torch.empty(3 * npix, device=dev, dtype=torch.float32)
            dep = torch.empty(npix, device=dev, dtype=torch.float32) if depth else None
            alp = torch.empty(npix, device=dev, dtype=torch.float32) if alpha else None
        self._check(self.lib.g4d_render(self.ctx, V, cams, tarr, _ptr(rgb), _ptr(dep), _ptr(alp)))
        self.generation += 1
        self._views = [(int(c.height), int(c.width)) for c in cameras]
        return rgb, dep, alp

    def render_noalloc(self, cameras: Sequence, times: Sequence[float], out: Sequence[Optional[torch.Tensor]]):
        """g4d_render_noalloc into the caller's `out` = (rgb, depth or None,
        alpha or None): the library allocates nothing (fixed per-GPU scratch,
        limits in the header); no state is kept for backward."""
        self._stream()
        V = len(cameras)
        cams = (G4DCamera * V)(*[to_camera(c) for c in cameras])
        tarr = (ctypes.c_float * V)(*[float(t) for t in times])
        npix = sum(int(c.width) * int(c.height) for c in cameras)
        rgb, dep, alp = out
        for t, k in ((rgb, 3), (dep, 1), (alp, 1)):
            if t is not None and not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                                      and t.numel() == k * npix):
                raise ValueError("render outputs must be contiguous float32 GPU tensors of the batch's size")
        self._check(self.lib.g4d_render_noalloc(self.ctx, V, cams, tarr, _ptr(rgb), _ptr(dep), _ptr(alp)))
        self.generation += 1
        self._views = [(int(c.height), int(c.width)) for c in cameras]
        return rgb, dep, alp

    def render_flow(self, cameras: Sequence, times: Sequence[float], frame_dt: float,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Flat [sum 2 H W] optical flow (du, dv planes per view) over t -> t + frame_dt."""
        self._stream()
        V = len(cameras)
        cams = (G4DCamera * V)(*[to_camera(c) for c in cameras])
        tarr = (ctypes.c_float * V)(*[float(t) for t in times])
        npix = sum(int(c.width) * int(c.height) for c in cameras)
        if out is None:
            out = torch.empty(2 * npix, device=torch.device("cuda", torch.cuda.current_device()))
        elif not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.numel() == 2 * npix):
            raise ValueError("flow output must be a contiguous float32 GPU tensor of 2 x pixels")
        self._check(self.lib.g4d_render_flow(self.ctx, V, cams, tarr, float(frame_dt), _ptr(out)))
        self.generation += 1
        self._views = [(int(c.height), int(c.width)) for c in cameras]
        return out

    def split(self, rgb, depth=None, alpha=None):
        """Per-view [3,H,W] / [H,W] views of the flat outputs."""
        out, o3, o1 = [], 0, 0
        for (h, w) in self._views:
            item = [rgb[o3:o3 + 3 * h * w].view(3, h, w)]
            if depth is not None:
                item.append(depth[o1:o1 + h * w].view(h, w))
            if alpha is not None:
                item.append(alpha[o1:o1 + h * w].view(h, w))
            out.append(item)
            o3 += 3 * h * w
            o1 += h * w
        return out

    def grad_buffers(self, device=None) -> List[torch.Tensor]:
        n = self.n
        dev = device or torch.device("cuda", torch.cuda.current_device())
        return [torch.empty(n, 4, device=dev), torch.empty(n, 4, device=dev), torch.empty(n, 4, device=dev),
                torch.empty(n, 4, device=dev), torch.empty(n, device=dev),
                torch.empty(n, self.n_coeffs, 3, device=dev)]

    def backward(self, dl_rgb, dl_depth=None, dl_alpha=None, out: Optional[List[torch.Tensor]] = None,
                 accumulate: bool = False) -> List[torch.Tensor]:
        """Gradients of the last render; into `out` when given (added to it
        with accumulate=True, overwritten otherwise)."""
        self._stream()
        g = out if out is not None else self.grad_buffers(dl_rgb.device)
        args = [dl_rgb.contiguous(), None if dl_depth is None else dl_depth.contiguous(),
                None if dl_alpha is None else dl_alpha.contiguous()]
        flags = G4D_GRAD_ACCUMULATE if accumulate else 0
        self._check(self.lib.g4d_render_backward(self.ctx, *[_ptr(a) for a in args], *[_ptr(t) for t in g], flags))
        self._keep = args
        return g

    def backward_loss(self, kind: int, img: torch.Tensor, target: torch.Tensor, scale: float,
                      loss_out: torch.Tensor, dl_depth=None, dl_alpha=None,
                      out: Optional[List[torch.Tensor]] = None, accumulate: bool = False) -> List[torch.Tensor]:
        """image_loss(kind, img, target, scale, loss_out) and the backward of
        the last render from its dL/dimg in one library call (img: the
        render's rgb output); loss_out (1 float) is added to."""
        self._stream()
        g = out if out is not None else self.grad_buffers(img.device)
        args = [img.contiguous(), target.contiguous(), None if dl_depth is None else dl_depth.contiguous(),
                None if dl_alpha is None else dl_alpha.contiguous()]
        flags = G4D_GRAD_ACCUMULATE if accumulate else 0
        self._check(self.lib.g4d_render_backward_loss(self.ctx, kind, _ptr(args[0]), _ptr(args[1]), float(scale),
                                                      _ptr(loss_out), _ptr(args[2]), _ptr(args[3]),
                                                      *[_ptr(t) for t in g], flags))
        self._keep = args
        return g

    def set_densify_stats(self, uv_grad_norm_sum: Optional[torch.Tensor], t_grad_abs_sum: Optional[torch.Tensor],
                          blend_count: Optional[torch.Tensor]):
        """Registers per-primitive accumulators (float32, float32, int32 [n] on
        the GPU) that every later backward adds the densification statistics
        to; None for all three switches them off."""
        ts = (uv_grad_norm_sum, t_grad_abs_sum, blend_count)
        if all(t is None for t in ts):
            self._densify = None
            self._check(self.lib.g4d_set_densify_stats(self.ctx, None, None, None))
            return
        for t, dt in zip(ts, (torch.float32, torch.float32, torch.int32)):
            if t is None or not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == self.n):
                raise ValueError("densify accumulators: contiguous GPU float32, float32, int32 tensors of n values")
        self._densify = ts  # keep alive
        self._check(self.lib.g4d_set_densify_stats(self.ctx, *[_ptr(t) for t in ts]))

    def adam_step(self, params: Sequence[torch.Tensor], grads: Sequence[torch.Tensor], exp_avg: torch.Tensor,
                  exp_avg_sq: torch.Tensor, step: int, lr: Sequence[float], betas=(0.9, 0.999), eps: float = 1e-15):
        """One fused Adam step over the six groups (updated in place); the
        moment buffers hold n (17 + 3K) floats each, group after group."""
        self._stream()
        n = int(params[0].shape[0])
        for t in (*params, *grads, exp_avg, exp_avg_sq):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("adam_step tensors must be contiguous float32 on the GPU")
        if exp_avg.numel() != n * (17 + 3 * self.n_coeffs) or exp_avg_sq.numel() != exp_avg.numel():
            raise ValueError("moment buffers must hold n (17 + 3K) floats")
        o = G4DAdamOptions()
        for i in range(6):
            o.lr[i] = float(lr[i])
        o.beta1, o.beta2, o.eps = float(betas[0]), float(betas[1]), float(eps)
        P = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in params])
        G = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in grads])
        self._check(self.lib.g4d_adam_step(self.ctx, n, ctypes.byref(o), int(step), P, G, _ptr(exp_avg),
                                           _ptr(exp_avg_sq)))

    def split_sample(self, idx: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
        """New 4D positions mu_i + R_i S_i z_k for i = idx[k] (int32 [K], z [K, 4])."""
        self._stream()
        if not (idx.is_cuda and idx.dtype == torch.int32 and z.is_cuda and z.dtype == torch.float32
                and z.is_contiguous() and idx.is_contiguous() and z.shape == (idx.numel(), 4)):
            raise ValueError("split_sample needs int32 idx [K] and float32 z [K, 4] on the GPU")
        out = torch.empty_like(z)
        self._check(self.lib.g4d_split_sample(self.ctx, idx.numel(), _ptr(idx), _ptr(z), _ptr(out)))
        return out

    def image_loss(self, kind: int, img: torch.Tensor, target: torch.Tensor, scale: float,
                   loss_out: torch.Tensor, grad_out: torch.Tensor):
        """loss_out (1 float, added to) and grad_out = dL/dimg, computed by the library."""
        self._stream()
        self._check(self.lib.g4d_image_loss(self.ctx, kind, img.numel(), _ptr(img), _ptr(target),
                                            float(scale), _ptr(loss_out), _ptr(grad_out)))

    def stage_timing(self, on: bool):
        self.set_tuning(G4D_TUNE_STAGE_TIMING, 1 if on else 0)

    def stage_times(self) -> Dict[str, tuple]:
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        self._check(self.lib.g4d_stage_times(self.ctx, ms, n))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def stats(self) -> Dict[str, int]:
        s = G4DStats()
        V = len(self._views)
        per = (ctypes.c_int64 * V)()
        self._check(self.lib.g4d_get_stats(self.ctx, ctypes.byref(s), per))
        d = {k: int(getattr(s, k)) for k, _ in G4DStats._fields_}
        d["active_per_view"] = list(per)
        return d

    def debug(self, what: str) -> np.ndarray:
        code = DBG[what]
        nb = ctypes.c_int64()
        self._check(self.lib.g4d_debug_size(self.ctx, code, ctypes.byref(nb)))
        dt = {"records": np.float32, "pix_t": np.float32, "grad2d": np.float64}.get(what, np.uint32)
        arr = np.empty(int(nb.value) // np.dtype(dt).itemsize, dtype=dt)
        if arr.size:
            self._check(self.lib.g4d_debug_copy(self.ctx, code, arr.ctypes.data_as(ctypes.c_void_p), nb.value))
        if what == "records":
            arr = arr.reshape(-1, 12)
        if what == "grad2d":
            arr = arr.reshape(-1, 16)
        if what == "ranges":
            arr = arr.reshape(-1, 2)
        return arr


class Render4DGS(torch.autograd.Function):
    """rgb, depth, alpha = Render4DGS.apply(renderer, cameras, times, means4,
    log_scales4, q_left, q_right, opacity_logit, coeffs); flat outputs over the
    concatenated views. Backward returns the library's summed gradients."""

    @staticmethod
    def forward(ctx, renderer: Renderer, cameras, times, means4, log_scales4, q_left, q_right, opacity_logit,
                coeffs):
        renderer.set_primitives(means4.contiguous(), log_scales4.contiguous(), q_left.contiguous(),
                                q_right.contiguous(), opacity_logit.contiguous(), coeffs.contiguous())
        rgb, dep, alp = renderer.render(cameras, times)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.save_for_backward(means4, log_scales4, q_left, q_right, opacity_logit, coeffs)
        return rgb, dep, alp

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha):
        # unpacking makes autograd check that no parameter was modified in
        # place since the forward: the library reads them again here
        _ = ctx.saved_tensors
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("g4d: another render ran on this Renderer before this backward")
        grads = r.backward(g_rgb, g_depth, g_alpha)
        return (None, None, None, *grads)


def render(renderer: Renderer, cameras, times, means4, log_scales4, q_left, q_right, opacity_logit, coeffs):
    return Render4DGS.apply(renderer, cameras, times, means4, log_scales4, q_left, q_right, opacity_logit, coeffs)
