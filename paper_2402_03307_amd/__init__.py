"""MI355X-native 4D-rotor Gaussian splatting renderer (forward + backward).

Thin ctypes binding of the HIP library libr4d.so (C ABI in include/r4d.h).
It only marshals arguments: every step of the render and of its derivative
runs in the library's HIP kernels.  PyTorch supplies device memory and the
current HIP stream.  If the library has not been built this module raises
ImportError; there is no fallback implementation.

    import paper_2402_03307_amd as r4d
    images = r4d.render(params, views, settings)     # list of [3, H, W] tensors
    loss = sum(...); loss.backward()                 # gradients via r4d_render_backward

params: dict of CUDA tensors (float32, or float64 for the test-only path):
    means [4, n], log_scales [4, n], rotors [8, n], opacity [n], sh [3k, n],
    plus "sh_degree" (int).
views: list of dicts with width, height, fx, fy, cx, cy, world_to_cam (3x4),
    t and bg (3 floats).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libr4d.so")

__all__ = ["render", "render_flow", "Renderer", "TrainState", "adam_config", "R4DError",
           "default_settings", "LIB_PATH", "BUF_RECORDS", "BUF_RECT", "BUF_DEPTHKEY",
           "BUF_VALUES", "BUF_RANGES", "BUF_TFINAL", "BUF_NCONTRIB", "BUF_NEVAL", "BUF_FLOW",
           "BUF_NBLEND", "BUF_REST", "EXPORTED_SYMBOLS", "MODE_PER_VIEW", "MODE_FUSED",
           "MODE_GRAPH"]

(BUF_RECORDS, BUF_RECT, BUF_DEPTHKEY, BUF_VALUES, BUF_RANGES, BUF_TFINAL, BUF_NCONTRIB,
 BUF_NEVAL, BUF_FLOW, BUF_NBLEND, BUF_REST) = range(11)

# execution modes of a multi-view call (see R4D_MODE_* in include/r4d.h)
MODE_PER_VIEW, MODE_FUSED, MODE_GRAPH = 0, 1, 2
_MODE_NAMES = {"per_view": MODE_PER_VIEW, "fused": MODE_FUSED, "graph": MODE_GRAPH}

EXPORTED_SYMBOLS = (
    "r4d_default_settings", "r4d_create", "r4d_destroy", "r4d_render_forward",
    "r4d_render_backward", "r4d_render_forward_f64", "r4d_render_backward_f64",
    "r4d_render_forward_noalloc",
    "r4d_render_forward_flow", "r4d_render_backward_flow", "r4d_render_forward_flow_f64",
    "r4d_render_backward_flow_f64", "r4d_knn4d", "r4d_consistency4d_loss_grad",
    "r4d_consistency4d_loss_grad_f64", "r4d_default_adam_config", "r4d_adam_step",
    "r4d_train_state_init", "r4d_opacity_reset", "r4d_entropy_loss_grad", "r4d_render_backward_stats",
    "r4d_default_densify_config", "r4d_densify", "r4d_render_forward_3d",
    "r4d_render_backward_3d", "r4d_render_forward_3d_f64", "r4d_render_backward_3d_f64",
    "r4d_saved_release", "r4d_l1_loss_grad", "r4d_l1_loss_grad_views", "r4d_saved_stats",
    "r4d_saved_front_stats", "r4d_saved_copy", "r4d_saved_check", "r4d_check_pending", "r4d_saved_config",
    "r4d_status_string",
    "r4d_last_error", "r4d_set_timing", "r4d_get_timings", "r4d_stage_name",
)
NUM_STAGES = 9


class R4DError(RuntimeError):
    pass


c_i32, c_f32, c_vp = ctypes.c_int32, ctypes.c_float, ctypes.c_void_p


class _Gaussians(ctypes.Structure):
    _fields_ = [("n", c_i32), ("sh_degree", c_i32), ("means", c_vp), ("log_scales", c_vp),
                ("rotors", c_vp), ("opacity", c_vp), ("sh", c_vp)]


class _View(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("fx", c_f32), ("fy", c_f32),
                ("cx", c_f32), ("cy", c_f32), ("world_to_cam", c_f32 * 12), ("t", c_f32),
                ("bg", c_f32 * 3)]


class _Settings(ctypes.Structure):
    _fields_ = [("tile_size", c_i32), ("near_plane", c_f32), ("time_cull", c_f32),
                ("extent_sigma", c_f32), ("alpha_min", c_f32), ("alpha_max", c_f32),
                ("T_min", c_f32), ("dilation", c_f32), ("guard_band", c_f32),
                ("fwd_pixels_per_thread", c_i32), ("bwd_pixels_per_thread", c_i32),
                ("mode", c_i32), ("sort_items", c_i32), ("front_fraction", c_f32),
                ("front_keep", c_i32)]


class _AdamConfig(ctypes.Structure):
    _fields_ = [("lr_means_init", c_f32), ("lr_means_final", c_f32), ("lr_means_steps", c_i32),
                ("lr_log_scales", c_f32), ("lr_rotors", c_f32), ("lr_opacity", c_f32),
                ("lr_sh_dc", c_f32), ("lr_sh_rest", c_f32), ("beta1", c_f32), ("beta2", c_f32),
                ("eps", c_f32)]


class _TrainState(ctypes.Structure):
    _fields_ = [("n", c_i32), ("sh_degree", c_i32), ("means", c_vp), ("log_scales", c_vp),
                ("rotors", c_vp), ("opacity", c_vp), ("sh", c_vp), ("opacity_logit", c_vp),
                ("adam_m", c_vp), ("adam_v", c_vp), ("step", c_vp)]


class _DensifyConfig(ctypes.Structure):
    _fields_ = [("grad_threshold", c_f32), ("size_threshold", c_f32), ("min_opacity", c_f32),
                ("max_size", c_f32)]


class _Grads(ctypes.Structure):
    _fields_ = [("means", c_vp), ("log_scales", c_vp), ("rotors", c_vp), ("opacity", c_vp),
                ("sh", c_vp)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2402_03307_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.r4d_default_settings.argtypes = [P(_Settings)]
    lib.r4d_default_settings.restype = None
    lib.r4d_create.argtypes = [P(c_vp), ctypes.c_int]
    lib.r4d_create.restype = ctypes.c_int
    lib.r4d_destroy.argtypes = [c_vp]
    lib.r4d_destroy.restype = None
    fwd_args = [c_vp, P(_Gaussians), P(_View), ctypes.c_int, P(_Settings), c_vp, P(c_vp), c_vp]
    bwd_args = [c_vp, P(_Gaussians), P(_View), ctypes.c_int, P(_Settings), c_vp, c_vp, P(_Grads),
                c_vp]
    for name, args in (("r4d_render_forward", fwd_args), ("r4d_render_forward_f64", fwd_args),
                       ("r4d_render_backward", bwd_args), ("r4d_render_backward_f64", bwd_args)):
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.r4d_render_forward_noalloc.argtypes = [c_vp, P(_Gaussians), P(_View), ctypes.c_int,
                                               P(_Settings), c_vp, c_vp]
    lib.r4d_render_forward_noalloc.restype = ctypes.c_int
    ffwd_args = [c_vp, P(_Gaussians), P(_View), ctypes.c_int, P(_Settings), c_vp, c_vp, P(c_vp),
                 c_vp]
    fbwd_args = [c_vp, P(_Gaussians), P(_View), ctypes.c_int, P(_Settings), c_vp, c_vp, c_vp,
                 P(_Grads), c_vp]
    for name, args in (("r4d_render_forward_flow", ffwd_args),
                       ("r4d_render_forward_flow_f64", ffwd_args),
                       ("r4d_render_backward_flow", fbwd_args),
                       ("r4d_render_backward_flow_f64", fbwd_args)):
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.r4d_knn4d.argtypes = [c_vp, c_vp, c_i32, c_i32, c_f32, c_f32, c_vp, c_vp]
    lib.r4d_knn4d.restype = ctypes.c_int
    lib.r4d_consistency4d_loss_grad.argtypes = [c_vp, P(_Gaussians), c_vp, c_i32, c_f32, c_vp,
                                                P(_Grads), c_vp]
    lib.r4d_consistency4d_loss_grad.restype = ctypes.c_int
    lib.r4d_consistency4d_loss_grad_f64.argtypes = [c_vp, P(_Gaussians), c_vp, c_i32,
                                                    ctypes.c_double, c_vp, P(_Grads), c_vp]
    lib.r4d_consistency4d_loss_grad_f64.restype = ctypes.c_int
    lib.r4d_default_adam_config.argtypes = [P(_AdamConfig)]
    lib.r4d_default_adam_config.restype = None
    lib.r4d_adam_step.argtypes = [c_vp, P(_TrainState), P(_Grads), P(_AdamConfig), c_vp]
    lib.r4d_adam_step.restype = ctypes.c_int
    lib.r4d_train_state_init.argtypes = [c_vp, P(_TrainState), c_vp]
    lib.r4d_train_state_init.restype = ctypes.c_int
    lib.r4d_opacity_reset.argtypes = [c_vp, P(_TrainState), c_f32, c_vp]
    lib.r4d_opacity_reset.restype = ctypes.c_int
    lib.r4d_entropy_loss_grad.argtypes = [c_vp, c_vp, c_i32, c_f32, c_vp, c_vp, c_vp]
    lib.r4d_entropy_loss_grad.restype = ctypes.c_int
    lib.r4d_render_backward_stats.argtypes = [c_vp, P(_Gaussians), P(_View), ctypes.c_int,
                                              P(_Settings), c_vp, c_vp, c_vp, P(_Grads), c_vp,
                                              c_vp, c_vp]
    lib.r4d_render_backward_stats.restype = ctypes.c_int
    lib.r4d_default_densify_config.argtypes = [P(_DensifyConfig)]
    lib.r4d_default_densify_config.restype = None
    lib.r4d_densify.argtypes = [c_vp, P(_TrainState), c_vp, c_vp, c_vp, P(_DensifyConfig),
                                P(_TrainState), P(c_i32), c_vp]
    lib.r4d_densify.restype = ctypes.c_int
    for name, args in (("r4d_render_forward_3d", fwd_args), ("r4d_render_forward_3d_f64", fwd_args),
                       ("r4d_render_backward_3d", bwd_args),
                       ("r4d_render_backward_3d_f64", bwd_args)):
        fn = getattr(lib, name)       # same argument layouts as the 4D calls
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.r4d_saved_release.argtypes = [c_vp]
    lib.r4d_saved_release.restype = None
    lib.r4d_l1_loss_grad.argtypes = [c_vp, c_vp, c_vp, ctypes.c_int64, c_vp, c_vp, c_vp]
    lib.r4d_l1_loss_grad.restype = ctypes.c_int
    lib.r4d_l1_loss_grad_views.argtypes = [c_vp, c_vp, c_vp, P(_View), ctypes.c_int, c_vp, c_vp,
                                           c_vp]
    lib.r4d_l1_loss_grad_views.restype = ctypes.c_int
    lib.r4d_saved_check.argtypes = [c_vp]
    lib.r4d_saved_check.restype = ctypes.c_int
    lib.r4d_check_pending.argtypes = [c_vp]
    lib.r4d_check_pending.restype = ctypes.c_int
    lib.r4d_saved_config.argtypes = [c_vp, P(c_i32), P(c_i32), P(c_i32)]
    lib.r4d_saved_config.restype = ctypes.c_int
    lib.r4d_saved_stats.argtypes = [c_vp, ctypes.c_int, P(ctypes.c_int64), P(ctypes.c_int64),
                                    P(c_i32), P(c_i32)]
    lib.r4d_saved_stats.restype = ctypes.c_int
    lib.r4d_saved_front_stats.argtypes = [c_vp, ctypes.c_int] + [P(ctypes.c_int64)] * 4
    lib.r4d_saved_front_stats.restype = ctypes.c_int
    lib.r4d_saved_copy.argtypes = [c_vp, ctypes.c_int, ctypes.c_int, c_vp, ctypes.c_size_t, c_vp]
    lib.r4d_saved_copy.restype = ctypes.c_int
    lib.r4d_status_string.argtypes = [ctypes.c_int]
    lib.r4d_status_string.restype = ctypes.c_char_p
    lib.r4d_last_error.argtypes = [c_vp]
    lib.r4d_last_error.restype = ctypes.c_char_p
    lib.r4d_set_timing.argtypes = [c_vp, ctypes.c_int]
    lib.r4d_set_timing.restype = ctypes.c_int
    lib.r4d_get_timings.argtypes = [c_vp, P(ctypes.c_double), P(ctypes.c_int64), ctypes.c_int]
    lib.r4d_get_timings.restype = ctypes.c_int
    lib.r4d_stage_name.argtypes = [ctypes.c_int]
    lib.r4d_stage_name.restype = ctypes.c_char_p
    return lib


_lib = _load()


def library():
    return _lib


def default_settings() -> dict:
    s = _Settings()
    _lib.r4d_default_settings(ctypes.byref(s))
    return {name: getattr(s, name) for name, _ in _Settings._fields_}


def _settings_dict(s: _Settings) -> dict:
    return {name: getattr(s, name) for name, _ in _Settings._fields_}


def _settings_struct(settings: dict | None) -> _Settings:
    s = _Settings()
    _lib.r4d_default_settings(ctypes.byref(s))
    for k, v in (settings or {}).items():
        if k == "mode" and isinstance(v, str):
            v = _MODE_NAMES[v]
        if hasattr(s, k):
            setattr(s, k, type(getattr(s, k))(v))
    return s


def _views_array(views):
    arr = (_View * len(views))()
    for i, v in enumerate(views):
        arr[i].width = int(v["width"])
        arr[i].height = int(v["height"])
        arr[i].fx, arr[i].fy = float(v["fx"]), float(v["fy"])
        arr[i].cx, arr[i].cy = float(v["cx"]), float(v["cy"])
        w2c = np.asarray(v["world_to_cam"], dtype=np.float32).reshape(12)
        for j in range(12):
            arr[i].world_to_cam[j] = float(w2c[j])
        arr[i].t = float(v["t"])
        bg = v.get("bg", (0.0, 0.0, 0.0))
        for j in range(3):
            arr[i].bg[j] = float(bg[j])
    return arr


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_PARAM_KEYS = ("means", "log_scales", "rotors", "opacity", "sh")


_STATIC_KEYS = ("means", "log_scales", "quats", "opacity", "sh")


def _check_params(p: dict, static: bool = False):
    deg = int(p["sh_degree"])
    n = p["opacity"].shape[-1]
    k = (deg + 1) ** 2
    if static:
        shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n), "opacity": (n,),
                  "sh": (3 * k, n)}
    else:
        shapes = {"means": (4, n), "log_scales": (4, n), "rotors": (8, n), "opacity": (n,),
                  "sh": (3 * k, n)}
    dtype = p["means"].dtype
    for key, shp in shapes.items():
        t = p[key]
        if tuple(t.shape) != shp:
            raise ValueError(f"{key}: expected shape {shp}, got {tuple(t.shape)}")
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
            raise ValueError(f"{key}: must be a contiguous CUDA tensor of one dtype")
    if dtype not in (torch.float32, torch.float64):
        raise ValueError("parameters must be float32 or float64")
    return n, deg, dtype


# Live library objects, released in a safe order (saved states, then contexts)
# at interpreter exit, before the HIP runtime goes away.
_live_saved = weakref.WeakSet()
_live_renderers = weakref.WeakSet()


def _split(flat: torch.Tensor, views, channels: int):
    """Per-view [channels, H, W] views of a flat output in the forward's layout."""
    out, off = [], 0
    for v in views:
        h, w = int(v["height"]), int(v["width"])
        out.append(flat[off:off + channels * h * w].view(channels, h, w))
        off += channels * h * w
    return out


def _flat(grads, dtype) -> torch.Tensor:
    """One contiguous tensor of `dtype` from a flat tensor or a list of per-view ones."""
    if isinstance(grads, torch.Tensor):
        d = grads.reshape(-1)
        if d.dtype != dtype or not d.is_contiguous():
            d = d.to(dtype).contiguous()
        return d
    return torch.cat([gi.reshape(-1).to(dtype) for gi in grads]).contiguous()


@atexit.register
def _release_all():
    for s in list(_live_saved):
        s.release()
    for r in list(_live_renderers):
        r.close(sync=False)


class SavedState:
    """Opaque per-forward state kept for the backward pass."""

    def __init__(self, renderer: "Renderer", handle: ctypes.c_void_p, views, dtype,
                 settings: dict | None = None):
        self.renderer = renderer
        self.handle = handle
        self.views = views
        self.dtype = dtype
        self.settings = dict(settings or {})  # as passed to the library (defaults filled in)
        _live_saved.add(self)

    def release(self):
        if self.handle is not None and self.handle.value:
            _lib.r4d_saved_release(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def check(self):
        """Waits for the forward call and raises if it overflowed or failed
        after returning (see r4d_saved_check)."""
        if self.handle is None:
            raise R4DError("saved state already released")
        self.renderer._check(_lib.r4d_saved_check(self.handle), "r4d_saved_check")

    def config(self) -> dict:
        ts, items, mode = c_i32(), c_i32(), c_i32()
        self.renderer._check(_lib.r4d_saved_config(self.handle, ctypes.byref(ts),
                                                   ctypes.byref(items), ctypes.byref(mode)),
                             "r4d_saved_config")
        return {"tile_size": ts.value, "sort_items": items.value, "mode": mode.value}

    def stats(self, view: int = 0) -> dict:
        if self.handle is None:
            raise R4DError("saved state already released")
        nv, nd = ctypes.c_int64(), ctypes.c_int64()
        tx, ty = c_i32(), c_i32()
        st = _lib.r4d_saved_stats(self.handle, view, ctypes.byref(nv), ctypes.byref(nd),
                                  ctypes.byref(tx), ctypes.byref(ty))
        self.renderer._check(st, "r4d_saved_stats")
        out = {"n_visible": nv.value, "n_dup": nd.value, "tiles_x": tx.value,
               "tiles_y": ty.value}
        f = [ctypes.c_int64() for _ in range(4)]
        st = _lib.r4d_saved_front_stats(self.handle, view, *[ctypes.byref(x) for x in f])
        self.renderer._check(st, "r4d_saved_front_stats")
        out.update(zip(("n_front", "n_values", "rest_tiles", "rest_entries"),
                       (x.value for x in f)))
        return out

    def copy(self, view: int, buffer: int, n_gaussians: int) -> torch.Tensor:
        """Device copy of one saved buffer (see r4d_saved_copy)."""
        v = self.views[view]
        hw = int(v["width"]) * int(v["height"])
        s = self.stats(view)
        fdt = self.dtype
        shapes = {BUF_RECORDS: ((n_gaussians, 12), fdt), BUF_RECT: ((n_gaussians, 4), torch.int16),
                  BUF_DEPTHKEY: ((n_gaussians,), torch.int32),
                  BUF_VALUES: ((s["n_values"],), torch.int32),
                  BUF_RANGES: ((s["tiles_x"] * s["tiles_y"], 2), torch.int32),
                  BUF_REST: ((s["tiles_x"] * s["tiles_y"], 2), torch.int32),
                  BUF_TFINAL: ((hw,), fdt), BUF_NCONTRIB: ((hw,), torch.int32),
                  BUF_NEVAL: ((hw,), torch.int32), BUF_NBLEND: ((hw,), torch.int32),
                  BUF_FLOW: ((n_gaussians, 2), fdt)}
        shape, dt = shapes[buffer]
        out = torch.empty(shape, dtype=dt, device=self.renderer.device)
        st = _lib.r4d_saved_copy(self.handle, view, buffer, _ptr(out),
                                 out.numel() * out.element_size(), _stream(self.renderer.device))
        self.renderer._check(st, "r4d_saved_copy")
        return out


class Renderer:
    """Owns one r4d context on one device."""

    def __init__(self, device: int | torch.device = 0):
        if isinstance(device, torch.device):
            device = device.index or 0
        self.device = torch.device("cuda", int(device))
        h = ctypes.c_void_p()
        st = _lib.r4d_create(ctypes.byref(h), int(device))
        if st != 0:
            raise R4DError(f"r4d_create failed: {_lib.r4d_status_string(st).decode()}")
        self.handle = h
        self._persistent = {}
        _live_renderers.add(self)

    def close(self, sync: bool = True):
        if getattr(self, "handle", None) is not None and self.handle.value:
            if sync:
                torch.cuda.synchronize(self.device)
            _lib.r4d_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check_pending(self):
        """Waits for the forwards whose status nobody has read (calls with
        save=False, saved states released unchecked) and raises if one of them
        overflowed its tile lists or failed to sort (r4d_check_pending)."""
        self._check(_lib.r4d_check_pending(self.handle), "r4d_check_pending")

    def _check(self, status: int, what: str):
        if status != 0:
            msg = _lib.r4d_last_error(self.handle).decode()
            raise R4DError(f"{what}: {_lib.r4d_status_string(status).decode()}: {msg}")

    def _buffer(self, key, shape, dtype, persistent: bool):
        """A fresh tensor, or in graph mode one kept per key (graph replays
        read and write fixed addresses)."""
        if not persistent:
            return torch.empty(shape, dtype=dtype, device=self.device)
        t = self._persistent.get(key)
        if t is None or tuple(t.shape) != tuple(shape) or t.dtype != dtype:
            t = torch.empty(shape, dtype=dtype, device=self.device)
            self._persistent[key] = t
        return t

    def forward(self, params: dict, views, settings: dict | None = None, save: bool = True,
                flat: bool = False, flow: bool = False):
        """Renders `views`; returns (list of [3, H, W] images, SavedState or
        None), or with flat=True the images as one 1-D tensor in the layout of
        r4d_render_forward.  With flow=True (r4d_render_forward_flow) it returns
        (images, flow images, SavedState or None), the flow images as [2, H, W]
        tensors (or one flat tensor).  In graph mode the outputs live in buffers
        that the next graph forward of the same shape overwrites."""
        n, deg, dtype = _check_params(params)
        g = _Gaussians(n, deg, *[_ptr(params[k]) for k in _PARAM_KEYS])
        varr = _views_array(views)
        st = _settings_struct(settings)
        graph = st.mode == MODE_GRAPH
        sizes = [3 * int(v["height"]) * int(v["width"]) for v in views]
        key = (dtype, tuple(sizes), n) + tuple(params[k].data_ptr() for k in _PARAM_KEYS)
        out = self._buffer(("img", flow) + key, (sum(sizes),), dtype, graph)
        handle = ctypes.c_void_p()
        hptr = ctypes.byref(handle) if save else None
        if flow:
            fout = self._buffer(("flow",) + key, (sum(sizes) // 3 * 2,), dtype, graph)
            fn = (_lib.r4d_render_forward_flow if dtype == torch.float32
                  else _lib.r4d_render_forward_flow_f64)
            status = fn(self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st),
                        _ptr(out), _ptr(fout), hptr, _stream(self.device))
            self._check(status, "r4d_render_forward_flow")
        else:
            fn = _lib.r4d_render_forward if dtype == torch.float32 else _lib.r4d_render_forward_f64
            status = fn(self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st),
                        _ptr(out), hptr, _stream(self.device))
            self._check(status, "r4d_render_forward")
        saved = (SavedState(self, handle, views, dtype, _settings_dict(st)) if save else None)
        if flat:
            return (out, fout, saved) if flow else (out, saved)
        images = _split(out, views, 3)
        return (images, _split(fout, views, 2), saved) if flow else (images, saved)

    def forward_noalloc(self, params: dict, views, settings: dict | None = None,
                        out: torch.Tensor | None = None, flat: bool = False):
        """Inference render through r4d_render_forward_noalloc: no device memory
        is allocated by the library (every buffer lies in its fixed region).
        `out`: optional preallocated float32 image buffer (views' [3, H, W]
        images back to back), so that the call allocates nothing at all."""
        n, deg, dtype = _check_params(params)
        if dtype != torch.float32:
            raise R4DError("the no-allocation forward is float32 only")
        g = _Gaussians(n, deg, *[_ptr(params[k]) for k in _PARAM_KEYS])
        varr = _views_array(views)
        st = _settings_struct(settings)
        total = sum(3 * int(v["height"]) * int(v["width"]) for v in views)
        if out is None:
            out = torch.empty((total,), dtype=dtype, device=self.device)
        if (out.dtype != dtype or out.device != self.device or not out.is_contiguous()
                or out.numel() < total):
            raise R4DError("out must be a contiguous float32 tensor of the images' size "
                           "on the renderer's device")
        status = _lib.r4d_render_forward_noalloc(self.handle, ctypes.byref(g), varr, len(views),
                                                 ctypes.byref(st), _ptr(out),
                                                 _stream(self.device))
        self._check(status, "r4d_render_forward_noalloc")
        return out if flat else _split(out, views, 3)

    def backward(self, params: dict, views, settings: dict | None, saved: SavedState,
                 grad_images, grad_flows=None, stats=None) -> dict:
        """Gradients w.r.t. the five parameter tensors.  grad_images (and
        grad_flows, for the saved state of a flow render): list of [3, H, W]
        ([2, H, W]) tensors or one flat tensor in the forward's layout.  In graph
        mode the returned tensors are buffers that the next graph backward of
        the same shape overwrites."""
        n, deg, dtype = _check_params(params)
        g = _Gaussians(n, deg, *[_ptr(params[k]) for k in _PARAM_KEYS])
        varr = _views_array(views)
        st = _settings_struct(settings)
        graph = st.mode == MODE_GRAPH
        dl = _flat(grad_images, dtype)
        grads = {k: self._buffer(("grad", k, dtype, n), tuple(params[k].shape), dtype, graph)
                 for k in _PARAM_KEYS}
        gs = _Grads(*[_ptr(grads[k]) for k in _PARAM_KEYS])
        if stats is not None:
            # densification statistics (grad_accum float [n], vis_count int32 [n]), added to
            accum, count = stats
            dlf = _flat(grad_flows, dtype) if grad_flows is not None else None
            status = _lib.r4d_render_backward_stats(
                self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st), saved.handle,
                _ptr(dl), _ptr(dlf), ctypes.byref(gs), _ptr(accum), _ptr(count),
                _stream(self.device))
            self._check(status, "r4d_render_backward_stats")
            return grads
        if grad_flows is not None:
            dlf = _flat(grad_flows, dtype)
            fn = (_lib.r4d_render_backward_flow if dtype == torch.float32
                  else _lib.r4d_render_backward_flow_f64)
            status = fn(self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st),
                        saved.handle, _ptr(dl), _ptr(dlf), ctypes.byref(gs), _stream(self.device))
            self._check(status, "r4d_render_backward_flow")
            return grads
        fn = _lib.r4d_render_backward if dtype == torch.float32 else _lib.r4d_render_backward_f64
        status = fn(self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st),
                    saved.handle, _ptr(dl), ctypes.byref(gs), _stream(self.device))
        self._check(status, "r4d_render_backward")
        return grads

    def knn4d(self, means: torch.Tensor, k: int = 8, spatial_scale: float = 1.0,
              temporal_scale: float = 1.0) -> torch.Tensor:
        """[n, k] int32 indices of each Gaussian's k nearest other Gaussians in
        scaled 4D space (r4d_knn4d); means: [4, n] float32 on this device."""
        if means.dtype != torch.float32 or means.dim() != 2 or means.shape[0] != 4:
            raise ValueError("means must be a [4, n] float32 tensor")
        means = means.contiguous()
        n = int(means.shape[1])
        out = torch.empty((n, int(k)), dtype=torch.int32, device=self.device)
        st = _lib.r4d_knn4d(self.handle, _ptr(means), n, int(k), float(spatial_scale),
                            float(temporal_scale), _ptr(out), _stream(self.device))
        self._check(st, "r4d_knn4d")
        return out

    def consistency4d(self, params: dict, neighbours: torch.Tensor, weight: float = 1.0,
                      grads: dict | None = None, need_grad: bool = True):
        """4D consistency loss (r4d_consistency4d_loss_grad): returns (loss
        tensor, grads) where grads["rotors"] and grads["log_scales"] have had
        weight * dL/d(.) added (fresh zero tensors when `grads` is None; no
        gradient when need_grad is False)."""
        n, deg, dtype = _check_params(params)
        g = _Gaussians(n, deg, *[_ptr(params[k]) for k in _PARAM_KEYS])
        nb = neighbours.to(torch.int32).contiguous()
        if nb.dim() != 2 or nb.shape[0] != n:
            raise ValueError("neighbours must be [n, k]")
        loss = torch.empty(1, dtype=dtype, device=self.device)
        gs = None
        if need_grad:
            if grads is None:
                grads = {k: torch.zeros_like(params[k]) for k in ("rotors", "log_scales")}
            gs = _Grads(None, _ptr(grads["log_scales"]), _ptr(grads["rotors"]), None, None)
        fn = (_lib.r4d_consistency4d_loss_grad if dtype == torch.float32
              else _lib.r4d_consistency4d_loss_grad_f64)
        st = fn(self.handle, ctypes.byref(g), _ptr(nb), int(nb.shape[1]), float(weight),
                _ptr(loss), ctypes.byref(gs) if gs is not None else None, _stream(self.device))
        self._check(st, "r4d_consistency4d_loss_grad")
        return loss[0], grads

    def entropy_loss_grad(self, opacity: torch.Tensor, weight: float = 1.0,
                          grad: torch.Tensor | None = None):
        """Entropy loss (r4d_entropy_loss_grad): returns (loss, grad) with
        grad += weight * dL/do (a fresh zero tensor when None)."""
        opacity = opacity.contiguous()
        grad = torch.zeros_like(opacity) if grad is None else grad
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        st = _lib.r4d_entropy_loss_grad(self.handle, _ptr(opacity), int(opacity.numel()),
                                        float(weight), _ptr(loss), _ptr(grad),
                                        _stream(self.device))
        self._check(st, "r4d_entropy_loss_grad")
        return loss[0], grad

    def adam_step(self, state: "TrainState", grads: dict, config: dict | None = None):
        """One fused Adam step (r4d_adam_step) of the train state's parameters."""
        gs = _Grads(*[_ptr(grads[k]) for k in _PARAM_KEYS])
        cfg = adam_config(config)
        st = _lib.r4d_adam_step(self.handle, ctypes.byref(state.struct()), ctypes.byref(gs),
                                ctypes.byref(cfg), _stream(self.device))
        self._check(st, "r4d_adam_step")

    def densify(self, state: "TrainState", grad_accum: torch.Tensor, vis_count: torch.Tensor,
                normals: torch.Tensor, config: dict | None = None) -> "TrainState":
        """Clone / split / prune (r4d_densify); returns the new TrainState (its
        tensors freshly allocated).  normals: [4, 2n] float32 N(0, 1) draws."""
        n, deg = state.n, state.deg
        cap = max(2 * n, 1)
        dev = state.params["means"].device
        rows = {k: int(state.params[k].shape[0]) if state.params[k].dim() == 2 else 1
                for k in _PARAM_KEYS}
        flat = {k: torch.empty(rows[k] * cap, dtype=torch.float32, device=dev) for k in _PARAM_KEYS}
        total_rows = sum(rows.values())
        logit = torch.empty(cap, dtype=torch.float32, device=dev)
        m = torch.empty(total_rows * cap, dtype=torch.float32, device=dev)
        v = torch.empty(total_rows * cap, dtype=torch.float32, device=dev)
        step = torch.zeros(1, dtype=torch.int32, device=dev)
        out = _TrainState(cap, deg, *[_ptr(flat[k]) for k in _PARAM_KEYS], _ptr(logit), _ptr(m),
                          _ptr(v), _ptr(step))
        cfg = _DensifyConfig()
        _lib.r4d_default_densify_config(ctypes.byref(cfg))
        for key, val in (config or {}).items():
            setattr(cfg, key, val)
        n_out = c_i32()
        st = _lib.r4d_densify(self.handle, ctypes.byref(state.struct()), _ptr(grad_accum),
                              _ptr(vis_count), _ptr(normals.contiguous()), ctypes.byref(cfg),
                              ctypes.byref(out), ctypes.byref(n_out), _stream(self.device))
        self._check(st, "r4d_densify")
        k = n_out.value
        params = {key: (flat[key][:rows[key] * k].view(rows[key], k) if state.params[key].dim() == 2
                        else flat[key][:k]) for key in _PARAM_KEYS}
        params["sh_degree"] = deg
        new = TrainState.__new__(TrainState)
        new.params, new.n, new.deg = params, k, deg
        new.opacity_logit = logit[:k]
        new.m = m[:total_rows * k]
        new.v = v[:total_rows * k]
        new.step = step
        return new

    def opacity_reset(self, state: "TrainState", cap: float = 0.01):
        st = _lib.r4d_opacity_reset(self.handle, ctypes.byref(state.struct()), float(cap),
                                    _stream(self.device))
        self._check(st, "r4d_opacity_reset")

    def forward_static(self, params: dict, views, settings: dict | None = None,
                       save: bool = True, flat: bool = False):
        """Render of static 3D Gaussians (r4d_render_forward_3d); params: means
        [3, n], log_scales [3, n], quats [4, n] (w, x, y, z), opacity [n], sh
        [3k, n], sh_degree.  Returns (images, SavedState or None)."""
        n, deg, dtype = _check_params(params, static=True)
        g = _Gaussians(n, deg, *[_ptr(params[k]) for k in _STATIC_KEYS])
        varr = _views_array(views)
        st = _settings_struct(settings)
        graph = st.mode == MODE_GRAPH
        sizes = [3 * int(v["height"]) * int(v["width"]) for v in views]
        key = ("img3d", dtype, tuple(sizes), n) + tuple(params[k].data_ptr() for k in _STATIC_KEYS)
        out = self._buffer(key, (sum(sizes),), dtype, graph)
        handle = ctypes.c_void_p()
        fn = _lib.r4d_render_forward_3d if dtype == torch.float32 else _lib.r4d_render_forward_3d_f64
        status = fn(self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st), _ptr(out),
                    ctypes.byref(handle) if save else None, _stream(self.device))
        self._check(status, "r4d_render_forward_3d")
        saved = (SavedState(self, handle, views, dtype, _settings_dict(st)) if save else None)
        return (out, saved) if flat else (_split(out, views, 3), saved)

    def backward_static(self, params: dict, views, settings: dict | None, saved: SavedState,
                        grad_images) -> dict:
        """Gradients of a static render w.r.t. means, log_scales, quats, opacity
        and sh (r4d_render_backward_3d)."""
        n, deg, dtype = _check_params(params, static=True)
        g = _Gaussians(n, deg, *[_ptr(params[k]) for k in _STATIC_KEYS])
        varr = _views_array(views)
        st = _settings_struct(settings)
        graph = st.mode == MODE_GRAPH
        dl = _flat(grad_images, dtype)
        grads = {k: self._buffer(("grad3d", k, dtype, n), tuple(params[k].shape), dtype, graph)
                 for k in _STATIC_KEYS}
        gs = _Grads(*[_ptr(grads[k]) for k in _STATIC_KEYS])
        fn = (_lib.r4d_render_backward_3d if dtype == torch.float32
              else _lib.r4d_render_backward_3d_f64)
        status = fn(self.handle, ctypes.byref(g), varr, len(views), ctypes.byref(st),
                    saved.handle, _ptr(dl), ctypes.byref(gs), _stream(self.device))
        self._check(status, "r4d_render_backward_3d")
        return grads

    def set_timing(self, enable: bool = True):
        self._check(_lib.r4d_set_timing(self.handle, int(bool(enable))), "r4d_set_timing")

    def timings(self, reset: bool = True) -> dict:
        """{stage name: (total ms, launches)} since the last reset."""
        ms = (ctypes.c_double * NUM_STAGES)()
        cnt = (ctypes.c_int64 * NUM_STAGES)()
        self._check(_lib.r4d_get_timings(self.handle, ms, cnt, int(bool(reset))),
                    "r4d_get_timings")
        return {_lib.r4d_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(NUM_STAGES)}

    def l1_loss_grad_views(self, images: torch.Tensor, targets: torch.Tensor, views,
                           grad: torch.Tensor | None = None):
        """L = sum over views of each view's mean |image - target| and dL/dimages,
        for flat tensors in the forward's layout (one launch)."""
        images = images.contiguous()
        targets = targets.contiguous()
        grad = torch.empty_like(images) if grad is None else grad
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        varr = _views_array(views)
        status = _lib.r4d_l1_loss_grad_views(self.handle, _ptr(images), _ptr(targets), varr,
                                             len(views), _ptr(grad), _ptr(loss),
                                             _stream(self.device))
        self._check(status, "r4d_l1_loss_grad_views")
        return loss[0], grad

    def l1_loss_grad(self, image: torch.Tensor, target: torch.Tensor,
                     grad: torch.Tensor | None = None):
        """(mean |image - target|, its gradient w.r.t. image), the gradient
        written into `grad` when given."""
        image = image.contiguous()
        target = target.contiguous()
        grad = torch.empty_like(image) if grad is None else grad
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        status = _lib.r4d_l1_loss_grad(self.handle, _ptr(image), _ptr(target), image.numel(),
                                       _ptr(grad), _ptr(loss), _stream(self.device))
        self._check(status, "r4d_l1_loss_grad")
        return loss[0], grad


def adam_config(overrides: dict | None = None) -> _AdamConfig:
    """The library's default Adam settings with `overrides` applied."""
    c = _AdamConfig()
    _lib.r4d_default_adam_config(ctypes.byref(c))
    for k, val in (overrides or {}).items():
        setattr(c, k, val)
    return c


class TrainState:
    """Optimiser state around a parameter dict (float32 CUDA tensors, updated
    in place): the opacity logit, the Adam moments and the device step count."""

    def __init__(self, params: dict, renderer: "Renderer | None" = None):
        n, deg, dtype = _check_params(params)
        if dtype != torch.float32:
            raise ValueError("the optimiser works on float32 parameters")
        self.params = params
        self.n, self.deg = n, deg
        total = sum(params[k].numel() for k in _PARAM_KEYS)
        dev = params["means"].device
        self.opacity_logit = torch.empty(n, dtype=torch.float32, device=dev)
        self.m = torch.empty(total, dtype=torch.float32, device=dev)
        self.v = torch.empty(total, dtype=torch.float32, device=dev)
        self.step = torch.empty(1, dtype=torch.int32, device=dev)
        # logit of the opacity, zero moments and step count: r4d_train_state_init
        rend = renderer if renderer is not None else _renderer_for(dev)
        st = _lib.r4d_train_state_init(rend.handle, ctypes.byref(self.struct()), _stream(dev))
        rend._check(st, "r4d_train_state_init")

    def struct(self) -> _TrainState:
        p = self.params
        return _TrainState(self.n, self.deg, _ptr(p["means"]), _ptr(p["log_scales"]),
                           _ptr(p["rotors"]), _ptr(p["opacity"]), _ptr(p["sh"]),
                           _ptr(self.opacity_logit), _ptr(self.m), _ptr(self.v), _ptr(self.step))


_default_renderers: dict = {}


def _renderer_for(device: torch.device) -> Renderer:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    r = _default_renderers.get(idx)
    if r is None:
        r = Renderer(idx)
        _default_renderers[idx] = r
    return r


class _Render4D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, views, settings, sh_degree, means, log_scales, rotors, opacity, sh):
        params = {"means": means, "log_scales": log_scales, "rotors": rotors, "opacity": opacity,
                  "sh": sh, "sh_degree": sh_degree}
        images, saved = renderer.forward(params, views, settings, save=True)
        ctx.renderer, ctx.views, ctx.settings, ctx.saved = renderer, views, settings, saved
        ctx.save_for_backward(means, log_scales, rotors, opacity, sh)
        ctx.sh_degree = sh_degree
        return tuple(images)

    @staticmethod
    def backward(ctx, *grad_images):
        means, log_scales, rotors, opacity, sh = ctx.saved_tensors
        params = {"means": means, "log_scales": log_scales, "rotors": rotors, "opacity": opacity,
                  "sh": sh, "sh_degree": ctx.sh_degree}
        gi = [g if g is not None else torch.zeros(3, int(v["height"]), int(v["width"]),
                                                  dtype=means.dtype, device=means.device)
              for g, v in zip(grad_images, ctx.views)]
        grads = ctx.renderer.backward(params, ctx.views, ctx.settings, ctx.saved, gi)
        ctx.saved.release()
        return (None, None, None, None, grads["means"], grads["log_scales"], grads["rotors"],
                grads["opacity"], grads["sh"])


def render(params: dict, views, settings: dict | None = None, renderer: Renderer | None = None):
    """Render `views` of the Gaussian set `params`; differentiable w.r.t. the
    five parameter tensors.  Returns a list of [3, H, W] tensors."""
    dev = params["means"].device
    renderer = renderer or _renderer_for(dev)
    return list(_Render4D.apply(renderer, list(views), settings, int(params["sh_degree"]),
                                params["means"], params["log_scales"], params["rotors"],
                                params["opacity"], params["sh"]))


class _Render4DFlow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, views, settings, sh_degree, means, log_scales, rotors, opacity, sh):
        params = {"means": means, "log_scales": log_scales, "rotors": rotors, "opacity": opacity,
                  "sh": sh, "sh_degree": sh_degree}
        images, flows, saved = renderer.forward(params, views, settings, save=True, flow=True)
        ctx.renderer, ctx.views, ctx.settings, ctx.saved = renderer, views, settings, saved
        ctx.save_for_backward(means, log_scales, rotors, opacity, sh)
        ctx.sh_degree = sh_degree
        return tuple(images) + tuple(flows)

    @staticmethod
    def backward(ctx, *grads):
        means, log_scales, rotors, opacity, sh = ctx.saved_tensors
        params = {"means": means, "log_scales": log_scales, "rotors": rotors, "opacity": opacity,
                  "sh": sh, "sh_degree": ctx.sh_degree}
        nv = len(ctx.views)

        def filled(g, v, c):
            return g if g is not None else torch.zeros(c, int(v["height"]), int(v["width"]),
                                                       dtype=means.dtype, device=means.device)
        gi = [filled(g, v, 3) for g, v in zip(grads[:nv], ctx.views)]
        gf = [filled(g, v, 2) for g, v in zip(grads[nv:], ctx.views)]
        out = ctx.renderer.backward(params, ctx.views, ctx.settings, ctx.saved, gi, gf)
        ctx.saved.release()
        return (None, None, None, None, out["means"], out["log_scales"], out["rotors"],
                out["opacity"], out["sh"])


def render_flow(params: dict, views, settings: dict | None = None,
                renderer: Renderer | None = None):
    """Colour and speed-field (optical flow) render of `views`; differentiable
    w.r.t. the five parameter tensors through both outputs.  Returns (list of
    [3, H, W] images, list of [2, H, W] flow images in pixels per unit of t)."""
    dev = params["means"].device
    renderer = renderer or _renderer_for(dev)
    out = _Render4DFlow.apply(renderer, list(views), settings, int(params["sh_degree"]),
                              params["means"], params["log_scales"], params["rotors"],
                              params["opacity"], params["sh"])
    nv = len(views)
    return list(out[:nv]), list(out[nv:])
