"""Thin ctypes binding of libomnigs.so (include/omnigs.h).

Argument marshalling only: every step of the render and its backward runs in
the HIP kernels of the library.  PyTorch provides the device memory (the
library's allocator callback hands out torch CUDA tensors, so the caching
allocator recycles them) and the stream (the current HIP stream of the
tensors' device).

The names mirror the C entry points: ``omnigs_forward``, ``omnigs_backward``,
``omnigs_l1_loss``, ``omnigs_forward_batch``, ``omnigs_last_error``,
``omnigs_default_settings`` and the ``omnigs_profile_*`` calls.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libomnigs.so")

OMNIGS_OK, OMNIGS_ERR_INVALID, OMNIGS_ERR_ALLOC, OMNIGS_ERR_HIP, OMNIGS_ERR_CAPACITY = 0, 1, 2, 3, 4
OMNIGS_MEM_SCRATCH, OMNIGS_MEM_STATE = 0, 1
STATUS_NAMES = {0: "OK", 1: "ERR_INVALID", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_CAPACITY"}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32)


class OmnigsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"omnigs {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class c_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("user", ctypes.c_void_p)]


class c_gaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("sh_degree", ctypes.c_int32), ("sh_coeffs", ctypes.c_int32)]


CAMERA_ERP, CAMERA_PINHOLE = 0, 1


class c_camera(ctypes.Structure):
    _fields_ = [("R_cw", ctypes.c_double * 9), ("t_cw", ctypes.c_double * 3), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("model", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double)]


class c_settings(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("T_min", ctypes.c_double),
                ("dilation", ctypes.c_double), ("near_plane", ctypes.c_double), ("bg", ctypes.c_double * 3)]


class c_image_out(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("final_T", ctypes.c_void_p), ("n_contrib", ctypes.c_void_p),
                ("n_blended", ctypes.c_void_p), ("depth", ctypes.c_void_p)]


class c_state(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_instances", ctypes.c_int64), ("n_entries", ctypes.c_int64),
                ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("records", ctypes.c_void_p), ("n_tiles", ctypes.c_void_p), ("depth_order", ctypes.c_void_p),
                ("inst_gauss", ctypes.c_void_p), ("tile_range", ctypes.c_void_p), ("tile_work", ctypes.c_void_p),
                ("radii", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("inst_quad", ctypes.c_void_p)]


class c_capacity(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_int64), ("entries", ctypes.c_int64), ("overflow", ctypes.c_void_p)]


class c_grads(ctypes.Structure):
    _fields_ = [("dmeans", ctypes.c_void_p), ("dscales", ctypes.c_void_p), ("dquats", ctypes.c_void_p),
                ("dopacities", ctypes.c_void_p), ("dsh", ctypes.c_void_p), ("dscreen", ctypes.c_void_p)]


class c_params(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("logits", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("sh_degree", ctypes.c_int32), ("sh_coeffs", ctypes.c_int32)]


class c_adam_settings(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("lr_means", "lr_sh_dc", "lr_sh_rest", "lr_logits", "lr_log_scales",
                                                 "lr_quats", "beta1", "beta2", "eps")] + [("step", ctypes.c_int32)]


class c_dens_stats(ctypes.Structure):
    _fields_ = [("accum", ctypes.c_void_p), ("denom", ctypes.c_void_p), ("max_radius", ctypes.c_void_p)]


class c_dens_settings(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("grad_threshold", "percent_dense", "extent", "min_opacity",
                                                 "max_screen", "big_fraction", "split_shrink")]


EXPORTS = ("omnigs_default_settings", "omnigs_forward", "omnigs_backward", "omnigs_l1_loss", "omnigs_photometric_loss",
           "omnigs_forward_batch",
           "omnigs_adam_step", "omnigs_accumulate_stats", "omnigs_densify", "omnigs_reset_opacity",
           "omnigs_last_error", "omnigs_profile_enable", "omnigs_profile_num_stages", "omnigs_profile_stage_name",
           "omnigs_profile_read", "omnigs_measure_ceilings",
           "omnigs_selftest_lookback", "omnigs_backward_noalloc", "omnigs_forward_batch_bytes",
           "omnigs_set_cover_key_blocks")

_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load libomnigs.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"libomnigs.so not found at {path}: build it with "
                               "`python -m paper_2404_03202_amd.build` (there is no CPU fallback)")
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        lib.omnigs_default_settings.argtypes = []
        lib.omnigs_default_settings.restype = c_settings
        lib.omnigs_forward.argtypes = [P(c_gaussians), P(c_camera), P(c_settings), c_allocator, P(c_image_out),
                                       P(c_state), P(c_capacity), vp]
        lib.omnigs_forward.restype = ctypes.c_int
        lib.omnigs_backward.argtypes = [P(c_gaussians), P(c_camera), P(c_settings), P(c_state), P(c_image_out), vp,
                                        vp, vp, P(c_grads), c_allocator, vp]
        lib.omnigs_backward.restype = ctypes.c_int
        lib.omnigs_backward_noalloc.argtypes = [P(c_gaussians), P(c_camera), P(c_settings), P(c_state),
                                                P(c_image_out), vp, vp, vp, P(c_grads), vp]
        lib.omnigs_backward_noalloc.restype = ctypes.c_int
        lib.omnigs_l1_loss.argtypes = [vp, vp, ctypes.c_int64, vp, vp, c_allocator, vp]
        lib.omnigs_l1_loss.restype = ctypes.c_int
        lib.omnigs_photometric_loss.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                                vp, vp, vp, c_allocator, vp]
        lib.omnigs_photometric_loss.restype = ctypes.c_int
        lib.omnigs_forward_batch.argtypes = [P(c_gaussians), P(c_camera), ctypes.c_int32, P(c_settings), c_allocator,
                                             P(c_image_out), ctypes.c_int64, vp, P(ctypes.c_int64), vp]
        lib.omnigs_forward_batch.restype = ctypes.c_int
        lib.omnigs_forward_batch_bytes.argtypes = [ctypes.c_int64, P(c_camera), ctypes.c_int32, ctypes.c_int64,
                                                   P(ctypes.c_uint64)]
        lib.omnigs_forward_batch_bytes.restype = ctypes.c_int
        lib.omnigs_adam_step.argtypes = [P(c_params), P(c_grads), P(c_params), P(c_params), P(c_adam_settings),
                                         P(c_gaussians), vp, vp]
        lib.omnigs_adam_step.restype = ctypes.c_int
        lib.omnigs_accumulate_stats.argtypes = [P(c_state), P(c_grads), P(c_dens_stats), vp, vp]
        lib.omnigs_accumulate_stats.restype = ctypes.c_int
        lib.omnigs_densify.argtypes = [P(c_params), P(c_params), P(c_params), P(c_dens_stats), vp, P(c_dens_settings),
                                       c_allocator, P(c_params), P(c_params), P(c_params), P(c_dens_stats),
                                       P(ctypes.c_int64), vp]
        lib.omnigs_densify.restype = ctypes.c_int
        lib.omnigs_reset_opacity.argtypes = [P(c_params), P(c_params), P(c_params), ctypes.c_double, vp]
        lib.omnigs_reset_opacity.restype = ctypes.c_int
        lib.omnigs_measure_ceilings.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, c_allocator,
                                                P(c_ceilings), vp]
        lib.omnigs_measure_ceilings.restype = ctypes.c_int
        lib.omnigs_selftest_lookback.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, c_allocator,
                                                 P(ctypes.c_uint32), P(ctypes.c_int32), vp]
        lib.omnigs_selftest_lookback.restype = ctypes.c_int
        lib.omnigs_set_cover_key_blocks.argtypes = [ctypes.c_uint32]
        lib.omnigs_set_cover_key_blocks.restype = ctypes.c_int
        lib.omnigs_last_error.argtypes = []
        lib.omnigs_last_error.restype = ctypes.c_char_p
        lib.omnigs_profile_enable.argtypes = [ctypes.c_uint32]
        lib.omnigs_profile_enable.restype = ctypes.c_int
        lib.omnigs_profile_num_stages.argtypes = []
        lib.omnigs_profile_num_stages.restype = ctypes.c_int32
        lib.omnigs_profile_stage_name.argtypes = [ctypes.c_int32]
        lib.omnigs_profile_stage_name.restype = ctypes.c_char_p
        lib.omnigs_profile_read.argtypes = [vp, vp]
        lib.omnigs_profile_read.restype = ctypes.c_int
        _lib = lib
        return lib


def omnigs_last_error() -> str:
    return load_library().omnigs_last_error().decode(errors="replace")


def _check(status):
    if status != OMNIGS_OK:
        raise OmnigsError(status, omnigs_last_error())


# ------------------------------------------------------------------ marshal
def omnigs_default_settings() -> dict:
    s = load_library().omnigs_default_settings()
    return dict(alpha_min=s.alpha_min, alpha_max=s.alpha_max, T_min=s.T_min, dilation=s.dilation,
                near_plane=s.near_plane, bg=tuple(s.bg))


def make_settings(settings: dict | None) -> c_settings:
    d = omnigs_default_settings()
    d.update(settings or {})
    s = c_settings()
    for k in ("alpha_min", "alpha_max", "T_min", "dilation", "near_plane"):
        setattr(s, k, float(d[k]))
    for k in range(3):
        s.bg[k] = float(d["bg"][k])
    return s


def camera_model(camera: dict) -> int:
    """CAMERA_ERP or CAMERA_PINHOLE from a camera dict's "model" ("erp",
    "pinhole" or the number; absent: ERP)."""
    m = camera.get("model", CAMERA_ERP)
    if isinstance(m, str):
        m = {"erp": CAMERA_ERP, "pinhole": CAMERA_PINHOLE}[m.lower()]
    return int(m)


def make_camera(camera: dict) -> c_camera:
    """camera: R [3,3] world->camera rotation, t [3], width, height; a pinhole
    camera (Eq. 2) also model="pinhole", fx, fy, cx, cy (pixels)."""
    c = c_camera()
    c.model = camera_model(camera)
    if c.model == CAMERA_PINHOLE:
        c.fx, c.fy, c.cx, c.cy = (float(camera[k]) for k in ("fx", "fy", "cx", "cy"))
    R = np.asarray(camera["R"], dtype=np.float64).reshape(9)
    t = np.asarray(camera["t"], dtype=np.float64).reshape(3)
    for k in range(9):
        c.R_cw[k] = float(R[k])
    for k in range(3):
        c.t_cw[k] = float(t[k])
    c.width = int(camera["width"])
    c.height = int(camera["height"])
    c.rows = int(camera.get("rows", 0))
    return c


def image_rows(camera: dict) -> int:
    """Rows of the rendered image: the camera's "rows" (top rows only) or
    its height."""
    r = int(camera.get("rows", 0))
    return r if r > 0 else int(camera["height"])


def _ptr(t):
    return None if t is None else t.data_ptr()


def make_gaussians(g: dict) -> c_gaussians:
    """g: means [N,3], scales [N,3], quats [N,4], opacities [N], sh [N,K,3]
    (contiguous float32 CUDA tensors), sh_degree."""
    sh = g["sh"]
    n = int(g["means"].shape[0])
    for k in ("means", "scales", "quats", "opacities", "sh"):
        t = g[k]
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
    c = c_gaussians()
    c.means, c.scales, c.quats = _ptr(g["means"]), _ptr(g["scales"]), _ptr(g["quats"])
    c.opacities, c.sh = _ptr(g["opacities"]), _ptr(sh)
    c.n = n
    c.sh_degree = int(g["sh_degree"])
    c.sh_coeffs = int(sh.shape[1]) if sh.dim() == 3 else int(sh.numel() // max(n, 1) // 3)
    return c


class Allocator:
    """Allocator callback backed by torch's caching allocator.  Scratch
    allocations are dropped when the call returns (stream-ordered reuse);
    state allocations stay referenced by the returned state."""

    def __init__(self, device, fail=False):
        self.device = device
        self.fail = fail
        self.scratch = []
        self.state = []
        self._cb = ALLOC_FN(self._alloc)
        self.c = c_allocator(self._cb, None)

    def _alloc(self, user, nbytes, kind):
        if self.fail:
            return None
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory: reported as OMNIGS_ERR_ALLOC
            return None
        (self.state if kind == OMNIGS_MEM_STATE else self.scratch).append(t)
        return t.data_ptr()


def _stream_ptr(device):
    return torch.cuda.current_stream(device).cuda_stream


class ForwardResult:
    """Outputs of omnigs_forward plus the saved state for omnigs_backward."""

    def __init__(self, image, final_T, n_contrib, state: c_state, keepalive, n_blended=None, depth=None,
                 overflow=None):
        self.image = image
        self.final_T = final_T
        self.n_contrib = n_contrib
        self.n_blended = n_blended
        self.depth = depth
        self.state = state
        self.overflow = overflow  # device int32 [1] with capacities, else None
        self._keep = keepalive

    @property
    def n_instances(self):
        """M, or -1 when the call read nothing back (see counts())."""
        return int(self.state.n_instances)

    @property
    def n_entries(self):
        return int(self.state.n_entries)

    def counts(self):
        """(S, M) as counted on the device (synchronises)."""
        c = self._view(self.state.counts, 2, torch.int32)
        return int(c[0]), int(c[1])

    def _view(self, ptr, count, dtype):
        """View a state buffer as a tensor (for tests / debugging)."""
        for t in self._keep:
            base = t.data_ptr()
            if base <= ptr < base + t.numel():
                off = ptr - base
                esz = torch.empty((), dtype=dtype).element_size()
                return t[off:off + count * esz].view(dtype)
        raise KeyError("pointer not in state buffers")

    def instance_lists(self):
        """Per-tile lists concatenated in tile-id order: (tile id [M] int32,
        Gaussian id [M] int32, ranges [tiles, 2] int32 of the library's own
        layout), device tensors (the tile ids are re-derived from the ranges)."""
        tiles = self.state.tiles_x * self.state.tiles_y
        rng = self._view(self.state.tile_range, 2 * tiles, torch.int32).view(tiles, 2)
        M = self.n_instances if self.n_instances >= 0 else int(rng[:, 1].max()) if tiles else 0
        gauss = self._view(self.state.inst_gauss, M, torch.int32)
        lens = (rng[:, 1] - rng[:, 0]).long()
        tile = torch.repeat_interleave(torch.arange(tiles, device=gauss.device, dtype=torch.int32), lens)
        starts = torch.repeat_interleave(rng[:, 0].long(), lens)
        first = torch.repeat_interleave(torch.cumsum(lens, 0) - lens, lens)
        idx = starts + torch.arange(int(lens.sum()), device=gauss.device) - first
        return tile, gauss[idx], rng

    def depth_order(self):
        return self._view(self.state.depth_order, int(self.state.n), torch.int32)

    def seam_fraction(self):
        """Fraction of the visible Gaussians (covering at least one tile)
        whose alpha >= alpha_min box crosses the longitude seam of the ERP
        image: centre column minus the screen radius below 0 or plus it past
        the width (synchronises)."""
        n = int(self.state.n)
        if n == 0:
            return 0.0
        rec = self._view(self.state.records, 12 * n, torch.float32).view(n, 12)
        px = rec[:, 0].double() + rec[:, 1].double()
        r = self._view(self.state.radii, n, torch.float32).double()
        vis = self.n_tiles() > 0
        W = float(self.state.width)
        cross = vis & ((px - r < 0.0) | (px + r > W))
        return float(cross.sum()) / max(int(vis.sum()), 1)


    def n_tiles(self):
        return self._view(self.state.n_tiles, int(self.state.n), torch.int32)


def omnigs_forward(g: dict, camera: dict, settings: dict | None = None, allocator: Allocator | None = None,
                   out: dict | None = None, with_blended: bool = False, with_depth: bool = False,
                   capacity=None) -> ForwardResult:
    """Render one camera: image [3,H,W], final_T, n_contrib (and n_blended,
    depth [H,W] on request), H the rendered rows; the alpha image is
    1 - final_T.  capacity None reads the instance counts back (one host
    sync); (instances, entries) sizes the instance and block-entry buffers
    instead, reads nothing back and flags overflow in result.overflow."""
    lib = load_library()
    dev = g["means"].device
    cg, cc, cs = make_gaussians(g), make_camera(camera), make_settings(settings)
    H, W = image_rows(camera), cc.width
    if out is None:
        out = dict(image=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                   final_T=torch.empty((H, W), dtype=torch.float32, device=dev),
                   n_contrib=torch.empty((H, W), dtype=torch.int32, device=dev))
        if with_blended:
            out["n_blended"] = torch.empty((H, W), dtype=torch.int32, device=dev)
        if with_depth:
            out["depth"] = torch.empty((H, W), dtype=torch.float32, device=dev)
    co = c_image_out(_ptr(out["image"]), _ptr(out["final_T"]), _ptr(out["n_contrib"]), _ptr(out.get("n_blended")),
                     _ptr(out.get("depth")))
    st = c_state()
    al = allocator or Allocator(dev)
    cap, overflow = None, None
    if capacity is not None:
        instances, entries = capacity
        overflow = torch.empty(1, dtype=torch.int32, device=dev)
        cap = c_capacity(int(instances), int(entries), _ptr(overflow))
    _check(lib.omnigs_forward(ctypes.byref(cg), ctypes.byref(cc), ctypes.byref(cs), al.c, ctypes.byref(co),
                              ctypes.byref(st), ctypes.byref(cap) if cap is not None else None,
                              ctypes.c_void_p(_stream_ptr(dev))))
    keep = list(al.state)
    al.scratch.clear()
    al.state.clear()
    return ForwardResult(out["image"], out["final_T"], out["n_contrib"], st, keep, out.get("n_blended"),
                         out.get("depth"), overflow)


def _backward_call(g, camera, settings, fwd, dL_dimage, grads, dL_ddepth, dL_dalpha, call):
    dev = g["means"].device
    n = int(g["means"].shape[0])
    cg, cc, cs = make_gaussians(g), make_camera(camera), make_settings(settings)
    for t in (dL_dimage, dL_ddepth, dL_dalpha):
        if t is not None and (t.dtype != torch.float32 or not t.is_contiguous()):
            raise ValueError("cotangents must be contiguous float32 tensors")
    if grads is None:
        z = lambda *shape: torch.empty(shape, dtype=torch.float32, device=dev)
        grads = dict(means=z(n, 3), scales=z(n, 3), quats=z(n, 4), opacities=z(n), sh=torch.empty_like(g["sh"]),
                     screen=z(n, 2))
    cgr = c_grads(_ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]), _ptr(grads["opacities"]),
                  _ptr(grads["sh"]), _ptr(grads["screen"]))
    co = c_image_out(_ptr(fwd.image), _ptr(fwd.final_T), _ptr(fwd.n_contrib), None, None)
    call(ctypes.byref(cg), ctypes.byref(cc), ctypes.byref(cs), ctypes.byref(fwd.state), ctypes.byref(co),
         ctypes.c_void_p(dL_dimage.data_ptr()), ctypes.c_void_p(_ptr(dL_ddepth)), ctypes.c_void_p(_ptr(dL_dalpha)),
         ctypes.byref(cgr), ctypes.c_void_p(_stream_ptr(dev)))
    return grads


def omnigs_backward(g: dict, camera: dict, settings: dict | None, fwd: ForwardResult, dL_dimage: torch.Tensor,
                    allocator: Allocator | None = None, grads: dict | None = None,
                    dL_ddepth: torch.Tensor | None = None, dL_dalpha: torch.Tensor | None = None) -> dict:
    """Gradients of <dL_dimage, image> (+ <dL_ddepth, depth> + <dL_dalpha,
    1 - final_T>, each optional) w.r.t. the parameters."""
    lib = load_library()
    al = allocator or Allocator(g["means"].device)
    grads = _backward_call(g, camera, settings, fwd, dL_dimage, grads, dL_ddepth, dL_dalpha,
                           lambda *a: _check(lib.omnigs_backward(*a[:9], al.c, a[9])))
    al.scratch.clear()
    return grads


def omnigs_backward_noalloc(g: dict, camera: dict, settings: dict | None, fwd: ForwardResult,
                            dL_dimage: torch.Tensor, grads: dict, dL_ddepth: torch.Tensor | None = None,
                            dL_dalpha: torch.Tensor | None = None) -> dict:
    """omnigs_backward on the library's fixed device scratch: the caller
    passes the gradient buffers, and the call allocates no device memory."""
    if grads is None:
        raise ValueError("omnigs_backward_noalloc writes into caller-provided gradient buffers")
    lib = load_library()
    return _backward_call(g, camera, settings, fwd, dL_dimage, grads, dL_ddepth, dL_dalpha,
                          lambda *a: _check(lib.omnigs_backward_noalloc(*a)))


def omnigs_l1_loss(image: torch.Tensor, target: torch.Tensor, grad: bool = True, allocator: Allocator | None = None):
    """(loss [1] float32, dL/dimage or None): mean |image - target| and sign/count."""
    lib = load_library()
    if image.shape != target.shape or image.dtype != torch.float32 or target.dtype != torch.float32:
        raise ValueError("image and target must be float32 tensors of one shape")
    image, target = image.contiguous(), target.contiguous()
    dev = image.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g = torch.empty_like(image) if grad else None
    al = allocator or Allocator(dev)
    _check(lib.omnigs_l1_loss(ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(target.data_ptr()), image.numel(),
                              ctypes.c_void_p(_ptr(g)), ctypes.c_void_p(loss.data_ptr()), al.c,
                              ctypes.c_void_p(_stream_ptr(dev))))
    al.scratch.clear()
    return loss, g


OMNIGS_MAX_BATCH = 16


class BatchResult:
    """Outputs of omnigs_forward_batch: one dict(image, final_T, n_contrib
    [, n_blended]) per camera, the device overflow flag and the instance
    count (-1 when it was not read back)."""

    def __init__(self, outs, overflow, n_instances, keepalive):
        self.outs = outs
        self.overflow = overflow
        self.n_instances = n_instances
        self._keep = keepalive


def omnigs_photometric_loss(image: torch.Tensor, target: torch.Tensor, lam: float, grad: bool = True,
                            allocator: Allocator | None = None, mask: torch.Tensor | None = None):
    """(loss [1] float32, dL/dimage or None) of (1 - lam) L1 + lam (1 - SSIM)
    for [C, H, W] float32 images, both means weighted by the [H, W] mask when
    one is given."""
    lib = load_library()
    if image.shape != target.shape or image.dim() != 3 or image.dtype != torch.float32 or \
            target.dtype != torch.float32:
        raise ValueError("image and target must be [C, H, W] float32 tensors of one shape")
    image, target = image.contiguous(), target.contiguous()
    C, H, W = image.shape
    if mask is not None:
        if mask.shape != (H, W) or mask.dtype != torch.float32:
            raise ValueError("mask must be a [H, W] float32 tensor")
        mask = mask.contiguous()
    dev = image.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g = torch.empty_like(image) if grad else None
    al = allocator or Allocator(dev)
    _check(lib.omnigs_photometric_loss(ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(target.data_ptr()), C, H, W,
                                       float(lam), ctypes.c_void_p(_ptr(mask)), ctypes.c_void_p(_ptr(g)),
                                       ctypes.c_void_p(loss.data_ptr()), al.c, ctypes.c_void_p(_stream_ptr(dev))))
    al.scratch.clear()
    return loss, g


def omnigs_forward_batch(g: dict, cameras: list, settings: dict | None = None, instance_capacity: int = 0,
                         allocator: Allocator | None = None, outs: list | None = None,
                         with_blended: bool = False, with_depth: bool = False) -> BatchResult:
    """Render up to OMNIGS_MAX_BATCH cameras (mixed resolutions) in one
    batched launch sequence on the current stream.  instance_capacity 0 reads
    the instance count back (one host sync); > 0 enqueues only and flags
    overflow on the device."""
    lib = load_library()
    dev = g["means"].device
    B = len(cameras)
    cg, cs = make_gaussians(g), make_settings(settings)
    cams = (c_camera * max(B, 1))(*[make_camera(c) for c in cameras])
    if outs is None:
        outs = []
        for c in cameras:
            H, W = image_rows(c), int(c["width"])
            o = dict(image=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                     final_T=torch.empty((H, W), dtype=torch.float32, device=dev),
                     n_contrib=torch.empty((H, W), dtype=torch.int32, device=dev))
            if with_blended:
                o["n_blended"] = torch.empty((H, W), dtype=torch.int32, device=dev)
            if with_depth:
                o["depth"] = torch.empty((H, W), dtype=torch.float32, device=dev)
            outs.append(o)
    couts = (c_image_out * max(B, 1))(*[c_image_out(_ptr(o["image"]), _ptr(o["final_T"]), _ptr(o["n_contrib"]),
                                                    _ptr(o.get("n_blended")), _ptr(o.get("depth"))) for o in outs])
    overflow = torch.empty(1, dtype=torch.int32, device=dev)
    m = ctypes.c_int64(-1)
    al = allocator or Allocator(dev)
    try:
        _check(lib.omnigs_forward_batch(ctypes.byref(cg), cams, B, ctypes.byref(cs), al.c, couts,
                                        int(instance_capacity), ctypes.c_void_p(overflow.data_ptr()),
                                        ctypes.byref(m), ctypes.c_void_p(_stream_ptr(dev))))
    finally:
        keep = list(al.scratch)
        al.scratch.clear()
    # scratch tensors go back to the caching allocator here; their reuse is
    # ordered after the enqueued kernels on this stream
    del keep
    return BatchResult(outs, overflow, int(m.value), [])


def omnigs_forward_batch_bytes(n: int, cameras: list, instance_capacity: int) -> int:
    """Device bytes omnigs_forward_batch requests from its allocator for n
    Gaussians, these cameras and an instance capacity (outputs excluded)."""
    lib = load_library()
    cams = (c_camera * max(len(cameras), 1))(*[make_camera(c) for c in cameras])
    out = ctypes.c_uint64(0)
    _check(lib.omnigs_forward_batch_bytes(int(n), cams, len(cameras), int(instance_capacity), ctypes.byref(out)))
    return int(out.value)


def output_bytes(camera: dict, with_blended: bool = False, with_depth: bool = False) -> int:
    """Bytes of one camera's forward outputs: image [3,H,W], final_T and
    n_contrib [H,W] (+ n_blended, depth)."""
    px = image_rows(camera) * int(camera["width"])
    return px * 4 * (5 + int(with_blended) + int(with_depth))


# ------------------------------------------------------------- optimisation
PARAM_KEYS = ("means", "log_scales", "quats", "logits", "sh")


def make_params(p: dict) -> c_params:
    """p: means [N,3], log_scales [N,3], quats [N,4], logits [N], sh [N,K,3]
    (contiguous float32 CUDA tensors), sh_degree."""
    for k in PARAM_KEYS:
        t = p[k]
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
    n = int(p["means"].shape[0])
    return c_params(_ptr(p["means"]), _ptr(p["log_scales"]), _ptr(p["quats"]), _ptr(p["logits"]), _ptr(p["sh"]), n,
                    int(p["sh_degree"]), int(p["sh"].shape[1]))


def _grads(grads: dict) -> c_grads:
    return c_grads(_ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]), _ptr(grads["opacities"]),
                   _ptr(grads["sh"]), _ptr(grads.get("screen")))


def omnigs_adam_step(p: dict, grads: dict, m1: dict, m2: dict, lrs: dict, step: int, act: dict | None = None,
                     beta1=0.9, beta2=0.999, eps=1e-15, skip: torch.Tensor | None = None):
    """In-place Adam step of p, m1, m2 (dicts of raw parameters); act (may be
    None): a Gaussian dict whose scales / opacities receive exp / sigmoid of
    the new log-scales / logits.  skip (device int32 [1], may be None): the
    step writes nothing when it is nonzero."""
    lib = load_library()
    s = c_adam_settings(lrs["means"], lrs["sh_dc"], lrs["sh_rest"], lrs["logits"], lrs["log_scales"], lrs["quats"],
                        beta1, beta2, eps, int(step))
    cp, c1, c2 = make_params(p), make_params(m1), make_params(m2)
    ca = None
    if act is not None:
        ca = c_gaussians()
        ca.scales, ca.opacities = _ptr(act["scales"]), _ptr(act["opacities"])
    _check(lib.omnigs_adam_step(ctypes.byref(cp), ctypes.byref(_grads(grads)), ctypes.byref(c1), ctypes.byref(c2),
                                ctypes.byref(s), ctypes.byref(ca) if ca is not None else None,
                                ctypes.c_void_p(_ptr(skip)), ctypes.c_void_p(_stream_ptr(p["means"].device))))


def omnigs_accumulate_stats(fwd: "ForwardResult", grads: dict, stats: dict, skip: torch.Tensor | None = None):
    """stats: accum, denom, max_radius ([N] float32 tensors), updated in place
    (nothing written when skip, a device int32 [1], is nonzero)."""
    lib = load_library()
    cs = c_dens_stats(_ptr(stats["accum"]), _ptr(stats["denom"]), _ptr(stats["max_radius"]))
    _check(lib.omnigs_accumulate_stats(ctypes.byref(fwd.state), ctypes.byref(_grads(grads)), ctypes.byref(cs),
                                       ctypes.c_void_p(_ptr(skip)), ctypes.c_void_p(_stream_ptr(stats["accum"].device))))


def omnigs_densify(p: dict, m1: dict, m2: dict, stats: dict, noise: torch.Tensor, settings: dict,
                   allocator: Allocator | None = None):
    """Densify and prune.  Returns (p, m1, m2, stats) as new tensor dicts."""
    lib = load_library()
    dev = p["means"].device
    cs = c_dens_settings(*(float(settings[k]) for k in ("grad_threshold", "percent_dense", "extent", "min_opacity",
                                                        "max_screen", "big_fraction", "split_shrink")))
    st_in = c_dens_stats(_ptr(stats["accum"]), _ptr(stats["denom"]), _ptr(stats["max_radius"]))
    outs = [c_params() for _ in range(3)]
    st_out = c_dens_stats()
    n_out = ctypes.c_int64(0)
    al = allocator or Allocator(dev)
    _check(lib.omnigs_densify(ctypes.byref(make_params(p)), ctypes.byref(make_params(m1)), ctypes.byref(make_params(m2)),
                              ctypes.byref(st_in), ctypes.c_void_p(_ptr(noise)), ctypes.byref(cs), al.c,
                              *[ctypes.byref(o) for o in outs], ctypes.byref(st_out), ctypes.byref(n_out),
                              ctypes.c_void_p(_stream_ptr(dev))))
    buf = al.state[-1] if al.state else None
    al.scratch.clear()
    al.state.clear()
    n = int(n_out.value)
    K = int(p["sh"].shape[1])

    def view(ptr, shape):
        if buf is None or n == 0:
            return torch.zeros(shape, dtype=torch.float32, device=dev)
        off = ptr - buf.data_ptr()
        cnt = int(np.prod(shape))
        return buf[off:off + 4 * cnt].view(torch.float32).view(shape)

    def as_dict(o):
        return dict(means=view(o.means, (n, 3)), log_scales=view(o.log_scales, (n, 3)), quats=view(o.quats, (n, 4)),
                    logits=view(o.logits, (n,)), sh=view(o.sh, (n, K, 3)), sh_degree=p["sh_degree"])
    stats_out = dict(accum=view(st_out.accum, (n,)), denom=view(st_out.denom, (n,)),
                     max_radius=view(st_out.max_radius, (n,)))
    return as_dict(outs[0]), as_dict(outs[1]), as_dict(outs[2]), stats_out


def omnigs_reset_opacity(p: dict, m1: dict, m2: dict, value: float = 0.01):
    lib = load_library()
    _check(lib.omnigs_reset_opacity(ctypes.byref(make_params(p)), ctypes.byref(make_params(m1)),
                                    ctypes.byref(make_params(m2)), float(value),
                                    ctypes.c_void_p(_stream_ptr(p["means"].device))))


# ---------------------------------------------------------------- profiling
def omnigs_profile_enable(on: bool = True, stages=None):
    """Stage timing on or off; `stages` (names) limits it to those stages."""
    lib = load_library()
    if not on:
        mask = 0
    elif stages is None:
        mask = 0xFFFFFFFF
    else:
        names = [lib.omnigs_profile_stage_name(k).decode() for k in range(lib.omnigs_profile_num_stages())]
        mask = 0
        for st in stages:
            mask |= 1 << names.index(st)
    _check(lib.omnigs_profile_enable(mask))


def omnigs_profile_read() -> dict:
    """{stage name: (total ms, launches)} since the last read (synchronises)."""
    lib = load_library()
    n = lib.omnigs_profile_num_stages()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib.omnigs_profile_read(ms, cnt))
    return {lib.omnigs_profile_stage_name(k).decode(): (ms[k], int(cnt[k])) for k in range(n)}


class c_ceilings(ctypes.Structure):
    _fields_ = [("fma_tflops", ctypes.c_double), ("exp_gops", ctypes.c_double), ("atomic_gops", ctypes.c_double),
                ("copy_gbps", ctypes.c_double)]


def omnigs_measure_ceilings(atomic_words: int = 10 << 20, copy_bytes: int = 256 << 20, repeats: int = 5,
                            device: str = "cuda:0", allocator: Allocator | None = None) -> dict:
    """Measured FP32 FMA (TFLOP/s), exp2 (G/s), scattered float atomic (G/s)
    and copy (GB/s, read + written) rates of the device."""
    lib = load_library()
    dev = torch.device(device)
    A = allocator or Allocator(dev)
    out = c_ceilings()
    with torch.cuda.device(dev):
        _check(lib.omnigs_measure_ceilings(int(atomic_words), int(copy_bytes), int(repeats), A.c, ctypes.byref(out),
                                           ctypes.c_void_p(_stream_ptr(dev))))
    A.scratch.clear()
    return {k: getattr(out, k) for k, _ in c_ceilings._fields_}


def omnigs_set_cover_key_blocks(blocks: int = 0) -> None:
    """Binning path for tests: covers from the sort keys while a call has at
    most `blocks` 8x8-tile blocks (0: the default, 65536), else from the
    Gaussians' rectangles; both give the same tile lists."""
    _check(load_library().omnigs_set_cover_key_blocks(int(blocks)))


def omnigs_selftest_lookback(primitive: str, n: int, max_polls: int = 0, device: str = "cuda:0") -> tuple:
    """(fault bits, exact) of the sort ("sort") or scan ("scan") primitive on
    n device-generated keys with the lookback poll bound set to max_polls (0:
    the library's)."""
    lib = load_library()
    dev = torch.device(device)
    A = Allocator(dev)
    fault, correct = ctypes.c_uint32(0), ctypes.c_int32(0)
    with torch.cuda.device(dev):
        _check(lib.omnigs_selftest_lookback({"sort": 0, "scan": 1}[primitive], int(n), int(max_polls), A.c,
                                            ctypes.byref(fault), ctypes.byref(correct),
                                            ctypes.c_void_p(_stream_ptr(dev))))
    return int(fault.value), bool(correct.value)


def tile_sort_bits(width: int, height: int) -> int:
    tiles = ((width + 15) // 16) * ((height + 15) // 16)
    return max(1, math.ceil(math.log2(max(tiles, 2))))
