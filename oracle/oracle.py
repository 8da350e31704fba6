"""Python face of the FP64 CPU oracle (``omnigs_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may call this module; the product path never does.  It shares
no code with the HIP implementation.  Inputs are the same float32 arrays the
GPU path receives, widened exactly to float64.

What each function computes, with the paper passages it follows, is stated in
``omnigs_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "omnigs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libomnigs_oracle.so")

# margins used to flag near-threshold discrete decisions (see DESIGN notes):
# relative for alpha and T decisions and for depth ties, absolute pixels for
# the rect bounds.
DEFAULT_FLAGS = dict(flag_rel_alpha=1e-5, flag_rel_T=1e-4, flag_rel_depth=2.0**-22, flag_abs_rect=1e-6)

DEFAULT_SETTINGS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, dilation=0.3, near_plane=0.2,
                        bg=(0.0, 0.0, 0.0))

REC = 48  # doubles per projection record
# depth: the sort key, t_r for the ERP camera and t_z for the pinhole camera;
# t_r: the distance to the camera centre in both
REC_FIELDS = dict(visible=0, t=slice(1, 4), depth=4, lon=5, lat=6, px=7, py=8, J=slice(9, 15), cov2d=slice(15, 18),
                  conic=slice(18, 21), ex=21, ey=22, xs=23, xe=24, ys=25, ye=26, full_x=27, tx0=28, ntx=29, ty0=30,
                  nty=31, ntiles=32, rgb=slice(33, 36), clamp=slice(36, 39), flag=39, dir=slice(40, 43), det=43,
                  t_r=44)

ERP, PINHOLE = 0, 1


def camera_model(camera) -> int:
    """0 (ERP, Eq. 3-5) or 1 (pinhole, Eq. 2) from a camera dict's "model"
    ("erp" / "pinhole" or the number; absent: ERP)."""
    m = camera.get("model", ERP)
    if isinstance(m, str):
        m = {"erp": ERP, "pinhole": PINHOLE}[m.lower()]
    return int(m)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scene(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("means", ctypes.c_void_p),
        ("scales", ctypes.c_void_p),
        ("quats", ctypes.c_void_p),
        ("opac", ctypes.c_void_p),
        ("sh", ctypes.c_void_p),
        ("sh_degree", ctypes.c_int32),
        ("sh_coeffs", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("R", ctypes.c_double * 9),
        ("t", ctypes.c_double * 3),
        ("alpha_min", ctypes.c_double),
        ("alpha_max", ctypes.c_double),
        ("T_min", ctypes.c_double),
        ("dilation", ctypes.c_double),
        ("near_plane", ctypes.c_double),
        ("bg", ctypes.c_double * 3),
        ("flag_rel_alpha", ctypes.c_double),
        ("flag_rel_T", ctypes.c_double),
        ("flag_rel_depth", ctypes.c_double),
        ("flag_abs_rect", ctypes.c_double),
        ("model", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("fx", ctypes.c_double),
        ("fy", ctypes.c_double),
        ("cx", ctypes.c_double),
        ("cy", ctypes.c_double),
        ("rows", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
        ("screen_shift", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        _lib.orc_project.argtypes = [P(_Scene), ctypes.c_void_p]
        _lib.orc_project.restype = ctypes.c_int
        _lib.orc_tile_lists.argtypes = [P(_Scene), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        _lib.orc_tile_lists.restype = ctypes.c_int64
        _lib.orc_render.argtypes = [P(_Scene)] + [ctypes.c_void_p] * 8
        _lib.orc_render.restype = ctypes.c_int
        _lib.orc_branches.argtypes = [P(_Scene), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32] + \
            [ctypes.c_void_p] * 5
        _lib.orc_branches.restype = ctypes.c_int
        _lib.orc_l1_tiles.argtypes = [P(_Scene)] + [ctypes.c_void_p] * 5
        _lib.orc_l1_tiles.restype = ctypes.c_int
        _lib.orc_backward.argtypes = [P(_Scene)] + [ctypes.c_void_p] * 17
        _lib.orc_backward.restype = ctypes.c_int
        _lib.orc_l1.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_l1.restype = ctypes.c_double
        _lib.orc_sh_eval.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib.orc_sh_eval.restype = None
        _lib.orc_num_threads.argtypes = []
        _lib.orc_num_threads.restype = ctypes.c_int
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Scene:
    """A Gaussian set, a camera and the raster settings, held in float64.

    ``gaussians``: dict with means [N,3], scales [N,3] (activated), quats
    [N,4] (w,x,y,z), opacities [N] (activated), sh [N,K,3], sh_degree.
    ``camera``: dict with R [3,3] (world -> camera rotation), t [3], width,
    height; for the pinhole camera of Eq. 2 also model="pinhole", fx, fy, cx,
    cy (pixels); optionally rows: render only the top ``rows`` rows (0 or
    absent: all), the image then has ``rows`` rows (``out_height``).
    """

    def __init__(self, gaussians, camera, settings=None, flags=None):
        st = dict(DEFAULT_SETTINGS)
        st.update(settings or {})
        fl = dict(DEFAULT_FLAGS)
        fl.update(flags or {})
        self.means = _f64(gaussians["means"]).reshape(-1, 3)
        self.n = self.means.shape[0]
        self.scales = _f64(gaussians["scales"]).reshape(self.n, 3)
        self.quats = _f64(gaussians["quats"]).reshape(self.n, 4)
        self.opac = _f64(gaussians["opacities"]).reshape(self.n)
        sh = _f64(gaussians["sh"])
        self.sh = sh.reshape(self.n, -1, 3)
        self.sh_coeffs = self.sh.shape[1]
        self.sh_degree = int(gaussians["sh_degree"])
        self.width = int(camera["width"])
        self.height = int(camera["height"])
        self.R = _f64(camera["R"]).reshape(3, 3)
        self.t = _f64(camera["t"]).reshape(3)
        self.model = camera_model(camera)
        self.rows = int(camera.get("rows", 0))
        self.intrinsics = tuple(float(camera[k]) for k in ("fx", "fy", "cx", "cy")) if self.model == PINHOLE \
            else (0.0, 0.0, 0.0, 0.0)
        self.settings = st
        self.flags = fl
        # [N,2] pixel offsets added to the projected centres (None: none):
        # moves p alone, for finite differences of dL/dp (not the method)
        self.screen_shift = None

    @property
    def tiles_x(self):
        return (self.width + 15) // 16 if self.model == PINHOLE else self.width // 16

    def camera(self, R=None, t=None):
        cam = dict(R=self.R if R is None else R, t=self.t if t is None else t, width=self.width,
                   height=self.height, model=self.model, rows=self.rows)
        if self.model == PINHOLE:
            cam.update(zip(("fx", "fy", "cx", "cy"), self.intrinsics))
        return cam

    @property
    def out_height(self):
        """Rows of the rendered image."""
        return self.rows if self.rows > 0 else self.height

    @property
    def tiles_y(self):
        return (self.out_height + 15) // 16

    def _struct(self):
        s = _Scene()
        s.n = self.n
        s.means = self.means.ctypes.data
        s.scales = self.scales.ctypes.data
        s.quats = self.quats.ctypes.data
        s.opac = self.opac.ctypes.data
        s.sh = self.sh.ctypes.data
        s.sh_degree = self.sh_degree
        s.sh_coeffs = self.sh_coeffs
        s.width = self.width
        s.height = self.height
        for k in range(9):
            s.R[k] = float(self.R.reshape(-1)[k])
        for k in range(3):
            s.t[k] = float(self.t[k])
        st = self.settings
        s.alpha_min = st["alpha_min"]
        s.alpha_max = st["alpha_max"]
        s.T_min = st["T_min"]
        s.dilation = st["dilation"]
        s.near_plane = st["near_plane"]
        for k in range(3):
            s.bg[k] = float(st["bg"][k])
        for k, v in self.flags.items():
            setattr(s, k, float(v))
        s.model = self.model
        s.fx, s.fy, s.cx, s.cy = self.intrinsics
        s.rows = self.rows
        if self.screen_shift is not None:
            self._shift = _f64(self.screen_shift).reshape(self.n, 2)
            s.screen_shift = self._shift.ctypes.data
        return s

    def with_params(self, **kw):
        """Copy with some parameter arrays replaced (float64)."""
        g = dict(means=self.means, scales=self.scales, quats=self.quats, opacities=self.opac, sh=self.sh,
                 sh_degree=self.sh_degree)
        g.update(kw)
        return Scene(g, self.camera(), self.settings, self.flags)

    def with_camera(self, R=None, t=None):
        g = dict(means=self.means, scales=self.scales, quats=self.quats, opacities=self.opac, sh=self.sh,
                 sh_degree=self.sh_degree)
        return Scene(g, self.camera(R, t), self.settings, self.flags)


def project(scene: Scene) -> np.ndarray:
    """Per-Gaussian projection records, [N, REC] float64 (fields: REC_FIELDS)."""
    lib = _load()
    rec = np.zeros((scene.n, REC), dtype=np.float64)
    s = scene._struct()
    if lib.orc_project(ctypes.byref(s), rec.ctypes.data) != 0:
        raise ValueError("oracle: invalid scene")
    return rec


def tile_lists(scene: Scene, tile_mask=None):
    """Sorted instances: (tile_id int32 [M], gaussian_id int32 [M], depth float64 [M]),
    of the tiles set in ``tile_mask`` ([tiles] bool; None: all)."""
    lib = _load()
    s = scene._struct()
    mk = _mask(scene, tile_mask)
    mp = mk.ctypes.data if mk is not None else None
    m = lib.orc_tile_lists(ctypes.byref(s), mp, 0, None, None, None)
    if m < 0:
        raise ValueError("oracle: invalid scene")
    tile = np.zeros(max(m, 1), dtype=np.int32)
    gid = np.zeros(max(m, 1), dtype=np.int32)
    tr = np.zeros(max(m, 1), dtype=np.float64)
    m2 = lib.orc_tile_lists(ctypes.byref(s), mp, m, tile.ctypes.data, gid.ctypes.data, tr.ctypes.data)
    assert m2 == m
    return tile[:m], gid[:m], tr[:m]


def _mask(scene, tile_mask):
    if tile_mask is None:
        return None
    m = np.ascontiguousarray(np.asarray(tile_mask, dtype=np.uint8).reshape(-1))
    assert m.size == scene.tiles_x * scene.tiles_y
    return m


MAX_BRANCHES = 64


def render(scene: Scene, alt: bool = True, tile_mask=None, max_branches: int = MAX_BRANCHES):
    """Forward render: dict(image [3,H,W], final_T [H,W], n_contrib [H,W],
    n_flags [H,W], n_grad_flags [H,W], n_blended [H,W], depth [H,W],
    alpha [H,W], branches) with H the rendered rows.  With ``tile_mask``
    ([tiles] bool) only those tiles are rendered (the other pixels stay
    zero).  With ``alt``, ``branches`` holds every result that each pixel
    with a flagged decision may take (``branches()``), else None."""
    lib = _load()
    H, W = scene.out_height, scene.width
    image = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), dtype=np.int32)
    nf = np.zeros((H, W), dtype=np.int32)
    ngf = np.zeros((H, W), dtype=np.int32)
    nbl = np.zeros((H, W), dtype=np.int32)
    depth = np.zeros((H, W))
    s = scene._struct()
    m = _mask(scene, tile_mask)
    rc = lib.orc_render(ctypes.byref(s), m.ctypes.data if m is not None else None, image.ctypes.data, T.ctypes.data,
                        nc.ctypes.data, nf.ctypes.data, ngf.ctypes.data, nbl.ctypes.data, depth.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid scene")
    out = dict(image=image, final_T=T, n_contrib=nc, n_flags=nf, n_grad_flags=ngf, n_blended=nbl,
               depth=depth, alpha=1.0 - T, branches=None)
    if alt:
        out["branches"] = branches(scene, np.flatnonzero(nf.reshape(-1) > 0), max_branches)
    return out


def branches(scene: Scene, pixels, max_branches: int = MAX_BRANCHES):
    """Every result that each of ``pixels`` (flat indices y * W + x) may take
    when its flagged decisions go either way: dict(pixels [P], count [P]
    (-1: more than ``max_branches``), image [P,B,3], final_T [P,B],
    n_contrib [P,B], n_blended [P,B]); branch 0 is the FP64 walk."""
    lib = _load()
    pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64).reshape(-1))
    P, B = len(pix), int(max_branches)
    out = dict(pixels=pix, count=np.zeros(P, np.int32), image=np.zeros((P, B, 3)), final_T=np.zeros((P, B)),
               n_contrib=np.zeros((P, B), np.int32), n_blended=np.zeros((P, B), np.int32))
    if P == 0:
        return out
    W = scene.width
    mask = np.zeros(scene.tiles_x * scene.tiles_y, np.uint8)
    mask[(pix // W) // 16 * scene.tiles_x + (pix % W) // 16] = 1
    s = scene._struct()
    rc = lib.orc_branches(ctypes.byref(s), mask.ctypes.data, P, pix.ctypes.data, B, out["count"].ctypes.data,
                          out["image"].ctypes.data, out["final_T"].ctypes.data, out["n_contrib"].ctypes.data,
                          out["n_blended"].ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid scene or pixel")
    return out


def l1(image, target):
    """L1 term of Eq. 17 (mean over all entries) and its gradient."""
    lib = _load()
    im = _f64(image)
    tg = _f64(target)
    g = np.zeros_like(im)
    loss = lib.orc_l1(im.size, im.ctypes.data, tg.ctypes.data, g.ctypes.data)
    return loss, g


def l1_tiles(scene: Scene, target, tile_mask, weight=None):
    """(sum over the masked tiles' pixels of w |C - target| / (3HW), decision
    hash); ``weight`` [H,W] or None (all ones)."""
    lib = _load()
    tg = _f64(target)
    w = None if weight is None else _f64(weight).reshape(scene.out_height, scene.width)
    mask = np.ascontiguousarray(np.asarray(tile_mask, dtype=np.uint8).reshape(-1))
    assert mask.size == scene.tiles_x * scene.tiles_y
    loss = ctypes.c_double(0.0)
    sig = ctypes.c_uint64(0)
    s = scene._struct()
    if lib.orc_l1_tiles(ctypes.byref(s), tg.ctypes.data, w.ctypes.data if w is not None else None, mask.ctypes.data,
                        ctypes.byref(loss), ctypes.byref(sig)) != 0:
        raise ValueError("oracle: invalid scene")
    return loss.value, sig.value


def backward(scene: Scene, dL_dimage, with_abs: bool = True, tile_mask=None, dL_ddepth=None, dL_dalpha=None):
    """Analytic gradient of <dL_dimage, image> + <dL_ddepth, depth> +
    <dL_dalpha, 1 - final_T> (the last two optional) w.r.t. the parameters.

    Returns dict(means, scales, quats, opacities, sh, screen, acc) and, with
    ``with_abs``, the same keys prefixed ``abs_``: sums of |per-pixel
    contributions| pushed through |chain| (the scale float32 sums of terms of
    both signs are judged against).  With ``tile_mask`` only those tiles are
    walked (exact when dL_dimage vanishes elsewhere).
    """
    lib = _load()
    n, K = scene.n, scene.sh_coeffs
    g = _f64(dL_dimage).reshape(3, scene.out_height, scene.width)
    gD = None if dL_ddepth is None else _f64(dL_ddepth).reshape(scene.out_height, scene.width)
    gA = None if dL_dalpha is None else _f64(dL_dalpha).reshape(scene.out_height, scene.width)
    out = dict(means=np.zeros((n, 3)), scales=np.zeros((n, 3)), quats=np.zeros((n, 4)), opacities=np.zeros(n),
               sh=np.zeros((n, K, 3)), screen=np.zeros((n, 2)), acc=np.zeros((n, 10)))
    names = ["means", "scales", "quats", "opacities", "sh", "screen"]
    if with_abs:
        for k in names:
            out["abs_" + k] = np.zeros_like(out[k])
    s = scene._struct()
    args = [out[k].ctypes.data for k in names] + [out["acc"].ctypes.data]
    args += [out["abs_" + k].ctypes.data for k in names] if with_abs else [None] * 6
    m = _mask(scene, tile_mask)
    if lib.orc_backward(ctypes.byref(s), m.ctypes.data if m is not None else None, g.ctypes.data,
                        gD.ctypes.data if gD is not None else None, gA.ctypes.data if gA is not None else None,
                        *args) != 0:
        raise ValueError("oracle: invalid scene")
    return out


def sh_eval(degree: int, direction):
    """Real SH basis values Y[(D+1)^2] and their derivatives dY/d(x,y,z)."""
    lib = _load()
    d = _f64(direction).reshape(3)
    K = (degree + 1) ** 2
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    lib.orc_sh_eval(degree, d.ctypes.data, Y.ctypes.data, dY.ctypes.data)
    return Y, dY


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for later oracle calls (n >= 1)."""
    lib = _load()
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads(int(n))
