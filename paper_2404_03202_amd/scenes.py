"""Seeded synthetic scenes and camera poses.

This module holds no rendering arithmetic: it only draws Gaussian parameter
sets, camera poses and request streams from seeded numpy generators.  It is
shared, as an input source, by the tests (which feed the same arrays to the
GPU path and to the FP64 oracle) and by the benchmark and serving demo.

Parameter conventions (the library's input layout):
  means [N,3] f32       world positions
  scales [N,3] f32      activated (positive) per-axis standard deviations
  quats [N,4] f32       rotation quaternion (w, x, y, z), not necessarily unit
  opacities [N] f32     activated opacity in (0, 1)
  sh [N,16,3] f32       real SH coefficients, degree <= 3, RGB innermost
Camera: R [3,3] f64 world->camera rotation, t [3] f64, width, height (ERP);
a pinhole camera (Eq. 2) adds model="pinhole", fx, fy, cx, cy (pixels).

Generators use ``np.random.default_rng([config, stream])`` with streams
0 = scene, 1 = target perturbation, 2 = poses, 3 = request stream,
4 = finite-difference parameter choice.
"""
from __future__ import annotations

import numpy as np

STREAM_SCENE, STREAM_TARGET, STREAM_POSES, STREAM_REQUESTS, STREAM_FD = 0, 1, 2, 3, 4


def rng_for(config: int, stream: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng([config, stream, extra])


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _uniform_shell(rng, n, r0, r1):
    """Points uniform in volume in the spherical shell r0 <= r <= r1."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = rng.uniform(size=n)
    r = (r0 ** 3 + u * (r1 ** 3 - r0 ** 3)) ** (1.0 / 3.0)
    return d * r[:, None]


def _attributes(rng, n, scale_lo, scale_hi, sh_degree=3):
    scales = np.exp(rng.uniform(np.log(scale_lo), np.log(scale_hi), size=(n, 3)))
    quats = rng.normal(size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    opac = _sigmoid(rng.normal(size=n))
    sh = np.zeros((n, 16, 3))
    sh[:, 0, :] = rng.normal(0.5, 0.2, size=(n, 3))
    k = (sh_degree + 1) ** 2
    if k > 1:
        sh[:, 1:k, :] = rng.normal(0.0, 0.1, size=(n, k - 1, 3))
    return scales, quats, opac, sh


def _pack(means, scales, quats, opac, sh, sh_degree):
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(means=f(means), scales=f(scales), quats=f(quats), opacities=f(opac), sh=f(sh),
                sh_degree=int(sh_degree))


def shell_scene(config: int, n: int, r0=1.0, r1=10.0, scale_lo=0.01, scale_hi=0.3, sh_degree=3):
    """Means uniform in the volume of a spherical shell; the attribute mix of
    the parity workloads (log-uniform scales, random unit quaternions,
    opacity sigmoid(N(0,1)), SH DC ~ N(0.5, 0.2), other SH ~ N(0, 0.1))."""
    rng = rng_for(config, STREAM_SCENE)
    means = _uniform_shell(rng, n, r0, r1)
    scales, quats, opac, sh = _attributes(rng, n, scale_lo, scale_hi, sh_degree)
    return _pack(means, scales, quats, opac, sh, sh_degree)


def room_scene(config: int, n: int, scale_lo=0.01, scale_hi=0.3, seam_fraction=0.2, sh_degree=3):
    """Indoor room layout: 70% of the means jittered (N(0, 0.05)) on the faces
    of an axis-aligned box with half-extents U(3, 8) per axis (face chosen in
    proportion to its area), 30% uniform in the shell 1 <= r <= 10; then a
    ``seam_fraction`` of all Gaussians is moved into a +-1 degree wedge around
    world longitude pi (keeping their horizontal radius and height) so that it
    straddles the ERP seam for a camera with identity yaw."""
    rng = rng_for(config, STREAM_SCENE)
    half = rng.uniform(3.0, 8.0, size=3)
    n_room = int(round(0.7 * n))
    n_shell = n - n_room
    # face areas: pair of faces normal to axis k has area (2 h_i)(2 h_j)
    areas = np.array([half[1] * half[2], half[1] * half[2], half[0] * half[2], half[0] * half[2],
                      half[0] * half[1], half[0] * half[1]])
    face = rng.choice(6, size=n_room, p=areas / areas.sum())
    pts = rng.uniform(-1.0, 1.0, size=(n_room, 3)) * half[None, :]
    axis = face // 2
    sign = np.where(face % 2 == 0, -1.0, 1.0)
    pts[np.arange(n_room), axis] = sign * half[axis]
    pts += rng.normal(0.0, 0.05, size=pts.shape)
    means = np.concatenate([pts, _uniform_shell(rng, n_shell, 1.0, 10.0)], axis=0)
    perm = rng.permutation(n)
    means = means[perm]
    n_seam = int(round(seam_fraction * n))
    if n_seam:
        idx = rng.choice(n, size=n_seam, replace=False)
        r_xz = np.hypot(means[idx, 0], means[idx, 2])
        lon = np.pi + np.deg2rad(rng.uniform(-1.0, 1.0, size=n_seam))
        means[idx, 0] = r_xz * np.sin(lon)
        means[idx, 2] = r_xz * np.cos(lon)
    scales, quats, opac, sh = _attributes(rng, n, scale_lo, scale_hi, sh_degree)
    return _pack(means, scales, quats, opac, sh, sh_degree)


def perturbed(config: int, g: dict, mean_sigma=0.01, dc_sigma=0.05, logit_sigma=0.1):
    """A perturbed copy of a scene (the target of the fwd+bwd workloads):
    means + N(0, 0.01), SH DC + N(0, 0.05), opacity logit + N(0, 0.1)."""
    rng = rng_for(config, STREAM_TARGET)
    n = g["means"].shape[0]
    means = g["means"].astype(np.float64) + rng.normal(0.0, mean_sigma, size=(n, 3))
    sh = g["sh"].astype(np.float64).copy()
    sh[:, 0, :] += rng.normal(0.0, dc_sigma, size=(n, 3))
    o = np.clip(g["opacities"].astype(np.float64), 1e-6, 1 - 1e-6)
    logit = np.log(o / (1.0 - o)) + rng.normal(0.0, logit_sigma, size=n)
    return _pack(means, g["scales"], g["quats"], _sigmoid(logit), sh, g["sh_degree"])


def rot_y(angle: float) -> np.ndarray:
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_x(angle: float) -> np.ndarray:
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def camera(width: int, height: int, R=None, centre=None) -> dict:
    """Camera dict from a world->camera rotation and a camera centre."""
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    c = np.zeros(3) if centre is None else np.asarray(centre, dtype=np.float64)
    return dict(R=R, t=-R @ c, width=int(width), height=int(height))


def pinhole_camera(width: int, height: int, fov_x_deg=90.0, R=None, centre=None, fy=None, cx=None, cy=None) -> dict:
    """Pinhole camera dict: f_x from the horizontal field of view, f_y = f_x
    (square pixels) and the principal point at the image centre unless
    given."""
    cam = camera(width, height, R, centre)
    fx = 0.5 * width / np.tan(np.radians(fov_x_deg) / 2.0)
    cam.update(model="pinhole", fx=float(fx), fy=float(fx if fy is None else fy),
               cx=float(0.5 * width if cx is None else cx), cy=float(0.5 * height if cy is None else cy))
    return cam


def crop_poses(config: int, count: int, width: int, height: int, fov_x_deg=90.0, radius=1.0):
    """Seeded perspective crops: centre uniform in the ball of ``radius``,
    yaw ~ U[-pi, pi), pitch ~ U[-pi/6, pi/6], world->camera rotation
    (R_y(yaw) R_x(pitch))^T."""
    rng = rng_for(config, STREAM_POSES, 1)
    out = []
    for _ in range(count):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = d * radius * rng.uniform() ** (1.0 / 3.0)
        yaw, pitch = rng.uniform(-np.pi, np.pi), rng.uniform(-np.pi / 6, np.pi / 6)
        out.append(pinhole_camera(width, height, fov_x_deg, (rot_y(yaw) @ rot_x(pitch)).T, c))
    return out


def cube_faces(cam: dict, size: int) -> list:
    """The six 90-degree pinhole faces (size x size) of a cube map around an
    ERP camera's centre: front, right, back, left (about the camera's Y
    axis), up and down.  Face k's world->camera rotation is F_k^T R with F_k
    the face's axes in the ERP camera frame."""
    R = np.asarray(cam["R"], dtype=np.float64)
    t = np.asarray(cam["t"], dtype=np.float64)
    faces = [rot_y(0.0), rot_y(np.pi / 2), rot_y(np.pi), rot_y(-np.pi / 2), rot_x(np.pi / 2), rot_x(-np.pi / 2)]
    out = []
    for F in faces:
        c = pinhole_camera(size, size, 90.0)
        c.update(R=F.T @ R, t=F.T @ t)
        out.append(c)
    return out


def poses(config: int, count: int, width: int, height: int, radius=1.0, yaw_zero=False):
    """Seeded poses: centre uniform in the ball of ``radius``, yaw ~ U[-pi, pi),
    world->camera rotation R_y(yaw)^T."""
    rng = rng_for(config, STREAM_POSES)
    out = []
    for _ in range(count):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = d * radius * rng.uniform() ** (1.0 / 3.0)
        yaw = 0.0 if yaw_zero else rng.uniform(-np.pi, np.pi)
        out.append(camera(width, height, rot_y(yaw).T, c))
    return out


SERVE_RESOLUTIONS = ((512, 256), (1024, 512), (2048, 1024), (3840, 1920))


def serve_cameras(config: int, count: int, resolutions=SERVE_RESOLUTIONS):
    """Cameras of a request stream: resolution uniform over `resolutions`,
    centre uniform in the unit ball, random yaw (the same sequence whatever
    the arrival rate)."""
    rng = rng_for(config, STREAM_REQUESTS)
    out = []
    for _ in range(count):
        w, h = resolutions[rng.integers(len(resolutions))]
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = d * rng.uniform() ** (1.0 / 3.0)
        yaw = rng.uniform(-np.pi, np.pi)
        out.append(camera(int(w), int(h), rot_y(yaw).T, c))
    return out


def arrival_times(config: int, count: int, rate_hz: float, run: int = 0):
    """Poisson arrivals: cumulative exponential gaps of mean 1 / rate_hz
    (seconds), seeded per run."""
    rng = rng_for(config, STREAM_REQUESTS, 1 + run)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))


# the workloads' scene definitions
def config0():
    """1,000 Gaussians in the shell, identity pose, 128x64."""
    return shell_scene(0, 1000), camera(128, 64)


def config1():
    """100k Gaussians in the shell at 1024x512 with a perturbed target set."""
    g = shell_scene(1, 100_000)
    return g, camera(1024, 512), perturbed(1, g)


def config2(n_poses=200):
    """1M Gaussians in the room layout at 2048x1024, 200 poses."""
    g = room_scene(2, 1_000_000)
    return g, poses(2, n_poses, 2048, 1024), perturbed(2, g)


def config3(n_poses=8):
    """3M Gaussians, room layout, scales log-uniform [0.002, 0.5], 3840x1920."""
    g = room_scene(3, 3_000_000, scale_lo=0.002, scale_hi=0.5)
    return g, poses(3, n_poses, 3840, 1920), perturbed(3, g)
