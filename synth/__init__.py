"""Seeded synthetic inputs shared by the FP64 oracle and the HIP library.

This module only *generates inputs*: voxel fields sampled at the key points
(the voxel vertices of the reconstruction grid, Sec. 3.3 "Key points") and
pinhole camera rigs. It contains none of the method's arithmetic (no ray
generation, marching, projection, back-projection or Planck integrals); each
side implements those on its own.

The workloads stand in for the paper's simulated fire and captured flames
(Sec. 5.1, Sec. 5.2), which are not available: Gaussian blob "plumes" on the
unit cube seen by a ring of cameras, shaped like the paper's rig (views spread
around the flame in one plane, perspective projection, Sec. 5.1).

Everything is generated in float64 at the node positions; callers cast to the
precision they need (the GPU path takes float32).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Grid",
    "Rig",
    "ring_rig",
    "grid_nodes",
    "blob_field",
    "tiny_volume",
    "colour_volume",
    "temperature_volume",
    "random_volume",
    "CONFIGS",
]


@dataclasses.dataclass(frozen=True)
class Grid:
    """Node-centred grid: n = (nx, ny, nz) key points spanning [lo, hi]."""

    nx: int
    ny: int
    nz: int
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)

    @property
    def shape_zyx(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Rig:
    """V pinhole cameras sharing one image size.

    World -> camera is x_c = R x_w + t; pixel u grows to the right, v grows
    downwards, the optical axis is +z_c, and pixel (u, v) covers
    [u, u+1) x [v, v+1) in the (fx, fy, cx, cy) intrinsics.
    """

    fx: np.ndarray  # [V]
    fy: np.ndarray  # [V]
    cx: np.ndarray  # [V]
    cy: np.ndarray  # [V]
    R: np.ndarray  # [V, 3, 3]
    t: np.ndarray  # [V, 3]
    width: int
    height: int

    @property
    def n_views(self) -> int:
        return int(self.fx.shape[0])

    def subset(self, views):
        views = list(views)
        return Rig(self.fx[views].copy(), self.fy[views].copy(), self.cx[views].copy(),
                   self.cy[views].copy(), self.R[views].copy(), self.t[views].copy(),
                   self.width, self.height)

    def centres(self) -> np.ndarray:
        """Camera centres in world coordinates (input bookkeeping only)."""
        return -np.einsum("vji,vj->vi", self.R, self.t)


def _look_at(eye, target, up):
    f = np.asarray(target, float) - np.asarray(eye, float)
    f /= np.linalg.norm(f)
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f])  # rows: camera x (right), y (down), z (forward)
    t = -R @ np.asarray(eye, float)
    return R, t


def ring_rig(n_views: int, width: int, height: int, *, radius: float = 3.0,
             fov_y_deg: float = 40.0, centre=(0.5, 0.5, 0.5), elevation_jitter_deg: float = 0.0,
             seed: int = 0, azimuth0_deg: float = 0.0) -> Rig:
    """Cameras at azimuth 2*pi*v/V on a circle around ``centre`` in its z-plane,
    each looking at ``centre`` with world +z up; vertical field of view
    ``fov_y_deg``; principal point at the image centre.

    ``elevation_jitter_deg`` > 0 lifts/lowers each camera by a seeded
    elevation angle in [-jitter, jitter] (the paper's virtual cameras look
    slightly up or down, Sec. 5.1).
    """
    rng = np.random.default_rng(seed)
    c = np.asarray(centre, float)
    fy = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    Rs, ts = [], []
    for v in range(n_views):
        az = math.radians(azimuth0_deg) + 2.0 * math.pi * v / n_views
        el = 0.0
        if elevation_jitter_deg > 0:
            el = math.radians(rng.uniform(-elevation_jitter_deg, elevation_jitter_deg))
        eye = c + radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                                     math.sin(el)])
        R, t = _look_at(eye, c, np.array([0.0, 0.0, 1.0]))
        Rs.append(R)
        ts.append(t)
    V = n_views
    return Rig(np.full(V, fy), np.full(V, fy), np.full(V, width / 2.0), np.full(V, height / 2.0),
               np.array(Rs), np.array(ts), int(width), int(height))


def grid_nodes(grid: Grid):
    """World coordinates of the key points as three [nz, ny, nx] arrays."""
    xs = np.linspace(grid.lo[0], grid.hi[0], grid.nx)
    ys = np.linspace(grid.lo[1], grid.hi[1], grid.ny)
    zs = np.linspace(grid.lo[2], grid.hi[2], grid.nz)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X, Y, Z


def blob_fields(grid: Grid, centres, covs, peaks) -> np.ndarray:
    """Several fields sharing the same Gaussian blobs: field f is
    sum_b peaks[b][f] * exp(-0.5 (x - c_b)^T cov_b^{-1} (x - c_b)) at every
    key point. peaks has shape [n_blobs, n_fields]; returns [n_fields, nz, ny, nx]."""
    xs = np.linspace(grid.lo[0], grid.hi[0], grid.nx)
    ys = np.linspace(grid.lo[1], grid.hi[1], grid.ny)
    zs = np.linspace(grid.lo[2], grid.hi[2], grid.nz)
    peaks = np.asarray(peaks, float).reshape(len(centres), -1)
    out = np.zeros((peaks.shape[1],) + grid.shape_zyx)
    for c, cov, pk in zip(centres, covs, peaks):
        A = np.linalg.inv(np.asarray(cov, float))
        dx = (xs - c[0])[None, None, :]
        dy = (ys - c[1])[None, :, None]
        dz = (zs - c[2])[:, None, None]
        q = (A[0, 0] * dx * dx + A[1, 1] * dy * dy + A[2, 2] * dz * dz
             + 2.0 * A[0, 1] * dx * dy + 2.0 * A[0, 2] * dx * dz + 2.0 * A[1, 2] * dy * dz)
        gb = np.exp(-0.5 * q)
        for f in range(peaks.shape[1]):
            out[f] += pk[f] * gb
    return out


def blob_field(grid: Grid, centres, covs, peaks) -> np.ndarray:
    """sum_b peak_b * exp(-0.5 (x - c_b)^T cov_b^{-1} (x - c_b)) at every key point."""
    return blob_fields(grid, centres, covs, np.asarray(peaks, float)[:, None])[0]


def tiny_volume(seed: int = 0, n: int = 32, n_blobs: int = 3):
    """Tiny plain-method instance: sum of isotropic Gaussian blobs (centres
    U[0.3,0.7]^3, std U[0.05,0.15], peak U[0.5,1]); emission = density,
    extinction = 2 * density. Returns (grid, emission [1,n,n,n], extinction [n,n,n])."""
    rng = np.random.default_rng(seed)
    g = Grid(n, n, n)
    centres = rng.uniform(0.3, 0.7, size=(n_blobs, 3))
    stds = rng.uniform(0.05, 0.15, size=n_blobs)
    peaks = rng.uniform(0.5, 1.0, size=n_blobs)
    covs = [np.eye(3) * s * s for s in stds]
    rho = blob_field(g, centres, covs, peaks)
    return g, rho[None].copy(), 2.0 * rho


def _plume_blobs(rng, n_blobs):
    centres, covs = [], []
    for _ in range(n_blobs):
        c = np.array([rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7), rng.uniform(0.25, 0.55)])
        s = rng.uniform(0.035, 0.08, size=3)
        kappa = rng.uniform(2.0, 4.0)  # stretch along +z: flame-like plume
        D = np.diag([s[0] ** 2, s[1] ** 2, (kappa * s[2]) ** 2])
        # small seeded tilt of the plume axis
        ax = rng.normal(size=3)
        ax[2] = 0.0
        ax /= np.linalg.norm(ax) + 1e-30
        ang = math.radians(rng.uniform(0.0, 12.0))
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        Rm = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)
        centres.append(c)
        covs.append(Rm @ D @ Rm.T)
    return centres, covs


def colour_blobs(seed: int = 0, n_blobs: int = 20):
    """The plume blobs of the colour workload: (centres, covariances, peaks
    [B, 4] = RGB emission and extinction) on the unit cube."""
    rng = np.random.default_rng(seed)
    centres, covs = _plume_blobs(rng, n_blobs)
    rgb = np.array([[1.0, rng.uniform(0.4, 0.8), rng.uniform(0.1, 0.3)] for _ in range(n_blobs)])
    rgb *= rng.uniform(0.5, 1.0, size=(n_blobs, 1))
    sig_pk = rng.uniform(0.5, 4.0, size=n_blobs)
    return centres, covs, np.concatenate([rgb, sig_pk[:, None]], axis=1)


def colour_volume(seed: int = 0, n: int = 128, n_blobs: int = 20):
    """Colour-intensity workload: 20 anisotropic plume blobs stretched along +z.
    Per-blob RGB emission (1, U[0.4,0.8], U[0.1,0.3]) * U[0.5,1]; per-blob peak
    extinction U[0.5,4] per unit length. Returns (grid, emission [3,n,n,n],
    extinction [n,n,n])."""
    g = Grid(n, n, n)
    fields = blob_fields(g, *colour_blobs(seed, n_blobs))
    return g, fields[:3].copy(), fields[3].copy()


def temperature_volume(seed: int = 0, n: int = 128, n_blobs: int = 20, t_bg: float = 800.0,
                       t_cap: float = 2200.0):
    """Temperature workload: T = 800 K + sum_b dT_b * blob_b, dT_b ~ U[200,1400],
    clamped to [800, 2200] K. Returns (grid, T [n,n,n])."""
    rng = np.random.default_rng(seed)
    g = Grid(n, n, n)
    centres, covs = _plume_blobs(rng, n_blobs)
    dT = rng.uniform(200.0, 1400.0, size=n_blobs)
    T = t_bg + blob_field(g, centres, covs, dT)
    return g, np.clip(T, t_bg, t_cap)


def random_volume(grid: Grid, channels: int, seed: int = 0, sigma_scale: float = 2.0,
                  positive: bool = True):
    """Unstructured random fields (for adjoint-identity style checks)."""
    rng = np.random.default_rng(seed)
    sh = grid.shape_zyx
    em = rng.uniform(0.0, 1.0, size=(channels,) + sh) if positive else \
        rng.normal(size=(channels,) + sh)
    sig = sigma_scale * rng.uniform(0.0, 1.0, size=sh)
    return em, sig


# Workload recipes (sizes of the hot-path configurations).
CONFIGS = {
    "tiny": dict(n=32, views=4, width=64, height=64, fov=40.0, radius=3.0, step_vox=0.5,
                 channels=1, albedo=0.0, iters=5),
    "colour": dict(n=128, views=8, width=512, height=512, fov=40.0, radius=3.0, step_vox=0.5,
                   channels=3, albedo=0.3, scatter_res=32, scatter_dirs=32, iters=20),
    "temperature": dict(n=128, views=8, width=512, height=512, fov=40.0, radius=3.0,
                        step_vox=0.5, channels=1, albedo=0.0, iters=30),
}


# ----------------------------------------------------------------- videos
@dataclasses.dataclass
class VideoSpec:
    """One synthetic flame video: a grid, a camera rig and plume blobs whose
    centres drift with a seeded per-blob velocity (frame-to-frame advection)."""

    video: int
    grid: Grid
    rig: Rig
    centres: np.ndarray   # [B, 3] at frame 0
    velocity: np.ndarray  # [B, 3] per frame
    covs: list
    peaks: np.ndarray     # [B, 4]: RGB emission, extinction

    def centres_at(self, frame: int) -> np.ndarray:
        c = self.centres + frame * self.velocity
        # keep the plumes inside the box: reflect at the [0.2, 0.8] walls
        c = np.abs(((c - 0.2) % 1.2) - 0.6) + 0.2
        return c


SERVE_GRIDS = (64, 128, 192, 256)
SERVE_IMAGES = ((256, 256), (512, 512), (640, 480), (1024, 768))


def video_spec(video: int, seed: int = 0, n_blobs: int = 12) -> VideoSpec:
    """Grid size from {64,128,192,256}^3, 4-12 ring views, image size from
    {256^2, 512^2, 640x480, 1024x768}, all drawn from the seed."""
    rng = np.random.default_rng([seed, video])
    n = int(rng.choice(SERVE_GRIDS))
    views = int(rng.integers(4, 13))
    W, H = SERVE_IMAGES[int(rng.integers(0, len(SERVE_IMAGES)))]
    centres, covs = _plume_blobs(rng, n_blobs)
    rgb = np.array([[1.0, rng.uniform(0.4, 0.8), rng.uniform(0.1, 0.3)] for _ in range(n_blobs)])
    rgb *= rng.uniform(0.5, 1.0, size=(n_blobs, 1))
    sig = rng.uniform(0.5, 4.0, size=(n_blobs, 1))
    vel = rng.normal(scale=0.004, size=(n_blobs, 3)) + np.array([0.0, 0.0, 0.003])
    rig = ring_rig(views, W, H, elevation_jitter_deg=10.0, seed=seed * 1000 + video)
    return VideoSpec(video, Grid(n, n, n), rig, np.array(centres), vel, covs,
                     np.concatenate([rgb, sig], axis=1))


def blob_fields_torch(grid: Grid, centres, covs, peaks, device="cuda"):
    """blob_fields evaluated with torch on `device` (float64 arithmetic, float32
    result) for large grids."""
    import torch
    xs = torch.linspace(grid.lo[0], grid.hi[0], grid.nx, dtype=torch.float64, device=device)
    ys = torch.linspace(grid.lo[1], grid.hi[1], grid.ny, dtype=torch.float64, device=device)
    zs = torch.linspace(grid.lo[2], grid.hi[2], grid.nz, dtype=torch.float64, device=device)
    peaks = np.asarray(peaks, float).reshape(len(centres), -1)
    out = torch.zeros((peaks.shape[1],) + grid.shape_zyx, dtype=torch.float64, device=device)
    for c, cov, pk in zip(centres, covs, peaks):
        A = np.linalg.inv(np.asarray(cov, float))
        dx = (xs - c[0])[None, None, :]
        dy = (ys - c[1])[None, :, None]
        dz = (zs - c[2])[:, None, None]
        q = (A[0, 0] * dx * dx + A[1, 1] * dy * dy + A[2, 2] * dz * dz
             + 2.0 * A[0, 1] * dx * dy + 2.0 * A[0, 2] * dx * dz + 2.0 * A[1, 2] * dy * dz)
        gb = torch.exp(-0.5 * q)
        for f in range(peaks.shape[1]):
            out[f] += float(pk[f]) * gb
    return out.float()


def video_frame(spec: VideoSpec, frame: int, device=None):
    """(emission [3,n,n,n], extinction [n,n,n]) of one frame: numpy when device
    is None, else torch tensors on that device."""
    c = spec.centres_at(frame)
    if device is None:
        f = blob_fields(spec.grid, c, spec.covs, spec.peaks)
        return f[:3].copy(), f[3].copy()
    f = blob_fields_torch(spec.grid, c, spec.covs, spec.peaks, device)
    return f[:3].contiguous(), f[3].contiguous()


def poisson_arrivals(n_jobs: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
