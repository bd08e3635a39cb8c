"""Thin ctypes binding of librte (include/rte.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of librte.so. Tensors must be float32, contiguous and on the GPU; each call is
enqueued on the current torch stream. There is no CPU fallback: importing the
binding without a built library, or calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

__all__ = [
    "LIB_PATH", "lib", "RteError", "Plan", "TempParams", "plan_create", "render", "inscatter",
    "backproject", "reconstruct", "reconstruct_temperature", "temperature_map",
    "temperature_invert", "KERNELS", "UPDATES", "job_step", "suggest_grid", "render_static",
    "STATIC_SCRATCH_BYTES", "STATIC_MAX_VIEWS",
]

# RTE_SANITIZE=1: the build with sanitized host code (python -m paper_1809_06417_amd.build --sanitize)
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "librte.asan.so" if os.environ.get("RTE_SANITIZE") == "1" else "librte.so")

RTE_OK, RTE_ERR_INVALID_ARG, RTE_ERR_BUDGET, RTE_ERR_HIP, RTE_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
KERNELS = {"rays": 0, "render": 1, "inscatter": 2, "gather": 3, "update": 4, "temp_map": 5,
           "pack": 6, "weights": 7, "colsum": 8, "adjoint": 9}
RTE_PLAN_GRADIENTS = 1
STATIC_SCRATCH_BYTES, STATIC_MAX_VIEWS = 128 << 20, 16  # RTE_STATIC_SCRATCH_BYTES, RTE_STATIC_MAX_VIEWS
UPDATES = {"sart": 0, "paper": 1, "mlem": 2}
BP_MODES = {"adjoint": 0, "paper": 1}


class RteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librte error {code}: {msg}")
        self.code = code


class Camera(ct.Structure):
    _fields_ = [("fx", ct.c_double), ("fy", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double),
                ("R", ct.c_double * 9), ("t", ct.c_double * 3), ("width", ct.c_int32),
                ("height", ct.c_int32)]


class Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("bbox_min", ct.c_double * 3), ("bbox_max", ct.c_double * 3)]


class RenderParams(ct.Structure):
    _fields_ = [("channels", ct.c_int32), ("step_vox", ct.c_float), ("albedo", ct.c_float),
                ("background", ct.c_float), ("scatter_res", ct.c_int32),
                ("scatter_dirs", ct.c_int32), ("scatter_step", ct.c_float), ("flags", ct.c_int32),
                ("phase_g", ct.c_float)]


class ReconParams(ct.Structure):
    _fields_ = [("update", ct.c_int32), ("lam", ct.c_float), ("clamp_nonneg", ct.c_int32),
                ("alpha_l", ct.c_float), ("alpha_d", ct.c_float), ("tau", ct.c_float),
                ("g_sigma", ct.c_float), ("seed", ct.c_uint64), ("use_mask", ct.c_int32),
                ("flame_threshold", ct.c_float), ("use_hull", ct.c_int32),
                ("outside_value", ct.c_float), ("stop_tol", ct.c_float), ("ordered_subsets", ct.c_int32)]


class _TempParams(ct.Structure):
    _fields_ = [("t_min", ct.c_float), ("t_max", ct.c_float), ("t_norm", ct.c_float),
                ("band_nm", ct.c_float * 3), ("band_std_nm", ct.c_float), ("lut_size", ct.c_int32),
                ("sigma_max", ct.c_float), ("soot_t0", ct.c_float), ("soot_span", ct.c_float),
                ("channel", ct.c_int32), ("panels", ct.c_int32)]


class TempParams:
    """Colour-temperature mapping parameters (see rte_temp_params)."""

    def __init__(self, t_min=800.0, t_max=2300.0, t_norm=2200.0, band_nm=(650.0, 550.0, 450.0),
                 band_std_nm=40.0, lut_size=4096, sigma_max=4.0, soot_t0=800.0, soot_span=1400.0,
                 channel=1, panels=4000):
        self.t_min, self.t_max, self.t_norm = t_min, t_max, t_norm
        self.band_nm = tuple(band_nm)
        self.band_std_nm, self.lut_size = band_std_nm, lut_size
        self.sigma_max, self.soot_t0, self.soot_span = sigma_max, soot_t0, soot_span
        self.channel, self.panels = channel, panels

    def c(self):
        s = _TempParams()
        s.t_min, s.t_max, s.t_norm = self.t_min, self.t_max, self.t_norm
        s.band_nm[:] = list(self.band_nm)
        s.band_std_nm, s.lut_size = self.band_std_nm, self.lut_size
        s.sigma_max, s.soot_t0, s.soot_span = self.sigma_max, self.soot_t0, self.soot_span
        s.channel, s.panels = self.channel, self.panels
        return s


_lib = None


def lib():
    """Load librte.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"librte.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ct.CDLL(LIB_PATH)
    P, vp, i32 = ct.POINTER, ct.c_void_p, ct.c_int32
    L.rte_plan_create.argtypes = [P(vp), P(Grid), P(Camera), i32, P(RenderParams), ct.c_size_t, vp]
    L.rte_plan_workspace_bytes.argtypes = [P(Grid), P(Camera), i32, P(RenderParams)]
    L.rte_plan_workspace_bytes.restype = ct.c_size_t
    L.rte_plan_device_bytes.argtypes = [vp]
    L.rte_plan_device_bytes.restype = ct.c_size_t
    L.rte_plan_destroy.argtypes = [vp]
    L.rte_plan_destroy.restype = None
    L.rte_plan_counts.argtypes = [vp, P(ct.c_uint64), P(ct.c_uint64)]
    L.rte_ray_table.argtypes = [vp, vp, vp, vp, vp]
    L.rte_render.argtypes = [vp, vp, vp, vp, vp, vp]
    L.rte_render_static.argtypes = [P(Grid), P(Camera), i32, P(RenderParams), vp, vp, vp, vp, vp]
    L.rte_render_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.rte_render_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.rte_inscatter.argtypes = [vp, vp, vp, vp, vp]
    L.rte_backproject.argtypes = [vp, vp, vp, vp, i32, P(ReconParams), vp]
    L.rte_reconstruct.argtypes = [vp, vp, vp, vp, i32, P(ReconParams), vp]
    L.rte_reconstruct_temperature.argtypes = [vp, vp, vp, i32, P(ReconParams), P(_TempParams), vp]
    L.rte_temperature_map.argtypes = [vp, vp, vp, vp, P(_TempParams), vp]
    L.rte_temperature_invert.argtypes = [vp, vp, vp, P(_TempParams), vp]
    L.rte_temperature_lut.argtypes = [vp, P(_TempParams), P(ct.c_float), i32]
    L.rte_suggest_grid.argtypes = [P(Camera), i32, P(ct.c_double), P(ct.c_double), ct.c_double, P(Grid),
                                   P(ct.c_double)]
    L.rte_job_begin.argtypes = [vp, vp, vp, vp, P(ReconParams), vp]
    L.rte_job_step.argtypes = [P(vp), i32, vp]
    L.rte_job_end.argtypes = [vp, vp, vp]
    L.rte_reconstruct_stats.argtypes = [vp, P(ct.c_int32), P(ct.c_int32), P(ct.c_float), i32]
    L.rte_flame_mask.argtypes = [vp, vp, ct.c_float, vp, vp]
    L.rte_visual_hull.argtypes = [vp, vp, vp, vp]
    L.rte_plan_set_timing.argtypes = [vp, i32]
    L.rte_plan_set_timing_mask.argtypes = [vp, ct.c_uint32]
    L.rte_plan_kernel_time.argtypes = [vp, i32, P(ct.c_double), P(ct.c_int64)]
    L.rte_last_error.restype = ct.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != RTE_OK:
        raise RteError(rc, lib().rte_last_error().decode())


def _grid(g):
    s = Grid()
    s.nx, s.ny, s.nz = int(g.nx), int(g.ny), int(g.nz)
    s.bbox_min[:] = [float(x) for x in g.lo]
    s.bbox_max[:] = [float(x) for x in g.hi]
    return s


def _cams(rig):
    V = int(len(rig.fx))
    arr = (Camera * V)()
    for v in range(V):
        c = arr[v]
        c.fx, c.fy, c.cx, c.cy = float(rig.fx[v]), float(rig.fy[v]), float(rig.cx[v]), float(rig.cy[v])
        c.R[:] = [float(x) for x in np.asarray(rig.R[v], dtype=np.float64).reshape(9)]
        c.t[:] = [float(x) for x in np.asarray(rig.t[v], dtype=np.float64).reshape(3)]
        c.width, c.height = int(rig.width), int(rig.height)
    return arr, V


def _params(channels, step_vox, albedo, background, scatter_res, scatter_dirs, scatter_step,
            flags=0, phase_g=0.0):
    p = RenderParams()
    p.channels, p.step_vox, p.albedo, p.background = int(channels), step_vox, albedo, background
    p.scatter_res, p.scatter_dirs, p.scatter_step = int(scatter_res), int(scatter_dirs), scatter_step
    p.flags = int(flags)
    p.phase_g = float(phase_g)
    return p


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, shape=None, name="tensor", fp64=False):
    """Device pointer of a float32/int32 (float64 with fp64=True) contiguous
    GPU tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if fp64 and t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64 (got {t.dtype})")
    if not fp64 and t.dtype not in (torch.float32, torch.int32):
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ct.c_void_p(t.data_ptr())


def workspace_bytes(grid, rig, channels=1, step_vox=0.5, albedo=0.0, background=0.0, scatter_res=0,
                    scatter_dirs=32, scatter_step=0.5, gradients=False, phase_g=0.0):
    cams, V = _cams(rig)
    p = _params(channels, step_vox, albedo, background, scatter_res, scatter_dirs, scatter_step,
                RTE_PLAN_GRADIENTS if gradients else 0, phase_g)
    return int(lib().rte_plan_workspace_bytes(ct.byref(_grid(grid)), cams, V, ct.byref(p)))


class Plan:
    """A grid + camera rig + forward-model setup with its device workspaces."""

    def __init__(self, grid, rig, channels=1, step_vox=0.5, albedo=0.0, background=0.0,
                 scatter_res=0, scatter_dirs=32, scatter_step=0.5, hbm_budget_bytes=0,
                 gradients=False, phase_g=0.0):
        import torch
        self._h = None
        self.grid = grid
        self.channels = int(channels)
        self.V, self.H, self.W = int(len(rig.fx)), int(rig.height), int(rig.width)
        self.scatter_res = int(scatter_res)
        self.phase_g = float(phase_g)
        cams, V = _cams(rig)
        self.gradients = bool(gradients)
        self._p = _params(channels, step_vox, albedo, background, scatter_res, scatter_dirs,
                          scatter_step, RTE_PLAN_GRADIENTS if gradients else 0, phase_g)
        h = ct.c_void_p()
        torch.cuda.init()
        _check(lib().rte_plan_create(ct.byref(h), ct.byref(_grid(grid)), cams, V,
                                     ct.byref(self._p), int(hbm_budget_bytes), _stream()))
        self._h = h
        s, hr = ct.c_uint64(), ct.c_uint64()
        _check(lib().rte_plan_counts(h, ct.byref(s), ct.byref(hr)))
        self.samples, self.hit_rays = int(s.value), int(hr.value)
        self.device_bytes = int(lib().rte_plan_device_bytes(h))

    # -- shapes
    @property
    def vol_shape(self):
        return (self.grid.nz, self.grid.ny, self.grid.nx)

    def img_shape(self, C=None):
        return (self.V, self.channels if C is None else C, self.H, self.W)

    @property
    def scat_shape(self):
        """[C, M, M, M], or [V, C, M, M, M] (one grid per view) when phase_g != 0."""
        M = self.scatter_res
        one = (self.channels, M, M, M)
        return (self.V,) + one if self.phase_g != 0.0 and M >= 2 else one

    def _new(self, shape, dtype=None):
        import torch
        return torch.empty(shape, device="cuda", dtype=dtype or torch.float32)

    # -- calls
    def ray_table(self):
        import torch
        tn = self._new((self.V, self.H, self.W))
        tf = self._new((self.V, self.H, self.W))
        K = self._new((self.V, self.H, self.W), torch.int32)
        _check(lib().rte_ray_table(self._h, _ptr(tn), _ptr(tf), _ptr(K), _stream()))
        return tn, tf, K

    def render(self, emission, extinction, inscatter=None, out=None):
        C = self.channels
        out = self._new(self.img_shape()) if out is None else out
        M = self.scatter_res
        _check(lib().rte_render(self._h, _ptr(emission, (C,) + self.vol_shape, "emission"),
                                _ptr(extinction, self.vol_shape, "extinction"),
                                _ptr(inscatter, self.scat_shape, "inscatter"),
                                _ptr(out, self.img_shape(), "images"), _stream()))
        return out

    def render_forward(self, emission, extinction, inscatter=None):
        """Images and the FP64 exit optical depth of every ray (for
        render_backward; the exit transmittance is exp(-depth))."""
        import torch
        C, M = self.channels, self.scatter_res
        out = self._new(self.img_shape())
        exit_tau = self._new((self.V, self.H, self.W), torch.float64)
        _check(lib().rte_render_forward(self._h, _ptr(emission, (C,) + self.vol_shape, "emission"),
                                        _ptr(extinction, self.vol_shape, "extinction"),
                                        _ptr(inscatter, self.scat_shape, "inscatter"),
                                        _ptr(out), _ptr(exit_tau, fp64=True), _stream()))
        return out, exit_tau

    def render_backward(self, emission, extinction, inscatter, exit_tau, grad_images):
        """(dL/d emission, dL/d extinction) given dL/d images."""
        C, M = self.channels, self.scatter_res
        g_em = self._new((C,) + self.vol_shape)
        g_sig = self._new(self.vol_shape)
        _check(lib().rte_render_backward(
            self._h, _ptr(emission, (C,) + self.vol_shape, "emission"),
            _ptr(extinction, self.vol_shape, "extinction"), _ptr(inscatter, self.scat_shape, "inscatter"),
            _ptr(exit_tau, (self.V, self.H, self.W), "exit_tau", fp64=True),
            _ptr(grad_images, self.img_shape(), "grad_images"), _ptr(g_em), _ptr(g_sig), _stream()))
        return g_em, g_sig

    def inscatter(self, emission, extinction, out=None):
        C = self.channels
        out = self._new(self.scat_shape) if out is None else out
        _check(lib().rte_inscatter(self._h, _ptr(emission, (C,) + self.vol_shape, "emission"),
                                   _ptr(extinction, self.vol_shape, "extinction"),
                                   _ptr(out, self.scat_shape, "inscatter"), _stream()))
        return out

    def backproject(self, extinction, residual, mode="adjoint", alpha_l=1e-3, alpha_d=1.0,
                    tau=0.05, out=None):
        C = self.channels
        out = self._new((C,) + self.vol_shape) if out is None else out
        rp = ReconParams(update=UPDATES["paper"], lam=1.0, clamp_nonneg=0, alpha_l=alpha_l,
                         alpha_d=alpha_d, tau=tau)
        _check(lib().rte_backproject(self._h, _ptr(extinction, self.vol_shape, "extinction"),
                                     _ptr(residual, self.img_shape(), "residual"),
                                     _ptr(out, (C,) + self.vol_shape, "delta"), BP_MODES[mode],
                                     ct.byref(rp), _stream()))
        return out

    def reconstruct(self, frames, extinction, emission, iters, update="sart", lam=1.0,
                    clamp_nonneg=True, alpha_l=1e-3, alpha_d=1.0, tau=0.05, g_sigma=0.0, seed=0,
                    flame_threshold=None, hull=False, outside_value=0.0, stop_tol=0.0, subsets=1):
        """In place on `emission` (warm start); returns it. flame_threshold
        (not None) restricts the adjustment to flame rays, hull=True to the
        visual hull; stop_tol > 0 turns on the stop rule (see stats());
        subsets > 1 makes ordered-subset updates (views v mod subsets)."""
        C = self.channels
        rp = ReconParams(update=UPDATES[update], lam=lam, clamp_nonneg=1 if clamp_nonneg else 0,
                         alpha_l=alpha_l, alpha_d=alpha_d, tau=tau, g_sigma=g_sigma, seed=int(seed),
                         use_mask=0 if flame_threshold is None else 1,
                         flame_threshold=0.0 if flame_threshold is None else flame_threshold,
                         use_hull=1 if hull else 0, outside_value=outside_value, stop_tol=stop_tol,
                         ordered_subsets=int(subsets))
        _check(lib().rte_reconstruct(self._h, _ptr(frames, self.img_shape(), "frames"),
                                     _ptr(extinction, self.vol_shape, "extinction"),
                                     _ptr(emission, (C,) + self.vol_shape, "emission"), int(iters),
                                     ct.byref(rp), _stream()))
        return emission

    def reconstruct_temperature(self, frames, temperature, iters, temp=None, lam=1.0):
        """In place on `temperature` [K]; frames are [V, 3, H, W]."""
        temp = temp or TempParams()
        rp = ReconParams(update=UPDATES["mlem"], lam=lam)
        _check(lib().rte_reconstruct_temperature(
            self._h, _ptr(frames, (self.V, 3, self.H, self.W), "frames"),
            _ptr(temperature, self.vol_shape, "temperature"), int(iters), ct.byref(rp),
            ct.byref(temp.c()), _stream()))
        return temperature

    def job_begin(self, frames, extinction, emission=None, update="sart", lam=1.0,
                  clamp_nonneg=True, flame_threshold=None, hull=False, outside_value=0.0, subsets=1):
        """Open a job; emission None keeps the volume resident in the plan."""
        C = self.channels
        rp = ReconParams(update=UPDATES[update], lam=lam, clamp_nonneg=1 if clamp_nonneg else 0,
                         alpha_l=1e-3, alpha_d=1.0, tau=0.05,
                         use_mask=0 if flame_threshold is None else 1,
                         flame_threshold=0.0 if flame_threshold is None else flame_threshold,
                         use_hull=1 if hull else 0, outside_value=outside_value, ordered_subsets=int(subsets))
        self._job_frames = frames  # keep the caller's frames alive while the job is open
        _check(lib().rte_job_begin(self._h, _ptr(frames, self.img_shape(), "frames"),
                                   _ptr(extinction, self.vol_shape, "extinction"),
                                   _ptr(emission, (C,) + self.vol_shape, "emission"), ct.byref(rp),
                                   _stream()))

    def job_end(self, emission=None):
        C = self.channels
        _check(lib().rte_job_end(self._h, _ptr(emission, (C,) + self.vol_shape, "emission"),
                                 _stream()))
        self._job_frames = None
        return emission

    def stats(self, max_errors=1024):
        """(updates made, per-iteration image RMS) of the last reconstruct()."""
        n, ne = ct.c_int32(), ct.c_int32()
        errs = (ct.c_float * max_errors)()
        _check(lib().rte_reconstruct_stats(self._h, ct.byref(n), ct.byref(ne), errs, max_errors))
        return int(n.value), [float(errs[i]) for i in range(min(int(ne.value), max_errors))]

    def flame_mask(self, frames, threshold):
        m = self._new((self.V, self.H, self.W))
        _check(lib().rte_flame_mask(self._h, _ptr(frames, self.img_shape(), "frames"),
                                    float(threshold), _ptr(m), _stream()))
        return m

    def visual_hull(self, mask=None):
        import torch
        inside = self._new(self.vol_shape, torch.int32)
        _check(lib().rte_visual_hull(self._h, _ptr(mask, (self.V, self.H, self.W), "mask"),
                                     _ptr(inside), _stream()))
        return inside

    def temperature_map(self, temperature, temp=None):
        temp = temp or TempParams()
        em = self._new((3,) + self.vol_shape)
        sig = self._new(self.vol_shape)
        _check(lib().rte_temperature_map(self._h, _ptr(temperature, self.vol_shape, "temperature"),
                                         _ptr(em), _ptr(sig), ct.byref(temp.c()), _stream()))
        return em, sig

    def temperature_invert(self, e, temp=None):
        temp = temp or TempParams()
        T = self._new(self.vol_shape)
        _check(lib().rte_temperature_invert(self._h, _ptr(e, self.vol_shape, "e"), _ptr(T),
                                            ct.byref(temp.c()), _stream()))
        return T

    def temperature_lut(self, temp=None):
        temp = temp or TempParams()
        out = np.zeros((3, temp.lut_size), dtype=np.float32)
        _check(lib().rte_temperature_lut(self._h, ct.byref(temp.c()),
                                         out.ctypes.data_as(ct.POINTER(ct.c_float)),
                                         int(temp.lut_size)))
        return out

    def set_timing(self, enable=True, kernels=None):
        """Per-kernel timing on or off; `kernels` (names or RTE_KERNEL ids)
        limits it to those kernels."""
        if kernels is None:
            _check(lib().rte_plan_set_timing(self._h, 1 if enable else 0))
            return
        mask = 0
        for k in kernels:
            mask |= 1 << (KERNELS[k] if isinstance(k, str) else int(k))
        _check(lib().rte_plan_set_timing_mask(self._h, mask if enable else 0))

    def kernel_time(self, kernel):
        ms, n = ct.c_double(), ct.c_int64()
        _check(lib().rte_plan_kernel_time(self._h, KERNELS[kernel] if isinstance(kernel, str)
                                          else int(kernel), ct.byref(ms), ct.byref(n)))
        return float(ms.value), int(n.value)

    def close(self):
        if self._h:
            lib().rte_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def suggest_grid(rig, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), alpha=1.5):
    """Key points per axis (nx, ny, nz) for the box [lo, hi] seen by `rig`, and
    the projected edge spans n_max (pixels) they come from (host only)."""
    cams, V = _cams(rig)
    lo_a, hi_a = (ct.c_double * 3)(*lo), (ct.c_double * 3)(*hi)
    g = Grid()
    nmax = (ct.c_double * 3)()
    _check(lib().rte_suggest_grid(cams, V, lo_a, hi_a, float(alpha), ct.byref(g), nmax))
    return (int(g.nx), int(g.ny), int(g.nz)), tuple(float(x) for x in nmax)


def job_step(plans):
    """One iteration for every plan with an open job, batched in one launch per phase."""
    arr = (ct.c_void_p * len(plans))(*[p._h for p in plans])
    _check(lib().rte_job_step(arr, len(plans), _stream()))


def render_static(grid, rig, emission, extinction, inscatter=None, channels=1, step_vox=0.5, albedo=0.0,
                  background=0.0, scatter_res=0, scatter_dirs=32, scatter_step=0.5, phase_g=0.0, out=None):
    """Images [V, C, H, W] of rte_render_static: the render of a plan built from
    these arguments, without a plan (the library's static device array holds
    the workspaces; nothing is allocated on the device by the call). `out`
    may be given to keep the call free of torch allocations too."""
    import torch
    cams, V = _cams(rig)
    p = _params(channels, step_vox, albedo, background, scatter_res, scatter_dirs, scatter_step, 0, phase_g)
    vol = (int(grid.nz), int(grid.ny), int(grid.nx))
    C, H, W = int(channels), int(rig.height), int(rig.width)
    M = int(scatter_res)
    scat_shape = ((V,) if phase_g != 0.0 and M >= 2 else ()) + (C, M, M, M)
    if out is None:
        torch.cuda.init()
        out = torch.empty((V, C, H, W), device="cuda", dtype=torch.float32)
    _check(lib().rte_render_static(ct.byref(_grid(grid)), cams, V, ct.byref(p),
                                   _ptr(emission, (C,) + vol, "emission"), _ptr(extinction, vol, "extinction"),
                                   _ptr(inscatter, scat_shape, "inscatter"), _ptr(out, (V, C, H, W), "images"),
                                   _stream()))
    return out


# Functional aliases with the ABI's names.
def plan_create(grid, rig, **kw):
    return Plan(grid, rig, **kw)


def render(plan, emission, extinction, inscatter=None):
    return plan.render(emission, extinction, inscatter)


def inscatter(plan, emission, extinction):
    return plan.inscatter(emission, extinction)


def backproject(plan, extinction, residual, mode="adjoint", **kw):
    return plan.backproject(extinction, residual, mode, **kw)


def reconstruct(plan, frames, extinction, emission, iters, **kw):
    return plan.reconstruct(frames, extinction, emission, iters, **kw)


def reconstruct_temperature(plan, frames, temperature, iters, temp=None, lam=1.0):
    return plan.reconstruct_temperature(frames, temperature, iters, temp, lam)


def temperature_map(plan, temperature, temp=None):
    return plan.temperature_map(temperature, temp)


def temperature_invert(plan, e, temp=None):
    return plan.temperature_invert(e, temp)
