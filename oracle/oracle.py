"""ctypes marshalling for the FP64 oracle (test infrastructure only).

Inputs come from :mod:`synth` (grids, rigs, fields); every array is converted
to float64 C-contiguous before the call. See ``rte_oracle.c`` for the
arithmetic and the passages of the paper each function follows.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

__all__ = [
    "lib", "ray_table", "render", "inscatter", "backproject_adjoint", "backproject_paper",
    "reconstruct", "planck", "band_radiance", "TempParams", "temp_lut", "temp_map",
    "temp_invert", "temperature_fit", "num_threads", "render_grad", "philox4x32_10",
    "sample_gain", "flame_mask", "visual_hull", "reconstruct_ext", "suggest_grid", "set_num_threads",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# RTE_SANITIZE=1: the AddressSanitizer/UBSan build (python -m oracle.build --sanitize)
_LIB_PATH = os.path.join(_HERE, "liboracle.asan.so" if os.environ.get("RTE_SANITIZE") == "1" else "liboracle.so")
_lib = None


class _Camera(ct.Structure):
    _fields_ = [("fx", ct.c_double), ("fy", ct.c_double), ("cx", ct.c_double), ("cy", ct.c_double),
                ("R", ct.c_double * 9), ("t", ct.c_double * 3), ("width", ct.c_int32),
                ("height", ct.c_int32)]


class _Grid(ct.Structure):
    _fields_ = [("n", ct.c_int32 * 3), ("lo", ct.c_double * 3), ("hi", ct.c_double * 3)]


class _ReconParams(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("lam", ct.c_double), ("clamp_nonneg", ct.c_int32),
                ("alpha_l", ct.c_double), ("alpha_d", ct.c_double), ("tau", ct.c_double),
                ("g_sigma", ct.c_double), ("seed", ct.c_uint64), ("use_mask", ct.c_int32),
                ("flame_threshold", ct.c_double), ("use_hull", ct.c_int32),
                ("outside_value", ct.c_double), ("stop_tol", ct.c_double), ("subsets", ct.c_int32)]


class _TempParams(ct.Structure):
    _fields_ = [("t_min", ct.c_double), ("t_max", ct.c_double), ("t_norm", ct.c_double),
                ("band_nm", ct.c_double * 3), ("band_std_nm", ct.c_double),
                ("lut_size", ct.c_int32), ("sigma_max", ct.c_double), ("soot_t0", ct.c_double),
                ("soot_span", ct.c_double), ("channel", ct.c_int32), ("panels", ct.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build(sanitize=_LIB_PATH.endswith(".asan.so"))
        _lib = ct.CDLL(_LIB_PATH)
        P = ct.POINTER
        d, i32 = ct.c_double, ct.c_int32
        dp = P(ct.c_double)
        _lib.orc_ray_table.argtypes = [P(_Grid), P(_Camera), i32, d, dp, dp, P(ct.c_int32)]
        _lib.orc_render.argtypes = [P(_Grid), P(_Camera), i32, i32, d, d, d, dp, dp, i32, dp, i32, dp, dp]
        _lib.orc_inscatter.argtypes = [P(_Grid), i32, dp, dp, i32, i32, d, dp]
        _lib.orc_inscatter_phase.argtypes = [P(_Grid), P(_Camera), i32, i32, dp, dp, i32, i32, d, d, dp]
        _lib.orc_backproject_adjoint.argtypes = [P(_Grid), P(_Camera), i32, i32, d, dp, dp, dp]
        _lib.orc_backproject_paper.argtypes = [P(_Grid), P(_Camera), i32, i32, d, d, d, d, dp, dp]
        _lib.orc_reconstruct.argtypes = [P(_Grid), P(_Camera), i32, i32, d, d, d, i32, i32, d, d, dp,
                                         dp, dp, i32, i32, d, i32, d, d, d, dp]
        _lib.orc_render_grad.argtypes = [P(_Grid), P(_Camera), i32, i32, d, d, d, dp, dp, i32, dp,
                                         i32, dp, dp, dp]
        u32p = P(ct.c_uint32)
        _lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        _lib.orc_philox4x32_10.restype = None
        _lib.orc_sample_gain.argtypes = [ct.c_uint64, i32, i32, ct.c_int64, i32, d]
        _lib.orc_sample_gain.restype = d
        _lib.orc_flame_mask.argtypes = [dp, i32, i32, ct.c_long, d, dp]
        _lib.orc_flame_mask.restype = None
        _lib.orc_visual_hull.argtypes = [P(_Grid), P(_Camera), i32, d, dp, P(ct.c_int32)]
        _lib.orc_reconstruct_ext.argtypes = [P(_Grid), P(_Camera), i32, i32, d, d, d, i32, i32, d, d,
                                             dp, dp, dp, i32, P(_ReconParams), dp, P(ct.c_int32)]
        _lib.orc_planck.argtypes = [d, d]
        _lib.orc_planck.restype = d
        _lib.orc_band_radiance.argtypes = [d, d, d, i32]
        _lib.orc_band_radiance.restype = d
        _lib.orc_temp_lut.argtypes = [P(_TempParams), dp]
        _lib.orc_temp_map.argtypes = [P(_TempParams), dp, dp, ct.c_long, dp, dp]
        _lib.orc_temp_map.restype = None
        _lib.orc_temp_invert.argtypes = [P(_TempParams), dp, dp, ct.c_long, dp]
        _lib.orc_temp_invert.restype = None
        _lib.orc_temperature_fit.argtypes = [P(_Grid), P(_Camera), i32, d, P(_TempParams), dp, dp,
                                             dp, i32, d, dp]
        _lib.orc_num_threads.restype = ct.c_int
        _lib.orc_set_num_threads.argtypes = [i32]
        _lib.orc_set_num_threads.restype = None
        _lib.orc_suggest_grid.argtypes = [P(_Camera), i32, dp, dp, d, P(ct.c_int32), dp]
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def suggest_grid(rig, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), alpha=1.5):
    """Voxels per axis (x, y, z) and the projected edge spans n_max (pixels)
    for the box [lo, hi] seen by `rig` (Sec. 4.2)."""
    lo_a, hi_a = np.array(lo, dtype=np.float64), np.array(hi, dtype=np.float64)
    vox = (ct.c_int32 * 3)()
    nmax = np.zeros(3)
    _check(lib().orc_suggest_grid(_cams(rig), rig.n_views, _dp(lo_a), _dp(hi_a), float(alpha), vox,
                                  _dp(nmax)), "suggest_grid")
    return tuple(int(v) for v in vox), nmax


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(g):
    s = _Grid()
    s.n[:] = [g.nx, g.ny, g.nz]
    s.lo[:] = list(map(float, g.lo))
    s.hi[:] = list(map(float, g.hi))
    return s


def _cams(rig):
    arr = (_Camera * rig.n_views)()
    for v in range(rig.n_views):
        c = arr[v]
        c.fx, c.fy, c.cx, c.cy = (float(rig.fx[v]), float(rig.fy[v]), float(rig.cx[v]),
                                  float(rig.cy[v]))
        c.R[:] = [float(x) for x in np.asarray(rig.R[v]).reshape(9)]
        c.t[:] = [float(x) for x in np.asarray(rig.t[v]).reshape(3)]
        c.width, c.height = rig.width, rig.height
    return arr


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def ray_table(grid, rig, step_vox=0.5):
    V, H, W = rig.n_views, rig.height, rig.width
    tn = np.zeros((V, H, W))
    tf = np.zeros((V, H, W))
    K = np.zeros((V, H, W), dtype=np.int32)
    _check(lib().orc_ray_table(ct.byref(_grid(grid)), _cams(rig), V, float(step_vox), _dp(tn),
                               _dp(tf), K.ctypes.data_as(ct.POINTER(ct.c_int32))), "ray_table")
    return tn, tf, K


def _scatter_views(S, V):
    """0 for one in-scatter grid [C, M, M, M], 1 for one per view [V, C, M, M, M]."""
    if S is None or S.ndim == 4:
        return 0
    if S.ndim != 5 or S.shape[0] != V:
        raise ValueError(f"in-scatter grids of shape {S.shape} do not match {V} views")
    return 1


def render(grid, rig, emission, extinction, *, step_vox=0.5, albedo=0.0, background=0.0,
           inscatter=None, rowsum=False):
    """Images [V, C, H, W] (and row sums [V, H, W] when rowsum=True).
    inscatter: [C, M, M, M] (isotropic) or [V, C, M, M, M] (one grid per view)."""
    em = _f64(emission)
    C = em.shape[0]
    sig = _f64(extinction)
    V, H, W = rig.n_views, rig.height, rig.width
    img = np.zeros((V, C, H, W))
    rs = np.zeros((V, H, W)) if rowsum else None
    S = None if inscatter is None else _f64(inscatter)
    s_res = 0 if S is None else S.shape[-1]
    _check(lib().orc_render(ct.byref(_grid(grid)), _cams(rig), V, C, float(step_vox),
                            float(albedo), float(background), _dp(em), _dp(sig), s_res,
                            _dp(S) if S is not None else None, _scatter_views(S, V), _dp(img),
                            _dp(rs) if rs is not None else None), "render")
    return (img, rs) if rowsum else img


def render_grad(grid, rig, emission, extinction, dLdI, *, step_vox=0.5, albedo=0.0,
                background=0.0, inscatter=None):
    """Gradients (d_emission [C,nz,ny,nx], d_extinction [nz,ny,nx]) of a loss with
    dL/dI = dLdI through the render (in-scatter grid held fixed)."""
    em = _f64(emission)
    C = em.shape[0]
    S = None if inscatter is None else _f64(inscatter)
    s_res = 0 if S is None else S.shape[-1]
    d_em = np.zeros(em.shape)
    d_sig = np.zeros(em.shape[1:])
    _check(lib().orc_render_grad(ct.byref(_grid(grid)), _cams(rig), rig.n_views, C,
                                 float(step_vox), float(albedo), float(background), _dp(em),
                                 _dp(_f64(extinction)), s_res, _dp(S) if S is not None else None,
                                 _scatter_views(S, rig.n_views), _dp(_f64(dLdI)), _dp(d_em),
                                 _dp(d_sig)), "render_grad")
    return d_em, d_sig


def inscatter(grid, emission, extinction, *, s_res=32, n_dirs=32, s_step=0.5, phase_g=0.0, rig=None,
              per_view=False):
    """In-scatter grid [C, M, M, M] (phase_g = 0), or one grid per view of
    `rig` [V, C, M, M, M] for the Henyey-Greenstein phase function (phase_g != 0,
    or per_view=True)."""
    em = _f64(emission)
    C = em.shape[0]
    if phase_g != 0.0 or per_view:
        if rig is None:
            raise ValueError("an anisotropic phase function needs the camera rig")
        S = np.zeros((rig.n_views, C, s_res, s_res, s_res))
        _check(lib().orc_inscatter_phase(ct.byref(_grid(grid)), _cams(rig), rig.n_views, C, _dp(em),
                                         _dp(_f64(extinction)), s_res, n_dirs, float(s_step),
                                         float(phase_g), _dp(S)), "inscatter_phase")
        return S
    S = np.zeros((C, s_res, s_res, s_res))
    _check(lib().orc_inscatter(ct.byref(_grid(grid)), C, _dp(em), _dp(_f64(extinction)), s_res,
                               n_dirs, float(s_step), _dp(S)), "inscatter")
    return S


def backproject_adjoint(grid, rig, extinction, residual, *, step_vox=0.5):
    res = _f64(residual)
    C = res.shape[1]
    out = np.zeros((C,) + (grid.nz, grid.ny, grid.nx))
    _check(lib().orc_backproject_adjoint(ct.byref(_grid(grid)), _cams(rig), rig.n_views, C,
                                         float(step_vox), _dp(_f64(extinction)), _dp(res),
                                         _dp(out)), "backproject_adjoint")
    return out


def backproject_paper(grid, rig, residual, *, step_vox=0.5, alpha_l=1e-3, alpha_d=1.0, tau=0.05):
    res = _f64(residual)
    C = res.shape[1]
    out = np.zeros((C,) + (grid.nz, grid.ny, grid.nx))
    _check(lib().orc_backproject_paper(ct.byref(_grid(grid)), _cams(rig), rig.n_views, C,
                                       float(step_vox), float(alpha_l), float(alpha_d),
                                       float(tau), _dp(res), _dp(out)), "backproject_paper")
    return out


def reconstruct(grid, rig, frames, extinction, emission0, iters, *, step_vox=0.5, albedo=0.0,
                background=0.0, s_res=32, n_dirs=32, s_step=0.5, phase_g=0.0, mode="sart", lam=1.0,
                clamp_nonneg=True, alpha_l=1e-3, alpha_d=1.0, tau=0.05, return_residuals=False):
    F = _f64(frames)
    em = np.array(emission0, dtype=np.float64, order="C", copy=True)
    C = em.shape[0]
    res = np.zeros(max(iters, 1))
    _check(lib().orc_reconstruct(ct.byref(_grid(grid)), _cams(rig), rig.n_views, C,
                                 float(step_vox), float(albedo), float(background), int(s_res),
                                 int(n_dirs), float(s_step), float(phase_g), _dp(F), _dp(_f64(extinction)),
                                 _dp(em), int(iters), {"sart": 0, "paper": 1, "mlem": 2}[mode], float(lam),
                                 1 if clamp_nonneg else 0, float(alpha_l), float(alpha_d),
                                 float(tau), _dp(res)), "reconstruct")
    return (em, res[:iters]) if return_residuals else em


def planck(lam_m, T):
    return float(lib().orc_planck(float(lam_m), float(T)))


def band_radiance(T, mu_nm, std_nm, panels=4000):
    return float(lib().orc_band_radiance(float(T), float(mu_nm), float(std_nm), int(panels)))


class TempParams:
    """Colour-temperature mapping parameters (defaults: the temperature workload)."""

    def __init__(self, t_min=800.0, t_max=2300.0, t_norm=2200.0, band_nm=(650.0, 550.0, 450.0),
                 band_std_nm=40.0, lut_size=4096, sigma_max=4.0, soot_t0=800.0, soot_span=1400.0,
                 channel=1, panels=4000):
        self.t_min, self.t_max, self.t_norm = t_min, t_max, t_norm
        self.band_nm = tuple(band_nm)
        self.band_std_nm = band_std_nm
        self.lut_size = lut_size
        self.sigma_max, self.soot_t0, self.soot_span = sigma_max, soot_t0, soot_span
        self.channel, self.panels = channel, panels

    def c(self):
        s = _TempParams()
        s.t_min, s.t_max, s.t_norm = self.t_min, self.t_max, self.t_norm
        s.band_nm[:] = list(self.band_nm)
        s.band_std_nm = self.band_std_nm
        s.lut_size = self.lut_size
        s.sigma_max, s.soot_t0, s.soot_span = self.sigma_max, self.soot_t0, self.soot_span
        s.channel, s.panels = self.channel, self.panels
        return s


def temp_lut(tp: TempParams):
    lut = np.zeros((3, tp.lut_size))
    _check(lib().orc_temp_lut(ct.byref(tp.c()), _dp(lut)), "temp_lut")
    return lut


def temp_map(tp: TempParams, lut, T):
    T = _f64(T)
    n = T.size
    em = np.zeros((3,) + T.shape)
    sig = np.zeros(T.shape)
    lib().orc_temp_map(ct.byref(tp.c()), _dp(_f64(lut)), _dp(T), n, _dp(em), _dp(sig))
    return em, sig


def temp_invert(tp: TempParams, lut, e):
    e = _f64(e)
    T = np.zeros(e.shape)
    lib().orc_temp_invert(ct.byref(tp.c()), _dp(_f64(lut)), _dp(e), e.size, _dp(T))
    return T


def temperature_fit(grid, rig, tp: TempParams, lut, frames, T0, iters, *, step_vox=0.5, lam=1.0,
                    return_residuals=False):
    T = np.array(T0, dtype=np.float64, order="C", copy=True)
    res = np.zeros(max(iters, 1))
    _check(lib().orc_temperature_fit(ct.byref(_grid(grid)), _cams(rig), rig.n_views,
                                     float(step_vox), ct.byref(tp.c()), _dp(_f64(lut)),
                                     _dp(_f64(frames)), _dp(T), int(iters), float(lam), _dp(res)),
           "temperature_fit")
    return (T, res[:iters]) if return_residuals else T


def philox4x32_10(ctr, key):
    c = (ct.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ct.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ct.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def sample_gain(seed, it, view, pixel, k, g_sigma):
    return float(lib().orc_sample_gain(int(seed), int(it), int(view), int(pixel), int(k),
                                       float(g_sigma)))


def flame_mask(frames, threshold):
    F = _f64(frames)
    V, C, H, W = F.shape
    m = np.zeros((V, H, W))
    lib().orc_flame_mask(_dp(F), V, C, H * W, float(threshold), _dp(m))
    return m


def visual_hull(grid, rig, mask, *, step_vox=0.5):
    inside = np.zeros(grid.shape_zyx, dtype=np.int32)
    _check(lib().orc_visual_hull(ct.byref(_grid(grid)), _cams(rig), rig.n_views, float(step_vox),
                                 _dp(_f64(mask)), inside.ctypes.data_as(ct.POINTER(ct.c_int32))),
           "visual_hull")
    return inside.astype(bool)


def reconstruct_ext(grid, rig, frames, extinction, emission0, iters, *, step_vox=0.5, albedo=0.0,
                    background=0.0, s_res=32, n_dirs=32, s_step=0.5, phase_g=0.0, mode="sart", lam=1.0,
                    clamp_nonneg=True, alpha_l=1e-3, alpha_d=1.0, tau=0.05, g_sigma=0.0, seed=0,
                    flame_threshold=None, hull=False, outside_value=0.0, stop_tol=0.0, subsets=1):
    """Reconstruction with the paper's variants (flame mask, visual hull, gains
    G(s), stop rule) and ordered subsets of views. Returns (emission,
    per-iteration image RMS, updates made); with subsets > 1 the RMS is not
    computed (zeros) and the update count is in iterations."""
    F = _f64(frames)
    em = np.array(emission0, dtype=np.float64, order="C", copy=True)
    rp = _ReconParams()
    rp.mode = {"sart": 0, "paper": 1, "mlem": 2}[mode]
    rp.lam, rp.clamp_nonneg = float(lam), 1 if clamp_nonneg else 0
    rp.alpha_l, rp.alpha_d, rp.tau = float(alpha_l), float(alpha_d), float(tau)
    rp.g_sigma, rp.seed = float(g_sigma), int(seed)
    rp.use_mask = 0 if flame_threshold is None else 1
    rp.flame_threshold = 0.0 if flame_threshold is None else float(flame_threshold)
    rp.use_hull, rp.outside_value, rp.stop_tol = 1 if hull else 0, float(outside_value), float(stop_tol)
    rp.subsets = int(subsets)
    res = np.zeros(max(iters, 1))
    done = ct.c_int32()
    _check(lib().orc_reconstruct_ext(ct.byref(_grid(grid)), _cams(rig), rig.n_views, em.shape[0],
                                     float(step_vox), float(albedo), float(background), int(s_res),
                                     int(n_dirs), float(s_step), float(phase_g), _dp(F),
                                     _dp(_f64(extinction)), _dp(em), int(iters), ct.byref(rp), _dp(res),
                                     ct.byref(done)),
           "reconstruct_ext")
    return em, res[:iters], int(done.value)
