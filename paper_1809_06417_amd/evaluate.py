"""Evaluation protocols of the paper on synthetic volumes (Sec. 5).

* Leave-one-view-out (the extra evaluation of Sec. 5.1): reconstruct from all
  views but one, render every view of the result, and report the pixel
  intensity error on the input views and on the held-out test view.
* Camera-count sweep (Sec. 5.2, temperature): reconstruct the temperature
  field with 4, 16, 28 ... ring cameras and report the image and temperature
  errors per count.

Errors follow the paper's definitions: pixel intensity error = RMSE per
channel over a bounding rectangle that holds the whole flame, on a [0, 255]
scale; volume (or temperature) error = RMSE over the key points inside the
visual hull. The rendering, reconstruction, flame mask and hull all run in
the HIP library; the metrics are plain host arithmetic on copied results.
"""
from __future__ import annotations

import time

import numpy as np

from . import rte

__all__ = ["flame_boxes", "image_rmse", "volume_rmse", "leave_one_view_out", "camera_sweep"]


def flame_boxes(frames, threshold):
    """Per view, the smallest pixel rectangle (v0, v1, u0, u1), half-open, that
    holds every pixel with a channel above `threshold`; the whole image when
    the view shows no flame. frames: host array [V, C, H, W]."""
    V, _, H, W = frames.shape
    boxes = []
    for v in range(V):
        hot = (frames[v] > threshold).any(axis=0)
        rows, cols = np.flatnonzero(hot.any(axis=1)), np.flatnonzero(hot.any(axis=0))
        if rows.size == 0:
            boxes.append((0, H, 0, W))
        else:
            boxes.append((int(rows[0]), int(rows[-1]) + 1, int(cols[0]), int(cols[-1]) + 1))
    return boxes


def image_rmse(images, frames, boxes, scale):
    """RMSE per view and channel inside each view's box, times `scale`
    (host arrays [V, C, H, W]; returns [V, C])."""
    V, C = frames.shape[:2]
    out = np.zeros((V, C))
    for v, (v0, v1, u0, u1) in enumerate(boxes):
        d = images[v, :, v0:v1, u0:u1].astype(np.float64) - frames[v, :, v0:v1, u0:u1]
        out[v] = np.sqrt((d * d).reshape(C, -1).mean(axis=1)) * scale
    return out


def volume_rmse(volume, truth, inside, scale):
    """RMSE per channel over the key points with inside != 0, times `scale`
    (host arrays [C, nz, ny, nx] and [nz, ny, nx]; returns [C])."""
    m = inside.astype(bool)
    if not m.any():
        return np.zeros(volume.shape[0])
    d = volume[:, m].astype(np.float64) - truth[:, m]
    return np.sqrt((d * d).mean(axis=1)) * scale


def _host(t):
    return t.detach().cpu().numpy()


def leave_one_view_out(grid, rig, emission, extinction, test_view, iters, *, step_vox=0.5, albedo=0.0,
                       background=0.0, scatter_res=0, scatter_dirs=32, phase_g=0.0, update="sart",
                       flame_frac=0.01, timing=False):
    """Frames of every view are rendered from the true (emission, extinction)
    (device tensors); the emission is reconstructed from zero with the views
    other than `test_view` at the known extinction; every view is rendered
    from the result. Returns a dict with per-channel errors: 'input' (mean
    over the input views), 'test', 'volume' (inside the visual hull of the
    input views' flame masks), plus the seconds spent reconstructing, the
    march samples and hit rays per iteration and (timing=True) per-kernel
    (ms, launches)
    of the reconstruction."""
    import torch
    C = emission.shape[0]
    kw = dict(channels=C, step_vox=step_vox, albedo=albedo, background=background,
              scatter_res=scatter_res, scatter_dirs=scatter_dirs, phase_g=phase_g)
    inputs = [v for v in range(rig.n_views) if v != test_view]
    with rte.Plan(grid, rig, **kw) as full, rte.Plan(grid, rig.subset(inputs), **kw) as sub:
        S = full.inscatter(emission, extinction) if albedo > 0 else None
        F = full.render(emission, extinction, S)
        Fin = F[inputs].contiguous()
        thr = flame_frac * float(F.max())
        x = torch.zeros_like(emission)
        sub.set_timing(timing)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sub.reconstruct(Fin, extinction, x, iters, update=update)
        torch.cuda.synchronize()
        seconds = time.perf_counter() - t0
        kernels = {k: sub.kernel_time(k) for k in rte.KERNELS} if timing else {}
        sub.set_timing(False)
        samples, hit_rays = sub.samples, sub.hit_rays
        Sx = full.inscatter(x, extinction) if albedo > 0 else None
        I = full.render(x, extinction, Sx)
        inside = sub.visual_hull(sub.flame_mask(Fin, thr))
        Fh, Ih, xh = _host(F), _host(I), _host(x)
        em_h, inside_h = _host(emission), _host(inside)
    scale = 255.0 / max(float(Fh.max()), 1e-30)
    err = image_rmse(Ih, Fh, flame_boxes(Fh, thr), scale)
    return {"input": err[inputs].mean(axis=0), "test": err[test_view],
            "volume": volume_rmse(xh, em_h, inside_h, 255.0 / max(float(em_h.max()), 1e-30)),
            "reconstruct_s": seconds, "iters": iters, "test_view": test_view, "samples_per_iter": samples,
            "hit_rays": hit_rays, "kernels": kernels}


def camera_sweep(grid, temperature, rigs, iters, *, temp=None, flame_frac=0.01, observable=1e-3):
    """Temperature reconstruction (green-band fit from t_min) with each camera
    rig of `rigs` (e.g. rings of 4, 16, 28 cameras). Per rig: the RGB pixel
    intensity error of the renders of the reconstructed field against the
    frames, and the temperature RMSE (K) over key points inside the visual
    hull whose true green emission is at least `observable` of its maximum
    (below that the colour does not determine T in FP32). temperature: device
    tensor [nz, ny, nx] in K."""
    import torch
    temp = temp or rte.TempParams()
    out = []
    for rig in rigs:
        n = rig.n_views
        with rte.Plan(grid, rig, channels=1) as p:
            em3, sg = p.temperature_map(temperature, temp)
            F = torch.stack([p.render(em3[c:c + 1].contiguous(), sg)[:, 0] for c in range(3)], dim=1)
            T = torch.full_like(temperature, float(temp.t_min))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.reconstruct_temperature(F.contiguous(), T, iters, temp)
            torch.cuda.synchronize()
            seconds = time.perf_counter() - t0
            e3, s3 = p.temperature_map(T, temp)
            I = torch.stack([p.render(e3[c:c + 1].contiguous(), s3)[:, 0] for c in range(3)], dim=1)
            thr = flame_frac * float(F.max())
            inside = p.visual_hull(p.flame_mask(F[:, 1:2].contiguous(), thr))
            samples = p.samples
            Fh, Ih = _host(F), _host(I)
            Th, Tg, inside_h, eg = _host(T), _host(temperature), _host(inside), _host(em3[1])
        err = image_rmse(Ih, Fh, flame_boxes(Fh, thr), 255.0 / max(float(Fh.max()), 1e-30))
        mask = inside_h.astype(bool) & (eg >= observable * eg.max())
        t_rmse = float(np.sqrt(((Th - Tg)[mask] ** 2).mean())) if mask.any() else 0.0
        out.append({"cameras": n, "image": err.mean(axis=0), "temperature_K": t_rmse,
                    "voxels": int(mask.sum()), "reconstruct_s": seconds, "samples_per_iter": samples})
    return out
