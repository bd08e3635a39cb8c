"""Helpers for the GPU parity tests: FP32 inputs shared by both sides,
device/host transfers and the comparison metrics with their tolerances."""
import sys

import numpy as np

# Tolerances (floating point, FP32 GPU vs FP64 oracle):
RENDER_REL = 1e-4   # max |I_gpu - I_orc| / max |I_orc|, per view and channel
VOLUME_RMS = 1e-3   # RMS(V_gpu - V_orc) / max |V_orc| after fixed iterations
BACKPROJ_REL = 1e-4  # max |d_gpu - d_orc| / max |d_orc| for one back-projection


def f32(a):
    """Round an input to FP32 once; both sides consume exactly these values."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def as64(a):
    return np.asarray(a, dtype=np.float64)


def dev(a):
    import torch
    return torch.tensor(f32(a), device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def say(*msg):
    """Name the case before any GPU step (flushed so it survives a crash)."""
    print("[gpu-case]", *msg, flush=True)
    sys.stdout.flush()


def render_rel(gpu, orc):
    """Worst per-(view, channel) max-abs error relative to that image's max."""
    worst = 0.0
    for v in range(orc.shape[0]):
        for c in range(orc.shape[1]):
            scale = np.abs(orc[v, c]).max()
            if scale == 0:
                worst = max(worst, np.abs(gpu[v, c]).max())
            else:
                worst = max(worst, np.abs(gpu[v, c] - orc[v, c]).max() / scale)
    return worst


def rel_max(gpu, orc):
    scale = np.abs(orc).max()
    return np.abs(gpu - orc).max() / (scale if scale > 0 else 1.0)


def rel_rms(gpu, orc):
    scale = np.abs(orc).max()
    return np.sqrt(np.mean((gpu - orc) ** 2)) / (scale if scale > 0 else 1.0)
