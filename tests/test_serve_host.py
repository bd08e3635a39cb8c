"""Host-side checks of the serving loop's admission arithmetic (no GPU): the
bytes a job holds on the device while in flight and the smallest HBM budget
that admits every job (the largest plan workspace, every video's resident
volume and the largest job's inputs)."""
import types

import numpy as np

from paper_1809_06417_amd import serve


class FakeTensor:
    def __init__(self, *shape):
        self.shape = shape

    def numel(self):
        return int(np.prod(self.shape))


def video(plan_bytes, n, channels=3):
    v = serve.VideoState.__new__(serve.VideoState)
    v.plan_bytes = plan_bytes
    v.volume_bytes = 4 * channels * n ** 3
    return v


def test_job_input_bytes_are_frames_and_extinction():
    j = serve.Job(0, 0, 0, 0.0, FakeTensor(4, 3, 64, 48), FakeTensor(20, 20, 20))
    assert j.input_bytes() == 4 * (4 * 3 * 64 * 48 + 20 ** 3)


def test_min_budget_counts_largest_plan_all_volumes_largest_inputs():
    videos = {0: video(1000, 10), 1: video(5000, 20), 2: video(3000, 15)}
    jobs = [serve.Job(0, 0, 0, 0.0, FakeTensor(2, 3, 8, 8), FakeTensor(10, 10, 10)),
            serve.Job(1, 1, 0, 0.1, FakeTensor(4, 3, 16, 16), FakeTensor(20, 20, 20)),
            serve.Job(2, 2, 0, 0.2, FakeTensor(3, 3, 12, 12), FakeTensor(15, 15, 15))]
    expect = 5000 + 4 * 3 * (10 ** 3 + 20 ** 3 + 15 ** 3) + max(j.input_bytes() for j in jobs)
    assert serve.min_budget(videos, jobs) == expect


def test_latency_summary():
    jobs = [types.SimpleNamespace(arrival=0.1 * i, done=0.1 * i + 0.05 * (i + 1)) for i in range(10)]
    s = serve.latency_summary(jobs)
    lat = np.array([0.05 * (i + 1) for i in range(10)])
    assert s["jobs"] == 10
    assert abs(s["p50_ms"] - np.percentile(lat, 50) * 1e3) < 1e-9
    assert abs(s["p99_ms"] - np.percentile(lat, 99) * 1e3) < 1e-9
    assert abs(s["span_s"] - (0.9 + 0.5 - 0.0)) < 1e-12
    assert abs(s["frames_per_s"] - 10 / 1.4) < 1e-9
