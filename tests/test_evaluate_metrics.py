"""Host-side metrics of the evaluation protocols (Sec. 5.1): flame bounding
rectangle, per-channel pixel RMSE on a [0, 255] scale, volume RMSE inside the
hull; checked on hand-made arrays."""
import numpy as np

from paper_1809_06417_amd import evaluate


def test_flame_box_is_the_tight_rectangle_and_whole_image_without_flame():
    F = np.zeros((2, 3, 7, 9))
    F[0, 2, 2, 3] = 1.0
    F[0, 0, 5, 6] = 0.5
    boxes = evaluate.flame_boxes(F, 0.1)
    assert boxes[0] == (2, 6, 3, 7)
    assert boxes[1] == (0, 7, 0, 9)


def test_image_rmse_inside_the_box_only():
    F = np.zeros((1, 2, 4, 4))
    I = np.zeros_like(F)
    I[0, 0, 1, 1] = 2.0          # inside the box
    I[0, 1, 3, 3] = 100.0        # outside: ignored
    err = evaluate.image_rmse(I, F, [(0, 2, 0, 2)], scale=10.0)
    np.testing.assert_allclose(err, [[10.0 * np.sqrt(4.0 / 4), 0.0]])


def test_volume_rmse_over_hull_key_points():
    truth = np.zeros((1, 2, 2, 2))
    vol = np.full_like(truth, 3.0)
    inside = np.zeros((2, 2, 2), dtype=np.int32)
    inside[0, 0, 0] = inside[1, 1, 1] = 1
    vol[0, 1, 0, 0] = 50.0       # outside the hull
    np.testing.assert_allclose(evaluate.volume_rmse(vol, truth, inside, 2.0), [6.0])
    assert evaluate.volume_rmse(vol, truth, np.zeros_like(inside), 1.0)[0] == 0.0
