"""Host logic of the serving loop (no GPU): queue arithmetic, shape classes, request sizing."""
import numpy as np

from paper_2607_12201_amd import colloc, serving, workloads


def test_fifo_latencies_closed_form():
    lat = serving.fifo_latencies([0.0, 0.1, 0.15], [0.2, 0.2, 0.05])
    assert np.allclose(lat, [0.2, 0.3, 0.3])


def test_request_bytes_grow_with_mesh_and_precision_keeps_fallback_room():
    a = workloads.random_network(1, n_s=4, n_r=8, N=50, n_obs=1, n_times=50)
    b = workloads.random_network(1, n_s=4, n_r=8, N=100, n_obs=1, n_times=50)
    assert serving.request_bytes(b, 3, colloc.FP64) > serving.request_bytes(a, 3, colloc.FP64)
    assert serving.request_bytes(a, 3, colloc.FP32_IR) == serving.request_bytes(a, 3, colloc.FP64)
    assert serving.shape_class(a, 3) == serving.shape_class(b, 3) == (4, 8, 8, 3)


def test_batch_bytes_cover_the_padded_batch():
    """A batch is sized by its longest mesh (per-chunk partials), so admission must use the
    batch's own size, not the sum of the members' sizes alone."""
    a = workloads.random_network(1, n_s=4, n_r=8, N=50, n_obs=1, n_times=50)
    b = workloads.random_network(1, n_s=4, n_r=8, N=400, n_obs=1, n_times=50)
    ab = serving.batch_bytes([a, b], 3, colloc.FP64)
    assert ab >= serving.request_bytes(b, 3, colloc.FP64)
    assert ab >= serving.request_bytes(a, 3, colloc.FP64)
    assert serving.batch_bytes([a], 3, colloc.FP64) == serving.request_bytes(a, 3, colloc.FP64)
