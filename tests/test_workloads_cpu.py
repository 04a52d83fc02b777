"""Host checks of the seeded input generators (no solver arithmetic)."""
import numpy as np
import torch

from paper_1804_09666_amd import workloads as wl


def test_interleaved_sweep_lines_bitwise_equal():
    """The interleaved-layout generator (used to build large batches directly
    in device memory) reproduces sweep_lines bit for bit, on numpy and on
    torch tensors, for both boundary orders."""
    v = wl.smooth_lines(37, 1001, 5)
    vt = np.ascontiguousarray(v.T)
    for order in (1, 2):
        ref = wl.sweep_lines(v, 4.0, order)
        for got in (wl.sweep_lines_interleaved(vt, 4.0, order),
                    {k: t.numpy() for k, t in
                     wl.sweep_lines_interleaved(torch.from_numpy(vt), 4.0, order).items()}):
            for k in ref:
                assert np.array_equal(ref[k], np.ascontiguousarray(got[k].T)), (order, k)


def test_config_shapes_and_seeds():
    pd, td, u0 = wl.config1(N=64, seed=3)
    assert pd["d"].shape == (64, 64) and td["d"].shape == (64, 64)
    assert np.abs(u0).max() == 1.0
    # second-order boundary rows are not diagonally dominant, interior rows are
    assert pd["d"][0, 0] == -3.0 and pd["a"][0, 0] == 4.0 and pd["b"][0, 0] == -1.0
    assert (np.abs(pd["d"][:, 1:-1]) >= np.abs(pd["c"][:, 1:-1]) + np.abs(pd["a"][:, 1:-1])).all()
    sizes = wl.config2_sizes(count=1000)
    assert sizes.min() >= 64 and sizes.max() <= 65536
    a = wl.config3(nsys=4, n=100)
    b = wl.config3(nsys=4, n=100)
    assert all(np.array_equal(a[k], b[k]) for k in a)
