"""Host checks of the seeded input generators (no solver arithmetic) and of the
host-side planning of uneven batches."""
import numpy as np
import pytest
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


def test_uneven_batch_layout_host():
    """Planning of an uneven batch (host only): groups of 16 sorted by length,
    disjoint row positions, tile counts per compiled shape, rejection of
    systems shorter than 8 rows."""
    from paper_1804_09666_amd import bandsolve as bs
    rng = np.random.default_rng(1)
    n = np.floor(np.exp(rng.uniform(np.log(8), np.log(5000), 101))).astype(np.int64)
    plan = bs.Varlen(n, device="cpu")
    assert plan.info.groups == 7 and plan.slots == 112
    order = np.argsort(plan.slot)
    assert (np.diff(n[order]) <= 0).all()                       # longest first
    pos = np.concatenate([plan.offset[i] + 16 * np.arange(n[i]) for i in range(n.size)])
    assert np.unique(pos).size == pos.size and pos.max() < plan.elems
    gn = [n[order[16 * g]] for g in range(plan.info.groups)]
    assert plan.elems == 16 * sum(gn)
    for v, (M, PW) in enumerate(plan.variants()):
        assert plan.info.tiles[v] == sum(-(-x // (M * PW)) for x in gn)
    with pytest.raises(bs.BandSolveError):
        bs.Varlen(np.array([100, 7]), device="cpu")


def test_uneven_batch_generator_structure():
    """The device generator of uneven batches, run on the CPU: nothing outside
    a matrix, strict diagonal dominance, and y = A x_true row by row (dense
    products of each extracted system)."""
    import torch
    from paper_1804_09666_amd import workloads as wl
    sizes = [40, 9, 0, 23] + [0] * 12 + [12, 12, 12, 8] + [0] * 12
    t = {k: v.numpy() for k, v in wl.dominant_groups(sizes, seed=5, device="cpu").items()}
    gn = [max(sizes[16 * g:16 * g + 16]) for g in range(2)]
    goff = [0, 16 * gn[0]]
    assert t["d"].size == 16 * sum(gn)
    covered = np.zeros(t["d"].size, bool)
    for slot, m in enumerate(sizes):
        if m == 0:
            continue
        g, lane = divmod(slot, 16)
        idx = goff[g] + lane + 16 * np.arange(m)
        covered[idx] = True
        A = np.zeros((m, m))
        for off, k in ((-2, "e"), (-1, "c"), (0, "d"), (1, "a"), (2, "b")):
            v = t[k][idx]
            rows = np.arange(max(0, -off), min(m, m - off))
            assert not v[np.setdiff1d(np.arange(m), rows)].any()   # slots outside the matrix are 0
            A[rows, rows + off] = v[rows]
        off_sum = np.abs(A).sum(1) - np.abs(np.diag(A))
        assert (np.diag(A) >= off_sum + 1.0).all()
        assert np.allclose(A @ t["x_true"][idx], t["y"][idx], rtol=0, atol=1e-13)
    for k in ("e", "c", "d", "a", "b", "y", "x_true"):
        assert not t[k][~covered].any()                              # padding holds 0
