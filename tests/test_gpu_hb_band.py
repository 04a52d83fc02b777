"""GPU parity of the explicit banded Hotelling-Bodewig inverses of the ILU(0)
factors (Remark of Sec. 2; Appendix, the matrix form of the HB recursion)
against the oracle's recursion on dense n x n matrices: every band entry
bitwise, every slot outside the matrix exactly zero."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, say, to_device

pytestmark = pytest.mark.gpu


def dense_factors(ws, j, kind):
    """Dense L and U of system j from the oracle's band ILU(0)."""
    e, b = (ws["e"][j], ws["b"][j]) if kind == 5 else (0 * ws["d"][j], 0 * ws["d"][j])
    l2, l1, u0, u1, info = oracle.ilu0_band(e, ws["c"][j], ws["d"][j], ws["a"][j], b)
    assert info == 0
    n = u0.shape[0]
    L = np.eye(n) + np.diag(l1[1:], -1) + np.diag(l2[2:], -2)
    U = np.diag(u0) + np.diag(u1[:-1], 1) + np.diag(b[:-2], 2)
    return L, U


def expected_planes(X, K, lower):
    """Dense X -> planes [K + 1, n]: plane d holds X[i, i - d] (lower) or
    X[i, i + d] (upper), 0 outside the matrix."""
    n = X.shape[0]
    P = np.zeros((K + 1, n))
    for d in range(K + 1):
        for i in range(n):
            k = i - d if lower else i + d
            if 0 <= k < n:
                P[d, i] = X[i, k]
    return P


def check(ws, kind, batch, sL, sU, ld=None, systems=None):
    n = ws["d"].shape[1]
    t = to_device(ws, batch, ld=ld)
    f, info = bs.factor(diags_of(t, kind), kind=kind, batch=batch)
    assert int(info.abs().sum()) == 0
    say(f"hb_inverse_band kind={kind} n={n} batch={batch} ld={t['d'].shape[1]} s=({sL},{sU})")
    XL, XU = bs.hb_inverse(diags_of(t, kind), f, s_L=sL, s_U=sU, kind=kind, batch=batch)
    torch.cuda.synchronize()
    KL, KU = bs.hb_band_width(kind, sL, n), bs.hb_band_width(kind, sU, n)
    assert XL.shape[0] == KL + 1 and XU.shape[0] == KU + 1
    gl = XL[:, :, :batch].cpu().numpy()
    gu = XU[:, :, :batch].cpu().numpy()
    for j in (range(batch) if systems is None else systems):
        L, U = dense_factors(ws, j, kind)
        xl, xu = oracle.hb_matrix(L, sL), oracle.hb_matrix(U, sU)
        # the band claim: nothing of the dense iterate lies outside width K
        assert not np.triu(xl, 1).any() and not np.tril(xl, -KL - 1).any()
        assert not np.tril(xu, -1).any() and not np.triu(xu, KU + 1).any()
        for got, want in ((gl[:, :, j], expected_planes(xl, KL, True)),
                          (gu[:, :, j], expected_planes(xu, KU, False))):
            bad = got.view(np.int64) != want.view(np.int64)
            assert not bad.any(), (j, np.argwhere(bad)[:4], got[bad][:4], want[bad][:4])


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("sL,sU", [(0, 0), (1, 2), (3, 3), (5, 6)])
def test_band_entries_bitwise(kind, sL, sU):
    ws = wl.dominant_batch(37, 48, kind=kind, seed=wl.BASE_SEED + 60 + sL)
    check(ws, kind, 37, sL, sU, ld=64)


@pytest.mark.parametrize("kind", [5, 3])
def test_nilpotent_cap_is_the_inverse(kind):
    """2^s >= n: the band fills the triangle and X_s is T^{-1} (G nilpotent)."""
    n, batch = 12, 5
    ws = wl.dominant_batch(batch, n, kind=kind, seed=wl.BASE_SEED + 70)
    check(ws, kind, batch, 4, 5)
    t = to_device(ws, batch)
    f, _ = bs.factor(diags_of(t, kind), kind=kind, batch=batch)
    XL, XU = bs.hb_inverse(diags_of(t, kind), f, s_L=4, s_U=5, kind=kind, batch=batch)
    assert XL.shape[0] == n and XU.shape[0] == n
    for j in range(batch):
        L, U = dense_factors(ws, j, kind)
        got = np.zeros((n, n))
        for d in range(n):
            for i in range(d, n):
                got[i, i - d] = XL[d, i, j].item()
        assert np.abs(got - np.linalg.inv(L)).max() <= 1e-12 * np.abs(np.linalg.inv(L)).max()


def test_one_factor_only_and_sampled_larger_batch():
    ws = wl.dominant_batch(700, 160, kind=5, seed=wl.BASE_SEED + 71)
    t = to_device(ws, 700)
    f, _ = bs.factor(diags_of(t), batch=700)
    XL, XU = bs.hb_inverse(diags_of(t), f, s_L=3, batch=700)
    assert XU is None and XL.shape == (15, 160, t["d"].shape[1])
    _, XU2 = bs.hb_inverse(diags_of(t), f, s_U=2, batch=700)
    XLj, XUj = bs.hb_inverse(diags_of(t), f, s_L=3, s_U=2, batch=700)
    torch.cuda.synchronize()
    assert torch.equal(XL.view(torch.int64), XLj.view(torch.int64))
    assert torch.equal(XU2.view(torch.int64), XUj.view(torch.int64))
    check(ws, 5, 700, 3, 2, systems=(0, 1, 345, 699))


def test_rejections():
    ws = wl.dominant_batch(4, 16, kind=5, seed=wl.BASE_SEED + 72)
    t = to_device(ws, 4)
    f, _ = bs.factor(diags_of(t), batch=4)
    with pytest.raises(bs.BandSolveError):
        bs.hb_inverse(diags_of(t), f, s_L=31, batch=4)
    small = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(bs.BandSolveError) as ei:
        bs.hb_inverse(diags_of(t), f, s_L=2, s_U=2, batch=4, workspace=small)
    assert ei.value.status == bs.BS_EWORKSPACE


def test_every_slot_written_into_given_outputs():
    """Outputs passed in (filled with NaN) come back with every slot of the
    live systems written: band entries, and zeros outside the matrix."""
    batch, n = 50, 40
    ws = wl.dominant_batch(batch, n, kind=5, seed=wl.BASE_SEED + 73)
    t = to_device(ws, batch, ld=64)
    f, _ = bs.factor(diags_of(t), batch=batch)
    ref = bs.hb_inverse(diags_of(t), f, s_L=4, s_U=3, batch=batch)
    outs = [torch.full_like(r, float("nan")) for r in ref]
    got = bs.hb_inverse(diags_of(t), f, s_L=4, s_U=3, batch=batch, out=outs)
    torch.cuda.synchronize()
    for g, r in zip(got, ref):
        assert torch.equal(g[:, :, :batch].contiguous().view(torch.int64),
                           r[:, :, :batch].contiguous().view(torch.int64))
        assert torch.isnan(g[:, :, batch:]).all()     # padding columns untouched


@pytest.mark.parametrize("kind", [5, 3])
def test_full_sweep_batch_sampled_against_vector_form(kind):
    """The 2048 x 2048 ADI sweep batch at s = (5, 6), as bench.py times it
    (pentadiagonal; and the tridiagonal sweep): for sampled systems, X_s v
    from the GPU's band planes equals the oracle's vector form of the same HB
    iterate (2^s - 1 sweeps) to rounding."""
    pd5, td, _ = wl.config1()
    pd = pd5 if kind == 5 else {**td, "e": 0 * td["d"], "b": 0 * td["d"]}
    n = batch = 2048
    t = to_device(pd, batch)
    f, info = bs.factor(diags_of(t, kind), kind=kind, batch=batch)
    assert int(info.abs().sum()) == 0
    say(f"hb_inverse_band full sweep batch kind={kind} s=(5,6)")
    XL, XU = bs.hb_inverse(diags_of(t, kind), f, s_L=5, s_U=6, kind=kind, batch=batch)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for j in (0, 1, 1023, 2047):
        l2, l1, u0, u1, finfo = oracle.ilu0_band(pd["e"][j], pd["c"][j], pd["d"][j], pd["a"][j],
                                                 pd["b"][j])
        assert finfo == 0
        v = rng.uniform(-1.0, 1.0, n)
        xl, xu = XL[:, :, j].cpu().numpy(), XU[:, :, j].cpu().numpy()
        yl, yu = np.zeros(n), np.zeros(n)
        for d in range(xl.shape[0]):
            yl[d:] += xl[d, d:] * v[:n - d]
        for d in range(xu.shape[0]):
            yu[:n - d] += xu[d, :n - d] * v[d:]
        rl = oracle.hb_lower_apply(l2, l1, 5, v)
        ru = oracle.hb_upper_apply(u0, u1, pd["b"][j], 6, v)
        assert np.abs(yl - rl).max() <= 1e-12 * np.abs(rl).max(), j
        assert np.abs(yu - ru).max() <= 1e-12 * np.abs(ru).max(), j


@pytest.mark.parametrize("kind", [5, 3])
def test_many_tiles_and_chunks_bitwise(kind):
    """n = 300 (19 row tiles of 16, the last ragged), s = (5, 6): bands up to
    126 wide, so the product steps take up to 8 distance chunks and both step
    forms run (M in registers below band 16, M through the workspace above);
    sampled systems of a ragged batch bitwise against the dense recursion."""
    ws = wl.dominant_batch(70, 300, kind=kind, seed=wl.BASE_SEED + 74)
    check(ws, kind, 70, 5, 6, ld=96, systems=(0, 33, 69))


def test_graph_replays_match_eager():
    """hb_inverse_band enqueues kernels only (no host synchronisation, no
    memset), so it can be captured in a HIP graph; every replay, with eager
    work and synchronisation between replays, equals the eager call bitwise."""
    batch, n = 40, 64
    ws = wl.dominant_batch(batch, n, kind=5, seed=wl.BASE_SEED + 75)
    t = to_device(ws, batch, ld=64)
    f, _ = bs.factor(diags_of(t), batch=batch)
    ref = bs.hb_inverse(diags_of(t), f, s_L=3, s_U=4, batch=batch)
    nb = bs.load().hb_inverse_band_workspace_bytes(5, n, batch, 64, 3, 4)
    wsb = torch.empty((nb + 7) // 8, dtype=torch.float64, device="cuda")
    outs = [torch.zeros_like(r) for r in ref]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bs.hb_inverse(diags_of(t), f, s_L=3, s_U=4, batch=batch, workspace=wsb, out=outs,
                          stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        wsb.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o[:, :, :batch].contiguous().view(torch.int64),
                               r[:, :, :batch].contiguous().view(torch.int64)), rep
