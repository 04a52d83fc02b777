"""GPU parity of band ILU(0) with the rows of a system split over lanes
(chunks with warm-up rows, a bitwise proof at every chunk boundary and a
sequential fallback): factors and info must be the sequential recurrence's to
the last bit, on systems where the warm-up converges, where it cannot (the
fallback) and with bad pivots placed around chunk boundaries."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, host, say, to_device

pytestmark = pytest.mark.gpu

KEYS = {5: ("e", "c", "d", "a", "b"), 3: ("c", "d", "a")}


def chunk_rows(n, batch, kind=5):
    """Rows per chunk the library picks: about 32768 lanes, chunks >= 64
    rows."""
    K = min(-(-32768 // batch), n // 64)
    if K <= 1:
        return n
    return -(-n // K)


def bits(t, batch=None):
    """Bit patterns (of the first `batch` columns: factor padding is never written)."""
    t = t if batch is None else t[..., :batch]
    return t.contiguous().view(torch.int64).cpu().numpy()


def factor_both(ws, kind, batch, ld=None):
    t = to_device(ws, batch, ld=ld, corner_nan=True)
    f, info = bs.factor(diags_of(t, kind), kind=kind, batch=batch)
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
    try:
        fl, infol = bs.factor(diags_of(t, kind), kind=kind, batch=batch)
    finally:
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
    torch.cuda.synchronize()
    return f, info, fl, infol


def check_against_oracle(ws, kind, f, info, systems):
    fh = [host(f[k], len(info)) for k in range(f.shape[0])]
    n = ws["d"].shape[1]
    for s in systems:
        e = ws["e"][s] if kind == 5 else np.zeros(n)
        b = ws["b"][s] if kind == 5 else np.zeros(n)
        l2, l1, u0, u1, oi = oracle.ilu0_band(e, ws["c"][s], ws["d"][s], ws["a"][s], b)
        assert int(info[s]) == oi
        if oi:
            continue    # the oracle stops at a bad pivot and returns no factors
        refs = (l2, l1, u0, u1) if kind == 5 else (l1, u0)
        for got, ref in zip(fh, refs):
            assert np.array_equal(got[s], ref)


def laplacian_batch(batch, n, kind):
    """d = 2, c = a = -1 (and e = b = 0): the pivots 2 - 1/u0 approach 1 only
    algebraically, so no warm-up reaches the sequential state to the bit."""
    z = np.zeros((batch, n))
    ws = {"e": z.copy(), "c": -np.ones((batch, n)), "d": 2.0 * np.ones((batch, n)),
          "a": -np.ones((batch, n)), "b": z.copy()}
    ws["y"] = np.ones((batch, n))
    return ws


@pytest.mark.parametrize("kind", [5, 3])
def test_pde_sweep_bitwise(kind):
    """96 systems of the 1024 x 1024 sweep batch (chunks of 64 or more rows)."""
    pd, td, _ = wl.config1(N=1024)
    ws = {k: v[:96] for k, v in (pd if kind == 5 else td).items()}
    say(f"pde kind={kind} n=1024 batch=96 chunk={chunk_rows(1024, 96, kind)}")
    f, info, fl, infol = factor_both(ws, kind, 96)
    assert np.array_equal(bits(f, len(info)), bits(fl, len(info))) and np.array_equal(info.cpu(), infol.cpu())
    assert (info.cpu().numpy() == 0).all()
    check_against_oracle(ws, kind, f, info.cpu().numpy(), range(0, 96, 11))


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("n,batch,ld", [(2048, 64, 64), (1000, 130, 136), (4099, 7, 8),
                                        (127, 200, 200), (64, 3, 3)])
def test_dominant_shapes_bitwise(kind, n, batch, ld):
    ws = wl.dominant_batch(batch, n, kind=kind, seed=300 + n)
    say(f"dominant kind={kind} n={n} batch={batch} ld={ld} chunk={chunk_rows(n, batch, kind)}")
    f, info, fl, infol = factor_both(ws, kind, batch, ld)
    assert np.array_equal(bits(f, len(info)), bits(fl, len(info))) and np.array_equal(info.cpu(), infol.cpu())
    check_against_oracle(ws, kind, f, info.cpu().numpy(), range(0, batch, max(1, batch // 5)))


@pytest.mark.parametrize("kind", [5, 3])
def test_fallback_mixed_batch(kind):
    """Laplacian rows (every chunk fails its proof: sequential fallback)
    interleaved with dominant systems (chunks kept) in one batch."""
    n, batch = 1536, 64
    dom = wl.dominant_batch(batch, n, kind=kind, seed=5)
    lap = laplacian_batch(batch, n, kind)
    ws = {k: np.where((np.arange(batch) % 3 == 0)[:, None], lap[k], dom[k])
          for k in ("e", "c", "d", "a", "b", "y")}
    say(f"fallback kind={kind} n={n} batch={batch} chunk={chunk_rows(n, batch, kind)}")
    f, info, fl, infol = factor_both(ws, kind, batch)
    assert np.array_equal(bits(f, len(info)), bits(fl, len(info))) and np.array_equal(info.cpu(), infol.cpu())
    check_against_oracle(ws, kind, f, info.cpu().numpy(), [0, 1, 3, 4, 62, 63])


@pytest.mark.parametrize("kind", [5, 3])
def test_bad_pivots_around_chunk_boundaries(kind):
    """Zero and non-finite pivots on a chunk's first rows, in the warm-up rows
    of the next chunk, mid-chunk and on the last row: info as the oracle's,
    every factor (also past the bad pivot) as the one-lane path's."""
    n, batch = 1024, 64
    M = chunk_rows(n, batch, kind)
    ws = wl.dominant_batch(batch, n, kind=kind, seed=9)
    rows = [M, M + 1, 2 * M - 3, 3 * M + M // 2, n - 1, 5 * M - 1, 2]
    for s, r in enumerate(rows):
        ws["d"][s, r] = np.inf if s % 2 else np.nan
    # u0 = 0 exactly at row 4M: d chosen so that the pivot cancels
    s0 = len(rows)
    r0 = 4 * M
    tmp = {k: v[s0:s0 + 1].copy() for k, v in ws.items() if k in KEYS[kind]}
    e = tmp["e"][0] if kind == 5 else np.zeros(n)
    b = tmp["b"][0] if kind == 5 else np.zeros(n)
    l2, l1, u0, u1, _ = oracle.ilu0_band(e, tmp["c"][0], tmp["d"][0], tmp["a"][0], b)
    ws["d"][s0, r0] = ws["d"][s0, r0] - u0[r0]
    say(f"bad pivots kind={kind} chunk={M} rows={rows + [r0]}")
    f, info, fl, infol = factor_both(ws, kind, batch)
    assert np.array_equal(bits(f, len(info)), bits(fl, len(info))) and np.array_equal(info.cpu(), infol.cpu())
    got = info.cpu().numpy()
    assert list(got[:len(rows)]) == [r + 1 for r in rows]
    check_against_oracle(ws, kind, f, got, list(range(s0 + 1)) + [s0 + 1, 63])


def test_sip_uses_the_same_factors():
    """SIP with its own ILU(0) (chunked) gives the same iterates as SIP on
    factors from the one-lane kernel."""
    pd, _, _ = wl.config1(N=1024)
    ws = {k: v[:128] for k, v in pd.items()}
    t = to_device(ws, 128)
    x, it, rr, info = bs.sip(diags_of(t), t["y"], tol=1e-10, max_iter=50, s_L=3, s_U=3,
                             batch=128)
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
    try:
        f, finfo = bs.factor(diags_of(t), batch=128)
    finally:
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
    x2, it2, rr2, info2 = bs.sip(diags_of(t), t["y"], tol=1e-10, max_iter=50, s_L=3, s_U=3,
                                 batch=128, factors=f)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    assert np.array_equal(bits(x), bits(x2)) and np.array_equal(it.cpu(), it2.cpu())


def subst_rows(n, batch):
    """Rows per chunk of the substitution: about 32768 lanes, chunks >= 128 rows."""
    K = min(-(-32768 // batch), n // 128)
    return n if K <= 1 else -(-n // K)


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("case,n,batch", [("pde", 1024, 96), ("dominant", 1000, 130),
                                          ("dominant", 4099, 7), ("dominant", 255, 9),
                                          ("mixed", 1536, 64)])
def test_substitution_split_bitwise(kind, case, n, batch):
    """Substitution with the factors, rows split over lanes, against the
    one-lane sweeps (bitwise) and the oracle's LU solve; the mixed batch has
    Laplacian systems whose chunks fail their proofs (sequential redo)."""
    if case == "pde":
        pd, td, _ = wl.config1(N=n)
        ws = {k: v[:batch] for k, v in (pd if kind == 5 else td).items()}
    else:
        ws = wl.dominant_batch(batch, n, kind=kind, seed=40 + n)
        if case == "mixed":
            lap = laplacian_batch(batch, n, kind)
            ws = {k: np.where((np.arange(batch) % 3 == 1)[:, None], lap[k], ws[k])
                  for k in ("e", "c", "d", "a", "b", "y")}
    say(f"subst {case} kind={kind} n={n} batch={batch} chunk={subst_rows(n, batch)}")
    t = to_device(ws, batch, corner_nan=True)
    f, finfo = bs.factor(diags_of(t, kind), kind=kind, batch=batch)
    x0 = torch.full_like(t["y"], 7.0)
    x, info = bs.solve(diags_of(t, kind), t["y"], x0.clone(), kind=kind, batch=batch, factors=f)
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
    try:
        xl, infol = bs.solve(diags_of(t, kind), t["y"], x0.clone(), kind=kind, batch=batch,
                             factors=f)
    finally:
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
    torch.cuda.synchronize()
    assert (finfo.cpu().numpy() == 0).all() and (info.cpu().numpy() == 0).all()
    assert np.array_equal(bits(x), bits(xl))          # padding columns untouched too
    fh = [host(f[k], batch) for k in range(f.shape[0])]
    xh = host(x, batch)
    for s in range(0, batch, max(1, batch // 6)):
        if kind == 5:
            l2, l1, u0, u1 = fh
            b = ws["b"][s]
        else:
            l1, u0 = fh
            l2, u1, b = np.zeros_like(l1), None, np.zeros(n)
        xo, _ = oracle.band_lu_solve(l2[s], l1[s], u0[s], u1[s] if kind == 5 else ws["a"][s],
                                     b, ws["y"][s])
        assert np.abs(xh[s] - xo).max() <= 1e-12 * np.abs(xo).max()


def test_factor_and_substitution_full_sweep_batch():
    """ILU(0) and the substitution split over lanes on the 2048 x 2048 sweep
    batch the benchmark times: factors, info and x bitwise the one-lane
    kernels on every system, and the oracle's factors (bitwise) and LU solve
    on a sample."""
    pd, _, _ = wl.config1()
    n, batch = 2048, 2048
    say(f"full sweep batch factor + substitution chunk={chunk_rows(n, batch)}")
    t = to_device(pd, batch)
    f, info = bs.factor(diags_of(t), batch=batch)
    x, xinfo = bs.solve(diags_of(t), t["y"], batch=batch, factors=f)
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
    try:
        fl, infol = bs.factor(diags_of(t), batch=batch)
        xl, _ = bs.solve(diags_of(t), t["y"], batch=batch, factors=fl)
    finally:
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (xinfo.cpu().numpy() == 0).all()
    assert np.array_equal(bits(f, batch), bits(fl, batch)) and torch.equal(info, infol)
    assert np.array_equal(bits(x, batch), bits(xl, batch))
    check_against_oracle(pd, 5, f, info.cpu().numpy(), (0, 777, 2047))
    fh = [host(f[k], batch) for k in range(4)]
    xh = host(x, batch)
    for s in (0, 777, 2047):
        xo, _ = oracle.band_lu_solve(fh[0][s], fh[1][s], fh[2][s], fh[3][s], pd["b"][s], pd["y"][s])
        assert np.abs(xh[s] - xo).max() <= 1e-12 * np.abs(xo).max()
