"""GPU parity of the direct solvers (NPDM, NTDM, MNPDM, band ILU(0) and
substitution) against the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, host, rel_err, say, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-12   # relative parity bar per system, FP64

PATHS = {"lane": bs.PATH_LANE, "part": bs.PATH_PART}
@pytest.fixture(params=["lane", "part"])
def path(request):
    """Run the test once with one lane per system and once with the rows of a
    system split over lanes (where the shape allows it)."""
    bs.set_option(bs.OPT_DIRECT_PATH, PATHS[request.param])
    yield request.param
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)


def oracle_direct(ws, kind):
    if kind == 5:
        return oracle.npdm_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"])
    return oracle.ntdm_batch(ws["c"], ws["d"], ws["a"], ws["y"])


@pytest.mark.parametrize("kind", [5, 3])
def test_config0_parity(kind, path):
    ws = wl.config0(kind)
    batch = 64
    say(f"config0 kind={kind} n=1024 batch=64 path={path}")
    t = to_device(ws, batch)
    x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=batch)
    torch.cuda.synchronize()
    xr, ir = oracle_direct(ws, kind)
    assert (info.cpu().numpy() == 0).all() and (ir == 0).all()
    err = rel_err(host(x, batch), xr)
    say(f"  max rel err {err.max():.3e}")
    assert err.max() <= TOL
    assert np.abs(host(x, batch) - ws["x_true"]).max() <= 1e-13


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("n,batch,ld", [(1, 5, 64), (2, 3, 3), (3, 70, 128), (4, 64, 64),
                                        (8, 9, 9), (37, 1, 1), (129, 67, 80), (1000, 200, 256),
                                        (2047, 33, 64), (2048, 5, 5), (3000, 9, 16),
                                        (4096, 20, 64)])
def test_shapes_ragged_and_tiny(kind, n, batch, ld, path):
    ws = wl.dominant_batch(batch, n, kind=kind, seed=1000 + n + batch)
    say(f"shape kind={kind} n={n} batch={batch} ld={ld} path={path}")
    t = to_device(ws, batch, ld=ld, corner_nan=True, pad_fill=np.nan)
    x0 = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    x, info = bs.solve(diags_of(t, kind), t["y"], x0, kind=kind, batch=batch)
    torch.cuda.synchronize()
    xr, ir = oracle_direct(ws, kind)
    assert (info.cpu().numpy() == 0).all() and (ir == 0).all()
    assert rel_err(host(x, batch), xr).max() <= TOL
    if ld > batch:   # padding columns are never written
        assert (x[:, batch:] == 7.0).all()


def test_config1_full_size_pd_and_td(path):
    """2048 x 2048 ADI sweep (r = 4): every system of both batches."""
    pd, td, _ = wl.config1()
    batch = 2048
    for kind, ws in ((5, pd), (3, td)):
        say(f"config1 kind={kind} n=2048 batch=2048 path={path}")
        t = to_device(ws, batch)
        x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=batch)
        torch.cuda.synchronize()
        xr, ir = oracle_direct(ws, kind)
        assert (info.cpu().numpy() == 0).all() and (ir == 0).all()
        err = rel_err(host(x, batch), xr)
        say(f"  max rel err {err.max():.3e}")
        assert err.max() <= TOL


@pytest.mark.parametrize("kind", [5, 3])
def test_every_split_variant(kind):
    """Each compiled split-row variant, on a ragged batch whose rows span
    several tiles and on a second-order PDE batch."""
    ws = wl.dominant_batch(45, 1999, kind=kind, seed=17)
    pd, td, _ = wl.config1(N=512, seed=23)
    pde = pd if kind == 5 else td
    xr, _ = oracle_direct(ws, kind)
    xp, _ = oracle_direct(pde, kind)
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_PART)
    key = bs.OPT_PART_PD_VARIANT if kind == 5 else bs.OPT_PART_TD_VARIANT
    try:
        for idx, shape in enumerate(bs.part_variants(kind)):
            bs.set_option(key, idx)
            say(f"variant kind={kind} (M, PW, G, TMAX)={shape}")
            for rep in range(2):   # the workspace is reused: counters reset
                t = to_device(ws, 45, ld=64, corner_nan=True)
                x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=45)
                t2 = to_device(pde, 512)
                x2, info2 = bs.solve(diags_of(t2, kind), t2["y"], kind=kind, batch=512)
                torch.cuda.synchronize()
                assert (info.cpu().numpy() == 0).all() and (info2.cpu().numpy() == 0).all()
                assert rel_err(host(x, 45), xr).max() <= TOL
                assert rel_err(host(x2, 512), xp).max() <= TOL
    finally:
        bs.set_option(key, 0)
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)


def test_split_workspace_reuse_and_graph_replay():
    """One persistent workspace, many calls and graph replays: the meeting
    counters return to zero after every call."""
    pd, _, _ = wl.config1(N=1024, seed=29)
    batch = 1024
    t = to_device(pd, batch)
    xr, _ = oracle_direct(pd, 5)
    nbytes = bs.workspace_bytes(bs.OP_SOLVE, 5, 1024, batch)
    assert nbytes > 0
    wsb = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    x = torch.empty_like(t["y"])
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    for _ in range(5):
        bs.solve(diags_of(t), t["y"], x, batch=batch, info=info, workspace=wsb)
    torch.cuda.synchronize()
    assert (info.cpu() == 0).all() and rel_err(host(x, batch), xr).max() <= TOL
    M, PW, G, TMAX = bs.part_variants(5)[0]
    groups = -(-batch // G)
    assert (wsb.view(torch.int32)[: 4 * groups] == 0).all()      # meeting counters reset
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bs.solve(diags_of(t), t["y"], x, batch=batch, info=info, workspace=wsb, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(4):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert (info.cpu() == 0).all(), rep
        assert rel_err(host(x, batch), xr).max() <= TOL, rep


def test_in_place_and_deterministic():
    ws = wl.dominant_batch(100, 300, kind=5, seed=5)
    t = to_device(ws, 100, ld=128)
    x1, _ = bs.solve(diags_of(t), t["y"], batch=100)
    x2, _ = bs.solve(diags_of(t), t["y"], batch=100)
    y = t["y"].clone()
    x3, _ = bs.solve(diags_of(t), y, y, batch=100)   # x aliases rhs
    torch.cuda.synchronize()
    assert torch.equal(x1[:, :100], x2[:, :100]) and torch.equal(x1[:, :100], x3[:, :100])


def test_zero_and_nonfinite_pivots_reported(path):
    ws = wl.dominant_batch(4, 50, kind=5, seed=6)
    ws["d"][0, 0] = 0.0            # system 0: mu_0 = 0
    ws["d"][1, 10] = np.inf        # system 1: non-finite pivot at row 10
    # system 2: mu_1 = d_1 - (a_0 / d_0) c_1 = 0 exactly
    ws["d"][2, 0], ws["a"][2, 0], ws["c"][2, 1], ws["d"][2, 1] = 2.0, 1.0, 2.0, 1.0
    for kind in (5, 3):
        t = to_device(ws, 4)
        _, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=4)
        got = info.cpu().numpy().tolist()
        if kind == 5:
            ref = [oracle.npdm(*[ws[k][s] for k in ("e", "c", "d", "a", "b", "y")])[1]
                   for s in range(4)]
        else:
            ref = [oracle.ntdm(*[ws[k][s] for k in ("c", "d", "a", "y")])[1] for s in range(4)]
        say(f"pivots kind={kind}: gpu {got} oracle {ref}")
        assert got == ref and got[:3] == [1, 11, 2] and got[3] == 0


def test_factor_and_factored_solve():
    for kind in (5, 3):
        ws = wl.dominant_batch(70, 513, kind=kind, seed=7)
        t = to_device(ws, 70, ld=128, corner_nan=True)
        f, finfo = bs.factor(diags_of(t, kind), kind=kind, batch=70)
        x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=70, factors=f)
        torch.cuda.synchronize()
        assert (finfo.cpu().numpy() == 0).all() and (info.cpu().numpy() == 0).all()
        fh = [host(f[k], 70) for k in range(f.shape[0])]
        for s in range(0, 70, 7):
            e = ws["e"][s] if kind == 5 else np.zeros(513)
            b = ws["b"][s] if kind == 5 else np.zeros(513)
            l2, l1, u0, u1, oi = oracle.ilu0_band(e, ws["c"][s], ws["d"][s], ws["a"][s], b)
            assert oi == 0
            if kind == 5:
                for got, ref in zip(fh, (l2, l1, u0, u1)):
                    assert np.array_equal(got[s], ref)
            else:
                assert np.array_equal(fh[0][s], l1) and np.array_equal(fh[1][s], u0)
            xo, _ = oracle.band_lu_solve(l2, l1, u0, u1, b, ws["y"][s])
            assert rel_err(host(x, 70)[s:s + 1], xo[None]).max() <= TOL


def test_mnpdm_matches_npdm_and_oracle(path):
    pd, _, _ = wl.config1(N=256, seed=11)
    batch, n = 256, 256
    t = to_device(pd, batch)
    kmax = 3
    rows = np.full((kmax, batch), -1, dtype=np.int32)
    oe = np.zeros((kmax, batch))
    ob = np.zeros((kmax, batch))
    rows[0], ob[0] = 0, pd["b"][:, 0]
    rows[1], oe[1] = n - 1, pd["e"][:, n - 1]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, info = bs.solve_mnpdm([t["c"], t["d"], t["a"]], dev(rows), dev(oe), dev(ob), t["y"],
                             batch=batch)
    xn, infon = bs.solve(diags_of(t), t["y"], batch=batch)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    # the skipped products are exact zeros: bitwise the NPDM of the same kernel
    assert torch.equal(x[:, :batch], xn[:, :batch])
    for s in range(0, batch, 17):
        xo, io = oracle.mnpdm(pd["c"][s], pd["d"][s], pd["a"][s], [0, n - 1],
                              [0.0, pd["e"][s][n - 1]], [pd["b"][s][0], 0.0], pd["y"][s])
        assert io == 0
        assert rel_err(host(x, batch)[s:s + 1], xo[None]).max() <= TOL
    # a bad list is reported per system
    rows[0, 5], rows[1, 5] = 9, 3
    _, info2 = bs.solve_mnpdm([t["c"], t["d"], t["a"]], dev(rows), dev(oe), dev(ob), t["y"],
                              batch=batch)
    torch.cuda.synchronize()
    i2 = info2.cpu().numpy()
    assert i2[5] == -3 and (np.delete(i2, 5) == 0).all()


def test_mnpdm_full_sweep_batch():
    """MNPDM on the 2048 x 2048 sweep batch as the benchmark runs it (c, d, a
    and the two outer entries of every system, K = 2): bitwise the split NPDM
    on every system, and the oracle's MNPDM on a sample."""
    pd, _, _ = wl.config1()
    batch, n = 2048, 2048
    t = to_device(pd, batch)
    rows = np.full((2, batch), -1, dtype=np.int32)
    oe, ob = np.zeros((2, batch)), np.zeros((2, batch))
    rows[0], ob[0] = 0, pd["b"][:, 0]
    rows[1], oe[1] = n - 1, pd["e"][:, n - 1]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    say("MNPDM n=2048 batch=2048 K=2")
    x, info = bs.solve_mnpdm([t["c"], t["d"], t["a"]], dev(rows), dev(oe), dev(ob), t["y"],
                             batch=batch)
    xn, infon = bs.solve(diags_of(t), t["y"], batch=batch)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (infon.cpu().numpy() == 0).all()
    assert torch.equal(x.view(torch.int64), xn.view(torch.int64))
    xh = host(x, batch)
    for s in (0, 1, 1023, 2046, 2047):
        xo, io = oracle.mnpdm(pd["c"][s], pd["d"][s], pd["a"][s], [0, n - 1],
                              [0.0, pd["e"][s][n - 1]], [pd["b"][s][0], 0.0], pd["y"][s])
        assert io == 0 and rel_err(xh[s:s + 1], xo[None]).max() <= TOL


@pytest.mark.parametrize("n,batch,ld,kmax", [(2048, 100, 128, 5), (3001, 33, 40, 9),
                                             (5000, 7, 8, 4), (300, 64, 64, 0),
                                             (2048, 64, 64, 64), (2048, 48, 64, 100),
                                             (1999, 40, 40, 300), (2048, 80, 128, 12)])
def test_mnpdm_random_lists(n, batch, ld, kmax, path):
    """Random sparse outer diagonals (K entries per system, some lists shorter
    than kmax): MNPDM against the oracle and bitwise against NPDM on the
    zero-filled diagonals; several tiles, ragged batch, padded ld, a length
    beyond the split variants (one lane per system), and lists up to the 64
    entries per system the split kernel stages in LDS and beyond (scanned in
    global memory)."""
    rng = np.random.default_rng(n + batch)
    ws = wl.dominant_batch(batch, n, kind=5, seed=600 + n)
    rows = np.full((max(kmax, 1), batch), -1, dtype=np.int32)
    oe = np.zeros((max(kmax, 1), batch))
    ob = np.zeros((max(kmax, 1), batch))
    e = np.zeros((batch, n))
    b = np.zeros((batch, n))
    for s in range(batch):
        k = int(rng.integers(0, kmax + 1)) if kmax else 0
        r = np.sort(rng.choice(n, size=k, replace=False))
        rows[:k, s] = r
        oe[:k, s] = rng.uniform(-1, 1, k)
        ob[:k, s] = rng.uniform(-1, 1, k)
        for q in range(k):
            if r[q] >= 2:
                e[s, r[q]] = oe[q, s]
            if r[q] <= n - 3:
                b[s, r[q]] = ob[q, s]
    ws["e"], ws["b"] = e, b
    ws["d"] = np.abs(ws["c"]) + np.abs(ws["a"]) + np.abs(e) + np.abs(b) + 1.5
    say(f"mnpdm random lists n={n} batch={batch} ld={ld} kmax={kmax} path={path}")
    t = to_device(ws, batch, ld=ld)
    row_t = torch.from_numpy(np.ascontiguousarray(
        np.pad(rows, ((0, 0), (0, ld - batch)), constant_values=-1))).cuda()
    oe_t = torch.from_numpy(np.ascontiguousarray(np.pad(oe, ((0, 0), (0, ld - batch))))).cuda()
    ob_t = torch.from_numpy(np.ascontiguousarray(np.pad(ob, ((0, 0), (0, ld - batch))))).cuda()
    if kmax == 0:
        row_t = oe_t = ob_t = None
    x, info = bs.solve_mnpdm([t["c"], t["d"], t["a"]], row_t, oe_t, ob_t, t["y"], batch=batch)
    xn, infon = bs.solve(diags_of(t), t["y"], batch=batch)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (infon.cpu().numpy() == 0).all()
    M, PW, G, TMAX = bs.part_variants(5)[1]
    if path == "lane" or n <= M * PW * TMAX:   # both calls ran the same kernel family
        assert torch.equal(x[:, :batch], xn[:, :batch])
    xr, _ = oracle.npdm_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"])
    assert rel_err(host(x, batch), xr).max() <= TOL


def test_stream_probe_sums():
    """The streaming ceiling probe computes what it claims (it is timed by the
    benchmark against the solver's traffic pattern)."""
    g = torch.Generator(device="cuda").manual_seed(3)
    ins = [torch.rand(2 * 12345, dtype=torch.float64, device="cuda", generator=g)
           for _ in range(6)]
    for k in (1, 3, 6):
        out = torch.empty_like(ins[0])
        bs.stream_probe(ins[:k], out)
        ref = ins[0].clone()
        for t in ins[1:k]:
            ref += t
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


@pytest.mark.parametrize("batch,n,ld,pitch", [(1, 1, 1, 1), (33, 70, 40, 70), (70, 33, 128, 41),
                                              (257, 1000, 264, 1000), (2, 4099, 64, 4100)])
def test_interleave_conversions(batch, n, ld, pitch):
    """Device pack/unpack against the host layout helpers, bitwise; padding
    columns and the gaps of a pitched buffer are left alone."""
    rng = np.random.default_rng(batch * n)
    lines = rng.normal(size=(batch, n))
    src = torch.full((batch, pitch), np.nan, dtype=torch.float64, device="cuda")
    src[:, :n] = torch.from_numpy(lines).cuda()
    out = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    bs.pack_interleave(src[:, :n], ld=ld, out=out)
    back = torch.full((batch, pitch), -3.0, dtype=torch.float64, device="cuda")
    bs.unpack_interleave(out, batch, out=back[:, :n])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), wl.interleave(lines, ld, fill=7.0))
    assert np.array_equal(back[:, :n].cpu().numpy(), lines)
    assert (back[:, n:].cpu().numpy() == -3.0).all()
