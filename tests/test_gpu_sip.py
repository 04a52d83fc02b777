"""GPU parity of the Stone method (SIP, Algorithm 1) with exact substitution
and with Hotelling-Bodewig approximate inverses, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, host, rel_err, say, to_device

pytestmark = pytest.mark.gpu

SIP_PATHS = {"lane": 1, "tile": 2, "tile1": 3}


@pytest.fixture(params=["lane", "tile", "tile1"])
def sip_path(request):
    """Run the test with one lane per system and with the rows of a system
    split over lanes (the latter only where both factors take HB steps), two
    steps per launch (where the halos fit) and one."""
    bs.set_option(bs.OPT_SIP_PATH, SIP_PATHS[request.param])
    yield request.param
    bs.set_option(bs.OPT_SIP_PATH, 0)


def host_relres(ws, x):
    """||b - A x||_inf / ||b||_inf per system, recomputed on the host."""
    r = ws["y"] - wl.band_matvec({k: ws[k] for k in ("e", "c", "d", "a", "b")}, x)
    bn = np.abs(ws["y"]).max(axis=1)
    return np.abs(r).max(axis=1) / np.where(bn > 0, bn, 1.0)


def check_relres(ws, x, rr, info, tol):
    """The reported relres is the host's ||b - A x|| / ||b|| of the returned x
    (to rounding), and every converged system is below tol by the host's count."""
    hr = host_relres(ws, x)
    ok = info == 0
    assert (hr[ok] < tol * 1.01).all(), hr[ok].max()
    bn = np.abs(ws["y"]).max(axis=1)
    assert (np.abs(hr[ok] - rr[ok]) <= 1e-15 * (1.0 + np.abs(x[ok]).max(axis=1) * 64 /
                                                 np.where(bn[ok] > 0, bn[ok], 1.0))).all()


def run_both(ws, batch, tol, max_iter, sL, sU, x0=None, ld=None):
    t = to_device(ws, batch, ld=ld)
    x0_t = None
    if x0 is not None:
        x0_t = torch.from_numpy(wl.interleave(x0, t["y"].shape[1])).cuda()
    x, it, rr, info = bs.sip(diags_of(t), t["y"], x0_t, tol=tol, max_iter=max_iter,
                             s_L=sL, s_U=sU, batch=batch)
    torch.cuda.synchronize()
    xo, ito, rro, sto = oracle.sip_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"],
                                         tol=tol, max_iter=max_iter, s_L=sL, s_U=sU, x0=x0)
    xh, rrh, ih = host(x, batch), rr.cpu().numpy(), info.cpu().numpy()
    check_relres(ws, xh, rrh, ih, tol)
    return (xh, it.cpu().numpy(), rrh, ih, xo, ito, rro, sto)


@pytest.mark.parametrize("sL,sU", [(-1, -1), (-1, 2), (1, 1), (2, 3), (3, 3), (5, 6), (11, 11)])
def test_config0_sip_parity(sL, sU, sip_path):
    ws = wl.config0(5)
    say(f"config0 SIP sL={sL} sU={sU} path={sip_path}")
    x, it, rr, info, xo, ito, rro, sto = run_both(ws, 64, 1e-12, 200, sL, sU)
    say(f"  iters gpu {it.min()}..{it.max()} oracle {ito.min()}..{ito.max()}")
    assert (sto == 0).all() and (info == 0).all()
    assert np.abs(it - ito).max() <= 1
    assert (rr < 1e-12).all()
    xd, _ = oracle.npdm_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"])
    assert rel_err(x, xd).max() <= 1e-10
    assert rel_err(x, xo).max() <= 1e-10


def test_pde_lines_warm_start_and_status_codes(sip_path):
    sw = wl.sweep_lines(wl.smooth_lines(64, 512, seed=21), r=4.0, order=2)
    say("PDE lines SIP sL=3 sU=4 zero and warm start")
    x, it, rr, info, xo, ito, rro, sto = run_both(sw, 64, 1e-10, 300, 3, 4)
    assert (info == 0).all() and (sto == 0).all() and np.abs(it - ito).max() <= 1
    # previous-step start (the sweep's own rhs, i.e. u) needs fewer steps
    x2, it2, rr2, info2, xo2, ito2, _, sto2 = run_both(sw, 64, 1e-10, 300, 3, 4, x0=sw["y"])
    assert (info2 == 0).all() and np.abs(it2 - ito2).max() <= 1
    assert it2.mean() <= it.mean()
    # not converged within max_iter
    x3, it3, rr3, info3, _, ito3, _, sto3 = run_both(sw, 64, 1e-10, 2, 1, 1)
    assert (info3 == -1).all() and (sto3 == -1).all() and (it3 == 2).all()


def test_divergence_and_zero_rhs(sip_path):
    sw = wl.sweep_lines(wl.smooth_lines(8, 512, seed=9), r=2047.0, order=2)
    x, it, rr, info, xo, ito, rro, sto = run_both(sw, 8, 1e-10, 200, 1, 1)
    say(f"divergence: gpu info {info.tolist()} oracle {sto.tolist()}")
    assert (sto == -2).all() and (info == -2).all()
    ws = wl.dominant_batch(3, 100, seed=3)
    ws["y"][1] = 0.0
    x, it, rr, info, *_ = run_both(ws, 3, 1e-12, 10, 2, 2, x0=np.ones((3, 100)))
    assert info[1] == 0 and it[1] == 0 and (x[1] == 0).all()


def test_precomputed_factors_and_ragged_batch(sip_path):
    ws = wl.dominant_batch(67, 700, seed=12)
    t = to_device(ws, 67, ld=128)
    f, finfo = bs.factor(diags_of(t), batch=67)
    x1, it1, rr1, i1 = bs.sip(diags_of(t), t["y"], tol=1e-12, max_iter=100, s_L=2, s_U=2,
                              batch=67, factors=f)
    x2, it2, rr2, i2 = bs.sip(diags_of(t), t["y"], tol=1e-12, max_iter=100, s_L=2, s_U=2,
                              batch=67)
    torch.cuda.synchronize()
    assert (i1.cpu() == 0).all() and torch.equal(it1, it2)
    assert torch.equal(x1[:, :67], x2[:, :67])


@pytest.mark.parametrize("n,batch,ld,sL,sU", [(40, 5, 64, 2, 2), (209, 16, 16, 3, 4),
                                              (5000, 33, 64, 3, 4), (3001, 17, 20, 1, 5),
                                              (1500, 3, 3, 4, 1)])
def test_split_rows_shapes(n, batch, ld, sL, sU):
    """Rows split over lanes: one tile, several tiles with a ragged last one,
    padded leading dimension, uneven halos."""
    ws = wl.dominant_batch(batch, n, seed=5000 + n)
    say(f"tile SIP n={n} batch={batch} ld={ld} sL={sL} sU={sU}")
    x, it, rr, info, xo, ito, rro, sto = run_both(ws, batch, 1e-12, 300, sL, sU, ld=ld)
    say(f"  iters gpu {it.min()}..{it.max()} oracle {ito.min()}..{ito.max()}")
    assert (sto == 0).all() and (info == 0).all()
    assert np.abs(it - ito).max() <= 1 and (rr < 1e-12).all()
    assert rel_err(x, xo).max() <= 1e-10


def test_split_rows_full_sweep_batch():
    """The 2048 x 2048 second-order sweep batch (r = 4), HB (3, 4), to 1e-10:
    iteration counts of every system against the oracle's."""
    pd, _, _ = wl.config1()
    say("tile SIP config1 n=2048 batch=2048 sL=3 sU=4")
    x, it, rr, info, xo, ito, rro, sto = run_both(pd, 2048, 1e-10, 100, 3, 4)
    say(f"  iters gpu {np.bincount(it).tolist()} oracle {np.bincount(ito).tolist()}")
    assert (sto == 0).all() and (info == 0).all()
    assert np.abs(it - ito).max() <= 1 and (rr < 1e-10).all()
    xd, _ = oracle.npdm_batch(pd["e"], pd["c"], pd["d"], pd["a"], pd["b"], pd["y"])
    assert rel_err(x, xd).max() <= 1e-7


def test_split_rows_learned_start_workload_size():
    """The learned-start workload's solve: 4096 second-order sweep systems of
    n = 4096 (r = 4), HB (3, 3), zero start, to 1e-10.  Status and residual
    of every system; iteration counts and x of a sample against the oracle."""
    N = 4096
    sw = wl.sweep_lines(wl.smooth_lines(N, N, seed=404), 4.0, 2)
    t = to_device(sw, N)
    say(f"tile SIP n={N} batch={N} sL=3 sU=3")
    x, it, rr, info = bs.sip(diags_of(t), t["y"], tol=1e-10, max_iter=100, s_L=3, s_U=3,
                             batch=N)
    torch.cuda.synchronize()
    it, rr, info = it.cpu().numpy(), rr.cpu().numpy(), info.cpu().numpy()
    say(f"  iters {np.bincount(it).tolist()}")
    assert (info == 0).all() and (rr < 1e-10).all()
    pick = [0, 1, 777, 2048, N - 1]
    sub = {k: v[pick] for k, v in sw.items()}
    xo, ito, rro, sto = oracle.sip_batch(sub["e"], sub["c"], sub["d"], sub["a"], sub["b"],
                                         sub["y"], tol=1e-10, max_iter=100, s_L=3, s_U=3)
    assert (sto == 0).all() and np.abs(it[pick] - ito).max() <= 1
    xs = x[:, pick].cpu().numpy().T
    xd, _ = oracle.npdm_batch(sub["e"], sub["c"], sub["d"], sub["a"], sub["b"], sub["y"])
    assert rel_err(xs, xd).max() <= 1e-7


@pytest.mark.parametrize("case,sL,sU", [("sweep", 3, 4), ("sweep", 2, 2), ("ragged", 3, 3),
                                         ("ragged", 4, 4), ("ragged", 1, 5)])
def test_several_steps_per_launch_same_iterates(case, sL, sU):
    """Several steps per launch (three for (2, 2) and (3, 3), two for the
    others: tests at k, k + 1, ... in one launch) against one step per
    launch: bitwise the same x, iteration counts, residuals and status, for
    max_iter of every residue (the last launch then has steps to spare) and
    with systems that stop at different counts."""
    if case == "sweep":
        pd, _, _ = wl.config1(N=1024)
        ws, batch, ld = {k: v[:200] for k, v in pd.items()}, 200, 256
    else:
        ws, batch, ld = wl.dominant_batch(37, 3001, seed=77), 37, 40
        ws["y"][5] = 0.0                    # b = 0: x = 0, no step
        ws["d"][9, 0] = 0.0                 # ILU(0) pivot u0_0 = 0: no step
        ws["y"][11] *= 1e-300               # stops at a different count
    t = to_device(ws, batch, ld=ld)
    x0 = torch.from_numpy(wl.interleave(np.full((batch, ws["d"].shape[1]), 0.5), ld)).cuda()
    for max_iter in (0, 1, 2, 3, 5, 6, 7, 100):
        out = {}
        for name, path in (("two", 2), ("one", 3)):
            bs.set_option(bs.OPT_SIP_PATH, path)
            try:
                out[name] = bs.sip(diags_of(t), t["y"], x0.clone(), tol=1e-11,
                                   max_iter=max_iter, s_L=sL, s_U=sU, batch=batch)
            finally:
                bs.set_option(bs.OPT_SIP_PATH, 0)
        torch.cuda.synchronize()
        (x2, it2, rr2, i2), (x1, it1, rr1, i1) = out["two"], out["one"]
        say(f"{case} s=({sL},{sU}) max_iter={max_iter}: iters {it2.min().item()}..{it2.max().item()} "
            f"status {sorted(set(i2.cpu().tolist()))}")
        assert torch.equal(it2, it1) and torch.equal(i2, i1)
        assert torch.equal(rr2.view(torch.int64), rr1.view(torch.int64))
        assert torch.equal(x2[:, :batch].contiguous().view(torch.int64),
                           x1[:, :batch].contiguous().view(torch.int64))
        i = i2.cpu().numpy()
        assert (it2.cpu().numpy() <= max_iter).all()
        if case == "ragged":
            assert i[9] == 1 and i[5] == 0 and it2[5].item() == 0


@pytest.mark.parametrize("sL,sU", [(3, 4), (1, 6)])
def test_split_rows_graph_replay(sL, sU):
    """One captured sip_solve (factorization, norms, every step launch and the
    final copy; two steps per launch for (3, 4), one for (1, 6)) replayed three times, with eager solves on other data in
    between: every replay bitwise the eager result (the arrival counter, the
    done flag and the accumulators start clean each time)."""
    ws = wl.dominant_batch(48, 2500, seed=31)
    other = wl.dominant_batch(48, 2500, seed=32)
    t, t2 = to_device(ws, 48, ld=64), to_device(other, 48, ld=64)
    nbytes = bs.workspace_bytes(bs.OP_SIP, 5, 2500, 48, ld=64)
    wsb = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(t["y"])
    x_ref, it_ref, rr_ref, i_ref = bs.sip(diags_of(t), t["y"], torch.zeros_like(t["y"]), tol=1e-11,
                                          max_iter=60, s_L=sL, s_U=sU, batch=48)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            out = bs.sip(diags_of(t), t["y"], x=x, tol=1e-11, max_iter=60, s_L=sL, s_U=sU,
                         batch=48, workspace=wsb, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        _, it, rr, info = out
        say(f"graph replay {rep} s=({sL},{sU}): iters {it.min().item()}..{it.max().item()}")
        assert torch.equal(x[:, :48].contiguous().view(torch.int64),
                           x_ref[:, :48].contiguous().view(torch.int64))
        assert torch.equal(it, it_ref) and torch.equal(info, i_ref)
        assert torch.equal(rr.view(torch.int64), rr_ref.view(torch.int64))
        # eager work on other data in between (its own workspace)
        bs.sip(diags_of(t2), t2["y"], tol=1e-11, max_iter=60, s_L=sL, s_U=sU, batch=48)
        torch.cuda.synchronize()


def test_exact_substitution_full_sweep_batch():
    """Algorithm 1 as printed (exact triangular solves; rows split over lanes:
    row-parallel K x + b and residual, split substitution) on the 2048 x 2048
    sweep batch: with the band's exact ILU(0) it stops after one step.  Every
    system bitwise the one-lane kernel's run; iterations, status and x of a
    sample against the oracle's run of the same algorithm; relres of every
    system recomputed on the host."""
    pd, _, _ = wl.config1()
    t = to_device(pd, 2048)
    say("exact SIP n=2048 batch=2048")
    x, it, rr, info = bs.sip(diags_of(t), t["y"], tol=1e-12, max_iter=5, batch=2048)
    bs.set_option(bs.OPT_SIP_PATH, 1)
    try:
        xl, itl, rrl, infol = bs.sip(diags_of(t), t["y"], tol=1e-12, max_iter=5, batch=2048)
    finally:
        bs.set_option(bs.OPT_SIP_PATH, 0)
    torch.cuda.synchronize()
    assert torch.equal(x.view(torch.int64), xl.view(torch.int64))
    assert torch.equal(it, itl) and torch.equal(info, infol)
    assert torch.equal(rr.view(torch.int64), rrl.view(torch.int64))
    it, rr, info = it.cpu().numpy(), rr.cpu().numpy(), info.cpu().numpy()
    assert (info == 0).all() and (it == 1).all() and (rr < 1e-12).all()
    check_relres(pd, host(x, 2048), rr, info, 1e-12)
    pick = [0, 1, 1000, 2047]
    sub = {k: v[pick] for k, v in pd.items()}
    xo, ito, rro, sto = oracle.sip_batch(sub["e"], sub["c"], sub["d"], sub["a"], sub["b"],
                                         sub["y"], tol=1e-12, max_iter=5)
    assert (sto == 0).all() and (ito == it[pick]).all()
    assert rel_err(x[:, pick].cpu().numpy().T, xo).max() <= 1e-12


@pytest.mark.parametrize("case", ["dominant", "sweep", "ragged"])
def test_exact_rows_bitwise_one_lane(case):
    """Algorithm 1 as printed with the rows split over lanes against the
    one-lane kernel (Algorithm 1 in one persistent launch): bitwise the same
    x, step counts, residuals and statuses for max_iter of 0 .. 3 and 50,
    from a non-zero start (so K x matters), with a tolerance below rounding
    (every step taken, status -1), and with systems whose b = 0, whose
    ILU(0) pivot is zero, or whose right-hand side is tiny."""
    if case == "dominant":
        ws, batch, ld = wl.dominant_batch(64, 1024, seed=61), 64, 64
    elif case == "sweep":
        pd, _, _ = wl.config1(N=1024)
        ws, batch, ld = {k: v[:300] for k, v in pd.items()}, 300, 320
    else:
        ws, batch, ld = wl.dominant_batch(37, 3001, seed=62), 37, 40
        ws["y"][5] = 0.0                    # b = 0: x = 0, no step
        ws["d"][9, 0] = 0.0                 # ILU(0) pivot u0_0 = 0: no step
        ws["y"][11] *= 1e-300               # tiny rhs
    t = to_device(ws, batch, ld=ld)
    rng = np.random.default_rng(63)
    x0 = torch.from_numpy(wl.interleave(rng.uniform(-1, 1, (batch, ws["d"].shape[1])),
                                        ld)).cuda()
    for tol in (1e-12, 1e-30):
        for max_iter in (0, 1, 2, 3, 50):
            out = {}
            for name, path in (("rows", 0), ("lane", 1)):
                bs.set_option(bs.OPT_SIP_PATH, path)
                try:
                    out[name] = bs.sip(diags_of(t), t["y"], x0.clone(), tol=tol,
                                       max_iter=max_iter, batch=batch)
                finally:
                    bs.set_option(bs.OPT_SIP_PATH, 0)
            torch.cuda.synchronize()
            (xr, itr, rrr, ir), (xl, itl, rrl, il) = out["rows"], out["lane"]
            say(f"exact {case} tol={tol} max_iter={max_iter}: iters "
                f"{itr.min().item()}..{itr.max().item()} status {sorted(set(ir.cpu().tolist()))}")
            assert torch.equal(itr, itl) and torch.equal(ir, il)
            assert torch.equal(rrr.view(torch.int64), rrl.view(torch.int64))
            assert torch.equal(xr[:, :batch].contiguous().view(torch.int64),
                               xl[:, :batch].contiguous().view(torch.int64))
            if tol == 1e-30 and case != "ragged":
                assert (itr.cpu().numpy() == max_iter).all()
            if case == "ragged":
                i = ir.cpu().numpy()
                assert i[9] == 1 and i[5] == 0 and itr[5].item() == 0
                assert (xr[:, 5] == 0).all()


def test_split_rows_bad_pivot_and_max_iter_zero():
    ws = wl.dominant_batch(4, 600, seed=13)
    ws["d"][2, 0] = 0.0     # ILU(0) pivot u0_0 = 0: no step, x untouched
    t = to_device(ws, 4)
    x0 = torch.full_like(t["y"], 3.0)
    x, it, rr, info = bs.sip(diags_of(t), t["y"], x0, tol=1e-12, max_iter=50, s_L=2, s_U=2,
                             batch=4)
    torch.cuda.synchronize()
    i = info.cpu().numpy()
    assert i[2] == 1 and (np.delete(i, 2) == 0).all()
    assert (x[:, 2] == 3.0).all()
    # max_iter = 0: the test alone; relres of x0 reported
    x, it, rr, info = bs.sip(diags_of(t), t["y"], tol=1e-12, max_iter=0, s_L=2, s_U=2, batch=4)
    torch.cuda.synchronize()
    i = info.cpu().numpy()
    assert (it.cpu().numpy() == 0).all() and i[2] == 1 and (np.delete(i, 2) == -1).all()
    assert (rr.cpu().numpy()[[0, 1, 3]] == 1.0).all()   # x0 = 0: ||b - A 0|| = ||b||
