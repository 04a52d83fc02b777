"""GPU parity of the FP32-storage solve, of the long-system (three-launch)
split path and of FP32 solves with FP64 iterative refinement, against the
FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import KEYS, diags_of, host, rel_err, say, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-12          # FP64 relative parity bar per system
U32 = 2.0 ** -24     # unit roundoff of FP32


def oracle_direct(ws, kind):
    if kind == 5:
        return oracle.npdm_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"])
    return oracle.ntdm_batch(ws["c"], ws["d"], ws["a"], ws["y"])


def fp32_rounded(ws):
    """The FP64 values an FP32 copy of the batch holds."""
    return {k: ws[k].astype(np.float32).astype(np.float64) for k in KEYS}


def host_residual(ws, kind, x):
    """Per-system ||y - A x||_inf / ||y||_inf in FP64 on the host."""
    d = {k: ws[k] for k in ("c", "d", "a", "y")}
    if kind == 5:
        d["e"], d["b"] = ws["e"], ws["b"]
    else:
        d["e"] = d["b"] = np.zeros_like(ws["d"])
    r = ws["y"] - wl.band_matvec(d, x)
    return np.abs(r).max(axis=1) / np.abs(ws["y"]).max(axis=1)


# ------------------------------------------------------------ FP32 storage --
# With the compact state (BS_OPT_F32_STATE = 1, the default) the backward
# substitution and the final x = p - V x_L - W x_R run in FP32.  A value of x
# passes through: one rounding of each forward (FP64) result, at most two per
# step of the backward sweep (a contraction where |alpha| + |beta| < 1, so
# earlier errors do not grow), two roundings of the outer pairs and four
# fused steps of the final sum: below 16 u of the terms' magnitude on
# diagonally dominant rows.  The bar on the normwise backward error
#     eta = ||y - A x||_inf / (||A||_inf ||x||_inf + ||y||_inf)
# is twice that, K_BWD u.  On a strictly diagonally dominant matrix
# ||A^-1||_inf <= 1 / delta, delta = min_i (|d_i| - sum of |off-diagonals|)
# (Varah), so the forward error is then at most ||y - A x||_inf / delta.
K_BWD = 32


def abs_rowsum(ws, kind):
    s = np.abs(ws["c"]) + np.abs(ws["d"]) + np.abs(ws["a"])
    if kind == 5:
        s = s + np.abs(ws["e"]) + np.abs(ws["b"])
    return s


def backward_error(ws, kind, x):
    """Per system: eta (above) and ||y - A x||_inf, in FP64 on the host."""
    d = {k: ws[k] for k in ("c", "d", "a")}
    d["e"] = ws["e"] if kind == 5 else np.zeros_like(ws["d"])
    d["b"] = ws["b"] if kind == 5 else np.zeros_like(ws["d"])
    r = np.abs(ws["y"] - wl.band_matvec(d, x)).max(axis=1)
    scale = abs_rowsum(ws, kind).max(axis=1) * np.abs(x).max(axis=1) + np.abs(ws["y"]).max(axis=1)
    return r / scale, r


def check_fp32(ws, kind, xg, xr, state, dominant):
    if state == 0:   # FP64 arithmetic: within one FP32 rounding of x, plus the FP64 bar
        bar = U32 * np.abs(xr) + 2 * TOL * np.abs(xr).max(axis=1, keepdims=True)
        worst = (np.abs(xg - xr) / bar).max()
        say(f"  FP64 state: max |x - x_orc| / bar = {worst:.3f}")
        assert worst <= 1.0
        return
    eta, r = backward_error(ws, kind, xg)
    say(f"  compact state: max eta = {eta.max() / U32:.2f} u")
    assert (eta <= K_BWD * U32).all()
    if dominant:
        delta = (2 * np.abs(ws["d"]) - abs_rowsum(ws, kind)).min(axis=1)
        assert (delta > 0).all()
        err = np.abs(xg - xr).max(axis=1)
        bound = r / delta + 2 * TOL * np.abs(xr).max(axis=1)
        say(f"  compact state: max forward error / Varah bound = {(err / bound).max():.3f}")
        assert (err <= bound).all()


@pytest.fixture(params=[1, 0], ids=["compact_state", "fp64_state"])
def f32_state(request):
    bs.set_option(bs.OPT_F32_STATE, request.param)
    yield request.param
    bs.set_option(bs.OPT_F32_STATE, 1)


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("n,batch,ld", [(8, 5, 64), (9, 33, 64), (100, 17, 17), (2047, 45, 64),
                                        (2048, 70, 96), (4096, 20, 64), (5000, 7, 8),
                                        (40000, 3, 64)])
def test_fp32_storage_parity(kind, n, batch, ld, f32_state):
    """FP32 inputs and x, FP64 pivots and forward recurrences.  FP64 state:
    every element within one FP32 rounding of the FP64 oracle solution of the
    same (FP32-valued) system, plus the FP64 parity bar.  Compact state: the
    backward-error bar and the forward bound it implies (Varah)."""
    ws = fp32_rounded(wl.dominant_batch(batch, n, kind=kind, seed=3000 + n + batch))
    say(f"fp32 kind={kind} n={n} batch={batch} ld={ld} state={f32_state}")
    t = to_device(ws, batch, ld=ld, corner_nan=True, dtype=torch.float32)
    x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=batch)
    torch.cuda.synchronize()
    xr, ir = oracle_direct(ws, kind)
    assert (info.cpu().numpy() == 0).all() and (ir == 0).all()
    check_fp32(ws, kind, host(x, batch), xr, f32_state, dominant=True)


def test_workspace_shared_across_dtypes_and_states():
    """One workspace serves FP32 calls with either state and FP64 calls in
    turn: the variants differ in systems per block, and their meeting
    counters share one leading region that every call leaves zero."""
    kind, n, batch = 5, 2048, 96
    ws = wl.dominant_batch(batch, n, kind=kind, seed=77)
    w32 = fp32_rounded(ws)
    xr, _ = oracle_direct(ws, kind)
    xr32, _ = oracle_direct(w32, kind)
    t64 = to_device(ws, batch)
    t32 = to_device(w32, batch, dtype=torch.float32)
    nbytes = max(bs.workspace_bytes(bs.OP_SOLVE, kind, n, batch, dt) for dt in (bs.BS_F64, bs.BS_F32))
    wsb = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    lead = (batch + 15) // 16 * 4
    try:
        for state in (1, 0, 1):
            bs.set_option(bs.OPT_F32_STATE, state)
            for t, ref, wsrc in ((t32, xr32, w32), (t64, xr, ws)):
                say(f"shared workspace: state={state} dtype={t['y'].dtype}")
                x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=batch, workspace=wsb)
                torch.cuda.synchronize()
                assert (info.cpu().numpy() == 0).all()
                assert (wsb.view(torch.int32)[:lead] == 0).all()
                if t is t64:
                    assert rel_err(host(x, batch), ref).max() <= TOL
                else:
                    check_fp32(wsrc, kind, host(x, batch), ref, state, dominant=True)
    finally:
        bs.set_option(bs.OPT_F32_STATE, 1)


def test_compact_state_gave_up_waiting_is_redone():
    """The compact-state kernels under forced give-ups (no time to wait for
    the other blocks of a system): the FP32 solve redoes the rows of the
    blocks that gave up sequentially (FP64 on the FP32 values), and in the
    refinement, whose solves add d into x, the redo adds too; every system
    reports 0, the results meet their bars, and the meeting counters are clean."""
    kind, n, batch = 5, 2048, 96
    ws = wl.dominant_batch(batch, n, kind=kind, seed=88)
    w32 = fp32_rounded(ws)
    xr32, _ = oracle_direct(w32, kind)
    xr, _ = oracle_direct(ws, kind)
    t32 = to_device(w32, batch, dtype=torch.float32)
    t64 = to_device(ws, batch)
    lead = (batch + 15) // 16 * 4
    nb = bs.workspace_bytes(bs.OP_SOLVE, kind, n, batch, bs.BS_F32)
    w_s = torch.zeros((nb + 7) // 8, dtype=torch.float64, device="cuda")
    nb = bs.workspace_bytes(bs.OP_REFINE, kind, n, batch, ld=t64["y"].shape[1])
    w_r = torch.zeros((nb + 7) // 8, dtype=torch.float64, device="cuda")
    try:
        bs.set_option(bs.OPT_EXCHANGE_WAIT_US, 0)
        for rep in range(5):
            say(f"compact state, no wait: rep {rep}")
            x, info = bs.solve(diags_of(t32, kind), t32["y"], kind=kind, batch=batch, workspace=w_s)
            torch.cuda.synchronize()
            assert (info.cpu().numpy() == 0).all()
            assert (w_s.view(torch.int32)[:lead] == 0).all()
            check_fp32(w32, kind, host(x, batch), xr32, 1, dominant=True)
            xi, steps, relres, info = bs.refine(diags_of(t64, kind), t64["y"], batch=batch,
                                                tol=1e-12, max_steps=6, workspace=w_r)
            torch.cuda.synchronize()
            assert (info.cpu().numpy() == 0).all() and (relres.cpu().numpy() < 1e-12).all()
            assert (w_r.view(torch.int32)[:lead] == 0).all()
            assert rel_err(host(xi, batch), xr).max() <= 1e-11
    finally:
        bs.set_option(bs.OPT_EXCHANGE_WAIT_US, 1000000)


def test_fp32_pde_lines_and_in_place(f32_state):
    """Second-order (non-dominant boundary) PDE rows in FP32 storage on the
    full 2048 x 2048 sweep batch the benchmark times, every element of every
    system; x may alias rhs."""
    pd, td, _ = wl.config1()
    for kind, ws in ((5, fp32_rounded(pd)), (3, fp32_rounded(td))):
        say(f"fp32 sweep batch kind={kind} state={f32_state}")
        t = to_device(ws, 2048, dtype=torch.float32)
        y = t["y"].clone()
        x, info = bs.solve(diags_of(t, kind), y, y, kind=kind, batch=2048)
        torch.cuda.synchronize()
        xr, _ = oracle_direct(ws, kind)
        assert (info.cpu().numpy() == 0).all()
        check_fp32(ws, kind, host(x, 2048), xr, f32_state, dominant=False)


# ---------------------------------------------------- long systems, FP64 ---
@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("n,batch,ld", [(4097, 5, 64), (5000, 33, 40), (20000, 17, 64),
                                        (70001, 2, 2)])
def test_long_path_parity(kind, n, batch, ld):
    ws = wl.dominant_batch(batch, n, kind=kind, seed=4000 + n + batch)
    say(f"long kind={kind} n={n} batch={batch} ld={ld}")
    t = to_device(ws, batch, ld=ld, corner_nan=True, pad_fill=np.nan)
    x0 = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    x, info = bs.solve(diags_of(t, kind), t["y"], x0, kind=kind, batch=batch)
    torch.cuda.synchronize()
    xr, ir = oracle_direct(ws, kind)
    assert (info.cpu().numpy() == 0).all() and (ir == 0).all()
    err = rel_err(host(x, batch), xr)
    say(f"  max rel err {err.max():.3e}")
    assert err.max() <= TOL
    if ld > batch:
        assert (x[:, batch:] == 7.0).all()


def test_long_path_pde_lines():
    """ADI lines of length 1e5 (r = 4): PD second-order and TD first-order."""
    v = wl.smooth_lines(16, 100_000, 77)
    for kind, order in ((5, 2), (3, 1)):
        ws = wl.sweep_lines(v, 4.0, order)
        t = to_device(ws, 16, ld=64)
        x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=16)
        torch.cuda.synchronize()
        xr, _ = oracle_direct(ws, kind)
        err = rel_err(host(x, 16), xr)
        say(f"pde lines kind={kind} n=1e5 max rel err {err.max():.3e}")
        assert (info.cpu().numpy() == 0).all() and err.max() <= TOL


def test_long_path_pivots_reported():
    ws = wl.dominant_batch(3, 9000, kind=5, seed=8)
    ws["d"][0, 0] = 0.0
    ws["d"][1, 4500] = np.inf
    for kind in (5, 3):
        t = to_device(ws, 3)
        _, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=3)
        got = info.cpu().numpy().tolist()
        say(f"long pivots kind={kind}: {got}")
        assert got == [1, 4501, 0]


def test_long_path_workspace_reuse_and_graph_replay():
    ws = wl.dominant_batch(40, 12345, kind=5, seed=9)
    t = to_device(ws, 40, ld=64)
    xr, _ = oracle_direct(ws, 5)
    nbytes = bs.workspace_bytes(bs.OP_SOLVE, 5, 12345, 40, ld=64)
    wsb = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    x = torch.empty_like(t["y"])
    info = torch.empty(40, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bs.solve(diags_of(t), t["y"], x, batch=40, info=info, workspace=wsb, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert (info.cpu() == 0).all() and rel_err(host(x, 40), xr).max() <= TOL, rep
        bs.solve(diags_of(t), t["y"], x, batch=40, info=info, workspace=wsb)   # eager between


# ------------------------------------------------------------- refinement ---
def refine_check(ws, kind, batch, tol, err_bar, max_steps=8, ld=None):
    t = to_device(ws, batch, ld=ld, corner_nan=True)
    x, steps, relres, info = bs.refine(diags_of(t, kind), t["y"], kind=kind, batch=batch,
                                       tol=tol, max_steps=max_steps)
    torch.cuda.synchronize()
    xr, _ = oracle_direct(ws, kind)
    xg = host(x, batch)
    err = rel_err(xg, xr)
    st, rr, inf = steps.cpu().numpy(), relres.cpu().numpy(), info.cpu().numpy()
    hr = host_residual(ws, kind, xg)
    say(f"  steps {np.bincount(st).tolist()} relres max {rr.max():.2e} host {hr.max():.2e} "
        f"err vs oracle {err.max():.2e}")
    assert (inf == 0).all()
    assert (rr < tol).all() and (hr < 1.01 * tol).all()
    assert err.max() <= err_bar
    return st


@pytest.mark.parametrize("kind", [5, 3])
def test_refine_dominant(kind, f32_state):
    ws = wl.dominant_batch(45, 1999, kind=kind, seed=51)
    say(f"refine dominant kind={kind} state={f32_state}")
    # kappa_inf of these matrices is below 10: error <= kappa * tol
    st = refine_check(ws, kind, 45, 1e-12, 1e-11, ld=64)
    assert st.max() <= 3


def test_refine_config1_pde_to_1e10(f32_state):
    pd, td, _ = wl.config1()
    for kind, ws in ((5, pd), (3, td)):
        say(f"refine config1 kind={kind} n=2048 batch=2048 state={f32_state}")
        # r = 4 lines: kappa_inf <= 164, so relres < 1e-10 bounds the error by 2e-8
        st = refine_check(ws, kind, 2048, 1e-10, 2e-8)
        assert st.max() <= 3


def test_refine_long_stiff_lines():
    """r = 2047 (kappa_inf ~ 1e6): more steps, same stopping rule."""
    v = wl.smooth_lines(8, 100_000, 91)
    ws = wl.sweep_lines(v, 2047.0, 2)
    say("refine r=2047 n=1e5 kind=5")
    st = refine_check(ws, 5, 8, 1e-10, 1e-3)
    assert st.max() <= 6


def test_refine_status_cases(f32_state):
    ws = wl.dominant_batch(6, 300, kind=5, seed=61)
    ws["y"][2] = 0.0                   # zero rhs: x = 0 after one solve, relres 0
    ws["d"][4, 0] = 0.0                # bad pivot of the FP32 elimination at row 0
    t = to_device(ws, 6)
    x, steps, relres, info = bs.refine(diags_of(t), t["y"], batch=6, tol=1e-12, max_steps=8)
    torch.cuda.synchronize()
    i, st, rr = info.cpu().numpy(), steps.cpu().numpy(), relres.cpu().numpy()
    say(f"refine status info={i.tolist()} steps={st.tolist()}")
    assert i[4] == 1 and st[4] == 1
    assert i[2] == 0 and st[2] == 1 and rr[2] == 0.0 and (host(x, 6)[2] == 0).all()
    assert (np.delete(i, 4) == 0).all()
    # one step cannot reach 1e-15: not converged, relres reported
    _, steps, relres, info = bs.refine(diags_of(t), t["y"], batch=6, tol=1e-15, max_steps=1)
    torch.cuda.synchronize()
    i = info.cpu().numpy()
    assert i[4] == 1 and i[2] == 0 and (np.delete(i, [2, 4]) == -1).all()
    assert (steps.cpu().numpy() == 1).all()


def test_refine_graph_replay(f32_state):
    ws = wl.dominant_batch(64, 3000, kind=5, seed=71)
    t = to_device(ws, 64)
    xr, _ = oracle_direct(ws, 5)
    nbytes = bs.workspace_bytes(bs.OP_REFINE, 5, 3000, 64)
    wsb = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    x = torch.empty_like(t["y"])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            out = bs.refine(diags_of(t), t["y"], x, batch=64, tol=1e-12, max_steps=6,
                            workspace=wsb, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    _, steps, relres, info = out
    for rep in range(3):
        x.fill_(123.0)
        g.replay()
        torch.cuda.synchronize()
        assert (info.cpu() == 0).all(), rep
        assert (relres.cpu() < 1e-12).all(), rep
        assert rel_err(host(x, 64), xr).max() <= 1e-11, rep
        bs.refine(diags_of(t), t["y"], x, batch=64, tol=1e-12, workspace=wsb)  # eager between


# ------------------------------------------------ full-size n = 1e6 batch ---
@pytest.fixture(scope="module")
def c3():
    """256 PD lines of length 1e6 (r = 4), built in device memory by the
    interleaved generator; the sampled systems are rebuilt on the host."""
    nsys, n = 256, 1_000_000
    v = wl.smooth_lines(nsys, n, wl.BASE_SEED + 3)
    vt = torch.from_numpy(np.ascontiguousarray(v.T)).cuda()
    dev = wl.sweep_lines_interleaved(vt, 4.0, 2)
    del vt
    sample = [0, 1, 77, 128, 200, 255]
    hostws = wl.sweep_lines(v[sample], 4.0, 2)
    for k in KEYS:   # the device batch holds exactly the host values
        assert np.array_equal(dev[k][:, sample].cpu().numpy().T, hostws[k]), k
    return dev, hostws, sample


def test_full_size_1e6_fp64_sampled(c3):
    dev, hostws, sample = c3
    say("n=1e6 batch=256 FP64 split path")
    x, info = bs.solve(diags_of(dev), dev["y"], batch=256)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    xr, _ = oracle_direct(hostws, 5)
    err = rel_err(x[:, sample].cpu().numpy().T, xr)
    say(f"  sampled max rel err {err.max():.3e}")
    assert err.max() <= TOL


def test_full_size_1e6_refine_sampled(c3):
    dev, hostws, sample = c3
    say("n=1e6 batch=256 FP32 + refinement to 1e-10")
    x, steps, relres, info = bs.refine(diags_of(dev), dev["y"], batch=256, tol=1e-10)
    torch.cuda.synchronize()
    st, rr = steps.cpu().numpy(), relres.cpu().numpy()
    assert (info.cpu().numpy() == 0).all() and (rr < 1e-10).all()
    xr, _ = oracle_direct(hostws, 5)
    xs = x[:, sample].cpu().numpy().T
    err = rel_err(xs, xr)
    hr = host_residual(hostws, 5, xs)
    say(f"  steps {np.bincount(st).tolist()} relres max {rr.max():.2e} host {hr.max():.2e} "
        f"sampled err vs oracle {err.max():.2e}")
    assert (hr < 1.01e-10).all() and err.max() <= 2e-8 and st.max() <= 3
