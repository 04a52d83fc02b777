"""Breakdown of NPDM / NTDM (LU without pivoting, Sec. 1) on the default
split-row solver: a system whose partitioned elimination meets a zero, tiny
or non-finite pivot is solved again with the sequential recurrence, so its x
and info are the sequential method's (bitwise the oracle's).  A sequential
pivot that cancels deep inside a chunk is met by the chunk's own recurrence
too (it has forgotten its start by then) and is reported exactly; one that
cancels in the first row of a chunk other than the first is not met by the
partitioned elimination, which solves the (regular) system instead.
Everything goes through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, host, rel_err, say, to_device

pytestmark = pytest.mark.gpu

TOL = 1e-12
KEYS = ("e", "c", "d", "a", "b", "y")


def oracle_direct(ws, kind, s=None):
    sl = slice(None) if s is None else s
    if kind == 5:
        return oracle.npdm(*[ws[k][sl] for k in KEYS], return_mu=True)
    return oracle.ntdm(*[ws[k][sl] for k in ("c", "d", "a", "y")], return_mu=True)


def fresh(batch, n, kind, seed):
    ws = wl.dominant_batch(batch, n, kind=kind, seed=seed)
    return {k: np.array(ws[k]) for k in KEYS}


def cancel_pivot(ws, s, i, kind):
    """Make the sequential pivot mu_i of system s exactly zero: with e_i = 0
    and b_{i-2} = 0, mu_i = d_i - alpha_{i-1} c_i and alpha_{i-1} =
    a_{i-1} / mu_{i-1} (IEEE operations, as Python floats)."""
    if kind == 5:
        ws["e"][s, i] = 0.0
        ws["b"][s, i - 2] = 0.0
    _, info, mu = oracle_direct(ws, kind, s)
    assert info == 0
    alpha = float(ws["a"][s, i - 1]) / float(mu[i - 1])
    ws["d"][s, i] = alpha * float(ws["c"][s, i])
    _, info, _ = oracle_direct(ws, kind, s)
    assert info == i + 1, (info, i)


def run(ws, kind, batch, dtype=torch.float64):
    t = to_device(ws, batch, dtype=dtype)
    x, info = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=batch)
    torch.cuda.synchronize()
    return host(x, batch), info.cpu().numpy()


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("value", [0.0, 1e-14])
def test_chunk_start_pivot_is_redone(kind, value):
    """A zero or 1e-14 diagonal at the first row of a chunk (row 32: second
    chunk of the first tile; 512 and 1536: first chunk of a later tile) is a
    bad local pivot of the partitioned elimination, while the sequential
    pivot there is regular: info = 0 and x is the oracle's, bitwise."""
    batch, n = 64, 2048
    ws = fresh(batch, n, kind, 41)
    hit = {3: 32, 17: 512, 40: 1536, 63: 32}
    for s, i in hit.items():
        ws["d"][s, i] = value
    xr, ir, _ = oracle_direct(ws, kind)
    assert (ir == 0).all()
    x, info = run(ws, kind, batch)
    say(f"kind {kind} d={value}: info {np.unique(info).tolist()}")
    assert (info == 0).all()
    for s in hit:
        assert np.array_equal(x[s], xr[s]), s              # the sequential redo
    assert rel_err(x, xr).max() <= TOL


@pytest.mark.parametrize("kind", [5, 3])
@pytest.mark.parametrize("state", [1, 0])
def test_fp32_storage_redo(kind, state):
    """The same with FP32 storage, with the compact (1) and the FP64 (0)
    chunk state: the redo runs the sequential recurrence in FP64 on the FP32
    values, so x is the oracle's solution of the FP32-valued system, rounded
    once to FP32.  Rows 64 and 512 start a chunk in both states (64 and 32
    rows per chunk)."""
    batch, n = 32, 2048
    ws = fresh(batch, n, kind, 42)
    ws32 = {k: ws[k].astype(np.float32).astype(np.float64) for k in KEYS}
    for s, i in {1: 64, 9: 512}.items():
        ws32["d"][s, i] = 0.0
    xr, ir, _ = oracle_direct(ws32, kind)
    assert (ir == 0).all()
    bs.set_option(bs.OPT_F32_STATE, state)
    try:
        x, info = run(ws32, kind, batch, torch.float32)
    finally:
        bs.set_option(bs.OPT_F32_STATE, 1)
    assert (info == 0).all()
    for s in (1, 9):
        assert np.array_equal(x[s], xr[s].astype(np.float32).astype(np.float64)), s


@pytest.mark.parametrize("kind", [5, 3])
def test_deep_cancellation_reported_exactly(kind):
    """mu_i = 0 exactly at rows well inside a chunk (row 568 = chunk 17's
    row 24, row 88 = chunk 2's row 24): the chunk's recurrence meets it too,
    so the system is redone and reports the oracle's info, i + 1."""
    batch, n = 16, 2048
    ws = fresh(batch, n, kind, 43)
    cancel_pivot(ws, 2, 568, kind)
    cancel_pivot(ws, 11, 88, kind)
    xr, ir, _ = oracle_direct(ws, kind)
    x, info = run(ws, kind, batch)
    say(f"kind {kind} deep cancellation: gpu {info[[2, 11]].tolist()} oracle {ir[[2, 11]].tolist()}")
    assert np.array_equal(info, ir)
    ok = ir == 0
    assert rel_err(x[ok], xr[ok]).max() <= TOL


@pytest.mark.parametrize("kind", [5, 3])
def test_cancellation_at_chunk_start(kind):
    """mu_i = 0 exactly at the first row of a later tile (row 512): the
    partitioned elimination starts that chunk afresh and never meets the
    vanishing leading minor, so it solves the system, which is regular
    there: info = 0 and x matches a dense LU solve with partial pivoting.
    With one lane per system the sequential recurrence reports row 513."""
    batch, n = 8, 1024
    ws = fresh(batch, n, kind, 44)
    i = 512
    cancel_pivot(ws, 5, i, kind)
    x, info = run(ws, kind, batch)
    A = np.diag(ws["d"][5]) + np.diag(ws["c"][5, 1:], -1) + np.diag(ws["a"][5, :-1], 1)
    if kind == 5:
        A += np.diag(ws["e"][5, 2:], -2) + np.diag(ws["b"][5, :-2], 2)
    xd = np.linalg.solve(A, ws["y"][5])
    kappa = np.linalg.cond(A, np.inf)
    err = np.abs(x[5] - xd).max() / np.abs(xd).max()
    say(f"kind {kind} cancellation at a tile start: info {info[5]}, err {err:.2e}, "
        f"kappa {kappa:.1e}")
    assert info[5] == 0 and err <= 1e-14 * kappa
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
    try:
        _, info_lane = run(ws, kind, batch)
    finally:
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
    assert info_lane[5] == i + 1 and (np.delete(info_lane, 5) == 0).all()


@pytest.mark.parametrize("kmax", [2, 20])
def test_mnpdm_redo(kmax):
    """MNPDM on the split kernels: a zero diagonal at a chunk start is redone
    sequentially with the outer entries taken from the list (kmax 2: each
    lane scans the list; 20: the list staged in LDS, unused entries -1)."""
    batch, n = 16, 2048
    ws = wl.sweep_lines(wl.smooth_lines(batch, n, 45), 4.0, 2)
    ws = {k: np.array(ws[k]) for k in KEYS}
    ws["d"][4, 512] = 0.0
    ws["d"][9, 32] = 0.0
    xr, ir, _ = oracle_direct(ws, 5)
    assert (ir == 0).all()
    t = to_device(ws, batch)
    ld = t["y"].shape[1]
    rows = np.full((kmax, ld), -1, dtype=np.int32)
    oe = np.zeros((kmax, ld))
    ob = np.zeros((kmax, ld))
    rows[0, :batch], ob[0, :batch] = 0, ws["b"][:, 0]
    rows[1, :batch], oe[1, :batch] = n - 1, ws["e"][:, n - 1]
    dev = lambda a: torch.from_numpy(a).cuda()
    x, info = bs.solve_mnpdm([t["c"], t["d"], t["a"]], dev(rows), dev(oe), dev(ob), t["y"],
                             batch=batch)
    torch.cuda.synchronize()
    x = host(x, batch)
    assert (info.cpu().numpy() == 0).all()
    for s in (4, 9):
        assert np.array_equal(x[s], xr[s]), s
    assert rel_err(x, xr).max() <= TOL


@pytest.mark.parametrize("kind", [5, 3])
def test_long_path_redo(kind):
    """Systems longer than one launch's tiles (three launches and the redo):
    a zero diagonal at a tile start is redone (info 0, x bitwise the
    oracle's), a deep cancellation is reported exactly."""
    batch, n = 6, 6000
    ws = fresh(batch, n, kind, 46)
    ws["d"][1, 512] = 0.0
    ws["d"][4, 4096] = 1e-14
    cancel_pivot(ws, 3, 2264, kind)            # row 24 of the chunk at 2240
    xr, ir, _ = oracle_direct(ws, kind)
    x, info = run(ws, kind, batch)
    say(f"long kind {kind}: gpu {info.tolist()} oracle {ir.tolist()}")
    assert np.array_equal(info, ir) and ir[3] == 2265
    for s in (1, 4):
        assert np.array_equal(x[s], xr[s]), s
    ok = ir == 0
    assert rel_err(x[ok], xr[ok]).max() <= TOL


def test_varlen_redo():
    """Uneven batch: a system with a zero diagonal at a tile start is redone
    sequentially (x bitwise the oracle's), the others are untouched."""
    sizes = np.array([3000, 700, 5000, 64, 1500, 2049], dtype=np.int64)
    systems = []
    for k, n in enumerate(sizes):
        w = wl.dominant_batch(1, int(n), kind=5, seed=470 + k)
        systems.append({key: np.array(w[key][0]) for key in KEYS})
    systems[2]["d"][512] = 0.0
    systems[5]["d"][1024] = 1e-14
    plan = bs.Varlen(sizes)
    arrs = {k: torch.from_numpy(plan.pack([s[k] for s in systems], fill=np.nan)).cuda()
            for k in KEYS}
    diags = [arrs["e"], arrs["c"], arrs["d"], arrs["a"], arrs["b"]]
    refs = [oracle.npdm(*[s[k] for k in KEYS]) for s in systems]
    for v in range(len(plan.variants())):
        x, info = plan.solve(5, diags, arrs["y"], variant=v)
        torch.cuda.synchronize()
        got = plan.unpack(x.cpu().numpy())
        inf = info.cpu().numpy()[plan.slot]
        assert (inf == 0).all(), (v, inf)
        for i, (xr, ir) in enumerate(refs):
            assert ir == 0
            if i in (2, 5):
                assert np.array_equal(got[i], xr), (v, i)
            assert np.abs(got[i] - xr).max() <= TOL * np.abs(xr).max()


@pytest.mark.parametrize("variant", [0, 1])
def test_gave_up_waiting_is_redone(variant):
    """With no time to wait (BS_OPT_EXCHANGE_WAIT_US = 0) most blocks give up
    on the others of their system and write no x; the last block of each
    group solves the rows of the blocks that gave up sequentially, so every
    system reports 0 and is solved, and the meeting counters are clean
    afterwards.  With x aliasing the rhs that is impossible (the other
    blocks have overwritten rhs rows): such systems report -4."""
    batch, n = 64, (2048, 4096)[variant]         # four and eight blocks per system
    ws = wl.dominant_batch(batch, n, kind=5, seed=77)
    t = to_device(ws, batch)
    xr, _ = oracle.npdm_batch(*[ws[k] for k in KEYS])
    bs.set_option(bs.OPT_PART_PD_VARIANT, variant)
    nbytes = bs.workspace_bytes(bs.OP_SOLVE, 5, n, batch)
    wsb = torch.zeros((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    x = torch.empty_like(t["y"])
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    groups = -(-batch // bs.part_variants(5)[variant][2])
    rt = bs.part_variants(5)[variant][0] * bs.part_variants(5)[variant][1]
    try:
        bs.set_option(bs.OPT_EXCHANGE_WAIT_US, 0)
        redone_tiles = timeouts = 0
        for _ in range(10):
            x.fill_(np.nan)
            bs.solve(diags_of(t), t["y"], x, batch=batch, info=info, workspace=wsb)
            torch.cuda.synchronize()
            got = info.cpu().numpy()
            xh = host(x, batch)
            assert (got == 0).all() and rel_err(xh, xr).max() <= TOL
            assert (wsb.view(torch.int32)[: 4 * groups] == 0).all()
            # tiles written by the sequential redo hold the oracle's x bitwise
            same = (xh == xr).reshape(batch, -1, rt).all(axis=2)
            redone_tiles += int(same.sum())
            y = t["y"].clone()
            bs.solve(diags_of(t), y, y, batch=batch, info=info, workspace=wsb)
            torch.cuda.synchronize()
            got = info.cpu().numpy()
            assert set(np.unique(got)) <= {0, -4}
            ok = got == 0
            timeouts += int((~ok).sum())
            assert rel_err(host(y, batch)[ok], xr[ok]).max(initial=0.0) <= TOL
            assert (wsb.view(torch.int32)[: 4 * groups] == 0).all()
        say(f"variant {variant}: {redone_tiles} tiles redone; aliased rhs: {timeouts} "
            f"of {10 * batch} systems gave up")
        assert redone_tiles > 0
    finally:
        bs.set_option(bs.OPT_EXCHANGE_WAIT_US, 1000000)
        bs.set_option(bs.OPT_PART_PD_VARIANT, 0)
    bs.solve(diags_of(t), t["y"], x, batch=batch, info=info, workspace=wsb)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    assert rel_err(host(x, batch), xr).max() <= TOL


@pytest.mark.parametrize("kind", [5, 3])
def test_adi_gave_up_waiting_is_redone(kind):
    """The assembled ADI sweep under forced give-ups: the redo assembles its
    rows from v the same way, so x matches the solve with the default wait."""
    n, batch = 2048, 256
    v = torch.from_numpy(wl.interleave(wl.smooth_lines(batch, n, 48))).cuda()
    xd, info = bs.solve_adi(v, 4.0, kind=kind)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    try:
        bs.set_option(bs.OPT_EXCHANGE_WAIT_US, 0)
        x, info = bs.solve_adi(v, 4.0, kind=kind)
        torch.cuda.synchronize()
    finally:
        bs.set_option(bs.OPT_EXCHANGE_WAIT_US, 1000000)
    assert (info.cpu().numpy() == 0).all()
    assert rel_err(host(x, batch), host(xd, batch)).max() <= 1e-13
