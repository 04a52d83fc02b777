"""GPU parity of the uneven-batch solver (systems of different lengths in one
solve) against the FP64 oracle, every compiled tile shape, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import say

pytestmark = pytest.mark.gpu
TOL = 1e-12
KEYS = ("e", "c", "d", "a", "b", "y")


def make_batch(sizes, kind, seed):
    rng = np.random.default_rng(seed)
    systems = []
    for k, n in enumerate(sizes):
        ws = wl.dominant_batch(1, int(n), kind=kind, seed=int(rng.integers(1 << 30)))
        systems.append({key: ws[key][0] for key in KEYS})
    return systems


def solve_oracle(sysd, kind):
    if kind == 5:
        return oracle.npdm(*[sysd[k] for k in KEYS])[0]
    return oracle.ntdm(sysd["c"], sysd["d"], sysd["a"], sysd["y"])[0]


def to_dev(plan, systems, kind):
    arrs = {}
    for k in KEYS:
        if kind == 3 and k in ("e", "b"):
            continue
        arrs[k] = torch.from_numpy(plan.pack([s[k] for s in systems], fill=np.nan)).cuda()
    diags = [arrs.get("e"), arrs["c"], arrs["d"], arrs["a"], arrs.get("b")]
    return diags, arrs["y"]


@pytest.mark.parametrize("kind", [5, 3])
def test_uneven_batch_every_variant(kind):
    rng = np.random.default_rng(7 + kind)
    sizes = np.floor(np.exp(rng.uniform(np.log(8), np.log(20000), 75))).astype(np.int64)
    sizes[:3] = [8, 512, 513]        # tile boundaries and the minimum length
    systems = make_batch(sizes, kind, 100 + kind)
    plan = bs.Varlen(sizes)
    diags, y = to_dev(plan, systems, kind)
    refs = [solve_oracle(s, kind) for s in systems]
    for v, shape in enumerate(plan.variants()):
        x = torch.full_like(y, 7.0)
        x, info = plan.solve(kind, diags, y, x, variant=v)
        torch.cuda.synchronize()
        inf = info.cpu().numpy()
        got = plan.unpack(x.cpu().numpy())
        err = max(np.abs(g - r).max() / np.abs(r).max() for g, r in zip(got, refs))
        say(f"varlen kind={kind} variant {v} {shape}: max rel err {err:.2e}")
        assert (inf[plan.slot] == 0).all() and err <= TOL
        used = np.zeros(plan.elems, dtype=bool)
        for i in range(plan.count):
            used[plan.offset[i] + 16 * np.arange(sizes[i])] = True
        assert (x.cpu().numpy()[~used] == 7.0).all()      # nothing outside the systems written


def test_uneven_pde_lines_and_pivots():
    rng = np.random.default_rng(3)
    sizes = np.floor(np.exp(rng.uniform(np.log(64), np.log(65536), 40))).astype(np.int64)
    systems = []
    for k, n in enumerate(sizes):
        ws = wl.sweep_lines(wl.smooth_lines(1, int(n), 50 + k), 4.0, 2)
        systems.append({key: ws[key][0] for key in KEYS})
    systems[5]["d"][0] = 0.0           # first pivot zero in system 5
    plan = bs.Varlen(sizes)
    diags, y = to_dev(plan, systems, 5)
    x, info = plan.solve(5, diags, y)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()[plan.slot]
    got = plan.unpack(x.cpu().numpy())
    say(f"PDE lines: info of system 5 = {inf[5]}")
    assert inf[5] == 1 and (np.delete(inf, 5) == 0).all()
    for i, s in enumerate(systems):
        if i == 5:
            continue
        r = solve_oracle(s, 5)
        assert np.abs(got[i] - r).max() <= TOL * np.abs(r).max()


def test_autotuner_and_graph_replay():
    rng = np.random.default_rng(11)
    sizes = np.floor(np.exp(rng.uniform(np.log(64), np.log(65536), 300))).astype(np.int64)
    systems = make_batch(sizes, 5, 9)
    plan = bs.Varlen(sizes)
    diags, y = to_dev(plan, systems, 5)
    x = torch.empty_like(y)
    info = torch.empty(plan.slots, dtype=torch.int32, device="cuda")
    ws = plan.workspace(5)
    best, ms = plan.tune(5, diags, y, x, info, ws, reps=3)
    say(f"autotuner: best variant {best}, ms per variant {ms}")
    assert 0 <= best < len(plan.variants()) and all(t > 0 for t in ms)
    ref, _ = plan.solve(5, diags, y, torch.empty_like(y), variant=best, workspace=ws)
    torch.cuda.synchronize()
    ref = plan.unpack(ref.cpu().numpy())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.solve(5, diags, y, x, info, variant=best, workspace=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = plan.unpack(x.cpu().numpy())
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), rep
        assert (info.cpu().numpy()[plan.slot] == 0).all()


def test_full_size_uneven_batch():
    """The uneven-batch workload at full size: 10 000 dominant PD systems with
    n log-uniform in [64, 65536] (about 1e8 rows), generated on the device,
    solved with the tile shape the autotuner picks (the measured launch).
    Every system against its manufactured solution (dominant, so the error
    is a few ulps of max|x|), sampled systems against the oracle."""
    sizes = wl.config2_sizes()
    plan = bs.Varlen(sizes)
    dev = wl.dominant_groups(plan.slot_sizes)
    say(f"uneven batch full size: {plan.count} systems, {int(sizes.sum())} rows, "
        f"{plan.elems} stored elements")
    diags = [dev[k] for k in ("e", "c", "d", "a", "b")]
    x = torch.zeros_like(dev["y"])
    info = torch.empty(plan.slots, dtype=torch.int32, device="cuda")
    ws = plan.workspace(5)
    best, ms = plan.tune(5, diags, dev["y"], x, info, ws, reps=2)
    x.zero_()
    plan.solve(5, diags, dev["y"], x, info, variant=best, workspace=ws)
    torch.cuda.synchronize()
    say(f"  autotuner picked variant {best} ({ms})")
    assert (info.cpu().numpy()[plan.slot] == 0).all()
    # per-slot max |x - x_true| and max |x_true| (positions outside every
    # system hold 0 in x_true and are never written, so they add nothing)
    sn = torch.as_tensor(plan.slot_sizes, device="cuda")
    gn = sn.view(-1, 16).max(dim=1).values
    gid = torch.repeat_interleave(torch.arange(gn.numel(), device="cuda"), gn * 16)
    slot = gid * 16 + torch.arange(plan.elems, device="cuda") % 16
    err = torch.zeros(plan.slots, dtype=torch.float64, device="cuda")
    err.scatter_reduce_(0, slot, (x - dev["x_true"]).abs(), "amax")
    scale = torch.zeros(plan.slots, dtype=torch.float64, device="cuda")
    scale.scatter_reduce_(0, slot, dev["x_true"].abs(), "amax")
    rel = (err / scale.clamp_min(1e-300)).cpu().numpy()[plan.slot]
    say(f"  max rel err vs manufactured solution over all systems {rel.max():.2e}")
    assert rel.max() <= TOL
    pick = [int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 4242, 9999]
    for i in pick:
        pos = torch.as_tensor(plan.offset[i] + 16 * np.arange(sizes[i]), device="cuda")
        sysd = {k: dev[k].index_select(0, pos).cpu().numpy() for k in KEYS}
        r = solve_oracle(sysd, 5)
        got = x.index_select(0, pos).cpu().numpy()
        assert np.abs(got - r).max() <= TOL * np.abs(r).max(), i
