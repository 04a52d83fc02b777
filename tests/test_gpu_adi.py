"""GPU parity of the ADI sweep assembled inside the solver (band_solve_adi):
bitwise the split solve of the host-generated sweep coefficients, and within
the FP64 bar of the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, host, rel_err, say

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.mark.parametrize("kind,order", [(5, 2), (3, 1)])
def test_sweep_batch_2048(kind, order):
    """The y-sweep of the 2048 x 2048 field: the lines are the columns of u."""
    u0 = wl.smooth_field(2048, wl.BASE_SEED + 1)
    v = torch.from_numpy(u0).cuda()
    x, info = bs.solve_adi(v, 4.0, kind=kind)
    sw = wl.sweep_lines_interleaved(v, 4.0, order)
    xr, inf2 = bs.solve(diags_of(sw, kind), sw["y"], kind=kind, batch=2048)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all() and (inf2.cpu().numpy() == 0).all()
    assert torch.equal(x, xr)                       # same coefficients, same elimination
    ws = wl.adi_sweep(u0, 4.0, order, "y")
    if kind == 5:
        xo, _ = oracle.npdm_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"])
    else:
        xo, _ = oracle.ntdm_batch(ws["c"], ws["d"], ws["a"], ws["y"])
    err = rel_err(host(x, 2048), xo)
    say(f"adi kind={kind}: max rel err vs oracle {err.max():.2e}")
    assert err.max() <= TOL


@pytest.mark.parametrize("kind,order", [(5, 2), (3, 1)])
@pytest.mark.parametrize("n,batch,ld", [(8, 3, 64), (513, 33, 40), (2047, 17, 17), (4096, 20, 64)])
def test_shapes_padding_and_in_place(kind, order, n, batch, ld):
    lines = wl.smooth_lines(batch, n, 700 + n)            # [batch, n]
    vt = np.full((n, ld), np.nan)
    vt[:, :batch] = lines.T
    v = torch.from_numpy(vt).cuda()
    x, info = bs.solve_adi(v, 4.0, torch.full_like(v, 7.0), kind=kind, batch=batch)
    y = v.clone()
    x2, _ = bs.solve_adi(y, 4.0, y, kind=kind, batch=batch)    # x aliases v
    torch.cuda.synchronize()
    ws = wl.sweep_lines(lines, 4.0, order)
    if kind == 5:
        xo, _ = oracle.npdm_batch(ws["e"], ws["c"], ws["d"], ws["a"], ws["b"], ws["y"])
    else:
        xo, _ = oracle.ntdm_batch(ws["c"], ws["d"], ws["a"], ws["y"])
    assert (info.cpu().numpy() == 0).all()
    assert rel_err(host(x, batch), xo).max() <= TOL
    assert torch.equal(x[:, :batch], x2[:, :batch])
    assert (x[:, batch:] == 7.0).all()              # padding columns never written


def test_length_beyond_split_variants_rejected():
    v = torch.zeros((5000, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(bs.BandSolveError):
        bs.solve_adi(v, 4.0)


def test_ten_adi_steps_against_the_oracle():
    """Ten time steps of the nonlinear ADI run on a 96 x 96 grid, every sweep
    on the GPU (coefficients, split-row solve, device layout conversion
    between sweeps), against the same run with the host generator and the
    oracle: the x-sweep solution of every step within the FP64 bar."""
    N, steps = 96, 10
    from paper_1804_09666_amd import warmstart as wsm
    got = []
    wsm.adi_trajectory(N, steps, r=4.0, on_xsweep=lambda k, planes, w: got.append(w.clone()))
    u = wl.smooth_field(N, wl.BASE_SEED + 4)      # [y, x], the trajectory's seed
    for k in range(steps):
        sx = wl.sweep_lines(u, 4.0, 2)            # lines along x, one per y
        w, info = oracle.npdm_batch(sx["e"], sx["c"], sx["d"], sx["a"], sx["b"], sx["y"])
        assert (info == 0).all()
        wg = host(got[k], N)                      # interleaved [x][y] -> [y][x]
        err = np.abs(wg - w).max() / np.abs(w).max()
        say(f"step {k}: x-sweep rel err vs oracle {err:.2e}")
        assert err <= TOL * (k + 1)
        sy = wl.sweep_lines(w.T.copy(), 4.0, 2)   # lines along y, one per x
        ut, info = oracle.npdm_batch(sy["e"], sy["c"], sy["d"], sy["a"], sy["b"], sy["y"])
        assert (info == 0).all()
        u = ut.T.copy()
