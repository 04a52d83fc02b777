"""band_solve_noalloc (the fused solve with the library's static scratch, for
callers that cannot allocate) against band_solve through the C ABI: two calls
in a row, the second with a smaller batch and shorter systems (so the second
call reuses the array the first one left behind), PD FP64 on the full sweep
batch, then TD, then FP32 storage.  Same kernels: x and info bitwise equal."""
import numpy as np
import pytest
import torch

from paper_1804_09666_amd import bandsolve as bs
from paper_1804_09666_amd import workloads as wl
from gpu_util import diags_of, say, to_device

pytestmark = pytest.mark.gpu


def both(ws, kind, batch, dtype=torch.float64):
    t = to_device(ws, batch, dtype=dtype)
    x_ref, i_ref = bs.solve(diags_of(t, kind), t["y"], kind=kind, batch=batch)
    x = torch.full_like(t["y"], 7.0)
    x, info = bs.solve_noalloc(diags_of(t, kind), t["y"], x, kind=kind, batch=batch)
    torch.cuda.synchronize()
    return x, info, x_ref, i_ref


def check(x, info, x_ref, i_ref, batch):
    ib = torch.int64 if x.dtype == torch.float64 else torch.int32
    assert torch.equal(info, i_ref)
    assert torch.equal(x[:, :batch].contiguous().view(ib), x_ref[:, :batch].contiguous().view(ib))


def test_noalloc_matches_band_solve_two_calls():
    pd, td, _ = wl.config1()
    say("noalloc: PD sweep batch n=2048 batch=2048")
    x, info, x_ref, i_ref = both(pd, 5, 2048)
    check(x, info, x_ref, i_ref, 2048)
    assert (info.cpu().numpy() == 0).all()
    small = wl.dominant_batch(100, 1000, kind=5, seed=90)
    small["d"][7, 500] = 0.0          # a chunk-start pivot: the sequential redo runs
    say("noalloc: PD n=1000 batch=100 (second call, smaller)")
    x, info, x_ref, i_ref = both(small, 5, 100)
    check(x, info, x_ref, i_ref, 100)
    say("noalloc: TD sweep batch")
    x, info, x_ref, i_ref = both(td, 3, 2048)
    check(x, info, x_ref, i_ref, 2048)
    say("noalloc: PD FP32 storage n=3000 batch=64")
    w32 = wl.dominant_batch(64, 3000, kind=5, seed=91)
    x, info, x_ref, i_ref = both(w32, 5, 64, torch.float32)
    check(x, info, x_ref, i_ref, 64)


def test_noalloc_rejects_oversize():
    """A shape whose scratch exceeds the static array is refused on the host."""
    n, batch = 4096, 4096
    t = {k: torch.zeros((n, batch), dtype=torch.float64, device="cuda") for k in
         ("e", "c", "d", "a", "b", "y")}
    assert bs.workspace_bytes(bs.OP_SOLVE, 5, n, batch) > bs.NOALLOC_SCRATCH_BYTES
    with pytest.raises(bs.BandSolveError) as exc:
        bs.solve_noalloc(diags_of(t), t["y"], batch=batch)
    assert exc.value.status == bs.BS_EWORKSPACE
