"""Benchmark: batched pentadiagonal NPDM solves of one ADI sweep (n = 2048,
2048 systems, FP64) on one MI355X, plus the other hot-path rows.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A timed step is one band_solve of the 2048 pentadiagonal systems (n = 2048)
of the first y-sweep of u_t = (k(u)u_x)_x + (k(u)u_y)_y, k = 1 + u^2, on a
2048 x 2048 grid (r = tau/h^2 = 4), inputs resident in HBM.  Steps rotate over
four copies of the inputs (4 x 235 MB, more than the 256 MB Infinity Cache)
so each step streams its operands from HBM.  Prints ONE JSON line.

Outside the timed region the run also measures the other rows of the hot
path on the same sweep (tridiagonal NTDM batch, MNPDM, band ILU(0), SIP with
Hotelling-Bodewig steps) and times the FP64 CPU oracle on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1804_09666_amd import bandsolve as bs  # noqa: E402
from paper_1804_09666_amd import workloads as wl  # noqa: E402

N_ROWS = 2048
BATCH = 2048
R_ADI = 4.0           # r = tau / h^2 of the sweep batch (--r)
SEED = None           # sweep-batch seed (--seed; None: the workloads' default)
HB_S = (3, 4)         # SIP-HB steps of the SIP row (--hb-s)
TOL = 1e-10           # SIP and refinement tolerance (--tol)
PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PD_BYTES_PER_ROW = 56            # e, c, d, a, b, y read + x written (FP64)
TD_BYTES_PER_ROW = 40            # c, d, a, y read + x written
ROTATE = 4
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_npdm_split_pd_n2048_b2048.txt")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1804_09666_amd", "csrc", f)
               for f in ("direct_part.hip", "split_core.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def to_dev(ws, keys=("e", "c", "d", "a", "b", "y")):
    return {k: torch.from_numpy(wl.interleave(ws[k])).cuda() for k in keys}


def diags_of(t, kind):
    if kind == 5:
        return [t["e"], t["c"], t["d"], t["a"], t["b"]]
    return [None, t["c"], t["d"], t["a"], None]


def timed_solves(sets, kind, steps, warmup, ws_buf, xs, info):
    """Warm up, then time `steps` solves: per-launch events plus the whole
    region, all on the current stream (the one the library launches on)."""
    stream = torch.cuda.current_stream()
    for w in range(warmup):
        t = sets[w % len(sets)]
        bs.solve(diags_of(t, kind), t["y"], xs[w % len(xs)], kind=kind, batch=BATCH,
                 info=info, workspace=ws_buf)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_all0.record(stream)
    for k in range(steps):
        t = sets[k % len(sets)]
        ev[k][0].record(stream)
        bs.solve(diags_of(t, kind), t["y"], xs[k % len(xs)], kind=kind, batch=BATCH,
                 info=info, workspace=ws_buf)
        ev[k][1].record(stream)
    t_all1.record(stream)
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in ev])   # ms
    return t_all0.elapsed_time(t_all1), per


def graph_solves(sets, kind, steps, ws_buf, xs, info):
    """The same `steps` solves captured once in a HIP graph (rotating input
    sets baked in); one untimed replay, then one timed replay.  Returns ms."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for k in range(steps):
                t = sets[k % len(sets)]
                bs.solve(diags_of(t, kind), t["y"], xs[k % len(xs)], kind=kind, batch=BATCH,
                         info=info, workspace=ws_buf, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    del g
    return e0.elapsed_time(e1)


def stream_ceiling(sets, reps=20):
    """GB/s of the library's plain streaming kernel over the same six input
    arrays and one output (the fused PD solve's bytes), rotating the sets."""
    keys = ("e", "c", "d", "a", "b", "y")
    k = [0]
    outs = [torch.empty_like(sets[0]["y"]) for _ in range(2)]

    def run():
        t = sets[k[0] % len(sets)]
        out = outs[k[0] % 2]
        k[0] += 1
        bs.stream_probe([t[q] for q in keys], out)
    ms = t_ms(run, reps=reps)
    return PD_BYTES_PER_ROW * N_ROWS * BATCH / ms / 1e6


def traffic_from_profile():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def config1():
    """The sweep batch (first y-sweep of the ADI step, n = batch = 2048)."""
    return wl.config1(r=R_ADI, N=N_ROWS) if SEED is None else wl.config1(r=R_ADI, N=N_ROWS,
                                                                        seed=SEED)


def cpu_baseline(pd, samples):
    """The CPU leg: the FP64 oracle (serial NPDM per system, OpenMP over
    systems) timed on the host cores on the full sweep batch, repeated to
    ~10 s of CPU work; it also solves the sampled systems (`samples`: name ->
    system-contiguous batch) whose GPU results are compared with it."""
    import oracle
    args = [np.ascontiguousarray(pd[k]) for k in ("e", "c", "d", "a", "b", "y")]
    nthreads = oracle.max_threads()
    oracle.npdm_batch(*args, nthreads=nthreads)          # warm-up
    t0 = time.perf_counter()
    oracle.npdm_batch(*args, nthreads=nthreads)
    one = time.perf_counter() - t0
    # about 10 s of CPU work in five timed runs; the median run is reported
    reps = int(max(1, min(40, 2.0 / max(one * nthreads, 1e-6))))
    runs = []
    for _ in range(5):
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.npdm_batch(*args, nthreads=nthreads)
        runs.append(time.perf_counter() - t0)
    wall = float(np.median(runs))
    # one core, a bounded sample of 128 systems, for the per-row figure
    sub = [a[:128] for a in args]
    t0 = time.perf_counter()
    oracle.npdm_batch(*sub, nthreads=1)
    one_core = time.perf_counter() - t0
    refs = {}
    for name, ws in samples.items():
        if "e" in ws:
            refs[name] = oracle.npdm_batch(*[ws[k] for k in ("e", "c", "d", "a", "b", "y")])[0]
        else:
            refs[name] = oracle.ntdm_batch(*[ws[k] for k in ("c", "d", "a", "y")])[0]
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "value": BATCH * reps / wall,
        "unit": "PD systems/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": f"full sweep batch ({BATCH} systems, n={N_ROWS}) x {reps} repetitions per run, "
                  f"median of 5 runs after a warm-up, system-contiguous copy (layout conversion "
                  f"not timed), {cpu}",
        "ns_per_row_1core": one_core / (128 * N_ROWS) * 1e9,
    }, refs


def t_ms(fn, reps=5):
    """Mean wall time of fn() on the current stream (after one untimed call)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def r_sensitivity_rows(rs=(1.0, 64.0, 2047.0)):
    """The sweep batch at other r = tau/h^2 (the condition number grows from
    ~10 to ~1e6 with r): split-row solve time, and the sampled solutions of
    the split kernel and of the one-lane (sequential-recurrence) kernel, whose
    errors against the oracle the caller fills in."""
    KEYS = ("e", "c", "d", "a", "b", "y")
    idx = np.arange(0, BATCH, 97)
    out, got, samples = {}, {}, {}
    for r in rs:
        pd = wl.config1(r=r, N=N_ROWS)[0]
        t = to_dev(pd)
        x = torch.empty_like(t["y"])
        info = torch.empty(BATCH, dtype=torch.int32, device="cuda")
        nb = bs.workspace_bytes(bs.OP_SOLVE, 5, N_ROWS, BATCH)
        wsb = torch.zeros(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
        ms = t_ms(lambda: bs.solve(diags_of(t, 5), t["y"], x, batch=BATCH, info=info,
                                   workspace=wsb), reps=10)
        ok = bool((info == 0).all())
        xs = wl.deinterleave(x.cpu().numpy(), BATCH)[idx]
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
        try:
            xl, il = bs.solve(diags_of(t, 5), t["y"], batch=BATCH)
        finally:
            bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
        ok = ok and bool((il == 0).all())
        name = f"r{r:g}"
        out[name] = {"r": r, "split_us": ms * 1e3, "info_ok": ok}
        got[name] = {"split": xs, "lane": wl.deinterleave(xl.cpu().numpy(), BATCH)[idx]}
        samples["r_" + name] = {k: pd[k][idx] for k in KEYS}
        del t, x, xl, wsb, pd
        torch.cuda.empty_cache()
    return out, got, samples


def precision_rows():
    """FP32 storage + FP64 refinement to 1e-10 against the FP64 solve, on the
    sweep batch (2048 x 2048) and on 256 pentadiagonal lines of length 1e6
    (r = 4), all inputs resident in HBM.  Returns (rows, sampled GPU results,
    sampled host batches) -- the errors against the oracle are filled in by
    the caller once the CPU leg has solved the samples."""
    KEYS = ("e", "c", "d", "a", "b", "y")
    out, got, samples = {}, {}, {}
    cases = []
    pd, _, _ = config1()
    c1 = {k: torch.from_numpy(wl.interleave(pd[k], BATCH)).cuda() for k in KEYS}
    idx = [0, 97, 1024, 2047]
    cases.append(("adi_sweep_pd_n2048_b2048", c1, BATCH, N_ROWS,
                  {k: pd[k][idx] for k in KEYS}, idx))
    nsys, n = 256, 1_000_000
    v = wl.smooth_lines(nsys, n, wl.BASE_SEED + 3)
    vt = torch.from_numpy(np.ascontiguousarray(v.T)).cuda()
    c3 = wl.sweep_lines_interleaved(vt, R_ADI, 2)
    del vt
    idx3 = [0, 128, 255]
    cases.append(("pd_lines_n1e6_b256", c3, nsys, n, wl.sweep_lines(v[idx3], R_ADI, 2), idx3))
    del v
    for name, dev, batch, n, host_ws, idx in cases:
        log(f"precision rows: {name}")
        info = torch.empty(batch, dtype=torch.int32, device="cuda")
        rows = n * batch
        ir_floor = 176 if n <= 4096 else 280  # the single-launch and the long-system path
        # FP64 direct solve
        x64 = torch.empty_like(dev["y"])
        w64 = torch.zeros(max(bs.workspace_bytes(bs.OP_SOLVE, 5, n, batch), 8) // 8,
                          dtype=torch.float64, device="cuda")
        ms64 = t_ms(lambda: bs.solve(diags_of(dev, 5), dev["y"], x64, batch=batch, info=info,
                                     workspace=w64))
        ok64 = bool((info == 0).all())
        # FP32 storage solve alone (the matrix already held in FP32)
        d32 = {k: dev[k].float() for k in KEYS}
        x32 = torch.empty_like(d32["y"])
        w32 = torch.zeros(max(bs.workspace_bytes(bs.OP_SOLVE, 5, n, batch, bs.BS_F32), 8) // 8,
                          dtype=torch.float64, device="cuda")
        ms32 = t_ms(lambda: bs.solve(diags_of(d32, 5), d32["y"], x32, batch=batch, info=info,
                                     workspace=w32))
        ok32 = bool((info == 0).all())
        del d32
        # FP32 solves + FP64 refinement to 1e-10 on the FP64 data
        xir = torch.empty_like(dev["y"])
        wir = torch.zeros(bs.workspace_bytes(bs.OP_REFINE, 5, n, batch) // 8 + 1,
                          dtype=torch.float64, device="cuda")
        res = {}

        def ir():
            _, st, rr, inf = bs.refine(diags_of(dev, 5), dev["y"], xir, batch=batch, tol=TOL,
                                       max_steps=8, workspace=wir)
            res.update(st=st, rr=rr, inf=inf)
        msir = t_ms(ir)
        steps = res["st"].cpu().numpy()
        out[name] = {
            "n": n, "batch": batch,
            "fp64_solve_us": ms64 * 1e3,
            "fp64_algorithmic_GBps": PD_BYTES_PER_ROW * rows / ms64 / 1e6,
            "fp32_storage_solve_us": ms32 * 1e3,
            "fp32_algorithmic_GBps": 28 * rows / ms32 / 1e6,
            "fp32_ir_to_1e-10_us": msir * 1e3,
            "fp32_ir_over_fp64_time": msir / ms64,
            # least bytes any verified refinement moves per row: a first solve
            # from the FP64 A and b, a residual-and-correction pass and a
            # final residual (56 + 64 + 56), with the inputs read twice per
            # solve on the long-system path (104 + 120 + 56)
            "fp32_ir_floor_B_per_row": ir_floor,
            "fp32_ir_GBps_at_floor": ir_floor * rows / msir / 1e6,
            "ir_steps_hist": np.bincount(steps).tolist(),
            "ir_relres_max": float(res["rr"].max()),
            "ir_converged": int((res["inf"] == 0).sum()),
            "info_ok": ok64 and ok32,
        }
        got[name] = {"fp64": x64[:, idx].cpu().numpy().T, "fp32": x32[:, idx].double().cpu().numpy().T,
                     "fp32_ir": xir[:, idx].cpu().numpy().T}
        samples["prec_" + name] = host_ws
        del x64, x32, xir, w64, w32, wir
    del c1, c3
    torch.cuda.empty_cache()
    return out, got, samples


def other_rows(pd, td):
    """Hot-path rows other than the timed PD solve, on the same sweep."""
    out = {}

    # NTDM on the tridiagonal (first-order) batch of the same sweep
    tds = [to_dev(td, ("c", "d", "a", "y")) for _ in range(ROTATE)]
    x = torch.empty_like(tds[0]["y"])
    info = torch.empty(BATCH, dtype=torch.int32, device="cuda")
    nb = bs.workspace_bytes(bs.OP_SOLVE, 3, N_ROWS, BATCH)
    wsb = torch.zeros(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
    k = [0]

    def td_solve():
        t = tds[k[0] % ROTATE]
        k[0] += 1
        bs.solve(diags_of(t, 3), t["y"], x, kind=3, batch=BATCH, info=info, workspace=wsb)
    ms = t_ms(td_solve, reps=20)
    out["ntdm_td"] = {"us": ms * 1e3, "systems_per_s": BATCH / ms * 1e3,
                      "algorithmic_GBps": TD_BYTES_PER_ROW * N_ROWS * BATCH / ms / 1e6,
                      "info_ok": bool((info == 0).all())}
    del tds

    # the sweep assembled inside the solver from the field: 8 B read + 8 B written per row
    u0 = torch.from_numpy(wl.smooth_field(N_ROWS, wl.BASE_SEED + 1)).cuda()
    us_ = [u0.clone() for _ in range(ROTATE)]
    xa = torch.empty_like(u0)
    for kind in (5, 3):
        nb = bs.workspace_bytes(bs.OP_ADI, kind, N_ROWS, BATCH)
        wsa = torch.zeros(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
        k[0] = 0

        def adi():
            v = us_[k[0] % ROTATE]
            k[0] += 1
            bs.solve_adi(v, R_ADI, xa, kind=kind, batch=BATCH, info=info, workspace=wsa)
        ms = t_ms(adi, reps=20)
        out["adi_fused_" + ("pd" if kind == 5 else "td")] = {
            "us": ms * 1e3, "systems_per_s": BATCH / ms * 1e3,
            "bytes_per_row": 16, "algorithmic_GBps": 16 * N_ROWS * BATCH / ms / 1e6,
            "info_ok": bool((info == 0).all())}
    del us_, xa, u0

    t = to_dev(pd)
    # MNPDM: outer diagonals given as the two entries per system (rows 0, n-1)
    rows = np.full((2, BATCH), -1, dtype=np.int32)
    oe = np.zeros((2, BATCH))
    ob = np.zeros((2, BATCH))
    rows[0], ob[0] = 0, pd["b"][:, 0]
    rows[1], oe[1] = N_ROWS - 1, pd["e"][:, N_ROWS - 1]
    dv = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (rows, oe, ob)]
    nb = bs.workspace_bytes(bs.OP_MNPDM, 5, N_ROWS, BATCH)
    wsm_ = torch.zeros(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
    ms = t_ms(lambda: bs.solve_mnpdm([t["c"], t["d"], t["a"]], *dv, t["y"], x, batch=BATCH,
                                     info=info, workspace=wsm_), reps=10)
    out["mnpdm_pd"] = {"us": ms * 1e3, "systems_per_s": BATCH / ms * 1e3,
                       "algorithmic_GBps": 40 * N_ROWS * BATCH / ms / 1e6,
                       "info_ok": bool((info == 0).all())}
    # ILU(0) = band Doolittle
    f = torch.empty((4, N_ROWS, BATCH), dtype=torch.float64, device="cuda")
    ms = t_ms(lambda: bs.factor(diags_of(t, 5), batch=BATCH, out=f, info=info), reps=3)
    out["ilu0_pd"] = {"us": ms * 1e3, "algorithmic_GBps": 72 * N_ROWS * BATCH / ms / 1e6}
    # substitution L z = y, U x = z with those factors (z through the workspace)
    nb = bs.workspace_bytes(bs.OP_SOLVE_FACTORED, 5, N_ROWS, BATCH)
    wsz = torch.empty(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
    ms = t_ms(lambda: bs.solve(diags_of(t, 5), t["y"], x, batch=BATCH, factors=f, info=info,
                               workspace=wsz), reps=3)
    out["subst_pd"] = {"us": ms * 1e3, "algorithmic_GBps": 72 * N_ROWS * BATCH / ms / 1e6}
    # both split over lanes by default; the one-lane sweeps give the same bits
    xs = x.clone()
    bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_LANE)
    try:
        f1 = torch.empty_like(f)
        bs.factor(diags_of(t, 5), batch=BATCH, out=f1, info=info)
        bs.solve(diags_of(t, 5), t["y"], x, batch=BATCH, factors=f1, info=info)
    finally:
        bs.set_option(bs.OPT_DIRECT_PATH, bs.PATH_AUTO)
    out["ilu0_pd"]["bitwise_one_lane"] = bool(torch.equal(f.view(torch.int64), f1.view(torch.int64)))
    out["subst_pd"]["bitwise_one_lane"] = bool(torch.equal(xs.view(torch.int64), x.view(torch.int64)))
    del f1, xs, wsz
    # SIP with HB steps (s_L, s_U) = (3, 4) from zero start to 1e-10
    res = {}

    def sip():
        xs, it, rr, si = bs.sip(diags_of(t, 5), t["y"], tol=TOL, max_iter=200, s_L=HB_S[0],
                                s_U=HB_S[1], factors=f, batch=BATCH)
        res.update(it=it, rr=rr, si=si)
    ms = t_ms(sip, reps=1)
    its = res["it"].float()
    out["sip_hb_pd"] = {"us": ms * 1e3, "hb_s": list(HB_S), "tol": TOL,
                        "iters_mean": float(its.mean()), "iters_max": int(res["it"].max()),
                        "us_per_iteration": ms * 1e3 / max(float(its.max()), 1.0),
                        "converged": int((res["si"] == 0).sum())}
    # explicit banded HB inverses of both factors, s = (5, 6)
    sL, sU = 5, 6
    KL, KU = bs.hb_band_width(5, sL, N_ROWS), bs.hb_band_width(5, sU, N_ROWS)
    XL = torch.empty((KL + 1, N_ROWS, BATCH), dtype=torch.float64, device="cuda")
    XU = torch.empty((KU + 1, N_ROWS, BATCH), dtype=torch.float64, device="cuda")
    wsh = torch.empty(bs.load().hb_inverse_band_workspace_bytes(5, N_ROWS, BATCH, BATCH, sL, sU)
                      // 8, dtype=torch.float64, device="cuda")
    ms = t_ms(lambda: bs.hb_inverse(diags_of(t, 5), f, s_L=sL, s_U=sU, batch=BATCH,
                                    workspace=wsh, out=(XL, XU)), reps=2)
    terms, planes = hb_work(2, (sL, sU), N_ROWS)
    gbps = planes * N_ROWS * BATCH * 8 / ms / 1e6
    out["hb_band_pd"] = {"us": ms * 1e3, "hb_s": [sL, sU], "output_GB": (KL + KU + 2) * N_ROWS *
                         BATCH * 8 / 1e9,
                         "hbm_GBps_algorithmic": gbps, "hbm_frac": gbps / 8000.0,
                         "fp64_GFLOPs": 2 * terms * BATCH / ms / 1e6,
                         # separate multiplies and adds: 39.3 T operations/s
                         "fp64_op_frac": 2 * terms * BATCH / ms / 1e6 / 39300.0}
    del XL, XU, wsh
    return out


def hb_work(q, steps, n):
    """Products and streamed planes of the banded HB recursion, per system:
    a step j with an output band of 16 or more reads X_j (b + 1 planes) to
    form M = 2I - T X_j (b + q + 1 planes, written), then reads both and
    writes X_{j+1}; a narrower step reads X_j once and writes X_{j+1} (M
    stays in registers).  A product entry of X_j M takes (b + 1)(b + q + 1)
    terms per row when the bands fit the matrix."""
    terms = planes = 0
    for s in steps:
        for j in range(s):
            b = min(n - 1, q * (2 ** j - 1))
            bm = min(n - 1, b + q)
            bo = min(n - 1, q * (2 ** (j + 1) - 1))
            terms += n * (b + 1) * (bm + 1) + n * (bm + 1) * (q + 1)
            if bo < 16:
                planes += (b + 1) + (bo + 1)
            else:
                planes += (b + 1) + (bm + 1) + (b + 1) + (bm + 1) + (bo + 1)
    return terms, planes


def varlen_rows(reps=5):
    """Uneven batch: 10 000 dominant PD systems with n log-uniform in
    [64, 65536] (about 1e8 rows).  The uneven-batch solver (tile shape from
    the autotuner) eagerly and as one captured graph, against one band_solve
    launch per size octave (systems padded with identity rows to the
    octave's longest).  Returns (row, sampled GPU results, sampled host
    systems)."""
    KEYS = ("e", "c", "d", "a", "b", "y")
    sizes = wl.config2_sizes()
    plan = bs.Varlen(sizes)
    dev = wl.dominant_groups(plan.slot_sizes)
    del dev["x_true"]
    assert dev["y"].numel() == plan.elems
    diags = [dev[k] for k in ("e", "c", "d", "a", "b")]
    x = torch.empty_like(dev["y"])
    info = torch.empty(plan.slots, dtype=torch.int32, device="cuda")
    ws = plan.workspace(5)
    best, tune_ms = plan.tune(5, diags, dev["y"], x, info, ws, reps=3)
    ms_eager = t_ms(lambda: plan.solve(5, diags, dev["y"], x, info, variant=best, workspace=ws),
                    reps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.solve(5, diags, dev["y"], x, info, variant=best, workspace=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    ms_graph = t_ms(g.replay, reps)
    torch.cuda.synchronize()
    ok = bool((info.cpu().numpy()[plan.slot] == 0).all())
    xh = x.cpu().numpy()
    t = {k: v.cpu().numpy() for k, v in dev.items()}
    pick = [int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 4242, 9999]
    got, samples = {}, {}
    for i in pick:
        p = plan.offset[i] + 16 * np.arange(sizes[i])
        samples[f"varlen_{i}"] = {k: t[k][p][None] for k in KEYS}
        got[f"varlen_{i}"] = xh[p][None]
    del dev, diags, x, ws, g
    torch.cuda.empty_cache()
    # one launch per size octave
    edges = 64 * 2 ** np.arange(11)
    buckets = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        idx = np.nonzero((sizes >= lo) & (sizes < hi if hi < edges[-1] else sizes <= hi))[0]
        if idx.size == 0:
            continue
        nb, batch = int(sizes[idx].max()), idx.size
        ld = wl.padded_ld(batch)
        arr = {k: np.zeros((nb, ld)) for k in KEYS}
        arr["d"][:] = 1.0                                  # padding rows: identity
        for col, i in enumerate(idx):
            p = plan.offset[i] + 16 * np.arange(sizes[i])
            for k in KEYS:
                arr[k][:sizes[i], col] = t[k][p]
        bt = {k: torch.from_numpy(v).cuda() for k, v in arr.items()}
        buckets.append((bt, batch, torch.empty_like(bt["y"]),
                        torch.empty(batch, dtype=torch.int32, device="cuda"),
                        torch.zeros(max(bs.workspace_bytes(bs.OP_SOLVE, 5, nb, batch, ld=ld), 8)
                                    // 8, dtype=torch.float64, device="cuda")))

    def per_bucket():
        for bt, batch, xb, ib, wsb in buckets:
            bs.solve([bt[k] for k in ("e", "c", "d", "a", "b")], bt["y"], xb, batch=batch,
                     info=ib, workspace=wsb)
    ms_bucket = t_ms(per_bucket, reps)
    pad_rows = sum(bt["y"].shape[0] * batch for bt, batch, *_ in buckets)
    rows = int(sizes.sum())
    del buckets, t
    torch.cuda.empty_cache()
    shapes = plan.variants()
    return {
        "systems": int(sizes.size), "rows": rows, "n_range": [int(sizes.min()), int(sizes.max())],
        "groups": int(plan.info.groups), "group_padding_rows": int(plan.elems // 16 * 16 - rows),
        "autotuner_ms": {f"M{m}xPW{pw}": v for (m, pw), v in zip(shapes, tune_ms)},
        "chosen_shape": list(shapes[best]),
        "varlen_eager_ms": ms_eager, "varlen_graph_ms": ms_graph,
        "varlen_algorithmic_GBps": PD_BYTES_PER_ROW * rows / ms_graph / 1e6,
        "per_octave_launches_ms": ms_bucket, "per_octave_buckets": len(edges) - 1,
        "per_octave_padded_rows": int(pad_rows),
        "speedup_graph_vs_per_octave": ms_bucket / ms_graph,
        "info_ok": ok,
    }, got, samples


def warmstart_rows(N=4096, steps=200, train_steps=150, eval_every=1, hb_s=(3, 3), tol=1e-10,
                   iters=2000, per_step=4096, batch=4096):
    """Learned SIP start vector on an N x N ADI run: train on the x-sweeps of
    the first `train_steps` steps (sampled patches), then start SIP-HB on
    held-out later steps from zero, from the previous step's solution and
    from the network's prediction; iterations and wall time to `tol`."""
    from paper_1804_09666_amd import warmstart as wsm
    t_start = time.perf_counter()
    net = wsm.WarmStart(wsm.WS_BF16, seed=7)
    gen = wsm.adi_steps(N)
    npatch = N * ((N + 63) // 64)
    g = torch.Generator(device="cuda").manual_seed(1)
    fit, Xs, Ts = [], [], []
    for step, planes, w in gen:
        if step == 0:
            continue
        if len(fit) < 8:                       # scaling from the first training sweeps
            fit.append(([p.clone() for p in planes], w.clone()))
            if len(fit) < 8:
                continue
            net.fit_scaling(fit, N, N)
            todo = fit
        else:
            todo = [(planes, w)]
        for pl, ww in todo:
            idx = torch.randint(0, npatch, (per_step,), device="cuda", generator=g)
            Xs.append(wsm.features(net.dtype, pl, net.norm, N, N)[idx])
            Ts.append(net.targets(pl, ww, N, N)[idx])
        if step >= train_steps - 1:
            break
    del fit
    X, T = torch.cat(Xs), torch.cat(Ts)
    del Xs, Ts
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t_start
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    losses = []
    for it in range(iters):
        idx = torch.randint(0, X.shape[0], (batch,), device="cuda", generator=g)
        loss = net.train_step(X[idx], T[idx], 1e-3 * 0.1 ** (it / iters))
        if it % 250 == 0 or it == iters - 1:
            losses.append(loss.item())
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    del X, T
    # held-out sweeps
    res = {k: {"iters_mean": [], "iters_max": [], "ms": []} for k in ("zero", "prev", "learned")}
    ws_fwd = wsm.workspace(wsm.OP_FORWARD, net.dtype, npatch)
    Xb = torch.empty((npatch, wsm.IN), dtype=torch.bfloat16, device="cuda")
    Yb = torch.empty((npatch, wsm.OUT), dtype=torch.float32, device="cuda")
    f = None
    infer_ms = []
    for step, planes, w in gen:
        if step >= steps:
            break
        if (step - train_steps) % eval_every:
            continue
        diags, rhs, up = planes[:5], planes[5], planes[6]
        if f is None:
            f = torch.empty((4, N, N), dtype=torch.float64, device="cuda")
            wsip = torch.empty(bs.workspace_bytes(bs.OP_SIP, 5, N, N) // 8 + 1,
                               dtype=torch.float64, device="cuda")
        bs.factor(diags, batch=N, out=f)
        for name in ("zero", "prev", "learned"):
            x0 = torch.zeros_like(rhs) if name != "prev" else up.clone()
            torch.cuda.synchronize()
            a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            a.record()
            if name == "learned":
                net.predict(diags, rhs, up, N, N, x0=x0, ws=ws_fwd, X=Xb, Y=Yb)
            b.record()
            x, it, rr, info = bs.sip(diags, rhs, None, tol=tol, max_iter=40, s_L=hb_s[0],
                                     s_U=hb_s[1], factors=f, batch=N, x=x0, workspace=wsip)
            c.record()
            torch.cuda.synchronize()
            if name == "learned":
                infer_ms.append(a.elapsed_time(b))
            res[name]["iters_mean"].append(float(it.float().mean()))
            res[name]["iters_max"].append(int(it.max()))
            res[name]["ms"].append(a.elapsed_time(c))
            res[name]["ok"] = bool((info == 0).all()) and res[name].get("ok", True)
            res[name]["err_vs_direct_max"] = max(
                res[name].get("err_vs_direct_max", 0.0),
                float((x - w).abs().max() / w.abs().max()))
    out = {"grid": N, "steps": steps, "train_steps": train_steps,
           "held_out_steps_evaluated": len(res["zero"]["ms"]), "hb_s": list(hb_s), "tol": tol,
           "dataset_s": t_data, "train_iters": iters, "train_batch": batch,
           "train_ms": train_ms, "loss_trace": losses,
           "inference_ms_mean": float(np.mean(infer_ms)),
           # network flops over the whole inference time (features, fused network, start)
           "inference_network_TFLOPs_whole": 2 * npatch * (wsm.IN * wsm.HIDDEN + 2 * wsm.HIDDEN ** 2
                                                           + wsm.HIDDEN * wsm.OUT) /
                                             (float(np.mean(infer_ms)) * 1e-3) / 1e12}
    for k, v in res.items():
        out[k] = {"iters_mean": float(np.mean(v["iters_mean"])),
                  "iters_max": int(max(v["iters_max"])), "ms_mean": float(np.mean(v["ms"])),
                  "converged": v["ok"], "err_vs_direct_max": v["err_vs_direct_max"]}
    return out


def profile_rows():
    """Workload for `rocprofv3 --kernel-trace --stats`: a few launches of every
    hot-path row (the per-kernel durations are read from the profiler)."""
    KEYS = ("e", "c", "d", "a", "b", "y")
    pd, td, _ = config1()
    t5 = {k: torch.from_numpy(wl.interleave(pd[k])).cuda() for k in KEYS}
    t3 = {k: torch.from_numpy(wl.interleave(td[k])).cuda() for k in ("c", "d", "a", "y")}
    D5, D3 = diags_of(t5, 5), diags_of(t3, 3)
    x = torch.empty_like(t5["y"])
    info = torch.empty(BATCH, dtype=torch.int32, device="cuda")

    def rep(name, fn, k=5):
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        log(f"profiled {name}")
    rep("npdm split PD", lambda: bs.solve(D5, t5["y"], x, batch=BATCH, info=info))
    rep("ntdm split TD", lambda: bs.solve(D3, t3["y"], x, kind=3, batch=BATCH, info=info))
    rows = np.full((2, BATCH), -1, dtype=np.int32)
    oe, ob = np.zeros((2, BATCH)), np.zeros((2, BATCH))
    rows[0], ob[0] = 0, pd["b"][:, 0]
    rows[1], oe[1] = N_ROWS - 1, pd["e"][:, N_ROWS - 1]
    dv = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (rows, oe, ob)]
    rep("mnpdm split", lambda: bs.solve_mnpdm([t5["c"], t5["d"], t5["a"]], *dv, t5["y"], x,
                                              batch=BATCH, info=info))
    t32 = {k: v.float() for k, v in t5.items()}
    x32 = torch.empty_like(t32["y"])
    rep("fp32 storage PD", lambda: bs.solve(diags_of(t32, 5), t32["y"], x32, batch=BATCH,
                                            info=info))
    f = torch.empty((4, N_ROWS, BATCH), dtype=torch.float64, device="cuda")
    rep("ilu0 factor", lambda: bs.factor(D5, batch=BATCH, out=f, info=info))
    nb = bs.workspace_bytes(bs.OP_SOLVE_FACTORED, 5, N_ROWS, BATCH)
    wsz = torch.empty(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
    rep("substitution", lambda: bs.solve(D5, t5["y"], x, batch=BATCH, factors=f, info=info,
                                         workspace=wsz))
    rep("sip hb(3,4)", lambda: bs.sip(D5, t5["y"], tol=1e-10, max_iter=12, s_L=3, s_U=4,
                                      factors=f, batch=BATCH), k=1)
    rep("sip exact", lambda: bs.sip(D5, t5["y"], tol=1e-10, max_iter=3, factors=f, batch=BATCH),
        k=1)
    rep("hb band inverses s=(5,6)", lambda: bs.hb_inverse(D5, f, s_L=5, s_U=6, batch=BATCH), k=2)
    del t5, t3, t32, x, x32, f
    nsys, n = 256, 1_000_000
    v = wl.smooth_lines(nsys, n, wl.BASE_SEED + 3)
    c3 = wl.sweep_lines_interleaved(torch.from_numpy(np.ascontiguousarray(v.T)).cuda(), R_ADI, 2)
    del v
    xc = torch.empty_like(c3["y"])
    ic = torch.empty(nsys, dtype=torch.int32, device="cuda")
    rep("long path n=1e6", lambda: bs.solve(diags_of(c3, 5), c3["y"], xc, batch=nsys, info=ic),
        k=2)
    rep("refine n=1e6", lambda: bs.refine(diags_of(c3, 5), c3["y"], xc, batch=nsys, tol=1e-10,
                                          max_steps=4), k=1)
    del c3, xc
    torch.cuda.empty_cache()
    from paper_1804_09666_amd import warmstart as wsm
    net = wsm.WarmStart(wsm.WS_BF16, seed=7)
    P = 4096 * 64
    X = torch.zeros((P, wsm.IN), dtype=torch.bfloat16, device="cuda")
    Y = torch.empty((P, wsm.OUT), dtype=torch.float32, device="cuda")
    wsf = wsm.workspace(wsm.OP_FORWARD, wsm.WS_BF16, P)
    rep("warm-start network forward, 262144 patches",
        lambda: wsm.forward(wsm.WS_BF16, X, net.p32, net.pT, Y, wsf), k=3)
    rep("warm-start fused inference, 262144 patches",
        lambda: wsm.infer(X, net.p32, net.pT, Y), k=3)
    del X, Y, wsf
    g = torch.Generator(device="cuda").manual_seed(3)
    planes = [torch.rand((4096, 4096), dtype=torch.float64, device="cuda", generator=g)
              for _ in range(7)]
    x0 = torch.empty_like(planes[6])
    rep("warm-start prediction (features, network, start vector), 4096 x 4096",
        lambda: wsm.predict_fused(planes, [0.0] * 7 + [1.0] * 7, net.p32, net.pT, 0.0, 1.0,
                                  4096, 4096, x0), k=3)
    Xf = wsm.features(wsm.WS_BF16, planes, [0.0] * 7 + [1.0] * 7, 4096, 4096)
    rep("warm-start separate features and start vector, 4096 x 4096",
        lambda: wsm.apply(wsm.infer(Xf, net.p32, net.pT), planes[6], 0.0, 1.0, 4096, 4096, x0),
        k=2)


def summarize_stats(csv_dir, out_path, title, command):
    """rocprofv3 kernel statistics (CSV) -> short text table."""
    import csv
    import glob
    import re
    rows = []
    for fn in glob.glob(os.path.join(csv_dir, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            name = r["Name"]
            if name.startswith("_Z"):
                import subprocess
                name = subprocess.run(["c++filt"], input=name, capture_output=True,
                                      text=True).stdout.strip() or name
            name = name.replace("(anonymous namespace)::", "")
            name = re.sub(r"\(.*", "", name)
            name = re.sub(r"^void ", "", name)
            rows.append((name[:100], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                         float(r["Percentage"])))
    rows.sort(key=lambda t: -t[5])
    with open(out_path, "w") as fh:
        fh.write(f"# rocprofv3 kernel statistics: {title}\n")
        fh.write(f"# command (from the repository root):\n#   {command}\n")
        fh.write("name | calls | avg_us | min_us | max_us | share_%\n")
        for t in rows:
            fh.write(f"{t[0]} | {t[1]} | {t[2]:.2f} | {t[3]:.2f} | {t[4]:.2f} | {t[5]:.2f}\n")
    print(open(out_path).read())


def pmc_run():
    """Workload for the rocprofv3 counter passes: 5 PD solves of the sweep
    batch (rotating inputs) and one plain 1 GiB device copy whose HBM bytes
    are known, to scale FETCH_SIZE / WRITE_SIZE."""
    pd, _, _ = config1()
    sets = [to_dev(pd) for _ in range(ROTATE)]
    x = torch.empty_like(sets[0]["y"])
    info = torch.empty(BATCH, dtype=torch.int32, device="cuda")
    nb = bs.workspace_bytes(bs.OP_SOLVE, 5, N_ROWS, BATCH)
    ws_buf = torch.zeros(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
    for k in range(5):
        t = sets[k % ROTATE]
        bs.solve(diags_of(t, 5), t["y"], x, batch=BATCH, info=info, workspace=ws_buf)
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log("pmc run done")


def summarize_pmc(fetch_dir, write_dir, out_path=TRAFFIC_FILE):
    """Turn the two counter passes into HBM bytes per launch of the split PD
    kernel, each counter scaled by its reading for the 1 GiB copy."""
    import csv
    import glob

    def read(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return rows

    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = read(d, counter)
        kern = [v for k, v in rows if "part_kernel<double, 5," in k]
        copy = [v for k, v in rows if "copybuffer" in k.lower()]
        if not kern or not copy:
            raise SystemExit(f"{counter}: kernel or copy dispatch not found in {d}")
        res[counter] = (float(np.mean(kern)), float(max(copy)))
    fetch_k, fetch_c = res["FETCH_SIZE"]
    write_k, write_c = res["WRITE_SIZE"]
    f_scale = COPY_BYTES / (fetch_c * 1024.0)
    w_scale = COPY_BYTES / (write_c * 1024.0)
    hbm = fetch_k * 1024.0 * f_scale + write_k * 1024.0 * w_scale
    src_hash = kernel_source_hash()
    alg = PD_BYTES_PER_ROW * N_ROWS * BATCH
    with open(out_path, "w") as fh:
        fh.write("# HBM traffic per launch of the split-row NPDM kernel on the n=2048 x 2048\n"
                 "# ADI pentadiagonal batch, from two rocprofv3 counter passes:\n"
                 "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -- python3 bench.py --pmc-run\n"
                 "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -- python3 bench.py --pmc-run\n"
                 "# Each counter (KiB per dispatch) is scaled by what it reads for a plain\n"
                 "# 1 GiB device copy (read 1 GiB, write 1 GiB) in the same run.\n")
        fh.write(f"kernel_source_sha256_16: {src_hash}\n")
        fh.write(f"fetch_kib_per_launch_raw: {fetch_k:.1f}\n")
        fh.write(f"write_kib_per_launch_raw: {write_k:.1f}\n")
        fh.write(f"copy_fetch_kib_raw: {fetch_c:.1f}\n")
        fh.write(f"copy_write_kib_raw: {write_c:.1f}\n")
        fh.write(f"fetch_scale: {f_scale:.4f}\n")
        fh.write(f"write_scale: {w_scale:.4f}\n")
        fh.write(f"hbm_bytes_per_launch: {hbm:.0f}\n")
        fh.write(f"algorithmic_bytes_per_launch: {alg}\n")
        fh.write(f"traffic_over_algorithmic: {hbm / alg:.4f}\n")
    print(open(out_path).read())


def main():
    global R_ADI, SEED, HB_S, TOL
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--r", type=float, default=R_ADI, help="r = tau / h^2 of the sweep batch")
    ap.add_argument("--seed", type=int, default=None, help="seed of the sweep batch")
    ap.add_argument("--hb-s", default=f"{HB_S[0]},{HB_S[1]}",
                    help="HB steps s_L,s_U of the SIP row")
    ap.add_argument("--tol", type=float, default=TOL, help="SIP and refinement tolerance")
    ap.add_argument("--no-rows", action="store_true", help="skip the other hot-path rows")
    ap.add_argument("--rows", default="all",
                    help="comma list of row groups to measure besides the headline: direct "
                         "(TD, ADI, MNPDM, ILU(0), SIP on the sweep batch), precision (FP32 + "
                         "refinement, sweep batch and 256 x 1e6), warmstart (4096 x 4096 ADI run), "
                         "varlen (10 000 systems), rsens (r = 1, 64, 2047); or all")
    ap.add_argument("--pmc-run", action="store_true",
                    help="only run the workload of the rocprofv3 counter passes")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM traffic summary from two counter passes")
    ap.add_argument("--profile-rows", action="store_true",
                    help="only run a few launches of every hot-path row (for rocprofv3)")
    ap.add_argument("--profile-hb", action="store_true",
                    help="only one call of the explicit HB band inverses, s = (5, 6), on the "
                         "sweep batch's factors (for rocprofv3 counters)")
    ap.add_argument("--summarize-stats", nargs=4,
                    metavar=("CSV_DIR", "OUT", "TITLE", "COMMAND"),
                    help="write a kernel-statistics table from rocprofv3 CSV output")
    args = ap.parse_args()
    R_ADI, SEED, TOL = args.r, args.seed, args.tol
    HB_S = tuple(int(v) for v in args.hb_s.split(","))
    if len(HB_S) != 2 or min(HB_S) < 0 or not (TOL > 0):
        raise SystemExit("--hb-s takes two non-negative integers s_L,s_U; --tol must be positive")
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return
    if args.profile_hb:
        pd, _, _ = config1()
        t5 = {k: torch.from_numpy(wl.interleave(pd[k])).cuda() for k in ("e", "c", "d", "a", "b")}
        f, _ = bs.factor(diags_of(t5, 5), batch=BATCH)
        bs.hb_inverse(diags_of(t5, 5), f, s_L=5, s_U=6, batch=BATCH)
        torch.cuda.synchronize()
        log("profiled hb band inverses s=(5,6)")
        return
    if args.profile_rows:
        profile_rows()
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.pmc_run:
        pmc_run()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(systems of a sweep would be sharded across GPUs; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    torch.cuda.init()
    log(f"device: {torch.cuda.get_device_name(0)}")
    pd, td, _ = config1()
    sets = [to_dev(pd) for _ in range(ROTATE)]
    xs = [torch.empty_like(sets[0]["y"]) for _ in range(ROTATE)]
    info = torch.empty(BATCH, dtype=torch.int32, device="cuda")
    nb = bs.workspace_bytes(bs.OP_SOLVE, 5, N_ROWS, BATCH)
    ws_buf = torch.zeros(max(nb, 8) // 8, dtype=torch.float64, device="cuda")
    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    eager_ms, per = timed_solves(sets, 5, args.steps, args.warmup, ws_buf, xs, info)
    ok = bool((info == 0).all())
    log("the same steps as one captured graph")
    total_ms = graph_solves(sets, 5, args.steps, ws_buf, xs, info)
    ok = ok and bool((info == 0).all())
    ceiling = stream_ceiling(sets)
    idx = np.arange(0, BATCH, 97)
    x_last = wl.deinterleave(xs[(args.steps - 1) % ROTATE].cpu().numpy(), BATCH)[idx]
    ms_step = total_ms / args.steps
    kern_ms = float(per.mean())
    alg_bytes = PD_BYTES_PER_ROW * N_ROWS * BATCH
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    line = {
        "metric": "PD systems/sec + HBM GB/s at n=2048; FP32+IR and warm-start vs FP64 at 1e-10",
        "value": BATCH / (ms_step * 1e-3),
        "unit": "PD systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "adi_sweep_pd_n2048_b2048", "n": N_ROWS, "batch": BATCH,
                   "r": R_ADI, "seed": SEED, "hb_s": list(HB_S), "tol": TOL,
                   "method": "NPDM (split-row band_solve)",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic_from_profile()},
        "hbm_GBps_algorithmic": alg_bytes / (ms_step * 1e-3) / 1e9,
        "timing": "one HIP graph of the timed steps (rotating 4 input sets); eager launches "
                  "beside it",
        "eager_ms_per_step": eager_ms / args.steps,
        "stream_ceiling_GBps": ceiling,
        "frac_of_stream_ceiling": achieved / ceiling,
        "kernel_us_mean": kern_ms * 1e3,
        "kernel_us_median": float(np.median(per) * 1e3),
        "kernel_us_p10_p90": [float(np.percentile(per, 10) * 1e3),
                              float(np.percentile(per, 90) * 1e3)],
        "info_ok": ok,
    }
    samples = {"timed": {k: pd[k][idx] for k in ("e", "c", "d", "a", "b", "y")}}
    groups = set() if args.no_rows else (
        {"direct", "precision", "warmstart", "varlen", "rsens"} if args.rows == "all"
        else set(args.rows.split(",")))
    unknown = groups - {"direct", "precision", "warmstart", "varlen", "rsens"}
    if unknown:
        raise SystemExit(f"--rows: unknown group(s) {sorted(unknown)}")
    prec_x, vl_x, rs_x = {}, {}, {}
    if "direct" in groups:
        log("measuring the other hot-path rows")
        line["rows"] = other_rows(pd, td)
    del sets, xs
    torch.cuda.empty_cache()
    if "precision" in groups:
        prec, prec_x, prec_samples = precision_rows()
        line["fp32_ir"] = prec
        samples.update(prec_samples)
    if "warmstart" in groups:
        log("learned warm start (4096 x 4096 ADI run)")
        line["warm_start"] = warmstart_rows()
        torch.cuda.empty_cache()
    if "varlen" in groups:
        log("uneven batch (10 000 systems, n log-uniform in [64, 65536])")
        line["uneven_batch"], vl_x, vl_samples = varlen_rows()
        samples.update(vl_samples)
    if "rsens" in groups:
        log("the sweep batch at r = 1, 64, 2047")
        line["r_sensitivity"], rs_x, rs_samples = r_sensitivity_rows()
        samples.update(rs_samples)
    if not args.no_cpu:
        log("timing the CPU oracle")
        line["cpu_baseline"], refs = cpu_baseline(pd, samples)

        def rel(x, ref):
            return float((np.abs(x - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())
        line["parity_max_rel_err_sampled"] = rel(x_last, refs["timed"])
        if vl_x:
            line["uneven_batch"]["sampled_err_vs_oracle"] = max(
                rel(xv, refs[k]) for k, xv in vl_x.items())
        for name, xsamp in rs_x.items():
            for key, xv in xsamp.items():
                line["r_sensitivity"][name][f"{key}_err_vs_oracle"] = rel(xv, refs["r_" + name])
        for name, xsamp in prec_x.items():
            ref = refs["prec_" + name]
            for key, xv in xsamp.items():
                line["fp32_ir"][name][f"{key}_err_vs_oracle"] = rel(xv, ref)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
