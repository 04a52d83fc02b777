"""The oracle's checks catch plausible mistakes: each test builds a copy of
the oracle with one planted error (a dropped term, a wrong sign, a wrong
index, a transposed operand, an absolute instead of a relative stopping test)
and requires that at least one check fails on it, while the unmodified source
passes all of them.  The checks use only numpy/LAPACK and the mathematics of
the methods (dense solves, L U = A, the HB closed form, Algorithm 1's stopping
rule), never the oracle itself."""
import ctypes
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import build_oracle

SRC = build_oracle.SRC
FLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-w"]

# (name, text in band_oracle.cpp, replacement, which occurrence: 0 = first)
MUTATIONS = [
    ("npdm: e-term of gamma dropped",
     "gamma = real(c[i]) - alpha[i - 2] * e[i];", "gamma = real(c[i]);", 0),
    ("npdm: sign of the alpha*gamma term in mu",
     "mu = (real(d[i]) - beta[i - 2] * e[i]) - alpha[i - 1] * gamma;",
     "mu = (real(d[i]) - beta[i - 2] * e[i]) + alpha[i - 1] * gamma;", 0),
    ("npdm: wrong index in the forward substitution",
     "z[i] = ((real(y[i]) - z[i - 2] * e[i]) - z[i - 1] * gamma) / mu;",
     "z[i] = ((real(y[i]) - z[i - 1] * e[i]) - z[i - 1] * gamma) / mu;", 0),
    ("npdm: beta term of the back substitution dropped",
     "xs[i] = (z[i] - alpha[i] * xs[i + 1]) - beta[i] * xs[i + 2];",
     "xs[i] = z[i] - alpha[i] * xs[i + 1];", 0),
    ("ntdm: pivot with a instead of c (transposed operand)",
     "mu = real(d[i]) - alpha[i - 1] * c[i];", "mu = real(d[i]) - alpha[i - 1] * a[i];", 0),
    ("mnpdm: outer b entries ignored",
     "if (r <= n - 3 && b_at[q] != 0.0) {", "if (false) {", 0),
    ("ilu0: l2 divides by the wrong pivot",
     "if (i >= 2) L2[i] = real(e[i]) / U0[i - 2];", "if (i >= 2) L2[i] = real(e[i]) / U0[i - 1];", 0),
    ("ilu0: sign of the u1 update",
     "U1[i] = real(a[i]) - L1[i] * U2[i - 1];", "U1[i] = real(a[i]) + L1[i] * U2[i - 1];", 0),
    ("substitution: l2 term of the forward sweep dropped",
     "if (i >= 2) t = t - l2[i] * z[i - 2];", "if (false) t = t - l2[i] * z[i - 2];", 0),
    ("hb lower: sign of the correction",
     "yn[i] = yo[i] + (v[i] - ty);", "yn[i] = yo[i] - (v[i] - ty);", 0),
    ("hb upper: u2 term dropped",
     "if (i + 2 < n) ty = ty + u2[i] * yo[i + 2];", "if (false) ty = ty + u2[i] * yo[i + 2];", 0),
    ("hb upper: start without the diagonal inverse",
     "for (int64_t i = 0; i < n; ++i) yo[i] = v[i] / u0[i];",
     "for (int64_t i = 0; i < n; ++i) yo[i] = v[i];", 0),
    ("hb matrix: transposed operand in T X",
     "acc = acc + T[i * n + l] * Xc[l * n + k];", "acc = acc + T[l * n + i] * Xc[l * n + k];", 0),
    ("sip: K = A - LU instead of LU - A", "K0[i] = t0 - d[i];", "K0[i] = d[i] - t0;", 0),
    ("sip: absolute instead of relative stopping test",
     "if (!(val(rn) >= tol * bnorm)) { status = 0; break; }",
     "if (!(val(rn) >= tol)) { status = 0; break; }", 0),
    ("sip: sign of the residual", "r[i] = real(y[i]) - ax;", "r[i] = ax - real(y[i]);", 0),
]


def _dense(e, c, d, a, b):
    n = d.size
    A = np.diag(d)
    if n > 1:
        A += np.diag(c[1:], -1) + np.diag(a[:-1], 1)
    if n > 2:
        A += np.diag(e[2:], -2) + np.diag(b[:-2], 2)
    return A


def _systems():
    """A dominant random system and a second-order PDE sweep line (n = 12)."""
    rng = np.random.default_rng(5)
    n = 12
    out = []
    e, c, a, b = (rng.uniform(-1, 1, n) for _ in range(4))
    e[:2] = 0.0
    c[0] = 0.0
    a[-1] = 0.0
    b[-2:] = 0.0
    d = np.abs(e) + np.abs(c) + np.abs(a) + np.abs(b) + rng.uniform(1, 2, n)
    out.append((e, c, d, a, b))
    from paper_1804_09666_amd import workloads as wl
    sw = wl.sweep_lines(wl.smooth_lines(1, n, seed=3), 4.0, 2)
    out.append(tuple(sw[k][0] for k in ("e", "c", "d", "a", "b")))
    return out


def _checks(lib):
    """Names of the checks that fail on `lib`."""
    failed = []

    def check(name, ok):
        if not ok:
            failed.append(name)

    rng = np.random.default_rng(11)
    for k, (e, c, d, a, b) in enumerate(_systems()):
        A = _dense(e, c, d, a, b)
        xt = rng.uniform(-1, 1, d.size)
        y = A @ xt
        try:
            x, info = oracle.npdm(e, c, d, a, b, y, lib=lib)
            check(f"npdm solves ({k})", info == 0 and np.allclose(x, xt, rtol=0, atol=1e-10))
            _, _, mu = oracle.npdm(e, c, d, a, b, y, return_mu=True, lib=lib)
            check(f"npdm pivots give det A ({k})",
                  np.isclose(np.prod(mu), np.linalg.det(A), rtol=1e-10))
            T = _dense(0 * e, c, d, a, 0 * b)
            yt = T @ xt
            xtd, info = oracle.ntdm(c, d, a, yt, lib=lib)
            check(f"ntdm solves ({k})", info == 0 and np.allclose(xtd, xt, rtol=0, atol=1e-10))
            rows = np.arange(d.size)
            xm, info = oracle.mnpdm(c, d, a, rows, e, b, y, lib=lib)
            check(f"mnpdm solves ({k})", info == 0 and np.allclose(xm, xt, rtol=0, atol=1e-10))
            l2, l1, u0, u1, info = oracle.ilu0_band(e, c, d, a, b, lib=lib)
            L = np.eye(d.size) + np.diag(l1[1:], -1) + np.diag(l2[2:], -2)
            U = np.diag(u0) + np.diag(u1[:-1], 1) + np.diag(b[:-2], 2)
            check(f"ilu0: L U = A ({k})", info == 0 and np.allclose(L @ U, A, rtol=0, atol=1e-12))
            xs, info = oracle.band_lu_solve(l2, l1, u0, u1, b, y, lib=lib)
            check(f"substitution solves ({k})",
                  info == 0 and np.allclose(xs, xt, rtol=0, atol=1e-10))
            v = rng.uniform(-1, 1, d.size)
            for s in (1, 2):
                m = 2 ** s
                XL = sum(np.linalg.matrix_power(np.eye(d.size) - L, j) for j in range(m))
                D = np.diag(1.0 / u0)
                XU = sum(np.linalg.matrix_power(np.eye(d.size) - D @ U, j) for j in range(m)) @ D
                ol = oracle.hb_lower_apply(l2, l1, s, v, lib=lib)
                ou = oracle.hb_upper_apply(u0, u1, b, s, v, lib=lib)
                check(f"hb lower = closed form (s={s}, {k})", np.allclose(ol, XL @ v, atol=1e-12))
                check(f"hb upper = closed form (s={s}, {k})", np.allclose(ou, XU @ v, atol=1e-12))
                if k == 0:
                    X = oracle.hb_matrix(A, s, lib=lib)
                    D0 = np.diag(1.0 / np.diag(A))
                    G = np.eye(d.size) - D0 @ A
                    Xs = sum(np.linalg.matrix_power(G, j) for j in range(m)) @ D0
                    check(f"hb matrix = closed form (s={s})", np.allclose(X, Xs, atol=1e-12))
            # Literal Algorithm 1 with inexact factors (K = LU - A != 0): one
            # step from a random x0 is (LU)^-1 (K x0 + y) by dense algebra.
            fu = (l2, l1, u0 * 1.05, u1)
            LU = L @ (np.diag(fu[2]) + np.diag(u1[:-1], 1) + np.diag(b[:-2], 2))
            x0 = rng.uniform(-1, 1, d.size)
            x1 = np.linalg.solve(LU, (LU - A) @ x0 + y)
            xo, it, _, _ = oracle.sip(e, c, d, a, b, y, tol=1e-14, max_iter=1, x0=x0,
                                      factors=fu, lib=lib)
            check(f"sip literal step with K != 0 ({k})",
                  it == 1 and np.allclose(xo, x1, rtol=0, atol=1e-10))
            for scale in (1.0, 1e-9):
                ys = y * scale
                for sL, sU in ((-1, -1), (3, 3)):
                    xx, it, rr, st = oracle.sip(e, c, d, a, b, ys, tol=1e-10, max_iter=60,
                                                s_L=sL, s_U=sU, lib=lib)
                    res = np.abs(ys - A @ xx).max() / np.abs(ys).max()
                    check(f"sip s=({sL},{sU}) meets the relative rule ({k}, b scale {scale})",
                          st == 0 and res < 1e-10 and np.allclose(xx, xt * scale, rtol=0,
                                                                  atol=1e-7 * scale))
        except Exception as exc:  # a crash or refusal counts as a caught mistake
            failed.append(f"raised {type(exc).__name__} ({k})")
    return failed


def _build(text, path):
    src = path + ".cpp"
    with open(src, "w") as fh:
        fh.write(text)
    subprocess.run(["g++", *FLAGS, src, "-o", path], check=True, timeout=300)
    return oracle.bind(ctypes.CDLL(path))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planted_mistakes_are_caught(tmp_path):
    base = open(SRC).read()
    jobs = [("unmodified", base)]
    for name, old, new, occ in MUTATIONS:
        parts = base.split(old)
        assert len(parts) > occ + 1, f"mutation site not found: {name}"
        text = old.join(parts[:occ + 1]) + new + old.join(parts[occ + 1:])
        jobs.append((name, text))
    paths = [os.path.join(tmp_path, f"m{i}.so") for i in range(len(jobs))]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        libs = list(ex.map(lambda jp: _build(jp[0][1], jp[1]), zip(jobs, paths)))
    assert _checks(libs[0]) == [], "the unmodified oracle must pass every check"
    missed = [name for (name, _), lib in zip(jobs[1:], libs[1:]) if not _checks(lib)]
    assert not missed, f"planted mistakes no check caught: {missed}"
