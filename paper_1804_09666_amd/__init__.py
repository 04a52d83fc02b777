"""Batched band-SLAE solvers for MI355X (gfx950).

Pentadiagonal and tridiagonal systems from ADI sweeps, solved by NPDM / NTDM /
MNPDM and by the Stone method (SIP) over ILU(0) with Hotelling-Bodewig
approximate inverses (Veneva & Ayriyan, arXiv:1804.09666), through a C ABI
(`libbandsolve.so`, declared in include/bandsolve.h) over hand-written HIP
kernels.  The Python side only marshals arguments.

Submodules are imported lazily: `workloads` (seeded inputs) needs only numpy;
`bandsolve` (the binding) loads the HIP library on first use.
"""

__all__ = ["bandsolve", "workloads"]
