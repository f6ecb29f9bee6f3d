"""Differentiable geometric-multigrid solver for -div(D grad rho) + mua rho = q
on MI355X (gfx950): forward solve, JVP and VJP with respect to (q, log D,
log mua) through hand-written HIP kernels behind a C ABI (include/dmgs.h).

The HIP library is loaded on first use; importing this package needs no GPU.
"""
