"""Pins of the coefficient transfer between levels (reading: coarse
coefficients by full weighting on coarse interior vertices, injection on
coarse boundary vertices; Sec. 2.2 rediscretisation, weights of Eq. (rest)).

Constants and linear fields do not pin the weights: every normalised
symmetric stencil reproduces them.  These tests do:

* a unit spike at each fine offset (a, b, c) in {-1, 0, 1}^3 around the
  fine image of a coarse interior vertex reaches that coarse vertex with
  the tensor product of the printed 1D stencil 1/4 [1 2 1], and no other
  coarse interior vertex it is not adjacent to;
* a spike on the fine image of a coarse boundary vertex is injected with
  weight 1, and a spike next to it (on the fine boundary) reaches no coarse
  boundary vertex;
* the quadratic x^2 + y^2 + z^2 (fine vertex indices) has the closed-form
  coarse value 4 (X^2 + Y^2 + Z^2) + 3/2 on interior vertices (the stencil's
  second moment is 1/2 per axis) and 4 (X^2 + Y^2 + Z^2) on boundary ones;
  the bilinear x y maps to 4 X Y on both.

Each check runs on the three oracles that coarsen coefficients: the C
oracle (3D), the unrolled-adjoint oracle (3D) and the 2D oracle.  A
uniform 27-point (9-point) average, which reproduces constants and linears,
is shown to fail them.
"""
import numpy as np
import pytest

from conftest import golden
from oracle import ref, ref2d, unrolled

W1 = np.array([float(v) for v in golden("restriction_1d.txt")[0]])


def _coarse_interior(Nc, ndim):
    return tuple(slice(1, Nc) for _ in range(ndim))


def spike_weights_ok(coarsen, Nf, ndim):
    """Every spike around the fine image of one coarse interior vertex and of
    one coarse boundary vertex lands with the expected weights."""
    Nc = Nf // 2
    shape = (Nf + 1,) * ndim
    Xc = (Nc // 2,) * ndim            # an interior coarse vertex
    expect_w = W1
    for off in np.ndindex(*(3,) * ndim):
        f = np.zeros(shape)
        pos = tuple(2 * X + o - 1 for X, o in zip(Xc, off))
        f[pos] = 1.0
        c = coarsen(f)
        w = np.prod([expect_w[o] for o in off])
        if abs(c[Xc] - w) > 1e-15:
            return False
        # the spike reaches exactly the coarse interior vertices whose
        # 3^ndim neighbourhood holds it, each with its own weight
        want = np.zeros(c.shape)
        for C in np.ndindex(*c.shape):
            if all(0 < Ci < Nc for Ci in C):
                d = [p - 2 * Ci for p, Ci in zip(pos, C)]
                if all(abs(di) <= 1 for di in d):
                    want[C] = np.prod([expect_w[di + 1] for di in d])
        if np.abs(c - want).max() > 1e-15:
            return False
    # injection on a coarse boundary vertex: (0, Nc/2, ...) takes the fine
    # value at its image with weight 1
    Cb = (0,) + (Nc // 2,) * (ndim - 1)
    f = np.zeros(shape)
    f[tuple(2 * C for C in Cb)] = 1.0
    c = coarsen(f)
    if c[Cb] != 1.0:
        return False
    # a fine boundary spike beside that image does not reach the coarse
    # boundary vertex
    f = np.zeros(shape)
    f[(0, Nc + 1) + (Nc,) * (ndim - 2)] = 1.0
    c = coarsen(f)
    if c[Cb] != 0.0:
        return False
    return True


def quadratic_ok(coarsen, Nf, ndim):
    Nc = Nf // 2
    xs = np.meshgrid(*(np.arange(Nf + 1, dtype=float),) * ndim, indexing="ij")
    Xs = np.meshgrid(*(np.arange(Nc + 1, dtype=float),) * ndim, indexing="ij")
    f = sum(x * x for x in xs)
    c = coarsen(f)
    inj = 4.0 * sum(X * X for X in Xs)
    want = inj.copy()
    want[_coarse_interior(Nc, ndim)] += ndim * 0.5
    if np.abs(c - want).max() > 1e-12:
        return False
    c = coarsen(xs[0] * xs[1])
    return np.abs(c - 4.0 * Xs[0] * Xs[1]).max() <= 1e-12


ORACLES = [
    ("c-oracle-3d", ref.coarsen_field, 3),
    ("unrolled-3d", unrolled.coarsen, 3),
    ("ref2d", ref2d.coarsen_field, 2),
]


@pytest.mark.parametrize("name,fn,ndim", ORACLES, ids=[o[0] for o in ORACLES])
@pytest.mark.parametrize("Nf", [8, 12])
def test_coarsening_spike_weights(name, fn, ndim, Nf):
    assert spike_weights_ok(fn, Nf, ndim)


@pytest.mark.parametrize("name,fn,ndim", ORACLES, ids=[o[0] for o in ORACLES])
@pytest.mark.parametrize("Nf", [8, 12, 16])
def test_coarsening_quadratic_closed_form(name, fn, ndim, Nf):
    assert quadratic_ok(fn, Nf, ndim)


def _uniform_average(f):
    """A wrong transfer that keeps constants and linears: the plain mean of
    the 3^ndim fine neighbours on interior vertices, injection elsewhere."""
    ndim = f.ndim
    Nc = (f.shape[0] - 1) // 2
    c = f[(slice(None, None, 2),) * ndim].copy()
    acc = np.zeros((Nc - 1,) * ndim)
    for off in np.ndindex(*(3,) * ndim):
        acc += f[tuple(slice(1 + o, 2 * Nc - 2 + o, 2) for o in off)]
    c[_coarse_interior(Nc, ndim)] = acc / 3 ** ndim
    return c


@pytest.mark.parametrize("ndim", [2, 3])
def test_pins_reject_a_uniform_average(ndim):
    """The planted mistake passes the constant and linear pins but fails
    both of these."""
    Nf = 8
    x = np.meshgrid(*(np.arange(Nf + 1, dtype=float),) * ndim, indexing="ij")
    lin = 0.3 + 0.1 * x[0] - 0.2 * x[1]
    Xc = np.meshgrid(*(np.arange(Nf // 2 + 1, dtype=float),) * ndim, indexing="ij")
    assert np.abs(_uniform_average(lin) - (0.3 + 0.2 * Xc[0] - 0.4 * Xc[1])).max() <= 1e-14
    assert np.abs(_uniform_average(np.full(lin.shape, 2.5)) - 2.5).max() <= 1e-15
    assert not spike_weights_ok(_uniform_average, Nf, ndim)
    assert not quadratic_ok(_uniform_average, Nf, ndim)
