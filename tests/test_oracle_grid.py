"""Pins of the oracle for grids with different cell counts and spacings per
axis (oracle/refgrid.py), none of which uses the oracle to check itself:

* on a cubic grid with one spacing it equals the C oracle (itself pinned by
  closed forms, brute force and complex steps): fixed-cycle forward,
  pull-back, push-forward and gradients, both face means, g != 0;
* constant coefficients on anisotropic grids: the DST-I closed form, whose
  eigenvalues are sum over axes of (4 D / h_a^2) sin^2(j_a pi / (2 n_a)) + mua;
* variable coefficients: the converged solution equals a dense solve of the
  operator assembled vertex by vertex with per-axis spacings (both face
  means, g != 0);
* the pull-back of n fixed cycles equals the transpose of S_n built column
  by column;
* push-forward and pull-back with coefficient gradients equal complex-step
  derivatives of <w, rho> along random directions in q, log D and log mua;
* restriction weights and the coarsening follow the (1,2,1)/4 stencil of
  Eq. (rest) on every axis; trilinear interpolation reproduces trilinear
  fields; the level shapes of the paper's data grid;
* the likelihood mask keeps vertices at least `mask` from every face on
  each axis of a non-cubic grid.
"""
import numpy as np
import pytest
import scipy.fft

from conftest import golden
from oracle import likelihood, ref, refgrid
from paper_2608_00760_amd import synth


def fields(n, seed, contrast=1.0):
    rng = np.random.default_rng(seed)
    shape = tuple(c + 1 for c in n)
    D = np.exp(contrast * rng.standard_normal(shape) * 0.5)
    mu = np.exp(-2.0 + 0.5 * rng.standard_normal(shape))
    q = rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    for a in (q, w):
        a[0], a[-1], a[:, 0], a[:, -1], a[:, :, 0], a[:, :, -1] = 0, 0, 0, 0, 0, 0
    return D, mu, q, w, rng


def dense(D, mu, h, g, harmonic):
    """A u_int = q_int + b for the interior unknowns, assembled vertex by
    vertex (per-axis spacing)."""
    n = tuple(s - 1 for s in D.shape)
    idx = -np.ones(D.shape, dtype=np.int64)
    m = 0
    for x in range(1, n[0]):
        for y in range(1, n[1]):
            for z in range(1, n[2]):
                idx[x, y, z] = m
                m += 1
    A = np.zeros((m, m), dtype=np.result_type(D, mu))
    b = np.zeros(m, dtype=A.dtype)
    face = (lambda a, c: 2 * a * c / (a + c)) if harmonic else (lambda a, c: 0.5 * (a + c))
    for x in range(1, n[0]):
        for y in range(1, n[1]):
            for z in range(1, n[2]):
                r = idx[x, y, z]
                A[r, r] += mu[x, y, z]
                for axis, d in ((0, (1, 0, 0)), (0, (-1, 0, 0)), (1, (0, 1, 0)), (1, (0, -1, 0)), (2, (0, 0, 1)),
                                (2, (0, 0, -1))):
                    j = (x + d[0], y + d[1], z + d[2])
                    c = face(D[x, y, z], D[j]) / h[axis] ** 2
                    A[r, r] += c
                    if idx[j] >= 0:
                        A[r, idx[j]] -= c
                    else:
                        b[r] += c * g
    return A, b, idx


def test_level_shapes_of_the_paper_grid():
    assert refgrid.level_shapes((128, 64, 64)) == [(128, 64, 64), (64, 32, 32), (32, 16, 16), (16, 8, 8), (8, 4, 4),
                                                   (4, 2, 2)]
    assert refgrid.level_shapes((96, 64, 48))[-1] == (6, 4, 3)
    with pytest.raises(ValueError):
        refgrid.level_shapes((10, 8, 8))


@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_cubic_grid_equals_the_c_oracle(face_mean):
    N = 16
    logD, logmu = synth.log_coefficients(N, 11, 12)
    D, mu = np.exp(logD), np.exp(logmu)
    q, w = synth.normal(N, 13), synth.normal(N, 14)
    t = synth.tangents(N, 15)
    g = 0.3
    C = ref.Hierarchy(D, mu, face_mean=face_mean, bc=g)
    G = refgrid.HierarchyGrid(D, mu, h=(1.0, 1.0, 1.0), g=g, face_mean=face_mean)
    rc, _ = C.forward(q, fixed_cycles=3)
    rg, _ = G.forward(q, fixed_cycles=3)
    assert np.abs(rc - rg).max() <= 1e-13 * np.abs(rc).max()
    (lc, dc, mc), _ = C.vjp(rc, w, fixed_cycles=3)
    (lg, dg, mg), _ = G.vjp(rg, w, fixed_cycles=3)
    for a, b in ((lc, lg), (dc, dg), (mc, mg)):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    jc, _ = C.jvp(rc, t["dq"], t["dlogD"], t["dlogmua"], fixed_cycles=3)
    jg, _ = G.jvp(rg, t["dq"], t["dlogD"], t["dlogmua"], fixed_cycles=3)
    assert np.abs(jc - jg).max() <= 1e-12 * np.abs(jc).max()


@pytest.mark.parametrize("n,h", [((16, 8, 8), (0.5, 1.0, 1.5)), ((12, 24, 6), (1.0, 0.25, 2.0)),
                                 ((32, 16, 16), (7.5 / 32, 3.5 / 16, 3.5 / 16))])
def test_constant_coefficients_closed_form(n, h):
    Dc, muc = 1.3, 0.2
    shape = tuple(c + 1 for c in n)
    G = refgrid.HierarchyGrid(np.full(shape, Dc), np.full(shape, muc), h=h)
    rng = np.random.default_rng(3)
    q = np.zeros(shape)
    q[1:-1, 1:-1, 1:-1] = rng.standard_normal(tuple(c - 1 for c in n))
    lam = muc
    grids = np.meshgrid(*[np.arange(1, c) for c in n], indexing="ij")
    for a in range(3):
        lam = lam + 4.0 * Dc / h[a] ** 2 * np.sin(grids[a] * np.pi / (2 * n[a])) ** 2
    exact = scipy.fft.idstn(scipy.fft.dstn(q[1:-1, 1:-1, 1:-1], type=1) / lam, type=1)
    rho, info = G.forward(q, rtol=1e-13)
    assert info["status"] == 0
    assert np.abs(rho[1:-1, 1:-1, 1:-1] - exact).max() <= 1e-11 * np.abs(exact).max()
    qb, _ = G.pullback(q, rtol=1e-13)
    assert np.abs(qb[1:-1, 1:-1, 1:-1] - exact).max() <= 1e-11 * np.abs(exact).max()


@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_variable_coefficients_equal_a_dense_solve(face_mean):
    n, h, g = (16, 8, 4), (0.7, 1.3, 1.0), 0.4
    D, mu, q, _, _ = fields(n, 21, contrast=2.0)
    G = refgrid.HierarchyGrid(D, mu, h=h, g=g, face_mean=face_mean)
    rho, info = G.forward(q, rtol=1e-14, max_cycles=100)
    A, b, idx = dense(D, mu, h, g, face_mean == "harmonic")
    u = np.linalg.solve(A, q[1:-1, 1:-1, 1:-1].reshape(-1) + b)
    assert np.abs(rho[1:-1, 1:-1, 1:-1].reshape(-1) - u).max() <= 1e-12 * np.abs(u).max()
    assert rho[0, 3, 2] == g and rho[5, 0, 1] == g


def test_pullback_is_the_transpose_of_the_fixed_cycle_map():
    n, h = (8, 4, 4), (1.0, 0.6, 1.4)
    D, mu, _, _, _ = fields(n, 31, contrast=1.5)
    G = refgrid.HierarchyGrid(D, mu, h=h)
    shape = tuple(c + 1 for c in n)
    inner = tuple(c - 1 for c in n)
    m = int(np.prod(inner))
    for nu1, nu2, cyc in ((2, 2, 2), (2, 1, 1), (1, 3, 2)):
        S = np.zeros((m, m))
        St = np.zeros((m, m))
        for j in range(m):
            ein = np.zeros(m)
            ein[j] = 1.0
            e = np.zeros(shape)
            e[1:-1, 1:-1, 1:-1] = ein.reshape(inner)
            S[:, j] = G.forward(e, fixed_cycles=cyc, nu1=nu1, nu2=nu2)[0][1:-1, 1:-1, 1:-1].reshape(-1)
            St[:, j] = G.pullback(e, fixed_cycles=cyc, nu1=nu1, nu2=nu2)[0][1:-1, 1:-1, 1:-1].reshape(-1)
        assert np.abs(St - S.T).max() <= 1e-13 * np.abs(S).max(), (nu1, nu2, cyc)


@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_derivatives_equal_complex_steps(face_mean):
    n, h, g = (8, 8, 4), (0.8, 1.1, 0.9), 0.25
    D, mu, q, w, rng = fields(n, 41, contrast=1.5)
    logD, logmu = np.log(D), np.log(mu)
    shape = D.shape
    G = refgrid.HierarchyGrid(D, mu, h=h, g=g, face_mean=face_mean)
    rho, _ = G.forward(q, rtol=1e-15, max_cycles=200)
    (lam, gD, gmu), _ = G.vjp(rho, w, rtol=1e-15, max_cycles=200)
    eps = 1e-30
    for trial in range(3):
        vq = rng.standard_normal(shape)
        vq[0], vq[-1], vq[:, 0], vq[:, -1], vq[:, :, 0], vq[:, :, -1] = 0, 0, 0, 0, 0, 0
        vD, vm = rng.standard_normal(shape), rng.standard_normal(shape)
        Gc = refgrid.HierarchyGrid(np.exp(logD + 1j * eps * vD), np.exp(logmu + 1j * eps * vm), h=h, g=g,
                                   face_mean=face_mean)
        rc, _ = Gc.forward(q + 1j * eps * vq, fixed_cycles=60)
        cs = float(np.sum(w * rc).imag / eps)
        adj = float(np.sum(lam * vq) + np.sum(gD * vD) + np.sum(gmu * vm))
        assert abs(cs - adj) <= 1e-11 * abs(cs), (trial, cs, adj)
        drho, _ = G.jvp(rho, vq, vD, vm, rtol=1e-15, max_cycles=200)
        assert abs(float(np.sum(w * drho)) - cs) <= 1e-11 * abs(cs)


def test_transfers_on_each_axis():
    w1 = np.array([float(v) for v in golden("restriction_1d.txt")[0]])
    n = (8, 4, 12)
    shape = tuple(c + 1 for c in n)
    X = (2, 1, 3)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                r = np.zeros(shape)
                r[2 * X[0] + a - 1, 2 * X[1] + b - 1, 2 * X[2] + c - 1] = 1.0
                assert refgrid.restrict(r)[X] == w1[a] * w1[b] * w1[c]
                assert refgrid.coarsen_field(r)[X] == w1[a] * w1[b] * w1[c]
    # boundary injection and a quadratic's closed form
    x, y, z = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    Xc, Yc, Zc = np.meshgrid(*[np.arange(s // 2 + 1, dtype=float) for s in n], indexing="ij")
    c = refgrid.coarsen_field(x * x + y * y + z * z)
    want = 4.0 * (Xc ** 2 + Yc ** 2 + Zc ** 2)
    want[1:-1, 1:-1, 1:-1] += 1.5
    assert np.abs(c - want).max() <= 1e-12
    # trilinear fields are reproduced by the interpolation
    f = 0.3 + 1.1 * Xc - 0.7 * Yc + 0.25 * Xc * Zc - 0.1 * Xc * Yc * Zc
    e = refgrid.interpolate(f)
    xf, yf, zf = x / 2.0, y / 2.0, z / 2.0
    assert np.abs(e - (0.3 + 1.1 * xf - 0.7 * yf + 0.25 * xf * zf - 0.1 * xf * yf * zf)).max() <= 1e-13


def test_likelihood_mask_on_a_non_cubic_grid():
    shape = (17, 9, 13)
    k = likelihood.kept(shape, 2)
    for x in range(shape[0]):
        for y in range(shape[1]):
            for z in range(shape[2]):
                d = min(x, shape[0] - 1 - x, y, shape[1] - 1 - y, z, shape[2] - 1 - z)
                assert k[x, y, z] == (d >= 2)
