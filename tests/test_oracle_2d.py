"""Pins of the two-dimensional oracle (oracle/ref2d.py) against what the
mathematics fixes, independently of the oracle's own code:

* a dense operator assembled here vertex by vertex (loops, not slices):
  A u, one red or black half-sweep by its splitting formula, the exact solve;
* the discrete sine transform (DST-I) solution for constant coefficients
  (closed form: sine modes are eigenvectors of the five-point operator);
* bilinear fields are reproduced exactly by the prolongation, constants by
  the coefficient transfer, and I = 4 R^T as matrices;
* the pull-back of n fixed cycles is the transpose of the forward map, with
  the whole matrix S_n built column by column (V(2,2), V(2,1), V(0,2), both
  face means);
* the coefficient gradients and the push-forward against complex-step
  derivatives of the dense solution (no cycle involved);
* second-order convergence to a manufactured solution with variable D;
* the cycle contracts the residual on log-normal coefficients.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import ref2d
from paper_2608_00760_amd import synth


def dense(D, mu, h=1.0, harmonic=False, g=0.0):
    """(A, b_g): A on interior unknowns (x-major), b_g the boundary
    contribution of Dirichlet values g; complex D and mu allowed."""
    N = D.shape[0] - 1
    m = N - 1
    dt = np.result_type(D, mu, float)
    A = np.zeros((m * m, m * m), dtype=dt)
    bg = np.zeros(m * m, dtype=dt)

    def face(a, b):
        return 2.0 * a * b / (a + b) if harmonic else (a + b) / 2.0

    for x in range(1, N):
        for y in range(1, N):
            r = (x - 1) * m + (y - 1)
            A[r, r] += mu[x, y]
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                xa, ya = x + dx, y + dy
                c = face(D[x, y], D[xa, ya]) / (h * h)
                A[r, r] += c
                if 1 <= xa <= N - 1 and 1 <= ya <= N - 1:
                    A[r, (xa - 1) * m + (ya - 1)] -= c
                else:
                    bg[r] += c * g
    return A, bg


def inner(f):
    return f[1:-1, 1:-1].reshape(-1)


def embed(v, N, bc=0.0):
    u = np.full((N + 1, N + 1), bc, dtype=v.dtype)
    u[1:-1, 1:-1] = v.reshape(N - 1, N - 1)
    return u


def grf2(N, seed, harmonic=False, **kw):
    logD, logmu = synth.log_coefficients(N, seed, seed + 1, ndim=2)
    D, mu = np.exp(logD), np.exp(logmu)
    return ref2d.Hierarchy2D(D, mu, face_mean="harmonic" if harmonic else "arith", **kw), D, mu


@pytest.mark.parametrize("N,harmonic", [(6, False), (8, True), (12, False)])
def test_operator_half_sweep_and_exact_solve_match_dense(N, harmonic):
    H, D, mu = grf2(N, 10 + N, harmonic)
    A, _ = dense(D, mu, harmonic=harmonic)
    u = synth.normal(N, 1, ndim=2)
    q = synth.normal(N, 2, ndim=2)
    assert np.abs(inner(H.apply(0, u)) - A @ inner(u)).max() <= 1e-13 * np.abs(A @ inner(u)).max()
    # half-sweep of colour c: u_c = diag(A_cc)^-1 (q_c - A_c,other u_other)
    x = np.arange(1, N)
    col = ((x[:, None] + x[None, :]) % 2).reshape(-1)
    for c in (0, 1):
        v = inner(u).copy()
        sel = col == c
        expect = v.copy()
        expect[sel] = (inner(q)[sel] - A[sel][:, ~sel] @ v[~sel]) / np.diag(A)[sel]
        w = u.copy()
        H.gs_half(0, w, q, c)
        assert np.abs(inner(w) - expect).max() <= 1e-13 * np.abs(expect).max()
    # exact solve with Dirichlet values g
    g = 0.7
    A, bg = dense(D, mu, harmonic=harmonic, g=g)
    Hg = ref2d.Hierarchy2D(D, mu, face_mean="harmonic" if harmonic else "arith", g=g)
    w = np.full_like(q, g)
    Hg.exact(0, q, w)
    assert np.abs(inner(w) - np.linalg.solve(A, inner(q) + bg)).max() <= 1e-12


@pytest.mark.parametrize("N,h", [(6, 1.0), (32, 1.0), (48, 0.5)])
def test_constant_coefficients_dst_closed_form(N, h):
    Dc, muc = 1.3, 0.2
    H = ref2d.Hierarchy2D(np.full((N + 1,) * 2, Dc), np.full((N + 1,) * 2, muc), h=h)
    q = synth.blob(N, (0.4 * N, 0.55 * N), 0.1 * N + 1.0)
    q = synth.zero_boundary(q)
    k = np.arange(1, N)
    lam = Dc / h ** 2 * ((2 - 2 * np.cos(np.pi * k / N))[:, None] + (2 - 2 * np.cos(np.pi * k / N))[None, :]) + muc
    exact = scipy.fft.idstn(scipy.fft.dstn(q[1:-1, 1:-1], type=1) / lam, type=1)
    rho, info = H.forward(q, rtol=1e-13)
    assert info["status"] == 0
    assert np.abs(rho[1:-1, 1:-1] - exact).max() <= 1e-11 * np.abs(exact).max()
    # A is symmetric: the pull-back of the same vector is the same solution
    qb, _ = H.pullback(q, rtol=1e-13)
    assert np.abs(qb[1:-1, 1:-1] - exact).max() <= 1e-11 * np.abs(exact).max()


def test_transfers():
    Nc = 6
    X = np.arange(Nc + 1, dtype=float)
    f = 0.3 + 1.1 * X[:, None] - 0.7 * X[None, :] + 0.25 * X[:, None] * X[None, :]
    e = ref2d.interpolate(f)
    x = np.arange(2 * Nc + 1) / 2.0
    assert np.abs(e - (0.3 + 1.1 * x[:, None] - 0.7 * x[None, :] + 0.25 * x[:, None] * x[None, :])).max() <= 1e-14
    c = ref2d.coarsen_field(np.full((2 * Nc + 1,) * 2, 2.5))
    assert np.abs(c - 2.5).max() <= 1e-15
    # I = 4 R^T on interior vertices (coarse corrections vanish on the boundary)
    N = 8
    m, mc = N - 1, N // 2 - 1
    R = np.zeros((mc * mc, m * m))
    I = np.zeros((m * m, mc * mc))
    for j in range(m * m):
        R[:, j] = inner(ref2d.restrict(embed(np.eye(m * m)[j], N)))
    for j in range(mc * mc):
        u = np.zeros((N + 1, N + 1))
        ref2d.prolong_add(embed(np.eye(mc * mc)[j], N // 2), u)
        I[:, j] = inner(u)
    assert np.abs(I - 4.0 * R.T).max() <= 1e-15


@pytest.mark.parametrize("N,n,nu1,nu2,harmonic", [(8, 2, 2, 2, False), (12, 2, 2, 1, True), (8, 3, 0, 2, False),
                                                  (6, 2, 1, 3, False)])
def test_pullback_is_transpose_of_fixed_cycles(N, n, nu1, nu2, harmonic):
    H, _, _ = grf2(N, 40 + N, harmonic)
    m = (N - 1) ** 2
    S = np.zeros((m, m))
    P = np.zeros((m, m))
    for j in range(m):
        e = embed(np.eye(m)[j], N)
        S[:, j] = inner(H.forward(e, fixed_cycles=n, nu1=nu1, nu2=nu2)[0])
        P[:, j] = inner(H.pullback(e, fixed_cycles=n, nu1=nu1, nu2=nu2)[0])
    assert np.abs(P - S.T).max() <= 1e-13 * np.abs(S).max()
    if nu1 != nu2:
        # the counts matter: black-first cycles with them in place are another map
        Q = np.zeros((m, m))
        for j in range(m):
            Q[:, j] = inner(H.solve(embed(np.eye(m)[j], N), 0.0, 1, nu1, nu2, 0, 0, n)[0])
        assert np.abs(Q - S.T).max() > 1e-6 * np.abs(S).max()


@pytest.mark.parametrize("harmonic,g", [(False, 0.0), (True, 0.4)])
def test_gradients_match_complex_step(harmonic, g):
    N = 6
    logD, logmu = synth.log_coefficients(N, 71, 72, ndim=2)
    q = synth.normal(N, 3, ndim=2)
    w = synth.normal(N, 4, ndim=2)
    H = ref2d.Hierarchy2D(np.exp(logD), np.exp(logmu), face_mean="harmonic" if harmonic else "arith", g=g)
    rho, _ = H.forward(q, rtol=1e-14)
    (qb, gD, gmu), _ = H.vjp(rho, w, rtol=1e-14)

    def functional(lD, lm):
        A, bg = dense(np.exp(lD), np.exp(lm), harmonic=harmonic, g=g)
        return inner(w) @ np.linalg.solve(A, inner(q) + bg)

    eps = 1e-30
    cD = np.zeros_like(gD)
    cm = np.zeros_like(gmu)
    for x in range(N + 1):
        for y in range(N + 1):
            d = np.zeros((N + 1, N + 1), dtype=complex)
            d[x, y] = 1j * eps
            cD[x, y] = functional(logD + d, logmu.astype(complex)).imag / eps
            cm[x, y] = functional(logD.astype(complex), logmu + d).imag / eps
    assert np.abs(gD - cD).max() <= 1e-9 * np.abs(cD).max()
    assert np.abs(gmu - cm).max() <= 1e-9 * np.abs(cm).max()
    # dq: the gradient in q is S^T w, i.e. the solution with A^T = A
    A, _ = dense(np.exp(logD), np.exp(logmu), harmonic=harmonic)
    assert np.abs(inner(qb) - np.linalg.solve(A.T, inner(w))).max() <= 1e-9 * np.abs(qb).max()
    # push-forward along a direction of (q, log D, log mua)
    dq, dlD, dlm = synth.normal(N, 5, ndim=2), synth.normal(N, 6, zero_bdry=False, ndim=2), synth.normal(N, 7, ndim=2)
    drho, _ = H.jvp(rho, dq, dlD, dlm, rtol=1e-14)
    Ac, bgc = dense(np.exp(logD + 1j * eps * dlD), np.exp(logmu + 1j * eps * dlm), harmonic=harmonic, g=g)
    cs = np.linalg.solve(Ac, inner(q) + 1j * eps * inner(dq) + bgc).imag / eps
    assert np.abs(inner(drho) - cs).max() <= 1e-9 * np.abs(cs).max()


def test_manufactured_solution_second_order():
    errs = []
    for N in (32, 64):
        h = 1.0 / N
        x = np.arange(N + 1) * h
        X, Y = x[:, None], x[None, :]
        u = np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
        D = 1.0 + 0.5 * np.sin(np.pi * X) * np.cos(np.pi * Y)
        mu = np.full_like(u, 0.3)
        # q = -div(D grad u) + mu u, by hand
        ux = np.pi * np.cos(np.pi * X) * np.sin(2 * np.pi * Y)
        uy = 2 * np.pi * np.sin(np.pi * X) * np.cos(2 * np.pi * Y)
        Dx = 0.5 * np.pi * np.cos(np.pi * X) * np.cos(np.pi * Y)
        Dy = -0.5 * np.pi * np.sin(np.pi * X) * np.sin(np.pi * Y)
        lap = -(np.pi ** 2 + 4 * np.pi ** 2) * u
        q = -(Dx * ux + Dy * uy + D * lap) + mu * u
        H = ref2d.Hierarchy2D(D, mu, h=h)
        rho, info = H.forward(q, rtol=1e-12)
        assert info["status"] == 0
        errs.append(np.abs(rho - u).max())
    assert 3.6 <= errs[0] / errs[1] <= 4.4, errs


def test_cycle_contracts_on_lognormal_coefficients():
    H, _, _ = grf2(64, 81)
    q = synth.blob_source(64, 82, ndim=2)
    rho, info = H.forward(q, rtol=1e-10)
    assert info["status"] == 0 and info["cycles"] <= 14, info
    r = H.defect(0, rho, q)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(H.defect(0, 0 * rho, q))
