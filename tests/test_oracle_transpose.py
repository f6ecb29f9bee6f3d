"""Transposition pins of the oracle (Sec. 2.3-2.4, Eq. (EqcompT)).

* every step's adjoint is its exact transpose: <K x, y> = <x, K^T y>;
* the pull-back of n fixed cycles is the transpose of the push-forward of
  n fixed cycles (dot-product identity), including the coefficient directions;
* the reversed composition of adjoints equals n black-before-red V-cycles;
* S_n is linear in q and the push-forward in q is S itself (Sec. 2.3).
"""
import numpy as np
import pytest

from oracle import ref
from paper_2608_00760_amd import synth


def grf_hier(N, seed, face_mean="arith"):
    logD, logmu = synth.log_coefficients(N, seed, seed + 1)
    return ref.Hierarchy(np.exp(logD), np.exp(logmu), face_mean=face_mean)


def rnd(N, seed, zero_bdry=True):
    return synth.normal(N, seed, zero_bdry)


def dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("colour", [0, 1])
def test_half_sweep_adjoint_is_transpose(k, colour):
    H = grf_hier(16, 11)
    N = H.Ns[k]
    u, q, ub = rnd(N, 1), rnd(N, 2), rnd(N, 3)
    # the half-sweep is linear in (u, q) on interior entries (boundary = 0)
    out = H.gs_half(k, colour, u, q)
    ubar, qbar = H.gs_half_adj(k, colour, ub, np.zeros_like(ub))
    lhs = dot(out, ub)
    rhs = dot(u, ubar) + dot(q, qbar)
    assert abs(lhs - rhs) <= 1e-14 * np.linalg.norm(out) * np.linalg.norm(ub)


def test_defect_adjoint_is_transpose():
    H = grf_hier(16, 12)
    N = 16
    u, q, rb = rnd(N, 4), rnd(N, 5), rnd(N, 6)
    r = H.defect(0, u, q)
    ubar, qbar = H.defect_adj(0, rb, np.zeros_like(u), np.zeros_like(u))
    assert abs(dot(r, rb) - (dot(u, ubar) + dot(q, qbar))) <= 1e-14 * np.linalg.norm(r) * np.linalg.norm(rb)


@pytest.mark.parametrize("N", [8, 12, 32])
def test_restriction_is_prolongation_transpose_over_8(N):
    """Sec. 2.3.3: I = 2^3 R^T."""
    H = grf_hier(N, 13)
    r, y = rnd(N, 7), rnd(N // 2, 8)
    Rr = H.restrict(0, r)
    Py = H.prolong_add(0, y, np.zeros_like(r))
    assert abs(dot(Rr, y) - dot(r, Py) / 8.0) <= 1e-14 * np.linalg.norm(Rr) * np.linalg.norm(y)


@pytest.mark.parametrize("N", [2, 3])
def test_exact_solve_is_symmetric(N):
    H = grf_hier(N, 14)
    x, y = rnd(N, 9), rnd(N, 10)
    ax, ay = H.exact_solve(0, x), H.exact_solve(0, y)
    assert abs(dot(ax, y) - dot(x, ay)) <= 1e-14 * np.linalg.norm(ax) * np.linalg.norm(y)


def test_operator_is_symmetric():
    H = grf_hier(16, 15)
    x, y = rnd(16, 11), rnd(16, 12)
    assert abs(dot(H.apply(0, x), y) - dot(x, H.apply(0, y))) <= 1e-14 * np.linalg.norm(H.apply(0, x)) * np.linalg.norm(y)


@pytest.mark.parametrize("N,n", [(8, 3), (32, 15), (48, 5), (96, 4)])
@pytest.mark.parametrize("face_mean", ["arith", "harmonic"])
def test_dot_product_identity_fixed_cycles(N, n, face_mean):
    """<S_n v, w> = <v, S_n^T w> with n fixed cycles both ways (Sec. 2.4)."""
    H = grf_hier(N, 100 + N, face_mean)
    v, w = rnd(N, 20), rnd(N, 21)
    Sv, _ = H.forward(v, fixed_cycles=n)
    (STw, _, _), _ = H.vjp(Sv, w, fixed_cycles=n)
    lhs, rhs = dot(Sv, w), dot(v, STw)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Sv) * np.linalg.norm(w)


@pytest.mark.parametrize("N", [8, 32])
def test_full_dot_product_identity_all_inputs(N):
    """<JVP_n(dq, dlogD, dlogmua), w> = <dq, qbar> + <dlogD, logD_bar> + <dlogmua, logmua_bar>."""
    H = grf_hier(N, 200 + N)
    q = synth.blob_source(N, 5)
    rho, _ = H.forward(q, rtol=1e-12)
    n = 6
    t = synth.tangents(N, 300)
    drho, _ = H.jvp(rho, t["dq"], t["dlogD"], t["dlogmua"], fixed_cycles=n)
    (qb, gD, gmu), _ = H.vjp(rho, t["rhobar"], fixed_cycles=n)
    lhs = dot(drho, t["rhobar"])
    rhs = dot(t["dq"], qb) + dot(t["dlogD"], gD) + dot(t["dlogmua"], gmu)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(drho) * np.linalg.norm(t["rhobar"])


@pytest.mark.parametrize("N,n,nu1,nu2", [(8, 4, 2, 2), (32, 9, 2, 2), (24, 6, 2, 2), (16, 3, 2, 1), (16, 3, 1, 3),
                                          (12, 2, 0, 2)])
def test_literal_pullback_equals_black_red_cycles(N, n, nu1, nu2):
    """The reversed composition of adjoint steps of n V(nu1,nu2)-cycles equals
    n black-before-red V(nu2,nu1)-cycles on A qbar = rhobar from qbar = 0."""
    H = grf_hier(N, 300 + N)
    w = rnd(N, 30)
    (lit, _, _), _ = H.vjp(np.zeros_like(w), w, fixed_cycles=n, nu1=nu1, nu2=nu2)
    br, _ = H.pullback_br(w, fixed_cycles=n, nu1=nu1, nu2=nu2)
    assert np.abs(lit - br).max() <= 1e-13 * np.abs(lit).max()
    if nu1 != nu2:
        # the counts matter: black-first cycles with them in place differ
        same = H.cycles(w, np.zeros_like(w), n, order=1, nu1=nu1, nu2=nu2)
        assert np.abs(lit - same).max() > 1e-6 * np.abs(lit).max()
    # and, for comparison, one red-first cycle is a different map from one
    # black-first cycle (so the test above can tell the two orders apart)
    rb1 = H.cycles(w, np.zeros_like(w), 1, order=0)
    br1 = H.cycles(w, np.zeros_like(w), 1, order=1)
    assert np.abs(rb1 - br1).max() > 1e-3 * np.abs(br1).max()


def test_pullback_tolerance_mode_residual():
    """Tolerance mode stops on ||rhobar - A qbar|| / ||rhobar|| <= rtol."""
    N = 32
    H = grf_hier(N, 40)
    w = rnd(N, 41)
    (qb, _, _), info = H.vjp(np.zeros_like(w), w, rtol=1e-10)
    res = w - H.apply(0, qb)
    assert np.linalg.norm(res) / np.linalg.norm(w) <= 1e-10
    assert abs(np.linalg.norm(res) / np.linalg.norm(w) - info["rel_residual"]) <= 1e-3 * info["rel_residual"]


def test_linearity_and_jvp_in_q_is_S():
    N = 16
    H = grf_hier(N, 50)
    q1, q2 = rnd(N, 51), rnd(N, 52)
    a, b = 0.3, -1.7
    S1, _ = H.forward(q1, fixed_cycles=5)
    S2, _ = H.forward(q2, fixed_cycles=5)
    S12, _ = H.forward(a * q1 + b * q2, fixed_cycles=5)
    assert np.abs(S12 - (a * S1 + b * S2)).max() <= 1e-14 * np.abs(S12).max()
    j, _ = H.jvp(S1, q2, None, None, fixed_cycles=5)
    assert np.abs(j - S2).max() <= 1e-15 * np.abs(S2).max()
