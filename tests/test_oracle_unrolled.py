"""Pins of the unrolled-adjoint oracle (oracle/unrolled.py):

* its forward map S_n equals the C oracle's fixed-cycle solve (an
  independent implementation) to rounding;
* its reverse pass against complex-step derivatives of <w, S_n(q; log D,
  log mua)> in every entry of log D and log mua (the complex step runs the
  same forward code in complex arithmetic, so it checks the reverse pass
  and nothing it shares), for V(2,2) and V(2,1), both face means, g != 0;
* its q-part equals the C oracle's fixed-cycle pull-back S_n^T w;
* the coarsening transpose is the transpose of the coarsening (as matrices).
"""
import numpy as np
import pytest

from oracle import ref, unrolled
from paper_2608_00760_amd import synth


def case(N, seed):
    logD, logmu = synth.log_coefficients(N, seed, seed + 1)
    return logD, logmu, synth.normal(N, seed + 2), synth.normal(N, seed + 3)


@pytest.mark.parametrize("N,n,harmonic", [(8, 2, False), (12, 3, True)])
def test_forward_equals_c_oracle(N, n, harmonic):
    logD, logmu, q, w = case(N, 10 + N)
    U = unrolled.Unrolled(np.exp(logD), np.exp(logmu), harmonic=harmonic)
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu), face_mean="harmonic" if harmonic else "arith")
    rr, _ = H.forward(q, fixed_cycles=n)
    assert np.abs(U.forward(q, n) - rr).max() <= 1e-13 * np.abs(rr).max()
    _, (qb, _, _) = U.vjp(q, w, n)
    (rqb, _, _), _ = H.vjp(rr, w, fixed_cycles=n)
    assert np.abs(qb - rqb).max() <= 1e-13 * np.abs(rqb).max()


@pytest.mark.parametrize("N,n,nu,harmonic,g", [(4, 2, (2, 2), False, 0.0), (6, 2, (2, 1), True, 0.3),
                                               (8, 1, (1, 2), False, 0.0)])
def test_reverse_pass_matches_complex_step(N, n, nu, harmonic, g):
    logD, logmu, q, w = case(N, 40 + N)
    U = unrolled.Unrolled(np.exp(logD), np.exp(logmu), g=g, harmonic=harmonic)
    _, (qb, gD, gmu) = U.vjp(q, w, n, nu[0], nu[1])
    eps = 1e-30

    def F(lD, lm):
        Uc = unrolled.Unrolled(np.exp(lD), np.exp(lm), g=g, harmonic=harmonic)
        return np.sum(w * Uc.forward(q.astype(complex), n, nu[0], nu[1]))

    cD = np.zeros_like(gD)
    cm = np.zeros_like(gmu)
    for v in np.ndindex(q.shape):
        e = np.zeros(q.shape, dtype=complex)
        e[v] = 1j * eps
        cD[v] = F(logD + e, logmu.astype(complex)).imag / eps
        cm[v] = F(logD.astype(complex), logmu + e).imag / eps
    assert np.abs(gD - cD).max() <= 1e-10 * np.abs(cD).max()
    assert np.abs(gmu - cm).max() <= 1e-10 * np.abs(cm).max()
    # and in q (S_n is affine in q)
    cq = np.zeros_like(qb)
    Uq = unrolled.Unrolled(np.exp(logD), np.exp(logmu), g=g, harmonic=harmonic)
    for v in np.ndindex(q.shape):
        if min(v) == 0 or max(v) == N:
            continue
        e = np.zeros(q.shape, dtype=complex)
        e[v] = 1j * eps
        cq[v] = np.sum(w * Uq.forward(q + e, n, nu[0], nu[1])).imag / eps
    assert np.abs(qb - cq).max() <= 1e-10 * np.abs(cq).max()


def test_coarsen_transpose():
    Nf = 8
    n = (Nf + 1) ** 3
    nc = (Nf // 2 + 1) ** 3
    C = np.zeros((nc, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        C[:, j] = unrolled.coarsen(e.reshape((Nf + 1,) * 3)).reshape(-1)
    CT = np.zeros((n, nc))
    for j in range(nc):
        e = np.zeros(nc)
        e[j] = 1.0
        CT[:, j] = unrolled.coarsen_T(e.reshape((Nf // 2 + 1,) * 3), Nf).reshape(-1)
    assert np.abs(CT - C.T).max() <= 1e-15
