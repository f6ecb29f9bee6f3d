"""Pins of the likelihood epilogue oracle (oracle/likelihood.py):

* the gradient of H = 1/2 sum w (d - mua rho)^2 in q, log D and log mua
  against complex-step derivatives of H evaluated with a dense solve
  assembled in the tests (no cycle involved), with g != 0 and both face
  means;
* the noise model and Eq. (chi2) together: data drawn as L_e + sigma xi with
  xi ~ N(0, 1) and sigma from the noise model give chi2 within a few
  standard errors of 1 (sqrt(2 / N_vox)), and chi2 of noise-free data is 0;
* the mask keeps exactly the vertices at least `mask` from every face.
"""
import numpy as np
import pytest

from oracle import likelihood, ref
from paper_2608_00760_amd import synth
from tests._dense import assemble_dense


def interior(f):
    return f[1:-1, 1:-1, 1:-1].reshape(-1)


@pytest.mark.parametrize("harmonic,g", [(False, 0.0), (True, 0.3)])
def test_gradient_matches_complex_step(harmonic, g):
    N = 4
    logD, logmu = synth.log_coefficients(N, 11, 12)
    q = synth.normal(N, 13)
    d = np.abs(synth.normal(N, 14, zero_bdry=False))
    w = np.abs(synth.normal(N, 15))          # any nonnegative weights, 0 on the boundary
    fm = "harmonic" if harmonic else "arith"
    H = ref.Hierarchy(np.exp(logD), np.exp(logmu), face_mean=fm, bc=g)
    rho, _, (qb, gD, gmu) = likelihood.likelihood_grad(H, np.exp(logmu), q, d, w, rtol=1e-14, max_cycles=300)

    def Hval(qq, lD, lm):
        A, bg, idx = assemble_dense(np.exp(lD), np.exp(lm), g=g, harmonic=harmonic)
        u = np.linalg.solve(A, interior(qq) + bg)
        rr = np.full(qq.shape, g, dtype=u.dtype)
        rr[1:-1, 1:-1, 1:-1] = u.reshape(N - 1, N - 1, N - 1)
        res = d - np.exp(lm) * rr
        return 0.5 * np.sum(w * res * res)

    eps = 1e-30
    cq, cD, cm = np.zeros_like(q), np.zeros_like(q), np.zeros_like(q)
    for v in np.ndindex(q.shape):
        e = np.zeros(q.shape, dtype=complex)
        e[v] = 1j * eps
        cD[v] = Hval(q.astype(complex), logD + e, logmu.astype(complex)).imag / eps
        cm[v] = Hval(q.astype(complex), logD.astype(complex), logmu + e).imag / eps
        if all(0 < c < N for c in v):
            cq[v] = Hval(q + e, logD.astype(complex), logmu.astype(complex)).imag / eps
    for got, want in ((qb, cq), (gD, cD), (gmu, cm)):
        assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_chi2_of_model_noise_is_one():
    N = 32
    c = synth.grf_case(N, 600)
    H = ref.Hierarchy(c["D"], c["mua"])
    rho, _ = H.forward(c["q"], rtol=1e-12)
    Le = c["mua"] * rho
    w = likelihood.noise_weights(Le, mask=3)
    sigma = np.maximum(0.05 * Le, 0.01 * Le.max())
    xi = np.random.default_rng(601).standard_normal(Le.shape)
    d = Le + sigma * xi
    Hv, chi2, nvox = likelihood.neg_log_likelihood(rho, c["mua"], d, w)
    assert nvox == (N + 1 - 6) ** 3
    assert abs(chi2 - 1.0) <= 4.0 * np.sqrt(2.0 / nvox), chi2
    assert likelihood.neg_log_likelihood(rho, c["mua"], Le, w)[1] == 0.0
    # the weights are 1 / sigma^2 where kept
    k = likelihood.kept(Le.shape, 3)
    assert np.allclose(w[k] * sigma[k] ** 2, 1.0, rtol=1e-14) and not w[~k].any()


def test_mask_keeps_the_inner_block():
    k = likelihood.kept((9, 9, 9), 2)
    brute = np.zeros((9, 9, 9), dtype=bool)
    for x in range(9):
        for y in range(9):
            for z in range(9):
                brute[x, y, z] = min(x, y, z) >= 2 and max(x, y, z) <= 6
    assert (k == brute).all()
    k2 = likelihood.kept((7, 7), 1)
    assert k2.sum() == 25 and not k2[0].any() and not k2[:, -1].any()
