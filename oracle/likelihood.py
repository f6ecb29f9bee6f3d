"""Oracle for the response and likelihood epilogue of the reconstruction
(Sec. 2.5): test infrastructure, used only by the tests and the smoke check.
Plain float64 numpy on the solver oracle's fields (3D or 2D arrays).

* Response (Sec. 2.5.2, Eq. (response)): the absorbed energy density L_e = mua rho (the
  paper writes lambda for mua), restricted by the mask M to the voxels that
  enter the comparison with data.
* Noise model (Sec. 2.5.1, Eq. (noise)): sigma_i = max(rel L_e,i,
  floor max_j L_e,j) with rel = 0.05 and floor = 0.01; the mask keeps
  vertices at least `mask` vertices from every face (the paper masks 0.2 cm
  on all edges).  Weights w_i = 1 / sigma_i^2 on kept vertices, 0 elsewhere.
* Likelihood (Sec. 2.5.4, Eq. (likelihood), Gaussian with diagonal covariance): the negative
  log-likelihood up to a constant, H = 1/2 sum_i w_i (d_i - L_e,i)^2, and
  Eq. (chi2), chi2 = 2 H / N_vox with N_vox the number of kept voxels.
* Gradient of H: with rho = S q, dH/drho = mua w (mua rho - d); the gradients
  in q, log D and log mua through the solver are its pull-back (the solver
  oracle's vjp), and log mua also enters L_e directly:
  dH/dlogmua_i += w_i (mua_i rho_i - d_i) mua_i rho_i.
"""
import numpy as np


def kept(shape, mask):
    """Boolean array: vertices at least `mask` vertices from every face
    (each axis with its own number of vertices)."""
    out = np.ones(shape, dtype=bool)
    for a, n in enumerate(shape):
        idx = np.arange(n)
        ok = (idx >= mask) & (idx <= n - 1 - mask)
        sh = [1] * len(shape)
        sh[a] = n
        out &= ok.reshape(sh)
    return out


def noise_weights(Le, mask, rel=0.05, floor=0.01):
    sigma = np.maximum(rel * Le, floor * Le.max())
    w = 1.0 / sigma ** 2
    return np.where(kept(Le.shape, mask), w, 0.0)


def neg_log_likelihood(rho, mua, d, w):
    """(H, chi2, N_vox)."""
    res = d - mua * rho
    H = 0.5 * float(np.sum(w * res * res))
    nvox = int(np.count_nonzero(w > 0))
    return H, 2.0 * H / max(nvox, 1), nvox


def likelihood_grad(H, mua, q, d, w, **solver_kw):
    """rho, (H, chi2), (qbar, g_logD, g_logmua) for the hierarchy H of the
    solver oracle (3D ref.Hierarchy or 2D ref2d.Hierarchy2D)."""
    rho, _ = H.forward(q, **solver_kw)
    value = neg_log_likelihood(rho, mua, d, w)
    rhobar = mua * w * (mua * rho - d)
    (qbar, gD, gmu), _ = H.vjp(rho, rhobar, **solver_kw)
    gmu = gmu + w * (mua * rho - d) * mua * rho
    return rho, value[:2], (qbar, gD, gmu)
