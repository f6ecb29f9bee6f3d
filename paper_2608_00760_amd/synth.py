"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module draws fields only; it contains none of the solver's arithmetic.
Every field is a float64 numpy array of shape (N+1, N+1, N+1) on the vertices
of an N-cell grid with unit spacing, x slowest, z fastest; with ndim=2 it is
(N+1, N+1), x slowest, y fastest, and the recipes below hold with two
coordinates in place of three.

Recipes (the paper's Monte Carlo tissue data are not available; these stand
in for coefficient fields and sources of the same kind):
  grf       Gaussian random field with power spectrum proportional to k^-3:
            white noise N(0,1), FFT, amplitude scaled by |k|^-3/2 with integer
            wavenumbers, k = 0 removed, inverse FFT, normalised to sample mean 0
            and standard deviation 1.
  log D     clip(grf, -ln 100, ln 100): mean log 1, std 1, contrast <= 1e4.
  log mua   ln 0.05 + grf (independent seed).
  blob      exp(-|x - c|^2 / (2 sigma^2)) on vertex coordinates.
  q         sum of 16 blobs, centres ~ U[0.15N, 0.85N]^3, sigma ~ U[2, 6],
            amplitude ~ U[0.5, 1.5], plus N(0, 0.01^2) noise.
  tangents  N(0, 1); boundary entries of dq, dlogmua and rhobar are zeroed
            (they are ignored by the operator), dlogD keeps them.
"""
import math

import numpy as np

try:
    import scipy.fft as _fft
    _FFT_KW = {"workers": -1}
except ImportError:  # numpy fallback
    _fft = np.fft
    _FFT_KW = {}


def shape(N, ndim=3):
    return (N + 1,) * ndim


def grf(N, seed, slope=-3.0, ndim=3):
    """Zero-mean unit-variance Gaussian random field with P(k) ~ k^slope."""
    rng = np.random.default_rng(seed)
    n = N + 1
    w = rng.standard_normal(shape(N, ndim))
    W = _fft.rfftn(w, **_FFT_KW)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    if ndim == 3:
        k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    else:
        k2 = kx[:, None] ** 2 + kz[None, :] ** 2
    k2.flat[0] = 1.0
    amp = k2 ** (slope / 4.0)          # |k|^(slope/2)
    amp.flat[0] = 0.0
    W *= amp
    f = _fft.irfftn(W, s=shape(N, ndim), **_FFT_KW)
    f -= f.mean()
    f /= f.std()
    return np.ascontiguousarray(f)


def coords(N):
    x = np.arange(N + 1, dtype=np.float64)
    return x[:, None, None], x[None, :, None], x[None, None, :]


def blob(N, centre, sigma, amplitude=1.0):
    """amplitude * exp(-|x - c|^2 / (2 sigma^2)), as a product of 1D factors
    (len(centre) = 3 or 2 coordinates)."""
    x = np.arange(N + 1, dtype=np.float64)
    g = [np.exp(-(x - centre[a]) ** 2 / (2.0 * sigma * sigma)) for a in range(len(centre))]
    if len(centre) == 2:
        return amplitude * g[0][:, None] * g[1][None, :]
    return amplitude * (g[0][:, None, None] * g[1][None, :, None]) * g[2][None, None, :]


def zero_boundary(f):
    f = f.copy()
    for a in range(f.ndim):
        idx = [slice(None)] * f.ndim
        idx[a] = 0
        f[tuple(idx)] = 0.0
        idx[a] = -1
        f[tuple(idx)] = 0.0
    return f


def normal(N, seed, zero_bdry=True, ndim=3):
    f = np.random.default_rng(seed).standard_normal(shape(N, ndim))
    return zero_boundary(f) if zero_bdry else f


def log_coefficients(N, seed_D, seed_mu, ndim=3):
    logD = np.clip(grf(N, seed_D, ndim=ndim), -math.log(100.0), math.log(100.0))
    logmua = math.log(0.05) + grf(N, seed_mu, ndim=ndim)
    return logD, logmua


def blob_source(N, seed, nblobs=16, noise=0.01, ndim=3):
    rng = np.random.default_rng(seed)
    q = np.zeros(shape(N, ndim))
    for _ in range(nblobs):
        c = rng.uniform(0.15 * N, 0.85 * N, size=ndim)
        s = rng.uniform(2.0, 6.0)
        a = rng.uniform(0.5, 1.5)
        q += blob(N, c, s, a)
    q += noise * rng.standard_normal(shape(N, ndim))
    return q


def constant_case(N=32):
    """Constant coefficients D = 1, mua = 0.1 and a centred blob (sigma 3)."""
    D = np.ones(shape(N))
    mua = np.full(shape(N), 0.1)
    q = blob(N, (N / 2, N / 2, N / 2), 3.0)
    return {"N": N, "logD": np.log(D), "logmua": np.log(mua), "D": D, "mua": mua, "q": q}


def grf_case(N, base_seed, ndim=3):
    """Log-normal GRF coefficients and a 16-blob source.  Seeds are
    base_seed+1 (log D), +2 (log mua), +3 (q), +4 (cotangent rhobar)."""
    logD, logmua = log_coefficients(N, base_seed + 1, base_seed + 2, ndim)
    q = blob_source(N, base_seed + 3, ndim=ndim)
    return {"N": N, "logD": logD, "logmua": logmua, "D": np.exp(logD), "mua": np.exp(logmua), "q": q,
            "rhobar": normal(N, base_seed + 4, ndim=ndim)}


def tangents(N, base_seed, ndim=3):
    """Tangents (dq, dlogD, dlogmua) and cotangent rhobar, seeds base_seed+1..+4."""
    return {"dq": normal(N, base_seed + 1, ndim=ndim), "dlogD": normal(N, base_seed + 2, zero_bdry=False, ndim=ndim),
            "dlogmua": normal(N, base_seed + 3, ndim=ndim), "rhobar": normal(N, base_seed + 4, ndim=ndim)}


# ---------------------------------------------------------------------------
# Grids with different cell counts per axis (the paper's data grid has
# (128, 64, 64) cells over 7.5 x 3.5 x 3.5 cm).  The same recipes on the
# vertex index grid: integer wavenumbers per axis for the GRF, blob centres
# ~ U[0.15 n_a, 0.85 n_a] per axis and sigma ~ U[2, 6] vertices.

def grf_shape(cells, seed, slope=-3.0):
    """grf on (nx+1, ny+1, nz+1) vertices."""
    rng = np.random.default_rng(seed)
    shp = tuple(c + 1 for c in cells)
    w = rng.standard_normal(shp)
    W = _fft.rfftn(w, **_FFT_KW)
    k0 = np.fft.fftfreq(shp[0]) * shp[0]
    k1 = np.fft.fftfreq(shp[1]) * shp[1]
    k2r = np.fft.rfftfreq(shp[2]) * shp[2]
    k2 = k0[:, None, None] ** 2 + k1[None, :, None] ** 2 + k2r[None, None, :] ** 2
    k2.flat[0] = 1.0
    amp = k2 ** (slope / 4.0)
    amp.flat[0] = 0.0
    W *= amp
    f = _fft.irfftn(W, s=shp, **_FFT_KW)
    f -= f.mean()
    f /= f.std()
    return np.ascontiguousarray(f)


def grid_case(cells, base_seed, nblobs=16, noise=0.01):
    """grf_case on a grid of `cells` = (nx, ny, nz): log D, log mua, a
    16-blob source and a cotangent (seeds base_seed+1..+4), plus tangents
    dq, dlogD, dlogmua (seeds base_seed+5..+7)."""
    shp = tuple(c + 1 for c in cells)
    logD = np.clip(grf_shape(cells, base_seed + 1), -math.log(100.0), math.log(100.0))
    logmua = math.log(0.05) + grf_shape(cells, base_seed + 2)
    rng = np.random.default_rng(base_seed + 3)
    idx = [np.arange(c, dtype=np.float64) for c in shp]
    q = np.zeros(shp)
    for _ in range(nblobs):
        c = [rng.uniform(0.15 * n, 0.85 * n) for n in cells]
        sg = rng.uniform(2.0, 6.0)
        a = rng.uniform(0.5, 1.5)
        g = [np.exp(-(idx[k] - c[k]) ** 2 / (2.0 * sg * sg)) for k in range(3)]
        q += a * (g[0][:, None, None] * g[1][None, :, None]) * g[2][None, None, :]
    q += noise * rng.standard_normal(shp)
    out = {"cells": tuple(cells), "logD": logD, "logmua": logmua, "D": np.exp(logD), "mua": np.exp(logmua), "q": q}
    for name, sd, zb in (("rhobar", 4, True), ("dq", 5, True), ("dlogD", 6, False), ("dlogmua", 7, True)):
        f = np.random.default_rng(base_seed + sd).standard_normal(shp)
        out[name] = zero_boundary(f) if zb else f
    return out


# Named workloads (sizes and seeds).
def small_constant():
    """32^3 cells, D = 1, mua = 0.1, centred blob; tangents seeds 1001-1004."""
    c = constant_case(32)
    c.update(tangents(32, 1000))
    return c


def grf_128():
    """128^3 cells, GRF coefficients, seeds 2001-2004."""
    return grf_case(128, 2000)


def grf_256():
    """256^3 cells, GRF coefficients, seeds 3001-3004."""
    return grf_case(256, 3000)


def grf_512():
    """512^3 cells, GRF coefficients, seeds 5001-5004."""
    return grf_case(512, 5000)


def serving_stream(nreq=512, sizes=(64, 96, 128, 192), seed=4999, rate=None):
    """Request descriptors for the serving stream: grid size, mode
    ('jvp' or 'vjp', 50/50), per-request field seed 4000+r and Poisson arrival
    times (exponential gaps with the given rate; None = all at t = 0)."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.array(sizes), size=nreq)
    modes = rng.choice(np.array(["jvp", "vjp"]), size=nreq)
    if rate is None:
        t = np.zeros(nreq)
    else:
        t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    return [{"id": r, "N": int(Ns[r]), "mode": str(modes[r]), "seed": 4000 + r, "arrival": float(t[r])}
            for r in range(nreq)]


# ---------------------------------------------------------------------------
# Device-side generators (serving requests draw their fields on the GPU from
# a per-request seeded torch generator; same recipes as above, a different
# random stream).

def grf_torch(N, gen, device, slope=-3.0, ndim=3):
    import torch
    n = N + 1
    w = torch.randn((n,) * ndim, generator=gen, device=device, dtype=torch.float64)
    W = torch.fft.rfftn(w)
    kx = torch.fft.fftfreq(n, device=device, dtype=torch.float64) * n
    kz = torch.fft.rfftfreq(n, device=device, dtype=torch.float64) * n
    if ndim == 3:
        k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    else:
        k2 = kx[:, None] ** 2 + kz[None, :] ** 2
    k2.view(-1)[0] = 1.0
    amp = k2 ** (slope / 4.0)
    amp.view(-1)[0] = 0.0
    f = torch.fft.irfftn(W * amp, s=(n,) * ndim)
    f = f - f.mean()
    f = f / f.std(correction=0)
    return f.contiguous()


def blob_source_torch(N, gen, device, nblobs=16, noise=0.01):
    import torch
    n = N + 1
    par = torch.rand((nblobs, 5), generator=gen, device=device, dtype=torch.float64).cpu().numpy()
    x = torch.arange(n, device=device, dtype=torch.float64)
    q = torch.zeros((n, n, n), device=device, dtype=torch.float64)
    for b in range(nblobs):
        c = 0.15 * N + 0.7 * N * par[b, :3]
        s = 2.0 + 4.0 * par[b, 3]
        a = 0.5 + par[b, 4]
        gx = torch.exp(-(x - c[0]) ** 2 / (2 * s * s))
        gy = torch.exp(-(x - c[1]) ** 2 / (2 * s * s))
        gz = torch.exp(-(x - c[2]) ** 2 / (2 * s * s))
        q += a * gx[:, None, None] * gy[None, :, None] * gz[None, None, :]
    q += noise * torch.randn((n, n, n), generator=gen, device=device, dtype=torch.float64)
    return q.contiguous()


def zero_boundary_torch(f):
    f[0] = 0
    f[-1] = 0
    f[:, 0] = 0
    f[:, -1] = 0
    if f.dim() == 3:
        f[:, :, 0] = 0
        f[:, :, -1] = 0
    return f
