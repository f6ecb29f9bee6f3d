"""Brute-force dense and sparse assembly of the discrete operator, for pins.

Written inside the tests from the definition of the discretisation, with no
use of the oracle or of the GPU library: for every interior vertex i and each
of its six neighbours j the face coefficient c_ij = D_f / h^2 (D_f the
arithmetic or harmonic mean of D_i and D_j) adds c_ij to A_ii and -c_ij to
A_ij, or c_ij * g to the right-hand side when j is a boundary vertex; mua_i
adds to A_ii.  Works in complex arithmetic for the complex-step derivative.
"""
import numpy as np
import scipy.sparse as sp


def interior_index(N):
    n = N + 1
    idx = -np.ones((n, n, n), dtype=np.int64)
    m = 0
    for x in range(1, N):
        for y in range(1, N):
            for z in range(1, N):
                idx[x, y, z] = m
                m += 1
    return idx, m


def _face(Da, Db, harmonic):
    return 2 * Da * Db / (Da + Db) if harmonic else 0.5 * (Da + Db)


def assemble_dense(D, mua, h=1.0, g=0.0, harmonic=False):
    """Return (A, bvec, idx): A u_int = q_int + bvec for the interior unknowns."""
    N = D.shape[0] - 1
    idx, m = interior_index(N)
    dt = np.result_type(D, mua, complex) if np.iscomplexobj(D) or np.iscomplexobj(mua) else np.float64
    A = np.zeros((m, m), dtype=dt)
    b = np.zeros(m, dtype=dt)
    nbrs = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for x in range(1, N):
        for y in range(1, N):
            for z in range(1, N):
                r = idx[x, y, z]
                A[r, r] += mua[x, y, z]
                for dx, dy, dz in nbrs:
                    j = (x + dx, y + dy, z + dz)
                    c = _face(D[x, y, z], D[j], harmonic) / h ** 2
                    A[r, r] += c
                    if idx[j] >= 0:
                        A[r, idx[j]] -= c
                    else:
                        b[r] += c * g
    return A, b, idx


def assemble_sparse(D, mua, h=1.0, harmonic=False):
    """CSR matrix of A on interior unknowns (homogeneous boundary), vectorised."""
    N = D.shape[0] - 1
    n = N + 1
    idx, m = interior_index(N)
    sl = slice(1, N)
    I = idx[sl, sl, sl].ravel()
    diag = mua[sl, sl, sl].ravel().astype(np.float64).copy()
    rows, cols, vals = [], [], []
    for ax in range(3):
        for s in (1, -1):
            sh = [slice(1, N)] * 3
            sh[ax] = slice(1 + s, N + s)
            Dj = D[tuple(sh)].ravel()
            c = _face(D[sl, sl, sl].ravel(), Dj, harmonic) / h ** 2
            diag += c
            J = idx[tuple(sh)].ravel()
            keep = J >= 0
            rows.append(I[keep]); cols.append(J[keep]); vals.append(-c[keep])
    rows.append(I); cols.append(I); vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))
    return A, idx


def scatter(vec, idx, bc=0.0):
    """Interior vector -> full (N+1)^3 array with boundary value bc."""
    out = np.full(idx.shape, bc, dtype=vec.dtype)
    mask = idx >= 0
    out[mask] = vec[idx[mask]]
    return out


def gather(f, idx):
    mask = idx >= 0
    out = np.empty(int(mask.sum()), dtype=f.dtype)
    out[idx[mask]] = f[mask]
    return out
