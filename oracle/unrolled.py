"""Oracle for the unrolled adjoint of the fixed-cycle solver: the exact
derivative of rho = S_n(q; log D, log mua), n V(nu1, nu2)-cycles of the
three-dimensional solver from rho = 0 (interior) / g (boundary), with
respect to q, log D and log mua, through every step of every cycle --
smoothing, defect, restriction, prolongation, the coarsest solve and the
coarse coefficients (Sec. 2.2 Eq. (Eqcomp), reversed as in Sec. 2.4 Eq.
(EqcompT), with the coefficients as further inputs of each step).

Test infrastructure: used only by the tests.  Plain numpy, slow on
purpose; every function accepts complex arrays, so that the forward map can
be differentiated by complex steps to pin the reverse pass.  The steps and
readings are those of the solver (red-black Gauss-Seidel, red = (x+y+z)
even first, full weighting (1/64)(1,2,1)^3, trilinear I = 8 R^T, coarse
coefficients by full weighting with injection on the boundary, exact
coarsest solve, coarse corrections from 0).

Reverse pass of one step, with bars for cotangents (c_f = D_f / h^2 on
face f, d_i = sum_f c_f + mua_i):
* half-sweep of colour C, u'_i = (q_i + sum_j c_ij u_j) / d_i for i in C:
  v_i = ubar_i / d_i (i in C); qbar_i += v_i; mubar_i -= v_i u'_i;
  cbar_f += (v_a - v_b)(u'_b - u'_a) for f = (a, b); ubar_j += sum_i v_i c_ij
  (j not in C); ubar_i = 0 (i in C);
* defect r = q - A u (then qc = R r): rbar = R^T qcbar = I qcbar / 8;
  qbar += rbar; ubar -= A rbar; cbar_f -= (rbar_a - rbar_b)(u_a - u_b);
  mubar_i -= rbar_i u_i;
* prolongation u += I ec: ecbar = I^T ubar = 8 R ubar;
* coarsest solve u = A^-1 q: lam = A^-1 ubar, qbar = lam and the defect's
  coefficient terms with lam for rbar;
* coefficients: c_f = face(D_a, D_b) / h_k^2 on every level, and
  D_k, mua_k = coarsening of D_{k-1}, mua_{k-1}, whose transpose carries the
  coarse cotangents to the finest level; finally logD_bar = D Dbar,
  logmua_bar = mua mubar.
"""
import numpy as np


def level_sizes(N):
    Ns = [N]
    while Ns[-1] > 3:
        Ns.append(Ns[-1] // 2)
    return Ns


_W = (1.0, 2.0, 1.0)


def _fw_interior(f, Nc):
    """sum over a, b, c in {-1,0,1} of w_a w_b w_c f[2X+a, 2Y+b, 2Z+c] / 64,
    coarse interior."""
    s = np.zeros((Nc - 1,) * 3, dtype=f.dtype)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                s = s + _W[a + 1] * _W[b + 1] * _W[c + 1] * f[2 + a:2 * Nc - 1 + a:2, 2 + b:2 * Nc - 1 + b:2,
                                                                2 + c:2 * Nc - 1 + c:2]
    return s / 64.0


def _fw_interior_T(s, Nf):
    """Transpose of _fw_interior: a fine array from coarse-interior values."""
    Nc = Nf // 2
    f = np.zeros((Nf + 1,) * 3, dtype=s.dtype)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                f[2 + a:2 * Nc - 1 + a:2, 2 + b:2 * Nc - 1 + b:2, 2 + c:2 * Nc - 1 + c:2] += (
                    _W[a + 1] * _W[b + 1] * _W[c + 1] / 64.0) * s
    return f


def coarsen(f):
    Nc = (f.shape[0] - 1) // 2
    c = f[::2, ::2, ::2].copy()
    c[1:-1, 1:-1, 1:-1] = _fw_interior(f, Nc)
    return c


def coarsen_T(cbar, Nf):
    """Transpose of coarsen (coarse cotangent -> fine cotangent)."""
    f = _fw_interior_T(cbar[1:-1, 1:-1, 1:-1], Nf)
    inj = cbar.copy()
    inj[1:-1, 1:-1, 1:-1] = 0.0
    f[::2, ::2, ::2] += inj
    return f


def restrict(r):
    Nc = (r.shape[0] - 1) // 2
    qc = np.zeros((Nc + 1,) * 3, dtype=r.dtype)
    qc[1:-1, 1:-1, 1:-1] = _fw_interior(r, Nc)
    return qc


def interpolate(ec):
    """Trilinear interpolation of a coarse field to every fine vertex."""
    e = ec
    for ax in range(3):
        n = e.shape[ax]
        sh = list(e.shape)
        sh[ax] = 2 * (n - 1) + 1
        out = np.zeros(sh, dtype=e.dtype)
        idx_even = [slice(None)] * 3
        idx_even[ax] = slice(0, None, 2)
        out[tuple(idx_even)] = e
        idx_odd = [slice(None)] * 3
        idx_odd[ax] = slice(1, None, 2)
        lo = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi = [slice(None)] * 3
        hi[ax] = slice(1, None)
        out[tuple(idx_odd)] = 0.5 * (e[tuple(lo)] + e[tuple(hi)])
        e = out
    return e


_NB = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def _sh(a, d):
    """a shifted so that out[i] = a[i + d] on the interior block (x, y, z in 1..N-1)."""
    N = a.shape[0] - 1
    return a[1 + d[0]:N + d[0], 1 + d[1]:N + d[1], 1 + d[2]:N + d[2]]


class Unrolled:
    def __init__(self, D, mua, h=1.0, g=0.0, harmonic=False):
        self.N = D.shape[0] - 1
        self.Ns = level_sizes(self.N)
        self.L = len(self.Ns)
        self.h = h
        self.g = g
        self.harmonic = harmonic
        self.set_coefficients(D, mua)

    def set_coefficients(self, D, mua):
        self.D = [D]
        self.mu = [mua]
        for _ in range(1, self.L):
            self.D.append(coarsen(self.D[-1]))
            self.mu.append(coarsen(self.mu[-1]))

    def face(self, a, b):
        return 2.0 * a * b / (a + b) if self.harmonic else 0.5 * (a + b)

    def dface(self, a, b):
        """(d face / d a, d face / d b)."""
        if self.harmonic:
            s = a + b
            return 2.0 * b * b / (s * s), 2.0 * a * a / (s * s)
        return 0.5 + 0 * a, 0.5 + 0 * b

    def coup(self, k):
        """couplings c to the six neighbours of the interior vertices."""
        D = self.D[k]
        ih2 = 1.0 / (self.h * 2.0 ** k) ** 2
        Di = _sh(D, (0, 0, 0))
        return [self.face(Di, _sh(D, d)) * ih2 for d in _NB]

    def colour_mask(self, k, colour):
        n = self.Ns[k] + 1
        x = np.arange(1, n - 1)
        return (x[:, None, None] + x[None, :, None] + x[None, None, :]) % 2 == colour

    def apply(self, k, u):
        cs = self.coup(k)
        ui = _sh(u, (0, 0, 0))
        out = np.zeros_like(u)
        acc = _sh(self.mu[k], (0, 0, 0)) * ui
        for c, d in zip(cs, _NB):
            acc = acc + c * (ui - _sh(u, d))
        out[1:-1, 1:-1, 1:-1] = acc
        return out

    def defect(self, k, u, q):
        r = np.zeros_like(u)
        r[1:-1, 1:-1, 1:-1] = _sh(q, (0, 0, 0)) - self.apply(k, u)[1:-1, 1:-1, 1:-1]
        return r

    def gs_half(self, k, u, q, colour):
        cs = self.coup(k)
        num = _sh(q, (0, 0, 0)) + sum(c * _sh(u, d) for c, d in zip(cs, _NB))
        den = sum(cs) + _sh(self.mu[k], (0, 0, 0))
        m = self.colour_mask(k, colour)
        ui = u[1:-1, 1:-1, 1:-1]
        ui[m] = (num / den)[m]

    def exact(self, k, q, u):
        N = self.Ns[k]
        m = N - 1
        idx = -np.ones((N + 1,) * 3, dtype=int)
        t = 0
        for x in range(1, N):
            for y in range(1, N):
                for z in range(1, N):
                    idx[x, y, z] = t
                    t += 1
        D, mu = self.D[k], self.mu[k]
        ih2 = 1.0 / (self.h * 2.0 ** k) ** 2
        dt = np.result_type(D, mu, q, u)
        A = np.zeros((m ** 3, m ** 3), dtype=dt)
        b = np.zeros(m ** 3, dtype=dt)
        for x in range(1, N):
            for y in range(1, N):
                for z in range(1, N):
                    r = idx[x, y, z]
                    A[r, r] += mu[x, y, z]
                    b[r] += q[x, y, z]
                    for d in _NB:
                        j = (x + d[0], y + d[1], z + d[2])
                        c = self.face(D[x, y, z], D[j]) * ih2
                        A[r, r] += c
                        if idx[j] >= 0:
                            A[r, idx[j]] -= c
                        else:
                            b[r] += c * u[j]
        u[1:-1, 1:-1, 1:-1] = np.linalg.solve(A, b).reshape(m, m, m)

    # -- forward ----------------------------------------------------------------------
    def vcycle(self, k, u, q, nu1, nu2, tape=None):
        """One V(nu1, nu2)-cycle in place; with a tape, record what the
        reverse pass needs (the state after every half-sweep, the state the
        defect reads, the coarsest solution)."""
        rec = {} if tape is not None else None
        if k == self.L - 1:
            self.exact(k, q, u)
            if rec is not None:
                rec["u"] = u.copy()
                tape.append((k, rec))
            return
        states = []
        for _ in range(nu1):
            for colour in (0, 1):
                self.gs_half(k, u, q, colour)
                states.append(u.copy())
        if rec is not None:
            rec["pre"] = states
            rec["u_def"] = u.copy()
            tape.append((k, rec))
        qc = restrict(self.defect(k, u, q))
        uc = np.zeros_like(qc)
        self.vcycle(k + 1, uc, qc, nu1, nu2, tape)
        u[1:-1, 1:-1, 1:-1] += interpolate(uc)[1:-1, 1:-1, 1:-1]
        states = []
        for _ in range(nu2):
            for colour in (0, 1):
                self.gs_half(k, u, q, colour)
                states.append(u.copy())
        if rec is not None:
            rec["post"] = states

    def forward(self, q, n, nu1=2, nu2=2):
        u = np.zeros(q.shape, dtype=np.result_type(q, self.D[0]))
        u[0, :, :] = u[-1, :, :] = u[:, 0, :] = u[:, -1, :] = u[:, :, 0] = u[:, :, -1] = self.g
        for _ in range(n):
            self.vcycle(0, u, q, nu1, nu2)
        return u

    # -- reverse ----------------------------------------------------------------------
    def _coef_terms(self, k, abar, u, Db, mb):
        """cbar_f -= (abar_a - abar_b)(u_a - u_b), mubar -= abar u (interior),
        carried to Dbar through the face derivative."""
        ih2 = 1.0 / (self.h * 2.0 ** k) ** 2
        D = self.D[k]
        mb[1:-1, 1:-1, 1:-1] -= _sh(abar, (0, 0, 0)) * _sh(u, (0, 0, 0))
        self._face_accumulate(k, -1.0, abar, u, Db)

    def _face_accumulate(self, k, sign, a, u, Db):
        """Db_v += sign * sum over faces f=(v,w) with an interior endpoint of
        (a_v - a_w)(u_v - u_w) dface/dD_v / h_k^2 (a vanishes off the interior)."""
        ih2 = 1.0 / (self.h * 2.0 ** k) ** 2
        D = self.D[k]
        N = self.Ns[k]
        for ax in range(3):
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, N)
            hi[ax] = slice(1, N + 1)
            lo, hi = tuple(lo), tuple(hi)
            t = sign * (a[lo] - a[hi]) * (u[lo] - u[hi]) * ih2
            da, db = self.dface(D[lo], D[hi])
            # faces between two boundary vertices carry a = 0 on both ends
            Db[lo] += t * da
            Db[hi] += t * db

    def vcycle_rev(self, tape, ubar, qbars, Dbs, mbs, nu1, nu2):
        """Reverse of one recorded V-cycle.  ubar: cotangent of the level-0
        iterate after the cycle; returns the cotangent before it.  qbars,
        Dbs, mbs: per-level accumulators (qbars[0] is qbar of the finest
        right-hand side)."""
        recs = dict()
        order = []
        for k, rec in tape:
            recs[k] = rec
            order.append(k)
        return self._rev_level(0, recs, ubar, qbars, Dbs, mbs, nu1, nu2)

    def _rev_half(self, k, colour, up, ubar, qbar, Db, mb):
        cs = self.coup(k)
        d = sum(cs) + _sh(self.mu[k], (0, 0, 0))
        m = self.colour_mask(k, colour)
        v = np.zeros_like(ubar)
        vi = v[1:-1, 1:-1, 1:-1]
        vi[m] = (_sh(ubar, (0, 0, 0)) / d)[m]
        qbar[1:-1, 1:-1, 1:-1] += vi
        mb[1:-1, 1:-1, 1:-1] -= vi * _sh(up, (0, 0, 0))
        # cbar_f = (v_a - v_b)(u'_b - u'_a)
        self._face_accumulate(k, -1.0, v, up, Db)
        # ubar_j += sum_i v_i c_ij for j not in C; ubar_i = 0 for i in C
        gath = sum(c * _sh(v, dd) for c, dd in zip(cs, _NB))
        ui = ubar[1:-1, 1:-1, 1:-1]
        ui[~m] += gath[~m]
        ui[m] = 0.0

    def _rev_level(self, k, recs, ubar, qbars, Dbs, mbs, nu1, nu2):
        rec = recs[k]
        qbar, Db, mb = qbars[k], Dbs[k], mbs[k]
        ubar = ubar.copy()
        ubar[0, :, :] = ubar[-1, :, :] = ubar[:, 0, :] = ubar[:, -1, :] = ubar[:, :, 0] = ubar[:, :, -1] = 0.0
        if k == self.L - 1:
            lam = np.zeros_like(ubar)
            self.exact(k, ubar, lam)
            qbar += lam
            self._coef_terms(k, lam, rec["u"], Db, mb)
            return np.zeros_like(ubar)
        post = rec["post"]
        colours = [0, 1] * nu2
        for h in range(len(post) - 1, -1, -1):
            self._rev_half(k, colours[h], post[h], ubar, qbar, Db, mb)
        # prolongation: ecbar = 8 R ubar
        ecbar = 8.0 * restrict(ubar)
        self._rev_level(k + 1, recs, ecbar, qbars, Dbs, mbs, nu1, nu2)
        # restriction: rbar = I qcbar / 8; defect: qbar += rbar, ubar -= A rbar
        rbar = np.zeros_like(ubar)
        rbar[1:-1, 1:-1, 1:-1] = interpolate(qbars[k + 1])[1:-1, 1:-1, 1:-1] / 8.0
        qbars[k + 1][...] = 0.0   # consumed
        qbar += rbar
        ubar -= self.apply(k, rbar)
        self._coef_terms(k, rbar, rec["u_def"], Db, mb)
        pre = rec["pre"]
        colours = [0, 1] * nu1
        for h in range(len(pre) - 1, -1, -1):
            self._rev_half(k, colours[h], pre[h], ubar, qbar, Db, mb)
        return ubar

    def vjp(self, q, w, n, nu1=2, nu2=2):
        """(rho, (qbar, logD_bar, logmua_bar)) of S_n at q, cotangent w."""
        u = np.zeros(q.shape, dtype=np.float64)
        u[0, :, :] = u[-1, :, :] = u[:, 0, :] = u[:, -1, :] = u[:, :, 0] = u[:, :, -1] = self.g
        tapes = []
        for _ in range(n):
            tape = []
            self.vcycle(0, u, q, nu1, nu2, tape)
            tapes.append(tape)
        rho = u.copy()
        zeros = lambda k: np.zeros((self.Ns[k] + 1,) * 3)
        qbars = [zeros(k) for k in range(self.L)]
        Dbs = [zeros(k) for k in range(self.L)]
        mbs = [zeros(k) for k in range(self.L)]
        ubar = np.array(w, dtype=np.float64)
        for tape in reversed(tapes):
            ubar = self.vcycle_rev(tape, ubar, qbars, Dbs, mbs, nu1, nu2)
        for k in range(self.L - 1, 0, -1):
            Dbs[k - 1] += coarsen_T(Dbs[k], self.Ns[k - 1])
            mbs[k - 1] += coarsen_T(mbs[k], self.Ns[k - 1])
        return rho, (qbars[0], Dbs[0] * self.D[0], mbs[0] * self.mu[0])
