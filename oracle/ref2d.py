"""Oracle for the two-dimensional five-point variant of the solver.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never imports it.  Plain float64 numpy,
written from the method's description (Sec. 2.2-2.4) in the order the paper
gives its steps; slow on purpose and vectorised only where the result does
not depend on the order (a red-black half-sweep updates points that are not
each other's neighbours, so all of them may be updated at once).

Grid: N cells per axis, (N+1)^2 vertices, arrays of shape (N+1, N+1), x
slowest, y fastest; spacing h on the finest level, 2^k h on level k;
Dirichlet values g on the boundary.  The readings are those of the
three-dimensional solver, with two coordinates:

* operator (Eq. (maineq), discretised): for interior i,
  (A u)_i = sum over the 4 neighbours j of D_f (u_i - u_j) / h^2 + mua_i u_i,
  with the face value D_f the arithmetic mean (D_i + D_j)/2 or, as an
  option, the harmonic mean 2 D_i D_j / (D_i + D_j);
* red-black Gauss-Seidel (Sec. 2.2): red = (x + y) even in the level's own
  coordinates; a half-sweep sets u_i = (q_i + sum_j c_ij u_j) / (sum_j c_ij
  + mua_i) on one colour; the forward cycle sweeps red before black;
* restriction (Eq. (rest), as a tensor product): full weighting
  (1/16)(1,2,1) x (1,2,1) on coarse interior vertices; prolongation
  (Sec. 2.3.3): bilinear interpolation, I = 4 R^T;
* coarse operators (Sec. 2.2): rediscretised with spacing 2^k h from D and
  mua transferred by full weighting (injection on coarse boundary
  vertices); coarse corrections start from 0 (Sec. 2.3.1); the coarsest
  level (N in {2, 3}) is solved exactly;
* solver: V(nu1, nu2)-cycles from u = 0 (interior) until ||q - A u|| /
  ||q - A u_0|| <= rtol, or exactly fixed_cycles cycles (Sec. 2.4);
* pull-back (Sec. 2.4, Eq. (EqcompT)): the steps of every cycle reversed and
  transposed, which is a black-before-red V(nu2, nu1)-cycle on A lam = w;
* coefficient gradients: the adjoint-state derivative of the discrete
  solution, g_logmua = -mua lam rho on interior vertices and
  g_logD_v = -sum over faces f = (a, b) at v of dD_f/dlogD_v (lam_a - lam_b)
  (rho_a - rho_b) / h^2, with lam = 0 and rho = g on boundary vertices.
"""
import numpy as np


def level_sizes(N):
    """N, N/2, ... down to the first size in {2, 3}; N must be c 2^m, c in {2, 3}."""
    Ns = [int(N)]
    while Ns[-1] > 3:
        if Ns[-1] % 2:
            raise ValueError("N = %d is not c*2^m with c in {2, 3}" % N)
        Ns.append(Ns[-1] // 2)
    if Ns[-1] not in (2, 3):
        raise ValueError("N = %d is not c*2^m with c in {2, 3}" % N)
    return Ns


_W = (1.0, 2.0, 1.0)


def _coarse_interior_sum(f, Nc):
    """sum over a, b in {-1, 0, 1} of w_a w_b f[2X + a, 2Y + b] for coarse
    interior (X, Y), w = (1, 2, 1)."""
    s = np.zeros((Nc - 1, Nc - 1), dtype=f.dtype)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            s += _W[a + 1] * _W[b + 1] * f[2 + a:2 * Nc - 1 + a:2, 2 + b:2 * Nc - 1 + b:2]
    return s


def coarsen_field(f):
    """Coefficient transfer: full weighting on coarse interior vertices,
    injection on coarse boundary vertices."""
    Nc = (f.shape[0] - 1) // 2
    c = f[::2, ::2].copy()
    c[1:-1, 1:-1] = _coarse_interior_sum(f, Nc) / 16.0
    return c


def restrict(r):
    """Full weighting of a fine defect to the coarse level (0 on the coarse
    boundary)."""
    Nc = (r.shape[0] - 1) // 2
    qc = np.zeros((Nc + 1, Nc + 1), dtype=r.dtype)
    qc[1:-1, 1:-1] = _coarse_interior_sum(r, Nc) / 16.0
    return qc


def interpolate(ec):
    """Bilinear interpolation of a coarse field to every fine vertex."""
    Nc = ec.shape[0] - 1
    e = np.zeros((2 * Nc + 1, 2 * Nc + 1), dtype=ec.dtype)
    e[::2, ::2] = ec
    e[1::2, ::2] = 0.5 * (ec[:-1, :] + ec[1:, :])
    e[::2, 1::2] = 0.5 * (ec[:, :-1] + ec[:, 1:])
    e[1::2, 1::2] = 0.25 * (ec[:-1, :-1] + ec[1:, :-1] + ec[:-1, 1:] + ec[1:, 1:])
    return e


def prolong_add(ec, u):
    """u += I ec on fine interior vertices (the boundary keeps its values)."""
    u[1:-1, 1:-1] += interpolate(ec)[1:-1, 1:-1]


class Hierarchy2D:
    def __init__(self, D, mua, h=1.0, g=0.0, face_mean="arith"):
        D = np.asarray(D)
        mua = np.asarray(mua)
        self.N = D.shape[0] - 1
        self.Ns = level_sizes(self.N)
        self.L = len(self.Ns)
        self.g = g
        self.harmonic = face_mean == "harmonic"
        self.hs = [h * 2.0 ** k for k in range(self.L)]
        self.D = [D]
        self.mu = [mua]
        for k in range(1, self.L):
            self.D.append(coarsen_field(self.D[-1]))
            self.mu.append(coarsen_field(self.mu[-1]))

    # -- the operator ---------------------------------------------------------
    def face(self, Da, Db):
        if self.harmonic:
            return 2.0 * Da * Db / (Da + Db)
        return 0.5 * (Da + Db)

    def couplings(self, k):
        """c_ij = D_f / h^2 of the interior vertices to their x-1, x+1, y-1,
        y+1 neighbours, each of shape (N-1, N-1)."""
        D = self.D[k]
        ih2 = 1.0 / self.hs[k] ** 2
        Di = D[1:-1, 1:-1]
        return (self.face(Di, D[:-2, 1:-1]) * ih2, self.face(Di, D[2:, 1:-1]) * ih2,
                self.face(Di, D[1:-1, :-2]) * ih2, self.face(Di, D[1:-1, 2:]) * ih2)

    def apply(self, k, u):
        """A u on interior vertices, 0 on the boundary."""
        cxm, cxp, cym, cyp = self.couplings(k)
        ui = u[1:-1, 1:-1]
        out = np.zeros_like(u)
        out[1:-1, 1:-1] = (cxm * (ui - u[:-2, 1:-1]) + cxp * (ui - u[2:, 1:-1]) + cym * (ui - u[1:-1, :-2])
                           + cyp * (ui - u[1:-1, 2:]) + self.mu[k][1:-1, 1:-1] * ui)
        return out

    def defect(self, k, u, q):
        """q - A u on interior vertices (Sec. 2.3.2), 0 on the boundary."""
        r = np.zeros_like(u)
        r[1:-1, 1:-1] = q[1:-1, 1:-1] - self.apply(k, u)[1:-1, 1:-1]
        return r

    def gs_half(self, k, u, q, colour):
        """One red (colour 0) or black (colour 1) half-sweep, in place."""
        cxm, cxp, cym, cyp = self.couplings(k)
        num = (q[1:-1, 1:-1] + cxm * u[:-2, 1:-1] + cxp * u[2:, 1:-1] + cym * u[1:-1, :-2]
               + cyp * u[1:-1, 2:])
        den = cxm + cxp + cym + cyp + self.mu[k][1:-1, 1:-1]
        n = self.Ns[k] + 1
        x = np.arange(1, n - 1)
        mask = (x[:, None] + x[None, :]) % 2 == colour
        ui = u[1:-1, 1:-1]
        ui[mask] = (num / den)[mask]

    def exact(self, k, q, u):
        """Solve A u = q exactly on level k's interior, the boundary values
        of u moved to the right-hand side."""
        N = self.Ns[k]
        m = N - 1
        D, mu = self.D[k], self.mu[k]
        ih2 = 1.0 / self.hs[k] ** 2
        A = np.zeros((m * m, m * m), dtype=np.result_type(D, u))
        b = np.zeros(m * m, dtype=np.result_type(q, u, D))
        for x in range(1, N):
            for y in range(1, N):
                t = (x - 1) * m + (y - 1)
                A[t, t] += mu[x, y]
                b[t] += q[x, y]
                for xa, ya in ((x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)):
                    c = self.face(D[x, y], D[xa, ya]) * ih2
                    A[t, t] += c
                    if 0 < xa < N and 0 < ya < N:
                        A[t, (xa - 1) * m + (ya - 1)] -= c
                    else:
                        b[t] += c * u[xa, ya]
        u[1:-1, 1:-1] = np.linalg.solve(A, b).reshape(m, m)

    # -- the cycle --------------------------------------------------------------
    def vcycle(self, k, u, q, order, nu1, nu2):
        """One V(nu1, nu2)-cycle in place on u; order 0 sweeps red before
        black, order 1 black before red."""
        if k == self.L - 1:
            self.exact(k, q, u)
            return
        first, second = (1, 0) if order else (0, 1)
        for _ in range(nu1):
            self.gs_half(k, u, q, first)
            self.gs_half(k, u, q, second)
        qc = restrict(self.defect(k, u, q))
        uc = np.zeros_like(qc)
        self.vcycle(k + 1, uc, qc, order, nu1, nu2)
        prolong_add(uc, u)
        for _ in range(nu2):
            self.gs_half(k, u, q, first)
            self.gs_half(k, u, q, second)

    def cycles(self, q, u, n, order=0, nu1=2, nu2=2):
        u = np.array(u, dtype=np.float64)
        for _ in range(n):
            self.vcycle(0, u, q, order, nu1, nu2)
        return u

    def solve(self, b, bc, order, nu1, nu2, rtol, max_cycles, fixed_cycles):
        u = np.zeros_like(b, dtype=np.float64)
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = bc
        r0 = np.linalg.norm(self.defect(0, u, b))
        info = {"cycles": 0, "rel_residual": 0.0, "status": 0}
        if fixed_cycles > 0:
            for _ in range(fixed_cycles):
                self.vcycle(0, u, b, order, nu1, nu2)
            info["cycles"] = fixed_cycles
            info["rel_residual"] = np.linalg.norm(self.defect(0, u, b)) / (r0 if r0 > 0 else 1.0)
            return u, info
        if r0 == 0.0:
            return u, info
        for c in range(1, max_cycles + 1):
            self.vcycle(0, u, b, order, nu1, nu2)
            rel = np.linalg.norm(self.defect(0, u, b)) / r0
            info["cycles"], info["rel_residual"] = c, rel
            if rel <= rtol:
                return u, info
        info["status"] = 3
        return u, info

    # -- solver, push-forward and pull-back ----------------------------------------
    def forward(self, q, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """rho = S q (Eq. (Eqcomp))."""
        return self.solve(q, self.g, 0, nu1, nu2, rtol, max_cycles, fixed_cycles)

    def dface(self, Da, Db):
        """(dD_f/dlogD_a, dD_f/dlogD_b)."""
        if self.harmonic:
            s = Da + Db
            return 2.0 * Db * Db * Da / (s * s), 2.0 * Da * Da * Db / (s * s)
        return 0.5 * Da, 0.5 * Db

    def tangent_rhs(self, rho, dq, dlogD, dlogmua):
        """dq - (dA) rho on interior vertices: the right-hand side of the
        push-forward solve (dA along dlogD and dlogmua)."""
        D = self.D[0]
        ih2 = 1.0 / self.hs[0] ** 2
        Di, dDi = D[1:-1, 1:-1], dlogD[1:-1, 1:-1]
        ri = rho[1:-1, 1:-1]
        acc = self.mu[0][1:-1, 1:-1] * dlogmua[1:-1, 1:-1] * ri
        for sl in ((slice(None, -2), slice(1, -1)), (slice(2, None), slice(1, -1)),
                   (slice(1, -1), slice(None, -2)), (slice(1, -1), slice(2, None))):
            da, db = self.dface(Di, D[sl])
            acc = acc + (da * dDi + db * dlogD[sl]) * ih2 * (ri - rho[sl])
        out = np.zeros_like(rho)
        out[1:-1, 1:-1] = dq[1:-1, 1:-1] - acc
        return out

    def jvp(self, rho, dq, dlogD, dlogmua, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """drho = S (dq - dA rho) (Sec. 2.4: S is linear in q for fixed
        coefficients, so its Jacobian in q is S itself)."""
        rhs = self.tangent_rhs(rho, dq, dlogD, dlogmua)
        return self.solve(rhs, 0.0, 0, nu1, nu2, rtol, max_cycles, fixed_cycles)

    def pullback(self, w, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """qbar = S^T w: black-before-red V(nu2, nu1)-cycles on A qbar = w."""
        w = np.array(w, dtype=np.float64)
        w[0, :] = w[-1, :] = w[:, 0] = w[:, -1] = 0.0
        return self.solve(w, 0.0, 1, nu2, nu1, rtol, max_cycles, fixed_cycles)

    def coef_grads(self, rho, lam):
        """(g_logD, g_logmua) from the forward solution and the adjoint state,
        face by face."""
        N = self.N
        D = self.D[0]
        ih2 = 1.0 / self.hs[0] ** 2
        lam = lam.copy()
        lam[0, :] = lam[-1, :] = lam[:, 0] = lam[:, -1] = 0.0
        gD = np.zeros_like(rho)
        gmu = np.zeros_like(rho)
        gmu[1:-1, 1:-1] = -self.mu[0][1:-1, 1:-1] * lam[1:-1, 1:-1] * rho[1:-1, 1:-1]
        for (xa, ya), (xb, yb) in self._faces():
            t = (lam[xa, ya] - lam[xb, yb]) * (rho[xa, ya] - rho[xb, yb]) * ih2
            da, db = self.dface(D[xa, ya], D[xb, yb])
            gD[xa, ya] -= da * t
            gD[xb, yb] -= db * t
        return gD, gmu

    def _faces(self):
        """Every face of the grid with at least one interior endpoint."""
        N = self.N
        inside = lambda x, y: 0 < x < N and 0 < y < N
        for x in range(N + 1):
            for y in range(N + 1):
                for xb, yb in ((x + 1, y), (x, y + 1)):
                    if xb <= N and yb <= N and (inside(x, y) or inside(xb, yb)):
                        yield (x, y), (xb, yb)

    def vjp(self, rho, w, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """(qbar, g_logD, g_logmua) = pull-back of the cotangent w."""
        lam, info = self.pullback(w, rtol, max_cycles, fixed_cycles, nu1, nu2)
        gD, gmu = self.coef_grads(rho, lam)
        return (lam, gD, gmu), info
