"""Oracle for three-dimensional grids whose axes have different cell counts
and spacings: the paper's data grid, (128, 64, 64) over (7.5, 3.5, 3.5) cm
(Sec. 2.5.1, Data), on which the response of Eq. (response) (Sec. 2.5.2) and
the likelihood of Eq. (likelihood) (Sec. 2.5.4) are evaluated.

Test infrastructure: only the tests use it; the product path never imports
it.  Plain float64 numpy, written from the method's description (Sec.
2.2-2.4) in the order the paper gives its steps, slow on purpose; a
red-black half-sweep updates points that are not each other's neighbours,
so all points of one colour are updated at once.  Every function accepts
complex arrays, so that the solver can be differentiated by complex steps.

Grid: n = (nx, ny, nz) cells, (nx+1, ny+1, nz+1) vertices, arrays of that
shape in C order (x slowest, z fastest); spacing h = (hx, hy, hz) on the
finest level, 2^k h on level k; Dirichlet values g on the boundary.  The
readings are those of the cubic solver, axis by axis:

* operator (Eq. (maineq), second-order finite differences): for interior i,
  (A u)_i = sum over the 6 neighbours j of D_f (u_i - u_j) / h_a^2 +
  mua_i u_i, with h_a the spacing of the axis the face lies along and the
  face value D_f the arithmetic mean (D_i + D_j)/2 or, as an option, the
  harmonic mean 2 D_i D_j / (D_i + D_j);
* levels: every axis halves its cell count from one level to the next until
  the smallest reaches 2 or 3 (so each count must be c 2^m with the same m
  below that axis's coarsest size); the coarsest level is solved exactly;
* red-black Gauss-Seidel: red = (x + y + z) even in the level's own
  coordinates, red first in the forward cycle;
* restriction: full weighting (1/64)(1,2,1)^3 (Eq. (rest) along each axis)
  on coarse interior vertices; prolongation: trilinear, I = 2^3 R^T;
* coarse coefficients: full weighting on coarse interior vertices,
  injection on coarse boundary vertices; coarse corrections start from 0;
* solver: V(nu1, nu2)-cycles from u = 0 (interior) / g (boundary) until
  ||q - A u|| / ||q - A u_0|| <= rtol, or exactly fixed_cycles (Sec. 2.4);
* pull-back: the transposed cycle, black before red with the smoothing
  counts exchanged, on A lam = w (pinned against S_n^T built column by
  column in the tests);
* coefficient gradients: the adjoint-state derivative of the discrete
  solution, g_logmua = -mua lam rho on interior vertices and
  g_logD_v = -sum over faces f = (a, b) at v of dD_f/dlogD_v (lam_a - lam_b)
  (rho_a - rho_b) / h_f^2, with lam = 0 and rho = g on boundary vertices.
"""
import numpy as np

_W = (1.0, 2.0, 1.0)


def level_shapes(n):
    """Cell counts of every level: all axes halve until the smallest count
    is 2 or 3."""
    shapes = [tuple(int(c) for c in n)]
    while min(shapes[-1]) > 3:
        if any(c % 2 for c in shapes[-1]):
            raise ValueError("cell counts %s do not halve down to 2 or 3" % (n,))
        shapes.append(tuple(c // 2 for c in shapes[-1]))
    if min(shapes[-1]) not in (2, 3) or min(shapes[-1]) < 2:
        raise ValueError("cell counts %s do not halve down to 2 or 3" % (n,))
    return shapes


def _fw_interior(f):
    """sum over a, b, c in {-1, 0, 1} of w_a w_b w_c f[2X+a, 2Y+b, 2Z+c] / 64
    on the coarse interior vertices."""
    nc = [(s - 1) // 2 for s in f.shape]
    out = np.zeros(tuple(c - 1 for c in nc), dtype=f.dtype)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                out = out + _W[a + 1] * _W[b + 1] * _W[c + 1] * f[
                    2 + a:2 * nc[0] - 1 + a:2, 2 + b:2 * nc[1] - 1 + b:2, 2 + c:2 * nc[2] - 1 + c:2]
    return out / 64.0


def coarsen_field(f):
    """Coefficient transfer: full weighting on coarse interior vertices,
    injection on coarse boundary vertices."""
    c = f[::2, ::2, ::2].copy()
    c[1:-1, 1:-1, 1:-1] = _fw_interior(f)
    return c


def restrict(r):
    """Full weighting of a fine defect (0 on the coarse boundary)."""
    qc = np.zeros(tuple((s - 1) // 2 + 1 for s in r.shape), dtype=r.dtype)
    qc[1:-1, 1:-1, 1:-1] = _fw_interior(r)
    return qc


def interpolate(ec):
    """Trilinear interpolation of a coarse field to every fine vertex, one
    axis at a time (even fine index: the coarse value; odd: the mean of the
    two coarse neighbours)."""
    e = ec
    for axis in range(3):
        n = e.shape[axis]
        shape = list(e.shape)
        shape[axis] = 2 * n - 1
        out = np.zeros(shape, dtype=e.dtype)
        even = [slice(None)] * 3
        odd = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        even[axis] = slice(0, None, 2)
        odd[axis] = slice(1, None, 2)
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        out[tuple(even)] = e
        out[tuple(odd)] = 0.5 * (e[tuple(lo)] + e[tuple(hi)])
        e = out
    return e


def prolong_add(ec, u):
    """u += I ec on fine interior vertices."""
    u[1:-1, 1:-1, 1:-1] += interpolate(ec)[1:-1, 1:-1, 1:-1]


def _axis_slices(axis):
    """(neighbour below, neighbour above) of the interior block along axis."""
    m = [slice(1, -1)] * 3
    p = [slice(1, -1)] * 3
    m[axis] = slice(None, -2)
    p[axis] = slice(2, None)
    return tuple(m), tuple(p)


INNER = (slice(1, -1),) * 3


class HierarchyGrid:
    def __init__(self, D, mua, h=(1.0, 1.0, 1.0), g=0.0, face_mean="arith"):
        D = np.asarray(D)
        mua = np.asarray(mua)
        self.n = tuple(s - 1 for s in D.shape)
        self.shapes = level_shapes(self.n)
        self.L = len(self.shapes)
        self.g = g
        self.harmonic = face_mean == "harmonic"
        self.h = [tuple(float(a) * 2.0 ** k for a in h) for k in range(self.L)]
        self.D = [D]
        self.mu = [mua]
        for _ in range(1, self.L):
            self.D.append(coarsen_field(self.D[-1]))
            self.mu.append(coarsen_field(self.mu[-1]))

    # -- the operator ---------------------------------------------------------
    def face(self, Da, Db):
        if self.harmonic:
            return 2.0 * Da * Db / (Da + Db)
        return 0.5 * (Da + Db)

    def couplings(self, k):
        """c_ij of the interior vertices to their neighbours below and above
        along x, y and z: six arrays of the interior's shape."""
        D = self.D[k]
        Di = D[INNER]
        out = []
        for axis in range(3):
            ih2 = 1.0 / self.h[k][axis] ** 2
            m, p = _axis_slices(axis)
            out.append(self.face(Di, D[m]) * ih2)
            out.append(self.face(Di, D[p]) * ih2)
        return out

    def apply(self, k, u):
        """A u on interior vertices, 0 on the boundary."""
        c = self.couplings(k)
        ui = u[INNER]
        acc = self.mu[k][INNER] * ui
        for axis in range(3):
            m, p = _axis_slices(axis)
            acc = acc + c[2 * axis] * (ui - u[m]) + c[2 * axis + 1] * (ui - u[p])
        out = np.zeros_like(u, dtype=np.result_type(u, self.D[k]))
        out[INNER] = acc
        return out

    def defect(self, k, u, q):
        """q - A u on interior vertices (Sec. 2.3.2), 0 on the boundary."""
        r = np.zeros_like(u, dtype=np.result_type(u, q, self.D[k]))
        r[INNER] = q[INNER] - self.apply(k, u)[INNER]
        return r

    def gs_half(self, k, u, q, colour):
        """One red (colour 0) or black (colour 1) half-sweep, in place."""
        c = self.couplings(k)
        num = q[INNER].astype(np.result_type(q, u, self.D[k]))
        den = self.mu[k][INNER] + 0.0
        for axis in range(3):
            m, p = _axis_slices(axis)
            num = num + c[2 * axis] * u[m] + c[2 * axis + 1] * u[p]
            den = den + c[2 * axis] + c[2 * axis + 1]
        nx, ny, nz = self.shapes[k]
        x, y, z = np.ix_(np.arange(1, nx), np.arange(1, ny), np.arange(1, nz))
        mask = (x + y + z) % 2 == colour
        ui = u[INNER]
        ui[mask] = (num / den)[mask]

    def exact(self, k, q, u):
        """Solve A u = q exactly on level k's interior (dense), the boundary
        values of u moved to the right-hand side."""
        nx, ny, nz = self.shapes[k]
        mx, my, mz = nx - 1, ny - 1, nz - 1
        m = mx * my * mz
        D, mu = self.D[k], self.mu[k]
        dt = np.result_type(D, u, q)
        A = np.zeros((m, m), dtype=dt)
        b = np.zeros(m, dtype=dt)
        t_of = lambda x, y, z: ((x - 1) * my + (y - 1)) * mz + (z - 1)
        for x in range(1, nx):
            for y in range(1, ny):
                for z in range(1, nz):
                    t = t_of(x, y, z)
                    A[t, t] += mu[x, y, z]
                    b[t] += q[x, y, z]
                    for axis, (xa, ya, za) in ((0, (x - 1, y, z)), (0, (x + 1, y, z)), (1, (x, y - 1, z)),
                                               (1, (x, y + 1, z)), (2, (x, y, z - 1)), (2, (x, y, z + 1))):
                        cf = self.face(D[x, y, z], D[xa, ya, za]) / self.h[k][axis] ** 2
                        A[t, t] += cf
                        if 0 < xa < nx and 0 < ya < ny and 0 < za < nz:
                            A[t, t_of(xa, ya, za)] -= cf
                        else:
                            b[t] += cf * u[xa, ya, za]
        u[INNER] = np.linalg.solve(A, b).reshape(mx, my, mz)

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

    def _start(self, b, bc):
        u = np.zeros_like(b, dtype=np.result_type(b, self.D[0]))
        u[0], u[-1] = bc, bc
        u[:, 0], u[:, -1] = bc, bc
        u[:, :, 0], u[:, :, -1] = bc, bc
        return u

    def solve(self, b, bc, order, nu1, nu2, rtol, max_cycles, fixed_cycles):
        u = self._start(b, bc)
        r0 = np.linalg.norm(self.defect(0, u, b))
        info = {"cycles": 0, "rel_residual": 0.0, "status": 0}
        if fixed_cycles > 0:
            for _ in range(fixed_cycles):
                self.vcycle(0, u, b, order, nu1, nu2)
            info["cycles"] = fixed_cycles
            info["rel_residual"] = float(abs(np.linalg.norm(self.defect(0, u, b)) / (r0 if r0 > 0 else 1.0)))
            return u, info
        if r0 == 0.0:
            return u, info
        for c in range(1, max_cycles + 1):
            self.vcycle(0, u, b, order, nu1, nu2)
            rel = float(np.linalg.norm(self.defect(0, u, b)) / r0)
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
        """dq - (dA) rho on interior vertices (dA along dlogD and dlogmua)."""
        D = self.D[0]
        Di, dDi, ri = D[INNER], dlogD[INNER], rho[INNER]
        acc = self.mu[0][INNER] * dlogmua[INNER] * ri
        for axis in range(3):
            ih2 = 1.0 / self.h[0][axis] ** 2
            for sl in _axis_slices(axis):
                da, db = self.dface(Di, D[sl])
                acc = acc + (da * dDi + db * dlogD[sl]) * ih2 * (ri - rho[sl])
        out = np.zeros_like(rho, dtype=np.result_type(rho, dq, dlogD, D))
        out[INNER] = dq[INNER] - acc
        return out

    def jvp(self, rho, dq, dlogD, dlogmua, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """drho = S (dq - dA rho)."""
        rhs = self.tangent_rhs(rho, dq, dlogD, dlogmua)
        return self.solve(rhs, 0.0, 0, nu1, nu2, rtol, max_cycles, fixed_cycles)

    def pullback(self, w, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """qbar = S^T w: black-before-red V(nu2, nu1)-cycles on A qbar = w."""
        w = np.array(w)
        w[0], w[-1], w[:, 0], w[:, -1], w[:, :, 0], w[:, :, -1] = 0, 0, 0, 0, 0, 0
        return self.solve(w, 0.0, 1, nu2, nu1, rtol, max_cycles, fixed_cycles)

    def coef_grads(self, rho, lam):
        """(g_logD, g_logmua) from the forward solution and the adjoint state,
        face by face along each axis."""
        D = self.D[0]
        lam = np.array(lam)
        lam[0], lam[-1], lam[:, 0], lam[:, -1], lam[:, :, 0], lam[:, :, -1] = 0, 0, 0, 0, 0, 0
        gD = np.zeros_like(rho, dtype=np.result_type(rho, lam, D))
        gmu = np.zeros_like(gD)
        gmu[INNER] = -self.mu[0][INNER] * lam[INNER] * rho[INNER]
        inside = np.zeros(rho.shape, dtype=bool)
        inside[INNER] = True
        for axis in range(3):
            ih2 = 1.0 / self.h[0][axis] ** 2
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[axis] = slice(0, -1)
            b[axis] = slice(1, None)
            a, b = tuple(a), tuple(b)
            # faces (a, b) along this axis with at least one interior end
            keep = inside[a] | inside[b]
            t = (lam[a] - lam[b]) * (rho[a] - rho[b]) * ih2 * keep
            da, db = self.dface(D[a], D[b])
            gD[a] -= da * t
            gD[b] -= db * t
        return gD, gmu

    def vjp(self, rho, w, rtol=1e-10, max_cycles=200, fixed_cycles=0, nu1=2, nu2=2):
        """(qbar, g_logD, g_logmua) = pull-back of the cotangent w."""
        lam, info = self.pullback(w, rtol, max_cycles, fixed_cycles, nu1, nu2)
        gD, gmu = self.coef_grads(rho, lam)
        return (lam, gD, gmu), info
