// kernels_2d.hpp -- kernels of the two-dimensional (five-point) variant.
//
// Grid: N cells per axis, (N+1)^2 vertices, x slowest, y fastest,
// v = x*(N+1) + y; interior vertices have both coordinates in [1, N-1].
// The operator is the two-dimensional form of Eq. (maineq):
//   (A u)_i = sum over the 4 neighbours j of c_ij (u_i - u_j) + mua_i u_i,
//   c_ij = D_f / h^2 with the arithmetic (or harmonic) face mean,
// red = (x + y) even, restriction (1/16)(1,2,1) x (1,2,1), bilinear
// prolongation, coefficients coarsened by full weighting (injection on the
// boundary) -- the readings of the three-dimensional solver.
//
// Every kernel here is float64 and memory-bound.  Kernels that read
// neighbouring rows take one item per thread over a grid of whole blocks
// rounded up to a multiple of 8, remapped so that each XCD walks a
// contiguous band of rows (the rows it reads twice stay in its L2).
#pragma once
#include "grid.hpp"
#include "kernels_basic.hpp"

namespace dmgs {

__device__ __forceinline__ bool interior2(int N, int x, int y) { return x > 0 && x < N && y > 0 && y < N; }

__device__ __forceinline__ int64_t item_of_thread2() {
    return (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// ---------------------------------------------------------------------------
// Coefficients.

__global__ void k2_validate(const double* __restrict__ D, const double* __restrict__ mu, int N, int* __restrict__ bad) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    int b = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(v / n), y = (int)(v % n);
        if (!coef_ok(D[v], mu[v], interior2(N, x, y))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

__global__ void k2_exp_validate(const double* __restrict__ logD, const double* __restrict__ logmu,
                                double* __restrict__ D, double* __restrict__ mu, int N, int* __restrict__ bad) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    int b = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(v / n), y = (int)(v % n);
        const double d = exp(logD[v]), m = exp(logmu[v]);
        D[v] = d;
        mu[v] = m;
        if (!coef_ok(d, m, interior2(N, x, y))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

// sum over a, b in {-1, 0, 1} of (2 - |a|)(2 - |b|) f[2X + a, 2Y + b] / 16
__device__ __forceinline__ double full_weight2(const double* __restrict__ f, int nf, int X, int Y) {
    double s = 0.0;
    for (int a = -1; a <= 1; a++) {
        const double* row = f + (int64_t)(2 * X + a) * nf + 2 * Y;
        s += (double)(2 - abs(a)) * (row[-1] + 2.0 * row[0] + row[1]);
    }
    return s * (1.0 / 16.0);
}

__global__ void k2_coarsen_coef(const double* __restrict__ fD, const double* __restrict__ fmu, double* __restrict__ cD,
                                double* __restrict__ cmu, int Nf) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nc * nc) return;
    const int X = (int)(v / nc), Y = (int)(v % nc);
    if (!interior2(Nc, X, Y)) {
        const int64_t i = (int64_t)(2 * X) * nf + 2 * Y;
        cD[v] = fD[i];
        cmu[v] = fmu[i];
        return;
    }
    cD[v] = full_weight2(fD, nf, X, Y);
    cmu[v] = full_weight2(fmu, nf, X, Y);
}

// ---------------------------------------------------------------------------
// The cycle.

// u = 0 on interior vertices, g on the boundary.
__global__ void k2_init_iterate(double* __restrict__ u, int N, double g) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x)
        u[v] = interior2(N, (int)(v / n), (int)(v % n)) ? 0.0 : g;
}

// One red (colour 0) or black (colour 1) half-sweep in place (Sec. 2.2):
// u_i = (q_i + sum_j c_ij u_j) / (sum_j c_ij + mua_i) on the interior
// vertices of the colour.  Item t = row (x - 1) * (N/2) + j is the j-th
// vertex of the colour in row x; N is even on every level that smooths.
template <bool HARM>
__global__ void k2_half_sweep(double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                              const double* __restrict__ mu, int N, Stencil<double> s, int colour) {
    const int S = N / 2;
    const int64_t t = item_of_thread2();
    if (t >= (int64_t)(N - 1) * S) return;
    const int x = 1 + (int)(t / S);
    const int y = (((colour - x) & 1) ? 1 : 2) + 2 * (int)(t % S);
    if (y >= N) return;
    const int n = N + 1;
    const int64_t i = (int64_t)x * n + y;
    const double Di = D[i];
    const double cxm = face<HARM>(Di, D[i - n], s), cxp = face<HARM>(Di, D[i + n], s);
    const double cym = face<HARM>(Di, D[i - 1], s), cyp = face<HARM>(Di, D[i + 1], s);
    u[i] = (q[i] + cxm * u[i - n] + cxp * u[i + n] + cym * u[i - 1] + cyp * u[i + 1]) / (cxm + cxp + cym + cyp + mu[i]);
}

// q - A u at the interior vertex i = (x, y) (row stride n).
template <bool HARM>
__device__ __forceinline__ double defect2_at(const double* __restrict__ u, const double* __restrict__ q,
                                             const double* __restrict__ D, const double* __restrict__ mu, int64_t i,
                                             int n, const Stencil<double>& s) {
    const double Di = D[i], ui = u[i];
    return q[i] - (mu[i] * ui + face<HARM>(Di, D[i - n], s) * (ui - u[i - n]) + face<HARM>(Di, D[i + n], s) * (ui - u[i + n]) +
                   face<HARM>(Di, D[i - 1], s) * (ui - u[i - 1]) + face<HARM>(Di, D[i + 1], s) * (ui - u[i + 1]));
}

// qc = R (q - A u) (Sec. 2.3.2 and Eq. (rest)): one coarse vertex per
// thread, its nine fine defects formed on the fly (0 on the coarse boundary).
template <bool HARM>
__global__ void k2_defect_restrict(const double* __restrict__ u, const double* __restrict__ q,
                                   const double* __restrict__ D, const double* __restrict__ mu, int Nf,
                                   Stencil<double> s, double* __restrict__ qc) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nc * nc) return;
    const int X = (int)(v / nc), Y = (int)(v % nc);
    if (!interior2(Nc, X, Y)) {
        qc[v] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int a = -1; a <= 1; a++) {
        const int64_t i = (int64_t)(2 * X + a) * nf + 2 * Y;
        const double row = defect2_at<HARM>(u, q, D, mu, i - 1, nf, s) + 2.0 * defect2_at<HARM>(u, q, D, mu, i, nf, s) +
                           defect2_at<HARM>(u, q, D, mu, i + 1, nf, s);
        acc += (double)(2 - abs(a)) * row;
    }
    qc[v] = acc * (1.0 / 16.0);
}

// u += I ec on fine interior vertices (Sec. 2.3.3, bilinear).
__global__ void k2_prolong_add(const double* __restrict__ ec, double* __restrict__ u, int Nf) {
    const int nf = Nf + 1, nc = Nf / 2 + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nf * nf) return;
    const int x = (int)(v / nf), y = (int)(v % nf);
    if (!interior2(Nf, x, y)) return;
    const int X0 = x >> 1, X1 = (x + 1) >> 1, Y0 = y >> 1, Y1 = (y + 1) >> 1;
    const double* r0 = ec + (int64_t)X0 * nc;
    const double* r1 = ec + (int64_t)X1 * nc;
    double e;
    if (X0 == X1) e = (Y0 == Y1) ? r0[Y0] : 0.5 * (r0[Y0] + r0[Y1]);
    else if (Y0 == Y1) e = 0.5 * (r0[Y0] + r1[Y0]);
    else e = 0.25 * (r0[Y0] + r1[Y0] + r0[Y1] + r1[Y1]);
    u[v] += e;
}

// Exact solve on the coarsest level (N in {2, 3}: at most 4 unknowns), the
// boundary values of u moved to the right-hand side; one thread, Cholesky.
template <bool HARM>
__global__ void k2_exact(const double* __restrict__ q, double* __restrict__ u, const double* __restrict__ D,
                         const double* __restrict__ mu, int N, Stencil<double> s) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int n = N + 1, m1 = N - 1, m = m1 * m1;
    double A[4][4], b[4];
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) A[r][c] = 0.0;
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++) {
            const int t = (x - 1) * m1 + (y - 1);
            const int i = x * n + y;
            A[t][t] = mu[i];
            b[t] = q[i];
            const int nb[4][2] = {{x - 1, y}, {x + 1, y}, {x, y - 1}, {x, y + 1}};
            for (int e = 0; e < 4; e++) {
                const int xa = nb[e][0], ya = nb[e][1], j = xa * n + ya;
                const double c = face<HARM>(D[i], D[j], s);
                A[t][t] += c;
                if (interior2(N, xa, ya)) A[t][(xa - 1) * m1 + (ya - 1)] -= c;
                else b[t] += c * u[j];
            }
        }
    for (int j = 0; j < m; j++) {
        double d = A[j][j];
        for (int p = 0; p < j; p++) d -= A[j][p] * A[j][p];
        d = sqrt(d);
        A[j][j] = d;
        for (int i = j + 1; i < m; i++) {
            double acc = A[i][j];
            for (int p = 0; p < j; p++) acc -= A[i][p] * A[j][p];
            A[i][j] = acc / d;
        }
    }
    for (int i = 0; i < m; i++) {
        double acc = b[i];
        for (int p = 0; p < i; p++) acc -= A[i][p] * b[p];
        b[i] = acc / A[i][i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double acc = b[i];
        for (int p = i + 1; p < m; p++) acc -= A[p][i] * b[p];
        b[i] = acc / A[i][i];
    }
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++) u[x * n + y] = b[(x - 1) * m1 + (y - 1)];
}

// partial[block] = sum over the block's interior vertices of (q - A u)^2.
template <bool HARM>
__global__ void k2_resid_sq(const double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                            const double* __restrict__ mu, int N, Stencil<double> s, double* __restrict__ partial) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    double acc = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        if (!interior2(N, (int)(v / n), (int)(v % n))) continue;
        const double r = defect2_at<HARM>(u, q, D, mu, v, n, s);
        acc += r * r;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// ---------------------------------------------------------------------------
// Derivatives (the adjoint-state formulas of the three-dimensional solver
// with four neighbours).

// rhs = dq - (dA) rho on interior vertices, 0 on the boundary; dA along
// dlogD (face values) and dlogmu (dmua = mua dlogmu).  dq, dlogD or dlogmu
// may be null (zero).
__global__ void k2_tangent_rhs(const double* __restrict__ rho, const double* __restrict__ dq,
                               const double* __restrict__ dlogD, const double* __restrict__ dlogmu,
                               const double* __restrict__ D, const double* __restrict__ mu, int N, double inv_h2,
                               int harmonic, double* __restrict__ rhs) {
    const int n = N + 1;
    const int64_t i = item_of_thread2();
    if (i >= (int64_t)n * n) return;
    const int x = (int)(i / n), y = (int)(i % n);
    if (!interior2(N, x, y)) {
        rhs[i] = 0.0;
        return;
    }
    const int off[4] = {n, -n, 1, -1};
    const double ri = rho[i], Di = D[i];
    double acc = dlogmu ? mu[i] * dlogmu[i] * ri : 0.0;
    if (dlogD) {
        const double dDi = Di * dlogD[i];
        for (int e = 0; e < 4; e++) {
            const int64_t j = i + off[e];
            const double Dj = D[j], dDj = Dj * dlogD[j];
            double dDf;
            if (harmonic) {
                const double sum = Di + Dj;
                dDf = 2.0 * (Dj * Dj * dDi + Di * Di * dDj) / (sum * sum);
            } else {
                dDf = 0.5 * (dDi + dDj);
            }
            acc += dDf * inv_h2 * (ri - rho[j]);
        }
    }
    rhs[i] = (dq ? dq[i] : 0.0) - acc;
}

// g_logmua = -mua lam rho (interior, 0 on the boundary);
// g_logD_v = -sum over faces (v, j) with an interior endpoint of
// dD_f/dlogD_v (lam_v - lam_j)(rho_v - rho_j) / h^2, lam = 0 on the boundary.
__global__ void k2_coef_grads(const double* __restrict__ rho, const double* __restrict__ lam,
                              const double* __restrict__ D, const double* __restrict__ mu, int N, double inv_h2,
                              int harmonic, double* __restrict__ gD, double* __restrict__ gmu) {
    const int n = N + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)n * n) return;
    const int x = (int)(v / n), y = (int)(v % n);
    const bool vin = interior2(N, x, y);
    const double lv = vin ? lam[v] : 0.0, rv = rho[v], Dv = D[v];
    if (gmu) gmu[v] = vin ? -mu[v] * lv * rv : 0.0;
    if (!gD) return;
    double acc = 0.0;
    const int o[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int e = 0; e < 4; e++) {
        const int xa = x + o[e][0], ya = y + o[e][1];
        if (xa < 0 || xa > N || ya < 0 || ya > N) continue;
        const bool jin = interior2(N, xa, ya);
        if (!vin && !jin) continue;
        const int64_t j = (int64_t)xa * n + ya;
        const double lj = jin ? lam[j] : 0.0, Dj = D[j];
        double dcdv;
        if (harmonic) {
            const double sum = Dv + Dj;
            dcdv = 2.0 * Dj * Dj * Dv / (sum * sum);
        } else {
            dcdv = 0.5 * Dv;
        }
        acc += dcdv * (lv - lj) * (rv - rho[j]);
    }
    gD[v] = -acc * inv_h2;
}

}  // namespace dmgs
