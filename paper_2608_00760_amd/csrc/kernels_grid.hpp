// kernels_grid.hpp -- float64 kernels of three-dimensional plans whose axes
// have different cell counts and spacings (the paper's data grid, Sec.
// 2.5.1: (128, 64, 64) over 7.5 x 3.5 x 3.5 cm).
//
// One vertex (or coarse vertex) per thread, one operation per launch, in
// the layout of every other plan: (nx+1)(ny+1)(nz+1) vertices, x slowest,
// z fastest.  The operator is the 7-point stencil of Eq. (maineq) with the
// face coefficient of each axis scaled by that axis's 1/h^2; smoothing,
// transfers, coarsening, the exact coarsest solve and the derivative
// kernels follow the cubic kernels axis by axis.  These grids are small
// (the paper's has 0.55 M vertices), so the kernels are written for
// clarity rather than streamed.
#pragma once
#include "kernels_basic.hpp"

namespace dmgs {

// cells per axis and the per-axis scale of the face coefficient
struct GridDims {
    int nx, ny, nz;
    double ih2[3];   // 1 / h_a^2
    int harmonic;

    __host__ __device__ int64_t nv() const { return (int64_t)(nx + 1) * (ny + 1) * (nz + 1); }
    __device__ int64_t at(int x, int y, int z) const { return ((int64_t)x * (ny + 1) + y) * (nz + 1) + z; }
    __device__ void coords(int64_t v, int& x, int& y, int& z) const {
        z = (int)(v % (nz + 1));
        y = (int)((v / (nz + 1)) % (ny + 1));
        x = (int)(v / ((int64_t)(nz + 1) * (ny + 1)));
    }
    __device__ bool interior(int x, int y, int z) const {
        return x > 0 && x < nx && y > 0 && y < ny && z > 0 && z < nz;
    }
    // c = D_f / h_a^2 of a face along axis a
    __device__ double face(double Da, double Db, int a) const {
        return (harmonic ? 2.0 * Da * Db / (Da + Db) : 0.5 * (Da + Db)) * ih2[a];
    }
    // the next coarser level's dimensions (same face mean, spacing doubled)
    __host__ __device__ GridDims coarser() const {
        GridDims c = *this;
        c.nx = nx / 2;
        c.ny = ny / 2;
        c.nz = nz / 2;
        for (int a = 0; a < 3; a++) c.ih2[a] = ih2[a] * 0.25;
        return c;
    }
};

// neighbour offsets in the order +x, -x, +y, -y, +z, -z, and their axes
__device__ __constant__ const int kGridOff[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

#define GRID_LOOP(G, v)                                                                                   \
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, nv_ = (G).nv(); v < nv_;            \
         v += (int64_t)gridDim.x * blockDim.x)

template <class T>
__global__ void k_g_fill(T* __restrict__ a, GridDims G, T val) {
    GRID_LOOP(G, v) a[v] = val;
}

// u = 0 on interior vertices, g on the boundary
__global__ void k_g_init(double* __restrict__ u, GridDims G, double g) {
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        u[v] = G.interior(x, y, z) ? 0.0 : g;
    }
}

// D > 0 and finite everywhere, mua >= 0 and finite on interior vertices;
// from the logarithms when logD is given (D = exp(log D), mua = exp(log mua)).
__global__ void k_g_coef_in(const double* __restrict__ logD, const double* __restrict__ logmu, double* __restrict__ D,
                            double* __restrict__ mu, GridDims G, int* __restrict__ bad) {
    int b = 0;
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        if (logD) {
            D[v] = exp(logD[v]);
            mu[v] = exp(logmu[v]);
        }
        if (!coef_ok(D[v], mu[v], G.interior(x, y, z))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

// coarse coefficients: full weighting (1/64)(1,2,1)^3 on coarse interior
// vertices, injection on coarse boundary vertices
__global__ void k_g_coarsen(const double* __restrict__ fD, const double* __restrict__ fmu, GridDims F,
                            double* __restrict__ cD, double* __restrict__ cmu) {
    const GridDims C = F.coarser();
    GRID_LOOP(C, v) {
        int X, Y, Z;
        C.coords(v, X, Y, Z);
        if (!C.interior(X, Y, Z)) {
            const int64_t f = F.at(2 * X, 2 * Y, 2 * Z);
            cD[v] = fD[f];
            cmu[v] = fmu[f];
            continue;
        }
        double sD = 0.0, sm = 0.0;
        for (int a = -1; a <= 1; a++)
            for (int b = -1; b <= 1; b++)
                for (int c = -1; c <= 1; c++) {
                    const double w = (double)((2 - abs(a)) * (2 - abs(b)) * (2 - abs(c)));
                    const int64_t f = F.at(2 * X + a, 2 * Y + b, 2 * Z + c);
                    sD += w * fD[f];
                    sm += w * fmu[f];
                }
        cD[v] = sD / 64.0;
        cmu[v] = sm / 64.0;
    }
}

// sum over the 6 faces of c_ij u_j (num) and of c_ij (diag, without mua)
__device__ __forceinline__ void g_stencil(const double* __restrict__ u, const double* __restrict__ D, const GridDims& G,
                                          int x, int y, int z, int64_t i, double& num, double& diag) {
    num = 0.0;
    diag = 0.0;
    const double Di = D[i];
    for (int e = 0; e < 6; e++) {
        const int64_t j = G.at(x + kGridOff[e][0], y + kGridOff[e][1], z + kGridOff[e][2]);
        const double c = G.face(Di, D[j], e >> 1);
        num += c * u[j];
        diag += c;
    }
}

// one red (colour 0: (x+y+z) even) or black half-sweep, in place
__global__ void k_g_half(double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                         const double* __restrict__ mu, GridDims G, int colour) {
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        if (!G.interior(x, y, z) || ((x + y + z) & 1) != colour) continue;
        double num, diag;
        g_stencil(u, D, G, x, y, z, v, num, diag);
        u[v] = (q[v] + num) / (diag + mu[v]);
    }
}

// The last half-sweep of a solve, with the likelihood epilogue of its
// result: the swept colour is updated as in k_g_half, and every vertex, its
// value now final, gets rhobar = mua w (mua u - d) (0 on the boundary) and
// adds w (mua u - d)^2 and [w > 0] to its block's sums at partial[block]
// and partial[gridDim + block].  The other colour is only read.
__global__ void k_g_half_epi(double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                             const double* __restrict__ mu, GridDims G, int colour, const double* __restrict__ d,
                             const double* __restrict__ w, double* __restrict__ rhobar, double* __restrict__ partial) {
    double acc = 0.0, cnt = 0.0;
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        if (!G.interior(x, y, z)) {
            rhobar[v] = 0.0;
            continue;
        }
        double uv;
        if (((x + y + z) & 1) == colour) {
            double num, diag;
            g_stencil(u, D, G, x, y, z, v, num, diag);
            uv = (q[v] + num) / (diag + mu[v]);
            u[v] = uv;
        } else {
            uv = u[v];
        }
        const double m = mu[v], wv = w[v];
        const double res = m * uv - d[v];
        rhobar[v] = m * wv * res;
        acc += wv * res * res;
        cnt += wv > 0.0 ? 1.0 : 0.0;
    }
    const double s = block_sum(acc);
    const double c = block_sum(cnt);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        partial[gridDim.x + blockIdx.x] = c;
    }
}

// r = q - A u on interior vertices, 0 on the boundary
__global__ void k_g_defect(const double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                           const double* __restrict__ mu, GridDims G, double* __restrict__ r) {
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        if (!G.interior(x, y, z)) {
            r[v] = 0.0;
            continue;
        }
        double num, diag;
        g_stencil(u, D, G, x, y, z, v, num, diag);
        r[v] = q[v] - ((diag + mu[v]) * u[v] - num);
    }
}

// qc = R r: full weighting on coarse interior vertices, 0 on the coarse boundary
__global__ void k_g_restrict(const double* __restrict__ r, GridDims F, double* __restrict__ qc) {
    const GridDims C = F.coarser();
    GRID_LOOP(C, v) {
        int X, Y, Z;
        C.coords(v, X, Y, Z);
        if (!C.interior(X, Y, Z)) {
            qc[v] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int a = -1; a <= 1; a++)
            for (int b = -1; b <= 1; b++)
                for (int c = -1; c <= 1; c++)
                    s += (double)((2 - abs(a)) * (2 - abs(b)) * (2 - abs(c))) * r[F.at(2 * X + a, 2 * Y + b, 2 * Z + c)];
        qc[v] = s / 64.0;
    }
}

// u += I ec on fine interior vertices (trilinear, I = 2^3 R^T)
__global__ void k_g_prolong_add(const double* __restrict__ ec, GridDims F, double* __restrict__ u) {
    const GridDims C = F.coarser();
    GRID_LOOP(F, v) {
        int x, y, z;
        F.coords(v, x, y, z);
        if (!F.interior(x, y, z)) continue;
        const int X0 = x >> 1, X1 = X0 + (x & 1), Y0 = y >> 1, Y1 = Y0 + (y & 1), Z0 = z >> 1, Z1 = Z0 + (z & 1);
        const double s = ((ec[C.at(X0, Y0, Z0)] + ec[C.at(X0, Y0, Z1)]) + (ec[C.at(X0, Y1, Z0)] + ec[C.at(X0, Y1, Z1)])) +
                         ((ec[C.at(X1, Y0, Z0)] + ec[C.at(X1, Y0, Z1)]) + (ec[C.at(X1, Y1, Z0)] + ec[C.at(X1, Y1, Z1)]));
        u[v] += 0.125 * s;
    }
}

// Inverse of the coarsest operator (at most kGridCoarseMax unknowns, row t
// of [A | I] per thread, Gauss-Jordan in LDS), written as inv[t * m + j].
constexpr int kGridCoarseMax = 64;
__global__ void k_g_inverse(const double* __restrict__ D, const double* __restrict__ mu, GridDims G,
                            double* __restrict__ inv) {
    extern __shared__ double M[];   // m rows of 2m entries
    const int mx = G.nx - 1, my = G.ny - 1, mz = G.nz - 1, m = mx * my * mz, t = threadIdx.x;
    double* Mt = M + 2 * m * t;
    if (t < m) {
        const int x = 1 + t / (my * mz), y = 1 + (t / mz) % my, z = 1 + t % mz;
        for (int j = 0; j < 2 * m; j++) Mt[j] = 0.0;
        const int64_t i = G.at(x, y, z);
        double d = mu[i];
        for (int e = 0; e < 6; e++) {
            const int xa = x + kGridOff[e][0], ya = y + kGridOff[e][1], za = z + kGridOff[e][2];
            const double c = G.face(D[i], D[G.at(xa, ya, za)], e >> 1);
            d += c;
            if (G.interior(xa, ya, za)) Mt[((xa - 1) * my + (ya - 1)) * mz + (za - 1)] = -c;
        }
        Mt[t] = d;
        Mt[m + t] = 1.0;
    }
    __syncthreads();
    for (int p = 0; p < m; p++) {
        // rows other than p change only their own entries and read row p
        if (t < m && t != p) {
            const double f = Mt[p] / M[2 * m * p + p];
            for (int j = 0; j < 2 * m; j++) Mt[j] -= f * M[2 * m * p + j];
        }
        __syncthreads();
    }
    if (t < m)
        for (int j = 0; j < m; j++) inv[t * m + j] = Mt[m + j] / Mt[t];
}

// Exact solve on the coarsest level: u = A^-1 (q + boundary terms) on the
// interior (the boundary values of u, g on a one-level plan and 0 for coarse
// corrections, move to the right-hand side).  One thread per unknown.
__global__ void k_g_exact(const double* __restrict__ q, double* __restrict__ u, const double* __restrict__ D,
                          const double* __restrict__ inv, GridDims G) {
    __shared__ double rhs[kGridCoarseMax];
    const int mx = G.nx - 1, my = G.ny - 1, mz = G.nz - 1, m = mx * my * mz, t = threadIdx.x;
    int x = 0, y = 0, z = 0;
    int64_t i = 0;
    if (t < m) {
        x = 1 + t / (my * mz);
        y = 1 + (t / mz) % my;
        z = 1 + t % mz;
        i = G.at(x, y, z);
        double b = q[i];
        for (int e = 0; e < 6; e++) {
            const int xa = x + kGridOff[e][0], ya = y + kGridOff[e][1], za = z + kGridOff[e][2];
            if (!G.interior(xa, ya, za)) b += G.face(D[i], D[G.at(xa, ya, za)], e >> 1) * u[G.at(xa, ya, za)];
        }
        rhs[t] = b;
    }
    __syncthreads();
    if (t < m) {
        double s = 0.0;
        for (int j = 0; j < m; j++) s += inv[t * m + j] * rhs[j];
        u[i] = s;
    }
}

// partial[block] = sum over the block's interior vertices of (q - A u)^2
__global__ void k_g_resid_sq(const double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                             const double* __restrict__ mu, GridDims G, double* __restrict__ partial) {
    double acc = 0.0;
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        if (!G.interior(x, y, z)) continue;
        double num, diag;
        g_stencil(u, D, G, x, y, z, v, num, diag);
        const double r = q[v] - ((diag + mu[v]) * u[v] - num);
        acc += r * r;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// rhs = dq - (dA) rho on interior vertices (0 on the boundary), dA along
// dlogD and dlogmua (null tangents are 0)
__global__ void k_g_tangent_rhs(const double* __restrict__ rho, const double* __restrict__ dq,
                                const double* __restrict__ dlogD, const double* __restrict__ dlogmu,
                                const double* __restrict__ D, const double* __restrict__ mu, GridDims G,
                                double* __restrict__ rhs) {
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        if (!G.interior(x, y, z)) {
            rhs[v] = 0.0;
            continue;
        }
        const double ri = rho[v], Di = D[v];
        double acc = dlogmu ? mu[v] * dlogmu[v] * ri : 0.0;
        if (dlogD) {
            const double dDi = Di * dlogD[v];
            for (int e = 0; e < 6; e++) {
                const int64_t j = G.at(x + kGridOff[e][0], y + kGridOff[e][1], z + kGridOff[e][2]);
                const double Dj = D[j], dDj = Dj * dlogD[j];
                double dDf;
                if (G.harmonic) {
                    const double sum = Di + Dj;
                    dDf = 2.0 * (Dj * Dj * dDi + Di * Di * dDj) / (sum * sum);
                } else {
                    dDf = 0.5 * (dDi + dDj);
                }
                acc += dDf * G.ih2[e >> 1] * (ri - rho[j]);
            }
        }
        rhs[v] = (dq ? dq[v] : 0.0) - acc;
    }
}

// Coefficient gradients from the adjoint state lam (0 on the boundary):
//   logmua_bar_i = -mua_i lam_i rho_i on interior vertices, 0 on the boundary
//   logD_bar_v   = -sum over faces (v, j) with v or j interior of
//                  dD_f/dlogD_v (lam_v - lam_j)(rho_v - rho_j) / h_a^2
// and, with data d and weights w, the likelihood's direct log mua term
// w_i (mua_i rho_i - d_i) mua_i rho_i.
__global__ void k_g_coef_grads(const double* __restrict__ rho, const double* __restrict__ lam,
                               const double* __restrict__ D, const double* __restrict__ mu, GridDims G,
                               double* __restrict__ gD, double* __restrict__ gmu, const double* __restrict__ d,
                               const double* __restrict__ w) {
    GRID_LOOP(G, v) {
        int x, y, z;
        G.coords(v, x, y, z);
        const bool vin = G.interior(x, y, z);
        const double lv = vin ? lam[v] : 0.0, rv = rho[v], Dv = D[v];
        if (gmu) {
            double g = vin ? -mu[v] * lv * rv : 0.0;
            if (d && vin) {
                const double Le = mu[v] * rv;
                g += w[v] * (Le - d[v]) * Le;
            }
            gmu[v] = g;
        }
        if (!gD) continue;
        double acc = 0.0;
        for (int e = 0; e < 6; e++) {
            const int xa = x + kGridOff[e][0], ya = y + kGridOff[e][1], za = z + kGridOff[e][2];
            if (xa < 0 || xa > G.nx || ya < 0 || ya > G.ny || za < 0 || za > G.nz) continue;
            const bool jin = G.interior(xa, ya, za);
            if (!vin && !jin) continue;
            const int64_t j = G.at(xa, ya, za);
            const double lj = jin ? lam[j] : 0.0, Dj = D[j];
            double dcdv;
            if (G.harmonic) {
                const double sum = Dv + Dj;
                dcdv = 2.0 * Dj * Dj * Dv / (sum * sum);
            } else {
                dcdv = 0.5 * Dv;
            }
            acc += dcdv * G.ih2[e >> 1] * (lv - lj) * (rv - rho[j]);
        }
        gD[v] = -acc;
    }
}

#undef GRID_LOOP

}  // namespace dmgs
