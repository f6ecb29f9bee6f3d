// kernels_basic.hpp -- one-operation-per-launch HIP kernels of the V-cycle:
// the coefficient hierarchy, red-black half-sweeps, defect, restriction,
// prolongation, the coarsest exact solve, residual norms, iterative
// refinement casts and the derivative kernels.  Used on every level whose
// arrays are too small for the fused streaming kernels, and by the
// diagnostic entry points.
#pragma once
#include "grid.hpp"

namespace dmgs {

// ---------------------------------------------------------------------------
// Fill, copy, cast

template <class T>
__global__ void k_init_iterate(T* __restrict__ u, int N, T g) {
    int n = N + 1;
    int64_t nv = (int64_t)n * n * n;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        int z = (int)(v % n), y = (int)((v / n) % n), x = (int)(v / ((int64_t)n * n));
        u[v] = is_interior(N, x, y, z) ? T(0) : g;
    }
}

template <class T>
__global__ void k_fill(T* __restrict__ a, int64_t nv, T val) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x)
        a[v] = val;
}

// Plain streaming copy of 16-byte words (used to calibrate memory counters).
__global__ void k_stream_copy(const float4* __restrict__ a, float4* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = a[i];
}

// D > 0 and finite on every vertex, mua >= 0 and finite on interior vertices.
__device__ __forceinline__ bool coef_ok(double d, double m, bool interior) {
    return d > 0.0 && isfinite(d) && (!interior || (m >= 0.0 && isfinite(m)));
}

__global__ void k_validate(const double* __restrict__ D, const double* __restrict__ mu, int N, int* __restrict__ bad) {
    const int n = N + 1, nv = n * n * n;
    int b = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        const int z = v % n, y = (v / n) % n, x = v / (n * n);
        if (!coef_ok(D[v], mu[v], is_interior(N, x, y, z))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

// Coefficients from their logarithms (D = exp(log D), mua = exp(log mua)),
// checked as k_validate checks them.
__global__ void k_exp_validate(const double* __restrict__ logD, const double* __restrict__ logmu, double* __restrict__ D,
                               double* __restrict__ mu, int N, int* __restrict__ bad) {
    const int n = N + 1, nv = n * n * n;
    int b = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        const int z = v % n, y = (v / n) % n, x = v / (n * n);
        const double d = exp(logD[v]), m = exp(logmu[v]);
        D[v] = d;
        mu[v] = m;
        if (!coef_ok(d, m, is_interior(N, x, y, z))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

// Kernels that read neighbours in the x +- 1 planes take one vertex per
// thread over a grid of whole blocks rounded up to a multiple of 8, blocks
// remapped so that each XCD walks a contiguous slab (the planes it reads
// stay in its L2).
__device__ __forceinline__ int vertex_of_thread() {
    return xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// Coefficient transfer to the next coarser level: full weighting
// (1/64)(1,2,1)^3 on coarse interior vertices, injection on coarse boundary
// vertices.  D and mua in one pass.
__device__ __forceinline__ double coarsen_at(const double* __restrict__ f, int Nc, int nf, int X, int Y, int Z) {
    if (!is_interior(Nc, X, Y, Z)) return f[vidx(nf, 2 * X, 2 * Y, 2 * Z)];
    double s = 0.0;
    for (int a = -1; a <= 1; a++)
        for (int b = -1; b <= 1; b++) {
            const double wab = (double)((2 - abs(a)) * (2 - abs(b)));
            const double* row = f + vidx(nf, 2 * X + a, 2 * Y + b, 2 * Z);
            s += wab * (row[-1] + 2.0 * row[0] + row[1]);
        }
    return s * (1.0 / 64.0);
}

__global__ void k_coarsen_coef(const double* __restrict__ fD, const double* __restrict__ fmu, double* __restrict__ cD,
                               double* __restrict__ cmu, int Nf) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1, nv = nc * nc * nc;
    const int v = vertex_of_thread();
    if (v >= nv) return;
    const int Z = v % nc, Y = (v / nc) % nc, X = v / (nc * nc);
    cD[v] = coarsen_at(fD, Nc, nf, X, Y, Z);
    cmu[v] = coarsen_at(fmu, Nc, nf, X, Y, Z);
}

// Smoother data of one level from its float64 coefficients: the inverse
// diagonal w = 1 / (sum_j c_ij + mua_i) on interior vertices (0 on the
// boundary), formed in float64 and stored as T, and, when D32 is given,
// float32 copies of D and mua.
template <class T>
__global__ void k_level_prep(const double* __restrict__ D, const double* __restrict__ mu, int N, Stencil<double> st,
                             T* __restrict__ w, float* __restrict__ D32, float* __restrict__ mu32) {
    const int n = N + 1, sx = n * n, nv = sx * n;
    const int i = vertex_of_thread();
    if (i >= nv) return;
    const int z = i % n, y = (i / n) % n, x = i / sx;
    const double Di = D[i], mi = mu[i];
    if (D32) {
        D32[i] = (float)Di;
        mu32[i] = (float)mi;
    }
    if (!is_interior(N, x, y, z)) {
        w[i] = T(0);
        return;
    }
    const double d = mi + face_coef(Di, D[i + sx], st) + face_coef(Di, D[i - sx], st) + face_coef(Di, D[i + n], st) +
                     face_coef(Di, D[i - n], st) + face_coef(Di, D[i + 1], st) + face_coef(Di, D[i - 1], st);
    w[i] = (T)(1.0 / d);
}

// Weighted-Jacobi sweep, out of place: on interior vertices
//   u_out = u_in + omega w (q - A u_in),   w = 1 / (sum_j c_ij + mua_i),
// and from a zero iterate (zero != 0) u_out = omega w q.  Boundary entries of
// u_out are not written (the ping-pong partner holds the same values).
template <class T>
__global__ void k_wj_sweep(const T* __restrict__ u, T* __restrict__ u_out, const T* __restrict__ q,
                           const T* __restrict__ D, const T* __restrict__ mu, const T* __restrict__ w, int N,
                           Stencil<T> s, T omega, int zero) {
    const int n = N + 1, sx = n * n, nv = sx * n;
    const int i = vertex_of_thread();
    if (i >= nv) return;
    const int z = i % n, y = (i / n) % n, x = i / sx;
    if (!is_interior(N, x, y, z)) return;
    if (zero) {
        u_out[i] = omega * w[i] * q[i];
        return;
    }
    const T Di = D[i], ui = u[i];
    const T Au = mu[i] * ui + face_coef(Di, D[i + sx], s) * (ui - u[i + sx]) + face_coef(Di, D[i - sx], s) * (ui - u[i - sx]) +
                 face_coef(Di, D[i + n], s) * (ui - u[i + n]) + face_coef(Di, D[i - n], s) * (ui - u[i - n]) +
                 face_coef(Di, D[i + 1], s) * (ui - u[i + 1]) + face_coef(Di, D[i - 1], s) * (ui - u[i - 1]);
    u_out[i] = ui + omega * w[i] * (q[i] - Au);
}

// ---------------------------------------------------------------------------
// Red-black Gauss-Seidel half-sweep on colour c (0 = red = (x+y+z) even), in
// place: u_i <- (q_i + sum_j c_ij u_j) / (sum_j c_ij + mua_i).  Each thread
// updates one vertex of the colour; rows are interleaved by colour.
template <class T>
__global__ void k_gs_half(T* __restrict__ u, const T* __restrict__ q, const T* __restrict__ D,
                          const T* __restrict__ mu, int N, Stencil<T> s, int colour) {
    int M = N / 2, Ni = N - 1;
    int64_t total = (int64_t)Ni * Ni * M;
    int64_t lin = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (lin >= total) return;
    int t = (int)(lin % M);
    int64_t rem = lin / M;
    int y = 1 + (int)(rem % Ni), x = 1 + (int)(rem / Ni);
    int z = 1 + ((x + y + 1 + colour) & 1) + 2 * t;
    if (z > N - 1) return;
    int n = N + 1;
    int64_t i = vidx(n, x, y, z);
    int64_t sx = (int64_t)n * n;
    T Di = D[i];
    T c0 = face_coef(Di, D[i + sx], s), c1 = face_coef(Di, D[i - sx], s);
    T c2 = face_coef(Di, D[i + n], s), c3 = face_coef(Di, D[i - n], s);
    T c4 = face_coef(Di, D[i + 1], s), c5 = face_coef(Di, D[i - 1], s);
    T num = q[i] + c0 * u[i + sx] + c1 * u[i - sx] + c2 * u[i + n] + c3 * u[i - n] + c4 * u[i + 1] + c5 * u[i - 1];
    T den = mu[i] + c0 + c1 + c2 + c3 + c4 + c5;
    u[i] = num / den;
}

// r = q - A u on interior vertices (0 on the boundary); mode 1 writes A u instead.
template <class T>
__global__ void k_defect(const T* __restrict__ u, const T* __restrict__ q, const T* __restrict__ D,
                         const T* __restrict__ mu, T* __restrict__ r, int N, Stencil<T> s, int apply_only) {
    int n = N + 1;
    int64_t nv = (int64_t)n * n * n, sx = (int64_t)n * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        int z = (int)(i % n), y = (int)((i / n) % n), x = (int)(i / sx);
        if (!is_interior(N, x, y, z)) { r[i] = T(0); continue; }
        T Di = D[i], ui = u[i];
        T Au = mu[i] * ui + face_coef(Di, D[i + sx], s) * (ui - u[i + sx]) + face_coef(Di, D[i - sx], s) * (ui - u[i - sx]) +
               face_coef(Di, D[i + n], s) * (ui - u[i + n]) + face_coef(Di, D[i - n], s) * (ui - u[i - n]) +
               face_coef(Di, D[i + 1], s) * (ui - u[i + 1]) + face_coef(Di, D[i - 1], s) * (ui - u[i - 1]);
        r[i] = apply_only ? Au : q[i] - Au;
    }
}

// Full-weighting restriction qc = R r (1/64)(1,2,1)^3 on coarse interior
// vertices, 0 on the coarse boundary.
template <class T>
__global__ void k_restrict(const T* __restrict__ r, T* __restrict__ qc, int Nf) {
    int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    int64_t nv = (int64_t)nc * nc * nc;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        int Z = (int)(v % nc), Y = (int)((v / nc) % nc), X = (int)(v / ((int64_t)nc * nc));
        if (!is_interior(Nc, X, Y, Z)) { qc[v] = T(0); continue; }
        T s = T(0);
        for (int a = -1; a <= 1; a++)
            for (int b = -1; b <= 1; b++) {
                T wab = T((2 - abs(a)) * (2 - abs(b)));
                const T* row = r + vidx(nf, 2 * X + a, 2 * Y + b, 2 * Z);
                s += wab * (row[-1] + T(2) * row[0] + row[1]);
            }
        qc[v] = s * T(1.0 / 64.0);
    }
}

// u += I ec on fine interior vertices (trilinear interpolation, I = 8 R^T).
template <class T>
__global__ void k_prolong_add(const T* __restrict__ ec, T* __restrict__ u, int Nf) {
    int nf = Nf + 1, nc = Nf / 2 + 1;
    int64_t nv = (int64_t)nf * nf * nf;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        int z = (int)(v % nf), y = (int)((v / nf) % nf), x = (int)(v / ((int64_t)nf * nf));
        if (!is_interior(Nf, x, y, z)) continue;
        int x0 = x >> 1, y0 = y >> 1, z0 = z >> 1;
        int x1 = x0 + (x & 1), y1 = y0 + (y & 1), z1 = z0 + (z & 1);
        T s = ec[vidx(nc, x0, y0, z0)] + ec[vidx(nc, x0, y0, z1)] + ec[vidx(nc, x0, y1, z0)] + ec[vidx(nc, x0, y1, z1)] +
              ec[vidx(nc, x1, y0, z0)] + ec[vidx(nc, x1, y0, z1)] + ec[vidx(nc, x1, y1, z0)] + ec[vidx(nc, x1, y1, z1)];
        // each of the 8 gathered corners repeats a corner when a coordinate is
        // even, so the sum equals 8 x (trilinear value); scale by 1/8.
        u[v] += s * T(0.125);
    }
}

// Exact solve on a level with at most 8 interior unknowns (N = 2 or 3), by
// one thread, in float64 whatever the storage types: assemble the dense
// matrix and factor it (Cholesky).  Boundary entries of u are the Dirichlet
// values and move to the right-hand side; interior entries of u are written.
template <class Tq, class Tu>
__device__ void dense_exact_solve(const Tq* q, Tu* u, const double* __restrict__ D, const double* __restrict__ mu, int N,
                                  Stencil<double> s) {
    int n = N + 1, m = (N - 1) * (N - 1) * (N - 1);
    double A[8][8], b[8];
    int64_t vid[8];
    int t = 0;
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) vid[t++] = vidx(n, x, y, z);
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) A[r][c] = 0.0;
    const int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    t = 0;
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++, t++) {
                int64_t i = vid[t];
                A[t][t] = mu[i];
                b[t] = (double)q[i];
                for (int e = 0; e < 6; e++) {
                    int xa = x + off[e][0], ya = y + off[e][1], za = z + off[e][2];
                    int64_t j = vidx(n, xa, ya, za);
                    double c = face_coef(D[i], D[j], s);
                    A[t][t] += c;
                    if (is_interior(N, xa, ya, za)) {
                        int tj = ((xa - 1) * (N - 1) + (ya - 1)) * (N - 1) + (za - 1);
                        A[t][tj] -= c;
                    } else {
                        b[t] += c * (double)u[j];
                    }
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
    for (int r = 0; r < m; r++) u[vid[r]] = (Tu)b[r];
}

// Inverse of the coarsest operator, for coarse solves by a matrix-vector
// product (corrections, whose boundary values are 0).  The unknowns are the
// m = (N-1)^3 <= 8 interior vertices in x, y, z order; A is assembled in
// float64 as above and inverted by Gauss-Jordan elimination without
// pivoting (A is symmetric positive definite and diagonally dominant).  One
// workgroup of 64 threads; thread t owns row t.  inv is m x m, row-major.
constexpr int kCoarseMax = 8;
__global__ void k_coarse_inverse(const double* __restrict__ D, const double* __restrict__ mu, int N, Stencil<double> s,
                                 double* __restrict__ inv) {
    __shared__ double M[kCoarseMax][2 * kCoarseMax];
    const int Nm = N - 1, m = Nm * Nm * Nm, n = N + 1, t = threadIdx.x;
    if (t < m) {
        const int x = 1 + t / (Nm * Nm), y = 1 + (t / Nm) % Nm, z = 1 + t % Nm;
        for (int j = 0; j < 2 * m; j++) M[t][j] = 0.0;
        const int64_t i = vidx(n, x, y, z);
        const int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        double d = mu[i];
        for (int e = 0; e < 6; e++) {
            const int xa = x + off[e][0], ya = y + off[e][1], za = z + off[e][2];
            const double c = face_coef(D[i], D[vidx(n, xa, ya, za)], s);
            d += c;
            if (is_interior(N, xa, ya, za)) M[t][((xa - 1) * Nm + (ya - 1)) * Nm + (za - 1)] = -c;
        }
        M[t][t] = d;
        M[t][m + t] = 1.0;
    }
    __syncthreads();
    for (int p = 0; p < m; p++) {
        // rows other than p only change their own entries and read row p
        if (t < m && t != p) {
            const double f = M[t][p] / M[p][p];
            for (int j = 0; j < 2 * m; j++) M[t][j] -= f * M[p][j];
        }
        __syncthreads();
    }
    if (t < m)
        for (int j = 0; j < m; j++) inv[t * m + j] = M[t][m + j] / M[t][t];
}

template <class T>
__global__ void k_exact_solve(const T* __restrict__ q, T* __restrict__ u, const double* __restrict__ D,
                              const double* __restrict__ mu, int N, Stencil<double> s) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    dense_exact_solve(q, u, D, mu, N, s);
}

// ---------------------------------------------------------------------------
// Norms (float64 accumulation, deterministic two-stage reduction).

// partial[block] = sum over the block's interior vertices of (q - A u)^2
// (or of q^2 when u == nullptr).
template <class T>
__global__ void k_resid_sq(const T* __restrict__ u, const T* __restrict__ q, const T* __restrict__ D,
                           const T* __restrict__ mu, int N, Stencil<T> s, double* __restrict__ partial) {
    int n = N + 1;
    int64_t nv = (int64_t)n * n * n, sx = (int64_t)n * n;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        int z = (int)(i % n), y = (int)((i / n) % n), x = (int)(i / sx);
        if (!is_interior(N, x, y, z)) continue;
        T r = q[i];
        if (u) {
            T Di = D[i], ui = u[i];
            r -= mu[i] * ui + face_coef(Di, D[i + sx], s) * (ui - u[i + sx]) + face_coef(Di, D[i - sx], s) * (ui - u[i - sx]) +
                 face_coef(Di, D[i + n], s) * (ui - u[i + n]) + face_coef(Di, D[i - n], s) * (ui - u[i - n]) +
                 face_coef(Di, D[i + 1], s) * (ui - u[i + 1]) + face_coef(Di, D[i - 1], s) * (ui - u[i - 1]);
        }
        acc += (double)r * (double)r;
    }
    double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// out[slot] = sum of partial[0..count) in a fixed order (one block).
__global__ void k_sum_partials(const double* __restrict__ partial, int count, double* __restrict__ out, int slot) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
    double b = block_sum(acc);
    if (threadIdx.x == 0) out[slot] = b;
}

// Iterative refinement, float64 step: r32 = float(q - A u) on interior
// vertices (0 on the boundary), partial[block] = sum of (q - A u)^2.
__global__ void k_resid_cast(const double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                             const double* __restrict__ mu, int N, Stencil<double> s, float* __restrict__ r32,
                             double* __restrict__ partial) {
    int n = N + 1;
    int64_t nv = (int64_t)n * n * n, sx = (int64_t)n * n;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        int z = (int)(i % n), y = (int)((i / n) % n), x = (int)(i / sx);
        if (!is_interior(N, x, y, z)) { r32[i] = 0.0f; continue; }
        double Di = D[i], ui = u[i];
        double r = q[i] - (mu[i] * ui + face_coef(Di, D[i + sx], s) * (ui - u[i + sx]) + face_coef(Di, D[i - sx], s) * (ui - u[i - sx]) +
                           face_coef(Di, D[i + n], s) * (ui - u[i + n]) + face_coef(Di, D[i - n], s) * (ui - u[i - n]) +
                           face_coef(Di, D[i + 1], s) * (ui - u[i + 1]) + face_coef(Di, D[i - 1], s) * (ui - u[i - 1]));
        r32[i] = (float)r;
        acc += r * r;
    }
    double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// Iterative refinement, float64 step: u += e (e float32; boundary of e is 0).
__global__ void k_add_correction(double* __restrict__ u, const float* __restrict__ e, int64_t nv) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x)
        u[v] += (double)e[v];
}

// ---------------------------------------------------------------------------
// Derivatives with respect to the coefficients (adjoint-state derivatives of
// the discrete solution).

// Column march of the derivative kernels: thread p = y (N+1) + z of a plane
// walks the planes [x0, x1) of chunk c and keeps its own values at x - 1, x
// and x + 1 in registers, so each field is read from memory about once
// (plus one plane at each end of a chunk).  In-plane neighbours p +- 1 and
// p +- (N+1) are loaded: the block itself or blocks running beside it load
// them at about the same time.  The flattened (plane block, chunk) index is
// remapped so that each XCD runs a contiguous range of it (whole chunks of
// consecutive rows), which keeps those neighbours in one L2.
struct ColMarch {
    int n, y, z, x0, x1;
    int64_t sx, p;
};

__device__ __forceinline__ bool col_march(int N, int chunk, ColMarch& c) {
    const int nb = (int)(gridDim.x * gridDim.y);
    const int L = xcd_remap((int)(blockIdx.y * gridDim.x + blockIdx.x), nb);
    const int bx = L % (int)gridDim.x, by = L / (int)gridDim.x;
    c.n = N + 1;
    c.sx = (int64_t)c.n * c.n;
    c.p = (int64_t)bx * blockDim.x + threadIdx.x;
    c.x0 = by * chunk;
    if (c.p >= c.sx || c.x0 >= c.n) return false;
    c.y = (int)(c.p / c.n);
    c.z = (int)(c.p % c.n);
    c.x1 = min(c.n, c.x0 + chunk);
    return true;
}

// d D_f along the tangent: D_f = (D_a + D_b)/2 or 2 D_a D_b / (D_a + D_b),
// with dD = D dlogD at both ends
__device__ __forceinline__ double dface(double Da, double dDa, double Db, double dDb, int harmonic) {
    if (harmonic) {
        const double sum = Da + Db;
        return 2.0 * (Db * Db * dDa + Da * Da * dDb) / (sum * sum);
    }
    return 0.5 * (dDa + dDb);
}

// rhs = dq - (dA) rho on interior vertices (0 on the boundary), where
// (dA rho)_i = sum_j dD_f,ij/h^2 (rho_i - rho_j) + mua_i dlogmua_i rho_i and
// dD_f is the derivative of the face mean along dlogD.  Null tangents are 0.
// Neighbours in the order +x, -x, +y, -y, +z, -z.
__global__ void k_tangent_rhs_col(const double* __restrict__ rho, const double* __restrict__ dq,
                                  const double* __restrict__ dlogD, const double* __restrict__ dlogmu,
                                  const double* __restrict__ D, const double* __restrict__ mu, int N, double inv_h2,
                                  int harmonic, double* __restrict__ rhs, int chunk) {
    ColMarch c;
    if (!col_march(N, chunk, c)) return;
    const int n = c.n;
    const bool yz = c.y > 0 && c.y < N && c.z > 0 && c.z < N;
    auto dD_at = [&](int64_t j) { return dlogD ? D[j] * dlogD[j] : 0.0; };
    double rm = 0.0, Dm = 0.0, dDm = 0.0;
    if (c.x0 > 0 && yz) {
        const int64_t j = (c.x0 - 1) * c.sx + c.p;
        rm = rho[j]; Dm = D[j]; dDm = dD_at(j);
    }
    const int64_t i0 = c.x0 * c.sx + c.p;
    double rc = rho[i0], Dc = D[i0], dDc = dD_at(i0);
    for (int x = c.x0; x < c.x1; x++) {
        const int64_t i = x * c.sx + c.p;
        double rp = 0.0, Dp = 0.0, dDp = 0.0;
        if (x < N && yz) {
            rp = rho[i + c.sx]; Dp = D[i + c.sx]; dDp = dD_at(i + c.sx);
        }
        double out = 0.0;
        if (yz && x > 0 && x < N) {
            double acc = dlogmu ? mu[i] * dlogmu[i] * rc : 0.0;
            if (dlogD) {
                auto nb = [&](double Dj, double dDj, double rj) { acc += dface(Dc, dDc, Dj, dDj, harmonic) * inv_h2 * (rc - rj); };
                nb(Dp, dDp, rp);
                nb(Dm, dDm, rm);
                nb(D[i + n], dD_at(i + n), rho[i + n]);
                nb(D[i - n], dD_at(i - n), rho[i - n]);
                nb(D[i + 1], dD_at(i + 1), rho[i + 1]);
                nb(D[i - 1], dD_at(i - 1), rho[i - 1]);
            }
            out = (dq ? dq[i] : 0.0) - acc;
        }
        rhs[i] = out;
        rm = rc; Dm = Dc; dDm = dDc;
        rc = rp; Dc = Dp; dDc = dDp;
    }
}

// Coefficient gradients from the adjoint state lam = qbar:
//   logmua_bar_i = -mua_i lam_i rho_i (interior, 0 on the boundary)
//   logD_bar_v   = -sum_{faces (v,j), v or j interior} dD_f/dlogD_v (lam_v - lam_j)(rho_v - rho_j) / h^2
// with lam = 0 on boundary vertices.  With data d and weights w (the
// likelihood's gradient) logmua_bar also takes the direct term of L_e =
// mua rho: w_i (mua_i rho_i - d_i) mua_i rho_i.  Neighbours in the order
// +x, -x, +y, -y, +z, -z.
__global__ void k_coef_grads_col(const double* __restrict__ rho, const double* __restrict__ lam,
                                 const double* __restrict__ D, const double* __restrict__ mu, int N, double inv_h2,
                                 int harmonic, double* __restrict__ gD, double* __restrict__ gmu,
                                 const double* __restrict__ d, const double* __restrict__ w, int chunk) {
    ColMarch c;
    if (!col_march(N, chunk, c)) return;
    const int n = c.n;
    const bool yz = c.y > 0 && c.y < N && c.z > 0 && c.z < N;
    auto lam_at = [&](int x, int y, int z, int64_t j) { return is_interior(N, x, y, z) ? lam[j] : 0.0; };
    double lm = 0.0, rm = 0.0, Dm = 0.0;
    if (c.x0 > 0) {
        const int64_t j = (c.x0 - 1) * c.sx + c.p;
        lm = lam_at(c.x0 - 1, c.y, c.z, j); rm = rho[j]; Dm = D[j];
    }
    const int64_t i0 = c.x0 * c.sx + c.p;
    double lc = lam_at(c.x0, c.y, c.z, i0), rc = rho[i0], Dc = D[i0];
    for (int x = c.x0; x < c.x1; x++) {
        const int64_t i = x * c.sx + c.p;
        double lp = 0.0, rp = 0.0, Dp = 0.0;
        if (x < N) {
            lp = lam_at(x + 1, c.y, c.z, i + c.sx); rp = rho[i + c.sx]; Dp = D[i + c.sx];
        }
        const bool vin = yz && x > 0 && x < N;
        if (gmu) {
            double g = vin ? -mu[i] * lc * rc : 0.0;
            if (d && vin) {
                const double Le = mu[i] * rc;
                g += w[i] * (Le - d[i]) * Le;
            }
            gmu[i] = g;
        }
        if (gD) {
            double acc = 0.0;
            auto nb = [&](bool jin, double lj, double rj, double Dj) {
                if (!vin && !jin) return;
                double dcdv;
                if (harmonic) {
                    const double sum = Dc + Dj;
                    dcdv = 2.0 * Dj * Dj * Dc / (sum * sum);
                } else {
                    dcdv = 0.5 * Dc;
                }
                acc += dcdv * (lc - lj) * (rc - rj);
            };
            if (x < N) nb(yz && x + 1 < N, lp, rp, Dp);
            if (x > 0) nb(yz && x - 1 > 0, lm, rm, Dm);
            const bool xin = x > 0 && x < N, zin = c.z > 0 && c.z < N, yin = c.y > 0 && c.y < N;
            if (c.y < N) nb(xin && zin && c.y + 1 < N, xin && zin && c.y + 1 < N ? lam[i + n] : 0.0, rho[i + n], D[i + n]);
            if (c.y > 0) nb(xin && zin && c.y - 1 > 0, xin && zin && c.y - 1 > 0 ? lam[i - n] : 0.0, rho[i - n], D[i - n]);
            if (c.z < N) nb(xin && yin && c.z + 1 < N, xin && yin && c.z + 1 < N ? lam[i + 1] : 0.0, rho[i + 1], D[i + 1]);
            if (c.z > 0) nb(xin && yin && c.z - 1 > 0, xin && yin && c.z - 1 > 0 ? lam[i - 1] : 0.0, rho[i - 1], D[i - 1]);
            gD[i] = -acc * inv_h2;
        }
        lm = lc; rm = rc; Dm = Dc;
        lc = lp; rc = rp; Dc = Dp;
    }
}

}  // namespace dmgs
