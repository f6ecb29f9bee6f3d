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
// The outputs w, D32, mu32 are laid out with row pitch py and plane pitch
// px (D and mu are dense).
__global__ void k_level_prep(const double* __restrict__ D, const double* __restrict__ mu, int N, Stencil<double> st,
                             T* __restrict__ w, float* __restrict__ D32, float* __restrict__ mu32, int py, int64_t px) {
    const int n = N + 1, sx = n * n, nv = sx * n;
    const int i = vertex_of_thread();
    if (i >= nv) return;
    const int z = i % n, y = (i / n) % n, x = i / sx;
    const int64_t o = x * px + (int64_t)y * py + z;
    const double Di = D[i], mi = mu[i];
    if (D32) {
        D32[o] = (float)Di;
        mu32[o] = (float)mi;
    }
    if (!is_interior(N, x, y, z)) {
        w[o] = T(0);
        return;
    }
    const double d = mi + face_coef(Di, D[i + sx], st) + face_coef(Di, D[i - sx], st) + face_coef(Di, D[i + n], st) +
                     face_coef(Di, D[i - n], st) + face_coef(Di, D[i + 1], st) + face_coef(Di, D[i - 1], st);
    w[o] = (T)(1.0 / d);
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

// r = q - A u on interior vertices (0 on the boundary); mode 1 writes A u
// instead.  u, q and r are dense; the coefficients D and mu have row pitch
// cpy and plane pitch cpx.
template <class T>
__global__ void k_defect(const T* __restrict__ u, const T* __restrict__ q, const T* __restrict__ D,
                         const T* __restrict__ mu, T* __restrict__ r, int N, Stencil<T> s, int apply_only, int cpy,
                         int64_t cpx) {
    int n = N + 1;
    int64_t nv = (int64_t)n * n * n, sx = (int64_t)n * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        int z = (int)(i % n), y = (int)((i / n) % n), x = (int)(i / sx);
        if (!is_interior(N, x, y, z)) { r[i] = T(0); continue; }
        const int64_t c = x * cpx + (int64_t)y * cpy + z;
        T Di = D[c], ui = u[i];
        T Au = mu[c] * ui + face_coef(Di, D[c + cpx], s) * (ui - u[i + sx]) + face_coef(Di, D[c - cpx], s) * (ui - u[i - sx]) +
               face_coef(Di, D[c + cpy], s) * (ui - u[i + n]) + face_coef(Di, D[c - cpy], s) * (ui - u[i - n]) +
               face_coef(Di, D[c + 1], s) * (ui - u[i + 1]) + face_coef(Di, D[c - 1], s) * (ui - u[i - 1]);
        r[i] = apply_only ? Au : q[i] - Au;
    }
}

// dst = src on every vertex of an n^3 field, between layouts of row pitch
// spy / dpy and plane pitch spx / dpx (padding entries of dst untouched).
template <class T>
__global__ void k_repitch(const T* __restrict__ src, int spy, int64_t spx, T* __restrict__ dst, int dpy, int64_t dpx,
                          int n) {
    const int64_t nv = (int64_t)n * n * n;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(v % n), y = (int)((v / n) % n), x = (int)(v / ((int64_t)n * n));
        dst[x * dpx + (int64_t)y * dpy + z] = src[x * spx + (int64_t)y * spy + z];
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

// Arguments of k_sum_partials; grouped form, one workgroup per member (the
// same sums, in the same order).
struct SumArgs {
    const double* partial;
    int count;
    double* out;
    int slot;
};

__global__ void k_sum_grp(const Group<SumArgs>* g) {
    int bid;
    const int m = group_member(g, &bid);
    if (bid < 0) return;
    const SumArgs a = g->a[m];
    double acc = 0.0;
    for (int i = threadIdx.x; i < a.count; i += blockDim.x) acc += a.partial[i];
    double b = block_sum(acc);
    if (threadIdx.x == 0) a.out[a.slot] = b;
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

}  // namespace dmgs
