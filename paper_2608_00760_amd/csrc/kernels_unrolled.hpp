// kernels_unrolled.hpp -- reverse pass of the fixed-cycle solver through
// every step (the unrolled adjoint), float64, three-dimensional plans.
//
// Cotangents (bars) of one recorded V-cycle are carried back step by step
// (Sec. 2.4, Eq. (EqcompT), with the coefficients as further inputs of each
// step).  With c_f = D_f / h^2 on face f and d_i = sum_f c_f + mua_i:
//   half-sweep of colour C (u'_i = (q_i + sum_j c_ij u_j) / d_i, i in C):
//     v_i = ubar_i / d_i; qbar_i += v_i; mubar_i -= v_i u'_i;
//     Dbar_v -= sum over faces (v, w) of (v_v - v_w)(u'_v - u'_w) dc/dD_v;
//     ubar_j += sum_i c_ij v_i (j not in C), ubar_i = 0 (i in C);
//   defect r = q - A u with cotangent rbar:
//     qbar += rbar; ubar -= A rbar; mubar_i -= rbar_i u_i;
//     Dbar_v -= sum over faces (v, w) of (rbar_v - rbar_w)(u_v - u_w) dc/dD_v;
//   coarsest solve u = A^-1 q: lam = A^-1 ubar, qbar += lam and the
//   defect's coefficient terms with lam;
//   coefficient coarsening (full weighting, injection on the boundary):
//     its transpose carries a coarse level's Dbar, mubar to the finer one.
// Every kernel takes one vertex per thread; cotangents are 0 on boundary
// vertices except Dbar, which boundary faces reach.
#pragma once
#include "kernels_basic.hpp"

namespace dmgs {

// d c_f / d D_a for the face coefficient c_f = face(D_a, D_b) / h^2
__device__ __forceinline__ double dface_da(double Da, double Db, const Stencil<double>& s) {
    if (s.harmonic) {
        const double t = Da + Db;
        return Db * Db / (t * t) * s.two_inv_h2;
    }
    return s.half_inv_h2;
}

__device__ __forceinline__ bool vertex3(int64_t i, int N, int& x, int& y, int& z) {
    const int n = N + 1;
    z = (int)(i % n);
    y = (int)((i / n) % n);
    x = (int)(i / ((int64_t)n * n));
    return is_interior(N, x, y, z);
}

// half-sweep reverse, part 1: V = ubar / d on the colour's interior vertices
// (0 elsewhere); qbar += V; mubar -= V u'
__global__ void k_un_half_v(const double* __restrict__ ubar, const double* __restrict__ up,
                            const double* __restrict__ D, const double* __restrict__ mu, int N, Stencil<double> s,
                            int colour, double* __restrict__ V, double* __restrict__ qbar, double* __restrict__ mubar) {
    const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int x, y, z;
    if (!vertex3(i, N, x, y, z) || ((x + y + z) & 1) != colour) {
        V[i] = 0.0;
        return;
    }
    const int n = N + 1;
    const int64_t sx = (int64_t)n * n;
    const double Di = D[i];
    const double d = mu[i] + face_coef(Di, D[i + sx], s) + face_coef(Di, D[i - sx], s) + face_coef(Di, D[i + n], s) +
                     face_coef(Di, D[i - n], s) + face_coef(Di, D[i + 1], s) + face_coef(Di, D[i - 1], s);
    const double v = ubar[i] / d;
    V[i] = v;
    qbar[i] += v;
    mubar[i] -= v * up[i];
}

// half-sweep reverse, part 2: Dbar on every vertex, ubar on interior ones
__global__ void k_un_half_gather(double* __restrict__ ubar, const double* __restrict__ V, const double* __restrict__ up,
                                 const double* __restrict__ D, int N, Stencil<double> s, int colour,
                                 double* __restrict__ Dbar) {
    const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int x, y, z;
    const bool in = vertex3(i, N, x, y, z);
    const int n = N + 1;
    const int64_t sx = (int64_t)n * n;
    const int o[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    const int64_t off[6] = {sx, -sx, n, -n, 1, -1};
    const double Di = D[i], Vi = V[i], ui = up[i];
    double dacc = 0.0, gath = 0.0;
    for (int e = 0; e < 6; e++) {
        const int xa = x + o[e][0], ya = y + o[e][1], za = z + o[e][2];
        if (xa < 0 || xa > N || ya < 0 || ya > N || za < 0 || za > N) continue;
        const int64_t j = i + off[e];
        const double Dj = D[j], Vj = V[j];
        dacc += (Vi - Vj) * (ui - up[j]) * dface_da(Di, Dj, s);
        gath += face_coef(Di, Dj, s) * Vj;
    }
    Dbar[i] -= dacc;
    if (in) ubar[i] = ((x + y + z) & 1) == colour ? 0.0 : ubar[i] + gath;
}

// defect (or coarsest-solve) reverse with cotangent rbar = scale * rb (rb
// read on interior vertices only): qbar += rbar, ubar -= A rbar (unless
// ubar is null), mubar -= rbar u, Dbar -= the face terms
__global__ void k_un_defect(double* __restrict__ ubar, const double* __restrict__ rb, double scale,
                            const double* __restrict__ u, const double* __restrict__ D, const double* __restrict__ mu,
                            int N, Stencil<double> s, double* __restrict__ qbar, double* __restrict__ Dbar,
                            double* __restrict__ mubar) {
    const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int x, y, z;
    const bool in = vertex3(i, N, x, y, z);
    const int n = N + 1;
    const int64_t sx = (int64_t)n * n;
    const int o[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    const int64_t off[6] = {sx, -sx, n, -n, 1, -1};
    const double Di = D[i], ui = u[i];
    const double ri = in ? scale * rb[i] : 0.0;
    double dacc = 0.0, Ar = in ? mu[i] * ri : 0.0;
    for (int e = 0; e < 6; e++) {
        const int xa = x + o[e][0], ya = y + o[e][1], za = z + o[e][2];
        if (xa < 0 || xa > N || ya < 0 || ya > N || za < 0 || za > N) continue;
        const int64_t j = i + off[e];
        const double rj = is_interior(N, xa, ya, za) ? scale * rb[j] : 0.0;
        const double Dj = D[j];
        dacc += (ri - rj) * (ui - u[j]) * dface_da(Di, Dj, s);
        Ar += face_coef(Di, Dj, s) * (ri - rj);
    }
    Dbar[i] -= dacc;
    if (!in) return;
    qbar[i] += ri;
    mubar[i] -= ri * ui;
    if (ubar) ubar[i] -= Ar;
}

// a *= f
__global__ void k_un_scale(double* __restrict__ a, int64_t n, double f) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] *= f;
}

// fbar += (coarsening)^T cbar: full weighting (2-|a|)(2-|b|)(2-|c|)/64 from
// coarse interior vertices, injection from coarse boundary ones
__global__ void k_un_coarsen_T(const double* __restrict__ cbar, double* __restrict__ fbar, int Nf) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t nv = (int64_t)nf * nf * nf;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int z = (int)(i % nf), y = (int)((i / nf) % nf), x = (int)(i / ((int64_t)nf * nf));
    double acc = 0.0;
    const int Xs[2] = {x >> 1, (x + 1) >> 1}, Ys[2] = {y >> 1, (y + 1) >> 1}, Zs[2] = {z >> 1, (z + 1) >> 1};
    const int nx = Xs[0] == Xs[1] ? 1 : 2, ny = Ys[0] == Ys[1] ? 1 : 2, nz = Zs[0] == Zs[1] ? 1 : 2;
    for (int a = 0; a < nx; a++)
        for (int b = 0; b < ny; b++)
            for (int c = 0; c < nz; c++) {
                const int X = Xs[a], Y = Ys[b], Z = Zs[c];
                if (!is_interior(Nc, X, Y, Z)) continue;
                const double w = (double)((2 - abs(x - 2 * X)) * (2 - abs(y - 2 * Y)) * (2 - abs(z - 2 * Z))) / 64.0;
                acc += w * cbar[((int64_t)X * nc + Y) * nc + Z];
            }
    if (!(x & 1) && !(y & 1) && !(z & 1) && !is_interior(Nc, x >> 1, y >> 1, z >> 1))
        acc += cbar[((int64_t)(x >> 1) * nc + (y >> 1)) * nc + (z >> 1)];
    fbar[i] += acc;
}

// out = a * b
__global__ void k_un_mul(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] * b[i];
}

}  // namespace dmgs
