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
// The stencil kernels march along x (see UnCol); the others take one vertex
// per thread.  Cotangents are 0 on boundary vertices except Dbar, which
// boundary faces reach.
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

// Column march: thread p of a plane (p = y (N+1) + z, so a plane is one
// coalesced run) walks the planes [x0, x0 + chunk) of chunk blockIdx.y and
// keeps the fields it needs at x - 1, x and x + 1 in registers; in-plane
// neighbours are read at p +- (N+1) and p +- 1.  Each field is read from
// memory about once, instead of three times for neighbours one plane away.
struct UnCol {
    int n, y, z, x0, x1;
    int64_t sx, p;
};

__device__ __forceinline__ bool un_col(int N, int chunk, UnCol& c) {
    c.n = N + 1;
    c.sx = (int64_t)c.n * c.n;
    c.p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    c.x0 = (int)blockIdx.y * chunk;
    if (c.p >= c.sx || c.x0 >= c.n) return false;
    c.y = (int)(c.p / c.n);
    c.z = (int)(c.p % c.n);
    c.x1 = min(c.n, c.x0 + chunk);
    return true;
}

// Recorded half-sweep of colour C, out of place: u_out = the Gauss-Seidel
// value on C's interior vertices (it reads only the other colour, so it
// equals the in-place sweep) and u_in elsewhere.  The recompute writes each
// state straight into its tape slot.
__global__ void k_un_gs_half(const double* __restrict__ u_in, double* __restrict__ u_out,
                             const double* __restrict__ q, const double* __restrict__ D,
                             const double* __restrict__ mu, int N, Stencil<double> s, int colour, int chunk) {
    UnCol c;
    if (!un_col(N, chunk, c)) return;
    const int n = c.n;
    const bool yz = c.y > 0 && c.y < N && c.z > 0 && c.z < N;
    double Dm = 0.0, um = 0.0;
    if (c.x0 > 0) {
        const int64_t j = (c.x0 - 1) * c.sx + c.p;
        Dm = D[j]; um = u_in[j];
    }
    const int64_t i0 = c.x0 * c.sx + c.p;
    double Dc = D[i0], uc = u_in[i0];
    for (int x = c.x0; x < c.x1; x++) {
        const int64_t i = x * c.sx + c.p;
        double Dp = 0.0, upp = 0.0;
        if (x < N) {
            Dp = D[i + c.sx]; upp = u_in[i + c.sx];
        }
        double v = uc;
        if (yz && x > 0 && x < N && ((x + c.y + c.z) & 1) == colour) {
            const double c0 = face_coef(Dc, Dp, s), c1 = face_coef(Dc, Dm, s);
            const double c2 = face_coef(Dc, D[i + n], s), c3 = face_coef(Dc, D[i - n], s);
            const double c4 = face_coef(Dc, D[i + 1], s), c5 = face_coef(Dc, D[i - 1], s);
            const double num = q[i] + c0 * upp + c1 * um + c2 * u_in[i + n] + c3 * u_in[i - n] + c4 * u_in[i + 1] +
                               c5 * u_in[i - 1];
            const double den = mu[i] + c0 + c1 + c2 + c3 + c4 + c5;
            v = num / den;
        }
        u_out[i] = v;
        Dm = Dc; um = uc;
        Dc = Dp; uc = upp;
    }
}

// half-sweep reverse, part 1: V = ubar / d on the colour's interior vertices
// (0 elsewhere); qbar += V; mubar -= V u'
__global__ void k_un_half_v(const double* __restrict__ ubar, const double* __restrict__ up,
                            const double* __restrict__ D, const double* __restrict__ mu, int N, Stencil<double> s,
                            int colour, double* __restrict__ V, double* __restrict__ qbar, double* __restrict__ mubar,
                            int chunk) {
    UnCol c;
    if (!un_col(N, chunk, c)) return;
    const int n = c.n;
    const bool yz = c.y > 0 && c.y < N && c.z > 0 && c.z < N;
    double Dm = c.x0 > 0 ? D[(c.x0 - 1) * c.sx + c.p] : 0.0, Dc = D[c.x0 * c.sx + c.p];
    for (int x = c.x0; x < c.x1; x++) {
        const int64_t i = x * c.sx + c.p;
        const double Dp = x < N ? D[i + c.sx] : 0.0;
        if (yz && x > 0 && x < N && ((x + c.y + c.z) & 1) == colour) {
            const double d = mu[i] + face_coef(Dc, Dp, s) + face_coef(Dc, Dm, s) + face_coef(Dc, D[i + n], s) +
                             face_coef(Dc, D[i - n], s) + face_coef(Dc, D[i + 1], s) + face_coef(Dc, D[i - 1], s);
            const double v = ubar[i] / d;
            V[i] = v;
            qbar[i] += v;
            mubar[i] -= v * up[i];
        } else {
            V[i] = 0.0;
        }
        Dm = Dc;
        Dc = Dp;
    }
}

// half-sweep reverse, part 2: Dbar on every vertex, ubar on interior ones
__global__ void k_un_half_gather(double* __restrict__ ubar, const double* __restrict__ V, const double* __restrict__ up,
                                 const double* __restrict__ D, int N, Stencil<double> s, int colour,
                                 double* __restrict__ Dbar, int chunk) {
    UnCol c;
    if (!un_col(N, chunk, c)) return;
    const int n = c.n;
    const bool yz = c.y > 0 && c.y < N && c.z > 0 && c.z < N;
    double Dm = 0.0, Vm = 0.0, um = 0.0;
    if (c.x0 > 0) {
        const int64_t j = (c.x0 - 1) * c.sx + c.p;
        Dm = D[j]; Vm = V[j]; um = up[j];
    }
    const int64_t i0 = c.x0 * c.sx + c.p;
    double Dc = D[i0], Vc = V[i0], uc = up[i0];
    for (int x = c.x0; x < c.x1; x++) {
        const int64_t i = x * c.sx + c.p;
        double Dp = 0.0, Vp = 0.0, upp = 0.0;
        if (x < N) {
            Dp = D[i + c.sx]; Vp = V[i + c.sx]; upp = up[i + c.sx];
        }
        double dacc = 0.0, gath = 0.0;
        // neighbours in the order +x, -x, +y, -y, +z, -z
        auto nb = [&](double Dj, double Vj, double uj) {
            dacc += (Vc - Vj) * (uc - uj) * dface_da(Dc, Dj, s);
            gath += face_coef(Dc, Dj, s) * Vj;
        };
        if (x < N) nb(Dp, Vp, upp);
        if (x > 0) nb(Dm, Vm, um);
        if (c.y < N) nb(D[i + n], V[i + n], up[i + n]);
        if (c.y > 0) nb(D[i - n], V[i - n], up[i - n]);
        if (c.z < N) nb(D[i + 1], V[i + 1], up[i + 1]);
        if (c.z > 0) nb(D[i - 1], V[i - 1], up[i - 1]);
        Dbar[i] -= dacc;
        if (yz && x > 0 && x < N) ubar[i] = ((x + c.y + c.z) & 1) == colour ? 0.0 : ubar[i] + gath;
        Dm = Dc; Vm = Vc; um = uc;
        Dc = Dp; Vc = Vp; uc = upp;
    }
}

// defect (or coarsest-solve) reverse with cotangent rbar = scale * rb (rb
// read on interior vertices only): qbar += rbar, ubar -= A rbar (unless
// ubar is null), mubar -= rbar u, Dbar -= the face terms
__global__ void k_un_defect(double* __restrict__ ubar, const double* __restrict__ rb, double scale,
                            const double* __restrict__ u, const double* __restrict__ D, const double* __restrict__ mu,
                            int N, Stencil<double> s, double* __restrict__ qbar, double* __restrict__ Dbar,
                            double* __restrict__ mubar, int chunk) {
    UnCol c;
    if (!un_col(N, chunk, c)) return;
    const int n = c.n;
    const bool yz = c.y > 0 && c.y < N && c.z > 0 && c.z < N;
    auto rx = [&](int x, int64_t j) { return yz && x > 0 && x < N ? scale * rb[j] : 0.0; };
    double Dm = 0.0, um = 0.0, rm = 0.0;
    if (c.x0 > 0) {
        const int64_t j = (c.x0 - 1) * c.sx + c.p;
        Dm = D[j]; um = u[j]; rm = rx(c.x0 - 1, j);
    }
    const int64_t i0 = c.x0 * c.sx + c.p;
    double Dc = D[i0], uc = u[i0], rc = rx(c.x0, i0);
    for (int x = c.x0; x < c.x1; x++) {
        const int64_t i = x * c.sx + c.p;
        double Dp = 0.0, upp = 0.0, rp = 0.0;
        if (x < N) {
            Dp = D[i + c.sx]; upp = u[i + c.sx]; rp = rx(x + 1, i + c.sx);
        }
        const bool in = yz && x > 0 && x < N;
        double dacc = 0.0, Ar = in ? mu[i] * rc : 0.0;
        // neighbours in the order +x, -x, +y, -y, +z, -z; rb is read only
        // on interior neighbours
        auto nb = [&](double Dj, double uj, double rj) {
            dacc += (rc - rj) * (uc - uj) * dface_da(Dc, Dj, s);
            Ar += face_coef(Dc, Dj, s) * (rc - rj);
        };
        const bool zin = c.z > 0 && c.z < N, yin = c.y > 0 && c.y < N, xin = x > 0 && x < N;
        if (x < N) nb(Dp, upp, rp);
        if (x > 0) nb(Dm, um, rm);
        if (c.y < N) nb(D[i + n], u[i + n], xin && zin && c.y + 1 < N ? scale * rb[i + n] : 0.0);
        if (c.y > 0) nb(D[i - n], u[i - n], xin && zin && c.y - 1 > 0 ? scale * rb[i - n] : 0.0);
        if (c.z < N) nb(D[i + 1], u[i + 1], xin && yin && c.z + 1 < N ? scale * rb[i + 1] : 0.0);
        if (c.z > 0) nb(D[i - 1], u[i - 1], xin && yin && c.z - 1 > 0 ? scale * rb[i - 1] : 0.0);
        Dbar[i] -= dacc;
        if (in) {
            qbar[i] += rc;
            mubar[i] -= rc * uc;
            if (ubar) ubar[i] -= Ar;
        }
        Dm = Dc; um = uc; rm = rc;
        Dc = Dp; uc = upp; rc = rp;
    }
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
