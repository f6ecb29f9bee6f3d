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
// On levels N >= 96 the stencil kernels march the column tiles of
// kernels_deriv.hpp and take a whole red-black sweep per pass: the recorded
// sweep (k_un_gs_sweep_t), its reverse (k_un_sweep_rev_t), and the defect's
// reverse (k_un_defect_t), with each plane's neighbours over the tile plus a
// ring in LDS.  Smaller levels march one thread per plane vertex (UnCol),
// one half-sweep per pass.  The rest take one vertex per thread.
// Cotangents are 0 on boundary vertices except Dbar, which boundary faces
// reach.
#pragma once
#include "kernels_basic.hpp"
#include "kernels_deriv.hpp"

namespace dmgs {

// d c_f / d D_a for the face coefficient c_f = face(D_a, D_b) / h^2
__device__ __forceinline__ double dface_da(double Da, double Db, const Stencil<double>& s) {
    if (s.harmonic) {
        const double t = Da + Db;
        return Db * Db / (t * t) * s.two_inv_h2;
    }
    return s.half_inv_h2;
}

// Levels below N = 96 run these x-march forms instead of the column tiles:
// a thread per vertex column of the plane gives small levels many more
// workgroups than whole 16 x 64 tiles would.
//
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

// The planes y = N and z = N that the column tiles leave out (taken by the
// extra workgroups of the same launches, see der_edge_block): boundary
// vertices, where only Dbar changes, by the one face to an interior
// neighbour j (the other faces join boundary vertices, whose cotangent terms
// are 0).

// defect reverse: rbar = 0 at the vertex, scale * rb_j at the interior neighbour
template <bool HARM>
__device__ __forceinline__ void un_defect_edge(const DerEdge& e, const double* __restrict__ rb, double scale,
                                               const double* __restrict__ u, const double* __restrict__ D,
                                               const Stencil<double>& s, double* __restrict__ Dbar) {
    double dacc = 0.0;
    if (e.jin) {
        const double rj = scale * rb[e.j];
        const double Dv = D[e.i], Dj = D[e.j];
        double dda;
        if (HARM) {
            const double t = Dv + Dj;
            dda = Dj * Dj / (t * t) * s.two_inv_h2;
        } else {
            dda = s.half_inv_h2;
        }
        dacc += (0.0 - rj) * (u[e.i] - u[e.j]) * dda;
    }
    Dbar[e.i] = Dbar[e.i] - dacc;
}

// A whole recorded sweep, out of place: u_mid = u_in after the half-sweep
// of colour c1 (the Gauss-Seidel value (q + sum_j c_ij u_j) w on c1's
// interior vertices, with the stored inverse diagonal w), u_out = u_mid
// after the half-sweep of the other colour c2; the recompute writes both
// states straight into their tape slots (each half-sweep reads only the
// other colour, so it equals the in-place sweep).  Each field is read once
// for the two half-sweeps.  The column tiles march along x with two stages:
// at step x, stage 1 forms u_mid on plane x over the tile plus a ring of
// one, and stage 2 forms u_out on plane x - 1 from u_mid of plane x - 1 in
// LDS and of planes x - 2 and x in registers.  u and D live in LDS over the
// tile plus a ring of two for five planes (x - 2 .. x + 2; plane x + 1 is
// published at step x, after it was loaded at step x - 1), so both stages
// take their x-neighbours from LDS and a thread keeps only the plane in
// flight and q, w of three planes in registers.  One barrier per step
// orders all LDS traffic: a plane's slot is rewritten four steps after its
// last reader's step ended, u_mid is double-buffered by plane parity.
// Neighbours in the order +x, -x, +y, -y, +z, -z.
constexpr int kSwRY = kDerTY + 4, kSwRZ = kDerTZ + 4, kSwCells = kSwRY * kSwRZ;
constexpr int kSwHalo = kSwCells - kDerThreads;   // ring-2 cells (336)
constexpr int kSwSlots = 5;

// A thread's cells in arrays over the tile plus a ring of two: its own
// column's, and its ring cell (tid < kSwHalo): rows y0 - 2, y0 - 1 and
// y0 + 16, y0 + 17 whole, then columns z0 - 2, z0 - 1, z0 + 64, z0 + 65 of
// the tile's rows.
struct SwRing {
    int cell2;            // own column in the ring-2 arrays
    int hy, hz;           // the ring cell
    bool halo, hv, r1;    // a ring thread; its cell inside the grid; at distance one
    int hcell2, hcell1;   // the ring cell in the ring-2 and ring-1 arrays
    int64_t hp;           // its in-plane offset
};

__device__ __forceinline__ void sw_ring(const DerTile& t, SwRing& r) {
    const int tid = (int)threadIdx.x, n = t.n;
    const int y0 = t.y - tid / kDerTZ, z0 = t.z - tid % kDerTZ;
    r.cell2 = (tid / kDerTZ + 2) * kSwRZ + tid % kDerTZ + 2;
    int ly, lz;
    if (tid < 2 * kSwRZ) {
        ly = tid / kSwRZ - 2; lz = tid % kSwRZ - 2;
    } else if (tid < 4 * kSwRZ) {
        ly = kDerTY + (tid - 2 * kSwRZ) / kSwRZ; lz = (tid - 2 * kSwRZ) % kSwRZ - 2;
    } else {
        const int u = tid - 4 * kSwRZ;   // < 4 * kDerTY for ring threads
        ly = u / 4;
        const int c = u % 4;
        lz = c < 2 ? c - 2 : kDerTZ + c - 2;
    }
    r.halo = tid < kSwHalo;
    r.hy = y0 + ly;
    r.hz = z0 + lz;
    r.hv = r.halo && r.hy >= 0 && r.hy < n && r.hz >= 0 && r.hz < n;
    r.r1 = r.halo && ly >= -1 && ly <= kDerTY && lz >= -1 && lz <= kDerTZ;
    r.hcell2 = (ly + 2) * kSwRZ + lz + 2;
    r.hcell1 = (ly + 1) * kDerRZ + lz + 1;
    r.hp = r.hv ? (int64_t)r.hy * n + r.hz : 0;
}

template <bool HARM>
__global__ __launch_bounds__(kDerThreads) void k_un_gs_sweep_t(const double* __restrict__ u_in,
                                                              double* __restrict__ u_mid, double* __restrict__ u_out,
                                                              const double* __restrict__ q,
                                                              const double* __restrict__ D,
                                                              const double* __restrict__ w, int N, Stencil<double> s,
                                                              int c1, int chunk, int cover) {
    // the planes y = N and z = N: boundary values are kept
    if (der_edge_block(N, chunk, [&](const DerEdge& e) {
            const double v = u_in[e.i];
            u_mid[e.i] = v;
            u_out[e.i] = v;
        }))
        return;
    __shared__ double sU[kSwSlots][kSwCells], sD[kSwSlots][kSwCells], sM[2][kDerCells];
    DerTile t;
    der_tile(N, chunk, cover, t);
    const int n = t.n;
    const int c2 = 1 - c1;
    SwRing rg;
    sw_ring(t, rg);
    const int cell2 = rg.cell2, hy = rg.hy, hz = rg.hz, hcell2 = rg.hcell2, hcell1 = rg.hcell1;
    const bool halo = rg.halo, hv = rg.hv, r1 = rg.r1;
    const int64_t hp = rg.hp;
    struct UD {
        double u, D;
    };
    struct QW {
        double q, w;
    };
    const DerSpan sp(t, n, 2);
    const auto rU = sp.rsrc(u_in), rD = sp.rsrc(D), rQ = sp.rsrc(q), rW = sp.rsrc(w);
    const int xs = t.x0 - 1, xlast = t.x1;   // stage 1 runs on planes [xs, xlast]
    auto load_ud = [&](int x, bool valid, int64_t p) -> UD {
        const int o = valid ? (int)(p * 8) : kOob, so = sp.off(x);
        return UD{buf_load_s(rU, o, so), buf_load_s(rD, o, so)};
    };
    auto load_qw = [&](int x, bool valid, int64_t p) -> QW {
        const int o = (valid && x >= xs && x <= xlast) ? (int)(p * 8) : kOob, so = sp.off(x);
        return QW{buf_load_s(rQ, o, so), buf_load_s(rW, o, so)};
    };
    const bool hq = r1 && hv;
    auto slot = [](int x) { return (x + 2 * kSwSlots) % kSwSlots; };   // x >= -3
    auto publish = [&](int x, const UD& own, const UD& ring) {
        const int k = slot(x);
        sU[k][cell2] = own.u; sD[k][cell2] = own.D;
        if (halo) { sU[k][hcell2] = ring.u; sD[k][hcell2] = ring.D; }
    };
    auto fc = [&](double Da, double Db) { return face<HARM>(Da, Db, s); };
    // stage 1 at one vertex (cell c of the ring-2 arrays) of plane x
    auto stage1 = [&](int x, int y, int z, int c, const QW& f) {
        const int k = slot(x), km = slot(x - 1), kp = slot(x + 1);
        const double u = sU[k][c];
        if (!is_interior(N, x, y, z) || ((x + y + z) & 1) != c1) return u;
        const double Dc = sD[k][c];
        const int e[4] = {c + kSwRZ, c - kSwRZ, c + 1, c - 1};
        double num = f.q + fc(Dc, sD[kp][c]) * sU[kp][c] + fc(Dc, sD[km][c]) * sU[km][c];
        for (int j = 0; j < 4; j++) num += fc(Dc, sD[k][e[j]]) * sU[k][e[j]];
        return num * f.w;
    };
    const bool yz = t.y > 0 && t.y < N && t.z > 0 && t.z < N;
    double m2 = 0.0, m1 = 0.0;   // own u_mid at planes x - 2, x - 1
    UD P, PH;                    // plane x + 1 (own, ring), published at step x
    // step x: qm, qc hold q, w of planes x - 1, x; qn receives plane x + 1
    auto step = [&](int x, QW& qm, QW& qc, QW& qn, QW& hqc, QW& hqn) {
        publish(x + 1, P, PH);
        lds_barrier();
        P = load_ud(x + 2, t.inb, t.p);
        PH = load_ud(x + 2, hv, hp);
        qn = load_qw(x + 1, t.inb, t.p);
        hqn = load_qw(x + 1, hq, hp);
        const double m0 = stage1(x, t.y, t.z, cell2, qc);
        sM[x & 1][t.cell] = m0;
        if (r1) sM[x & 1][hcell1] = stage1(x, hy, hz, hcell2, hqc);
        if (t.own && x >= t.x0 && x < t.x1) u_mid[x * t.sx + t.p] = m0;
        // stage 2 on plane x - 1 (its u_mid from the previous step's slot)
        const int xm = x - 1;
        if (t.own && xm >= t.x0 && xm < t.x1) {
            double v = m1;
            if (yz && xm > 0 && xm < N && ((xm + t.y + t.z) & 1) == c2) {
                const int k = slot(xm), bm = xm & 1;
                const double Dc = sD[k][cell2];
                const int e[4] = {t.cell + kDerRZ, t.cell - kDerRZ, t.cell + 1, t.cell - 1};
                const int e2[4] = {cell2 + kSwRZ, cell2 - kSwRZ, cell2 + 1, cell2 - 1};
                double num = qm.q + fc(Dc, sD[slot(x)][cell2]) * m0 + fc(Dc, sD[slot(xm - 1)][cell2]) * m2;
                for (int j = 0; j < 4; j++) num += fc(Dc, sD[k][e2[j]]) * sM[bm][e[j]];
                v = num * qm.w;
            }
            u_out[xm * t.sx + t.p] = v;
        }
        m2 = m1;
        m1 = m0;
    };
    publish(xs - 1, load_ud(xs - 1, t.inb, t.p), load_ud(xs - 1, hv, hp));
    publish(xs, load_ud(xs, t.inb, t.p), load_ud(xs, hv, hp));
    P = load_ud(xs + 1, t.inb, t.p);
    PH = load_ud(xs + 1, hv, hp);
    QW Q0{0.0, 0.0}, Q1 = load_qw(xs, t.inb, t.p), Q2;
    QW G0{0.0, 0.0}, G1 = load_qw(xs, hq, hp), G2;
    for (int x = xs; x <= xlast; x += 3) {
        step(x, Q0, Q1, Q2, G1, G2);
        step(x + 1, Q1, Q2, Q0, G2, G0);
        step(x + 2, Q2, Q0, Q1, G0, G1);
    }
}

// The planes y = N and z = N in the reverse of a whole sweep: Dbar of the
// boundary vertex, by its one face to an interior neighbour j, first with
// V^A_j (the later half-sweep's), then with V^B_j, which needs ubar' of j
// after the first reverse: ubar_j + sum_k c_jk V^A_k over j's neighbours.
template <bool HARM>
__device__ __forceinline__ void un_sweep_rev_edge(const DerEdge& e, const double* __restrict__ ubar,
                                                  const double* __restrict__ uA, const double* __restrict__ uB,
                                                  const double* __restrict__ D, const double* __restrict__ w, int N,
                                                  const Stencil<double>& s, int c1, double* __restrict__ Dbar) {
    const int n = N + 1;
    const int64_t nn = (int64_t)n * n;
    double dA = 0.0, dB = 0.0;
    if (e.jin) {
        const int jx = (int)(e.j / nn), jy = (int)((e.j / n) % n), jz = (int)(e.j % n);
        const bool jc1 = ((jx + jy + jz) & 1) == c1;
        const double Dv = D[e.i], Dj = D[e.j];
        double dd;
        if (HARM) {
            const double t = Dv + Dj;
            dd = Dj * Dj / (t * t) * s.two_inv_h2;
        } else {
            dd = s.half_inv_h2;
        }
        const double VAj = jc1 ? ubar[e.j] * w[e.j] : 0.0;
        dA += (0.0 - VAj) * (uA[e.i] - uA[e.j]) * dd;
        double VBj = 0.0;
        if (!jc1) {
            const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
            double g = 0.0;
            for (int m = 0; m < 6; m++) {
                const int kx = jx + d[m][0], ky = jy + d[m][1], kz = jz + d[m][2];
                const int64_t k = ((int64_t)kx * n + ky) * n + kz;
                const double VAk = (is_interior(N, kx, ky, kz) && ((kx + ky + kz) & 1) == c1) ? ubar[k] * w[k] : 0.0;
                g += face<HARM>(Dj, D[k], s) * VAk;
            }
            VBj = (ubar[e.j] + g) * w[e.j];
        }
        dB += (0.0 - VBj) * (uB[e.i] - uB[e.j]) * dd;
    }
    Dbar[e.i] = (Dbar[e.i] - dA) - dB;
}

// The reverse of a whole recorded sweep in one pass (levels the column
// tiles cover): the half-sweep of colour c1 (which ran last; its state uA)
// reversed, then that of c2 = 1 - c1 (state uB), the two reverses in
// sequence.  Per vertex i (V^A = ubar w on c1's interior, V^B = ubar' w
// on c2's, ubar' = ubar + sum_j c_ij V^A_j on c2's interior, 0 elsewhere):
//   c1's interior: qbar += V^A, mubar -= V^A uA, ubar_out = sum_j c_ij V^B_j
//   c2's interior: qbar += V^B, mubar -= V^B uB, ubar_out = 0
//   every vertex:  Dbar -= the face terms of V^A with uA, then of V^B with uB.
// 96 instead of 2 x 88 bytes per vertex.  The column tiles march along x in
// two stages: at step x, stage 1 forms V^B on plane x over the tile plus a
// ring of one, from X (V^A on c1's interior, ubar on c2's, 0 elsewhere) and
// D in LDS over a ring of two for four planes (x - 2 .. x + 1; plane x + 1
// is published at step x); stage 2 forms the outputs on plane x - 1 from V^B,
// uA and uB of that plane in LDS over a ring of one and the own column's
// values of planes x - 2 and x in registers.  One barrier per step orders
// all LDS traffic.  Neighbours in the order +x, -x, +y, -y, +z, -z.
template <bool HARM>
__global__ __launch_bounds__(kDerThreads) void k_un_sweep_rev_t(const double* __restrict__ ubar_in,
                                                               double* __restrict__ ubar_out,
                                                               const double* __restrict__ uA,
                                                               const double* __restrict__ uB,
                                                               const double* __restrict__ D,
                                                               const double* __restrict__ w, int N, Stencil<double> s,
                                                               int c1, double* __restrict__ qbar,
                                                               double* __restrict__ mubar, double* __restrict__ Dbar,
                                                               int chunk, int cover) {
    if (der_edge_block(N, chunk, [&](const DerEdge& e) {
            un_sweep_rev_edge<HARM>(e, ubar_in, uA, uB, D, w, N, s, c1, Dbar);
        }))
        return;
    __shared__ double sX[4][kSwCells], sD[4][kSwCells], sVB[2][kDerCells], sUA[2][kDerCells], sUB[2][kDerCells];
    DerTile t;
    der_tile(N, chunk, cover, t);
    const int n = t.n;
    const int c2 = 1 - c1;
    SwRing rg;
    sw_ring(t, rg);
    struct L {
        double b, w, D;   // ubar, w, D
    };
    struct U {
        double a, b;      // uA, uB
    };
    struct A {
        double q, m, d;   // qbar, mubar, Dbar (own column)
    };
    const DerSpan sp(t, n, 2);
    const auto rB = sp.rsrc(ubar_in), rW = sp.rsrc(w), rD = sp.rsrc(D), rA = sp.rsrc(uA), rBb = sp.rsrc(uB);
    const auto rQ = sp.rsrc(qbar), rM = sp.rsrc(mubar), rDb = sp.rsrc(Dbar);
    const int xs = t.x0 - 1, xlast = t.x1;   // stage 1 runs on planes [xs, xlast]
    auto load_l = [&](int x, bool valid, int64_t p) -> L {
        const int o = valid ? (int)(p * 8) : kOob, so = sp.off(x);
        return L{buf_load_s(rB, o, so), buf_load_s(rW, o, so), buf_load_s(rD, o, so)};
    };
    auto load_u = [&](int x, bool valid, int64_t p) -> U {
        const int o = valid ? (int)(p * 8) : kOob, so = sp.off(x);
        return U{buf_load_s(rA, o, so), buf_load_s(rBb, o, so)};
    };
    auto load_a = [&](int x) -> A {
        const int o = (t.own && x >= t.x0 && x < t.x1) ? (int)(t.p * 8) : kOob, so = sp.off(x);
        return A{buf_load_s(rQ, o, so), buf_load_s(rM, o, so), buf_load_s(rDb, o, so)};
    };
    const bool hu = rg.r1 && rg.hv;
    auto slot = [](int x) { return (x + 8) & 3; };   // x >= -3
    auto interior_c = [&](int x, int y, int z, int c) { return is_interior(N, x, y, z) && ((x + y + z) & 1) == c; };
    // X of a vertex from its own fields
    auto xof = [&](const L& f, int x, int y, int z) {
        return interior_c(x, y, z, c1) ? f.b * f.w : (interior_c(x, y, z, c2) ? f.b : 0.0);
    };
    auto vaof = [&](const L& f, int x, int y, int z) { return interior_c(x, y, z, c1) ? f.b * f.w : 0.0; };
    auto fc = [&](double Da, double Db) { return face<HARM>(Da, Db, s); };
    auto dda = [&](double Da, double Db) {
        if (HARM) {
            const double u = Da + Db;
            return Db * Db / (u * u) * s.two_inv_h2;
        }
        return s.half_inv_h2;
    };
    // stage 1 at one vertex (cell c of the ring-2 arrays) of plane x: V^B
    auto stage1 = [&](int x, int y, int z, int c, double wc) {
        if (!interior_c(x, y, z, c2)) return 0.0;
        const int k = slot(x), km = slot(x - 1), kp = slot(x + 1);
        const double Dc = sD[k][c];
        double g = 0.0;
        g += fc(Dc, sD[kp][c]) * sX[kp][c];
        g += fc(Dc, sD[km][c]) * sX[km][c];
#pragma unroll 1
        for (int j = 0; j < 4; j++) {
            const int e = c + ((j & 1) ? -1 : 1) * (j < 2 ? kSwRZ : 1);
            g += fc(Dc, sD[k][e]) * sX[k][e];
        }
        return (sX[k][c] + g) * wc;
    };
    const bool yz = t.y > 0 && t.y < N && t.z > 0 && t.z < N;
    double m2 = 0.0, m1 = 0.0;   // own V^B at planes x - 2, x - 1
    // step x: l2 .. lp hold planes x - 2 .. x + 1 (l2 receives x + 2), h* the
    // same for the ring cell; u3 .. uc hold uA, uB of x - 3 (receives x + 1)
    // .. x; g1 holds the ring cell's uA, uB of x - 1, g0 receives x.  The
    // accumulators of plane x - 1 are loaded in the same step (stage 1 runs
    // while they arrive; a register ring for them would spill).
    auto step = [&](int x, L& l2, L& lm, L& lc, L& lp, L& h2, L& hm, L& hc, L& hp, U& u3, U& u2, U& um, U& uc,
                    U& g1, U& g0) {
        const int kp = slot(x + 1);
        sX[kp][rg.cell2] = xof(lp, x + 1, t.y, t.z);
        sD[kp][rg.cell2] = lp.D;
        lp.b = vaof(lp, x + 1, t.y, t.z);   // from here on the field holds V^A
        if (rg.halo) {
            sX[kp][rg.hcell2] = xof(hp, x + 1, rg.hy, rg.hz);
            sD[kp][rg.hcell2] = hp.D;
        }
        const int bm = (x - 1) & 1;
        sUA[bm][t.cell] = um.a; sUB[bm][t.cell] = um.b;
        if (rg.r1) { sUA[bm][rg.hcell1] = g1.a; sUB[bm][rg.hcell1] = g1.b; }
        lds_barrier();
        // plane x - 2's own values (its registers take plane x + 2 now)
        const double D2 = l2.D, VA2 = l2.b;
        l2 = load_l(x + 2, t.inb, t.p);
        h2 = load_l(x + 2, rg.hv, rg.hp);
        u3 = load_u(x + 1, t.inb, t.p);
        g0 = load_u(x, hu, rg.hp);
        const A a1 = load_a(x - 1);
        const double m0 = stage1(x, t.y, t.z, rg.cell2, lc.w);
        sVB[x & 1][t.cell] = m0;
        if (rg.r1) sVB[x & 1][rg.hcell1] = stage1(x, rg.hy, rg.hz, rg.hcell2, hc.w);
        // stage 2 on plane q = x - 1
        const int q = x - 1;
        if (t.own && q >= t.x0 && q < t.x1) {
            const bool intq = yz && q > 0 && q < N;
            const bool own2 = ((q + t.y + t.z) & 1) == c2;
            const double Dc = lm.D, VAc = lm.b, VBc = m1;
            const double uAc = um.a, uBc = um.b;
            double dA = 0.0, dB = 0.0, gB = 0.0;
            auto nb = [&](double Dj, double VAj, double VBj, double uAj, double uBj) {
                const double dd = dda(Dc, Dj);
                dA += (VAc - VAj) * (uAc - uAj) * dd;
                dB += (VBc - VBj) * (uBc - uBj) * dd;
                gB += fc(Dc, Dj) * VBj;
            };
            if (q < N) nb(lc.D, lc.b, m0, uc.a, uc.b);
            if (q > 0) nb(D2, VA2, m2, u2.a, u2.b);
            const int kq = slot(q);
            // in-plane neighbours one at a time (few LDS values in flight)
#pragma unroll 1
            for (int j = 0; j < 4; j++) {
                const int sgn = (j & 1) ? -1 : 1;
                const bool ok = j < 2 ? (j == 0 ? t.y < N : t.y > 0) : (j == 2 ? t.z < N : t.z > 0);
                const int e = t.cell + sgn * (j < 2 ? kDerRZ : 1), e2 = rg.cell2 + sgn * (j < 2 ? kSwRZ : 1);
                if (ok) nb(sD[kq][e2], own2 ? sX[kq][e2] : 0.0, sVB[bm][e], sUA[bm][e], sUB[bm][e]);
            }
            const int64_t i = q * t.sx + t.p;
            Dbar[i] = (a1.d - dA) - dB;
            if (intq) {
                if (!own2) {
                    qbar[i] = a1.q + VAc;
                    mubar[i] = a1.m - VAc * uAc;
                    ubar_out[i] = 0.0 + gB;
                } else {
                    qbar[i] = a1.q + VBc;
                    mubar[i] = a1.m - VBc * uBc;
                    ubar_out[i] = 0.0;
                }
            }
        }
        m2 = m1;
        m1 = m0;
    };
    L L0{0.0, 0.0, 0.0}, L1 = load_l(xs - 1, t.inb, t.p), L2 = load_l(xs, t.inb, t.p), L3 = load_l(xs + 1, t.inb, t.p);
    L H0{0.0, 0.0, 0.0}, H1 = load_l(xs - 1, rg.hv, rg.hp), H2 = load_l(xs, rg.hv, rg.hp),
        H3 = load_l(xs + 1, rg.hv, rg.hp);
    {
        const int k0 = slot(xs - 1), k1 = slot(xs);
        sX[k0][rg.cell2] = xof(L1, xs - 1, t.y, t.z); sD[k0][rg.cell2] = L1.D;
        sX[k1][rg.cell2] = xof(L2, xs, t.y, t.z); sD[k1][rg.cell2] = L2.D;
        L1.b = vaof(L1, xs - 1, t.y, t.z);
        L2.b = vaof(L2, xs, t.y, t.z);
        if (rg.halo) {
            sX[k0][rg.hcell2] = xof(H1, xs - 1, rg.hy, rg.hz); sD[k0][rg.hcell2] = H1.D;
            sX[k1][rg.hcell2] = xof(H2, xs, rg.hy, rg.hz); sD[k1][rg.hcell2] = H2.D;
        }
    }
    U U0{0.0, 0.0}, U1{0.0, 0.0}, U2{0.0, 0.0}, U3 = load_u(xs, t.inb, t.p);
    U G0{0.0, 0.0}, G1{0.0, 0.0};
    for (int x = xs; x <= xlast; x += 4) {
        step(x, L0, L1, L2, L3, H0, H1, H2, H3, U0, U1, U2, U3, G1, G0);
        step(x + 1, L1, L2, L3, L0, H1, H2, H3, H0, U1, U2, U3, U0, G0, G1);
        step(x + 2, L2, L3, L0, L1, H2, H3, H0, H1, U2, U3, U0, U1, G1, G0);
        step(x + 3, L3, L0, L1, L2, H3, H0, H1, H2, U3, U0, U1, U2, G0, G1);
    }
}

// Defect (or coarsest-solve) reverse with cotangent rbar = scale * rb on
// interior vertices (0 elsewhere; rb is read there only): qbar += rbar,
// ubar -= A rbar (unless ubar is null), mubar -= rbar u on interior vertices,
// and Dbar -= the face terms on every vertex.  Only the own vertex's ubar is
// read and written.
template <bool HARM>
__global__ __launch_bounds__(kDerThreads) void k_un_defect_t(double* __restrict__ ubar, const double* __restrict__ rb,
                                                            double scale, const double* __restrict__ u,
                                                            const double* __restrict__ D,
                                                            const double* __restrict__ mu, int N, Stencil<double> s,
                                                            double* __restrict__ qbar, double* __restrict__ Dbar,
                                                            double* __restrict__ mubar, int chunk, int cover) {
    if (der_edge_block(N, chunk, [&](const DerEdge& e) { un_defect_edge<HARM>(e, rb, scale, u, D, s, Dbar); }))
        return;
    __shared__ double sR[2][kDerCells], sU[2][kDerCells], sD[2][kDerCells];
    DerTile t;
    der_tile(N, chunk, cover, t);
    const int n = t.n;
    struct H {
        double r, u, D;   // rb (scaled where used), u, D
    };
    struct Vp : H {
        double m, qb, mb, Db, ub;   // own column only
    };
    const DerSpan sp(t, n);
    const auto rR = sp.rsrc(rb), rU = sp.rsrc(u), rD = sp.rsrc(D), rM = sp.rsrc(mu);
    const auto rQ = sp.rsrc(qbar), rMb = sp.rsrc(mubar), rDb = sp.rsrc(Dbar), rUb = sp.rsrc(ubar);
    // rb is read on interior vertices only
    auto load_h = [&](int x, bool valid, int y, int z, int64_t p) -> H {
        const int o = valid ? (int)(p * 8) : kOob, so = sp.off(x);
        const int orb = (valid && is_interior(N, x, y, z)) ? o : kOob;
        return H{buf_load_s(rR, orb, so), buf_load_s(rU, o, so), buf_load_s(rD, o, so)};
    };
    auto load_v = [&](int x) -> Vp {
        Vp v;
        static_cast<H&>(v) = load_h(x, t.inb, t.y, t.z, t.p);
        const int oo = (t.own && x < t.x1) ? (int)(t.p * 8) : kOob, so = sp.off(x);
        v.m = buf_load_s(rM, oo, so);
        v.qb = buf_load_s(rQ, oo, so);
        v.mb = buf_load_s(rMb, oo, so);
        v.Db = buf_load_s(rDb, oo, so);
        v.ub = buf_load_s(rUb, oo, so);
        return v;
    };
    auto dda = [&](double Da, double Db) {
        if (HARM) {
            const double w = Da + Db;
            return Db * Db / (w * w) * s.two_inv_h2;
        }
        return s.half_inv_h2;
    };
    const bool halo = threadIdx.x < kDerHalo;
    const bool yz = t.y > 0 && t.y < N && t.z > 0 && t.z < N;
    auto step = [&](int x, Vp& Rm, Vp& Rc, Vp& Rp, Vp& Rl, H& Hc, H& Hl) {
        const int b = x & 1;
        sR[b][t.cell] = scale * Rc.r; sU[b][t.cell] = Rc.u; sD[b][t.cell] = Rc.D;
        if (halo) { sR[b][t.hcell] = scale * Hc.r; sU[b][t.hcell] = Hc.u; sD[b][t.hcell] = Hc.D; }
        lds_barrier();
        Rl = load_v(x + 3);
        Hl = load_h(x + 2, t.hv, t.hy, t.hz, t.hp);
        if (t.own && x < t.x1) {
            const int64_t i = x * t.sx + t.p;
            const bool in = yz && x > 0 && x < N;
            const double rc = scale * Rc.r;
            double dacc = 0.0, Ar = in ? Rc.m * rc : 0.0;
            auto nb = [&](double Dj, double uj, double rj) {
                dacc += (rc - rj) * (Rc.u - uj) * dda(Rc.D, Dj);
                Ar += face<HARM>(Rc.D, Dj, s) * (rc - rj);
            };
            if (x < N) nb(Rp.D, Rp.u, scale * Rp.r);
            if (x > 0) nb(Rm.D, Rm.u, scale * Rm.r);
            auto cell = [&](int e) { nb(sD[b][e], sU[b][e], sR[b][e]); };
            if (t.y < N) cell(t.cell + kDerRZ);
            if (t.y > 0) cell(t.cell - kDerRZ);
            if (t.z < N) cell(t.cell + 1);
            if (t.z > 0) cell(t.cell - 1);
            Dbar[i] = Rc.Db - dacc;
            if (in) {
                qbar[i] = Rc.qb + rc;
                mubar[i] = Rc.mb - rc * Rc.u;
                if (ubar) ubar[i] = Rc.ub - Ar;
            }
        }
    };
    const int x0 = t.x0;
    Vp R0 = load_v(x0 - 1), R1 = load_v(x0), R2 = load_v(x0 + 1), R3 = load_v(x0 + 2), R4;
    H H0 = load_h(x0, t.hv, t.hy, t.hz, t.hp), H1 = load_h(x0 + 1, t.hv, t.hy, t.hz, t.hp), H2, H3, H4;
    for (int x = x0; x < t.x1; x += kDerRing) {
        step(x, R0, R1, R2, R4, H0, H2);
        step(x + 1, R1, R2, R3, R0, H1, H3);
        step(x + 2, R2, R3, R4, R1, H2, H4);
        step(x + 3, R3, R4, R0, R2, H3, H0);
        step(x + 4, R4, R0, R1, R3, H4, H1);
    }
}

// u = u_pre + I ec (the trilinear prolongation of the coarse correction
// added on interior vertices), u = u_pre on boundary ones: the recorded
// cycle's post-smoothing input, formed out of place from the pre-smoothed
// state; with u_pre null, from zero (the reverse pass's rbar = I qcbar).
__global__ void k_un_prolong_to(const double* __restrict__ ec, const double* __restrict__ u_pre,
                                double* __restrict__ u, int Nf) {
    const int nf = Nf + 1, nc = Nf / 2 + 1;
    const int64_t nv = (int64_t)nf * nf * nf;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(v % nf), y = (int)((v / nf) % nf), x = (int)(v / ((int64_t)nf * nf));
        double r = u_pre ? u_pre[v] : 0.0;
        if (is_interior(Nf, x, y, z)) {
            const int x0 = x >> 1, y0 = y >> 1, z0 = z >> 1;
            const int x1 = x0 + (x & 1), y1 = y0 + (y & 1), z1 = z0 + (z & 1);
            // the eight corners repeat one where a coordinate is even: 8 x the trilinear value
            const double s = ec[vidx(nc, x0, y0, z0)] + ec[vidx(nc, x0, y0, z1)] + ec[vidx(nc, x0, y1, z0)] +
                             ec[vidx(nc, x0, y1, z1)] + ec[vidx(nc, x1, y0, z0)] + ec[vidx(nc, x1, y0, z1)] +
                             ec[vidx(nc, x1, y1, z0)] + ec[vidx(nc, x1, y1, z1)];
            r += s * 0.125;
        }
        u[v] = r;
    }
}

// qc = 8 R r on coarse interior vertices (full weighting, then times 8: the
// transpose of the prolongation I = 8 R^T), 0 on coarse boundary ones.
__global__ void k_un_restrict8(const double* __restrict__ r, double* __restrict__ qc, int Nf) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t nv = (int64_t)nc * nc * nc;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int Z = (int)(v % nc), Y = (int)((v / nc) % nc), X = (int)(v / ((int64_t)nc * nc));
        if (!is_interior(Nc, X, Y, Z)) {
            qc[v] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int a = -1; a <= 1; a++)
            for (int b = -1; b <= 1; b++) {
                const double wab = (double)((2 - abs(a)) * (2 - abs(b)));
                const double* row = r + vidx(nf, 2 * X + a, 2 * Y + b, 2 * Z);
                s += wab * (row[-1] + 2.0 * row[0] + row[1]);
            }
        qc[v] = (s * (1.0 / 64.0)) * 8.0;
    }
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
