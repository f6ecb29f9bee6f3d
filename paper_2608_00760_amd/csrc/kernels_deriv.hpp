// kernels_deriv.hpp -- derivatives with respect to the coefficients on the
// finest level of cubic plans (adjoint-state derivatives of the discrete
// solution): the push-forward's right-hand side q' - A' rho and the
// pull-back's coefficient gradients.
//
// A workgroup owns a tile of kDerTY x kDerTZ vertex columns (y, z), one
// thread each, and marches them along x over a chunk of planes.  The tiles
// cover y, z < cover.  On large levels cover = N: the boundary planes
// y = N and z = N (a single row or column beyond whole tiles when N is a
// multiple of the tile) are left to extra workgroups of the same launch,
// one vertex per thread (grid rows past the chunks), so no workgroup holds
// a nearly empty tile.  Their outputs are disjoint from the tiles' and they
// read nothing the tiles write.  On small levels, where idle lanes cost
// little, cover = N + 1 and the tiles take every vertex.  Each
// thread keeps its own column's values at x - 1, x and x + 1 in registers
// (and the planes after them in flight).  The in-plane neighbours come from
// an LDS copy of plane x over the tile plus a ring of one vertex: the
// tile's threads publish their own values, and the first kDerHalo threads
// load the ring (into registers, two steps ahead).  The copy is double
// buffered by plane parity, so one barrier per plane orders every write
// before the reads of that plane and after the reads of the plane two
// steps back.  Every field is then read from memory about once (the ring
// adds 2 / kDerTY + 2 / kDerTZ, mostly cache hits).  Blocks are remapped so
// that each XCD runs a contiguous range of (tile, chunk) indices.
#pragma once
#include "kernels_stream.hpp"

namespace dmgs {

constexpr int kDerTY = 16, kDerTZ = 64, kDerThreads = kDerTY * kDerTZ;
constexpr int kDerRY = kDerTY + 2, kDerRZ = kDerTZ + 2, kDerCells = kDerRY * kDerRZ;
constexpr int kDerHalo = 2 * kDerRZ + 2 * kDerTY;   // ring cells

struct DerTile {
    int n, x0, x1;       // vertices per axis; chunk of planes [x0, x1)
    int y, z, cell;      // this thread's column and its LDS cell
    bool inb;            // the column lies inside the grid (its values are loaded)
    bool own;            // ... and below y = N, z = N (its outputs are formed here)
    int hy, hz, hcell;   // this thread's ring cell (tid < kDerHalo)
    bool hv;             // ... inside the grid
    int64_t sx, p, hp;   // plane stride; in-plane offsets of the column and the ring cell
};

// Chunks of planes along x (grid rows of tiles); rows past them take the
// boundary planes.
__device__ __forceinline__ int der_chunks(int N, int chunk) { return (N + chunk) / chunk; }

__device__ __forceinline__ void der_tile(int N, int chunk, int cover, DerTile& t) {
    const int nb = (int)gridDim.x * der_chunks(N, chunk);
    const int L = xcd_remap((int)(blockIdx.y * gridDim.x + blockIdx.x), nb);
    const int tile = L % (int)gridDim.x, ch = L / (int)gridDim.x;
    t.n = N + 1;
    t.sx = (int64_t)t.n * t.n;
    const int tiles_z = (cover + kDerTZ - 1) / kDerTZ;
    const int y0 = (tile / tiles_z) * kDerTY, z0 = (tile % tiles_z) * kDerTZ;
    t.x0 = ch * chunk;
    t.x1 = min(t.n, t.x0 + chunk);
    const int tid = (int)threadIdx.x, ty = tid / kDerTZ, tz = tid % kDerTZ;
    t.y = y0 + ty;
    t.z = z0 + tz;
    // with cover = N, a column at y = N or z = N inside the tile (N not a
    // multiple of the tile) is loaded for its neighbours; its outputs are the
    // companion kernel's
    t.inb = t.y < t.n && t.z < t.n;
    t.own = t.y < cover && t.z < cover;
    t.cell = (ty + 1) * kDerRZ + tz + 1;
    t.p = t.inb ? (int64_t)t.y * t.n + t.z : 0;
    // ring: the row above, the row below, then the left and right columns
    int ly = -1, lz = -1;
    if (tid < kDerRZ) {
        ly = -1; lz = tid - 1;
    } else if (tid < 2 * kDerRZ) {
        ly = kDerTY; lz = tid - kDerRZ - 1;
    } else if (tid < 2 * kDerRZ + kDerTY) {
        ly = tid - 2 * kDerRZ; lz = -1;
    } else {
        ly = tid - 2 * kDerRZ - kDerTY; lz = kDerTZ;
    }
    t.hy = y0 + ly;
    t.hz = z0 + lz;
    t.hv = tid < kDerHalo && t.hy >= 0 && t.hy < t.n && t.hz >= 0 && t.hz < t.n;
    t.hcell = (ly + 1) * kDerRZ + lz + 1;
    t.hp = t.hv ? (int64_t)t.hy * t.n + t.hz : 0;
}

// Vertices the tiles leave out: the boundary planes y = N (index t < n^2:
// (x, N, z)) and z = N (t >= n^2: (x, y, N), y < N), every x.  Each has at
// most one interior neighbour j: (x, N - 1, z), or (x, y, N - 1).
struct DerEdge {
    int64_t i, j;   // the vertex and its neighbour
    bool jin;       // the neighbour is interior
};

__device__ __forceinline__ void der_edge_at(int N, int64_t t, DerEdge& e) {
    const int n = N + 1;
    const int64_t nn = (int64_t)n * n;
    int x, y, z;
    if (t < nn) {
        x = (int)(t / n); y = N; z = (int)(t % n);
        e.jin = x > 0 && x < N && z > 0 && z < N;
        e.j = ((int64_t)x * n + (N - 1)) * n + z;
    } else {
        const int64_t u = t - nn;
        x = (int)(u / N); y = (int)(u % N); z = N;
        e.jin = x > 0 && x < N && y > 0 && y < N;
        e.j = ((int64_t)x * n + y) * n + (N - 1);
    }
    e.i = ((int64_t)x * n + y) * n + z;
}

// Vertices of the boundary planes y = N and z = N (all 2 n^2 - n of them).
__host__ __device__ inline int64_t der_edge_count(int N) { return (int64_t)(N + 1) * (2 * N + 1); }

// In a workgroup of the grid rows past the chunks, runs f(e) for this
// thread's share of the boundary-plane vertices and returns true (the whole
// workgroup then leaves before the march and its barriers).
template <class F>
__device__ __forceinline__ bool der_edge_block(int N, int chunk, F&& f) {
    const int nch = der_chunks(N, chunk);
    if ((int)blockIdx.y < nch) return false;
    const int64_t cnt = der_edge_count(N);
    const int64_t stride = (int64_t)(gridDim.y - nch) * gridDim.x * blockDim.x;
    for (int64_t t = ((int64_t)(blockIdx.y - nch) * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; t < cnt;
         t += stride) {
        DerEdge e;
        der_edge_at(N, t, e);
        f(e);
    }
    return true;
}

// d D_f along the tangent: D_f = (D_a + D_b)/2 or 2 D_a D_b / (D_a + D_b),
// with dD = D dlogD at both ends
template <bool HARM>
__device__ __forceinline__ double dface(double Da, double dDa, double Db, double dDb) {
    if (HARM) {
        const double sum = Da + Db;
        return 2.0 * (Db * Db * dDa + Da * Da * dDb) / (sum * sum);
    }
    return 0.5 * (dDa + dDb);
}

// The march: planes are loaded two steps before their first use into a
// named register ring of five planes (own column) and five ring cells
// (halo), unrolled by five so that no in-flight register is ever copied.
// A chunk runs a multiple of five steps; steps past its last plane load
// nothing, store nothing and keep the barriers uniform.
constexpr int kDerRing = 5;

// The planes a block reads, [x0 - m, x1 + m - 1] within the grid (m = 1, or
// 2 for the two-stage sweep), through one buffer resource per field; a plane
// is selected by a wave-uniform offset, and planes outside the span, null
// fields and lanes without a column read 0.  The host keeps (chunk + 5)
// planes below 2^31 bytes.
struct DerSpan {
    int xb, xe;        // planes [xb, xe)
    int pb;            // bytes per plane
    int64_t base;      // byte offset of plane xb
    __device__ DerSpan(const DerTile& t, int n, int m = 1)
        : xb(max(0, t.x0 - m)), xe(min(n, t.x1 + m)), pb((int)(t.sx * 8)), base((int64_t)xb * t.sx * 8) {}
    __device__ __amdgpu_buffer_rsrc_t rsrc(const double* f) const {
        const char* b = reinterpret_cast<const char*>(f) + (f ? base : 0);
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), 0, f ? (xe - xb) * pb : 0, 0x00020000);
    }
    __device__ int off(int x) const { return (x >= xb && x < xe) ? (x - xb) * pb : kOob; }
};

// rhs = dq - (dA) rho on interior vertices (0 on the boundary), where
// (dA rho)_i = sum_j dD_f,ij/h^2 (rho_i - rho_j) + mua_i dlogmua_i rho_i and
// dD_f is the derivative of the face mean along dlogD.  Null tangents are 0.
// Neighbours in the order +x, -x, +y, -y, +z, -z.
template <bool HARM>
__global__ __launch_bounds__(kDerThreads) void k_tangent_rhs_col(const double* __restrict__ rho,
                                                                const double* __restrict__ dq,
                                                                const double* __restrict__ dlogD,
                                                                const double* __restrict__ dlogmu,
                                                                const double* __restrict__ D,
                                                                const double* __restrict__ mu, int N, double inv_h2,
                                                                double* __restrict__ rhs, int chunk, int cover) {
    // the planes y = N and z = N: 0 (boundary)
    if (der_edge_block(N, chunk, [&](const DerEdge& e) { rhs[e.i] = 0.0; })) return;
    __shared__ double sR[2][kDerCells], sD[2][kDerCells], sT[2][kDerCells];
    DerTile t;
    der_tile(N, chunk, cover, t);
    const int n = t.n;
    struct H {
        double r, D, g;   // rho, D, dlogD (products formed when used, so loads stay in flight)
    };
    struct V : H {
        double m, gm, q;  // own column only: mua, dlogmua, dq
    };
    const DerSpan sp(t, n);
    const auto rR = sp.rsrc(rho), rD = sp.rsrc(D), rG = sp.rsrc(dlogD);
    const auto rM = sp.rsrc(dlogmu ? mu : nullptr), rGm = sp.rsrc(dlogmu), rQ = sp.rsrc(dq);
    auto load_h = [&](int x, bool valid, int64_t p) -> H {
        const int o = valid ? (int)(p * 8) : kOob, so = sp.off(x);
        return H{buf_load_s(rR, o, so), buf_load_s(rD, o, so), buf_load_s(rG, o, so)};
    };
    auto load_v = [&](int x) -> V {
        V v;
        static_cast<H&>(v) = load_h(x, t.inb, t.p);
        const int oo = (t.own && x < t.x1) ? (int)(t.p * 8) : kOob, so = sp.off(x);
        v.m = buf_load_s(rM, oo, so);
        v.gm = buf_load_s(rGm, oo, so);
        v.q = buf_load_s(rQ, oo, so);
        return v;
    };
    const bool yz = t.y > 0 && t.y < N && t.z > 0 && t.z < N;
    const bool halo = threadIdx.x < kDerHalo;
    // step x: plane x - 1 in Rm, x in Rc, x + 1 in Rp; plane x + 3 is loaded
    // into Rl (which held x - 2) and halo x + 2 into Hl (which held x - 3)
    auto step = [&](int x, V& Rm, V& Rc, V& Rp, V& Rl, H& Hc, H& Hl) {
        const int b = x & 1;
        sR[b][t.cell] = Rc.r; sD[b][t.cell] = Rc.D; sT[b][t.cell] = Rc.D * Rc.g;
        if (halo) { sR[b][t.hcell] = Hc.r; sD[b][t.hcell] = Hc.D; sT[b][t.hcell] = Hc.D * Hc.g; }
        lds_barrier();
        Rl = load_v(x + 3);
        Hl = load_h(x + 2, t.hv, t.hp);
        if (t.own && x < t.x1) {
            double out = 0.0;
            if (yz && x > 0 && x < N) {
                // a null dlogD reads 0, and every face term vanishes
                double acc = Rc.m * Rc.gm * Rc.r;
                const double dDc = Rc.D * Rc.g;
                auto nb = [&](double Dj, double dDj, double rj) {
                    acc += dface<HARM>(Rc.D, dDc, Dj, dDj) * inv_h2 * (Rc.r - rj);
                };
                nb(Rp.D, Rp.D * Rp.g, Rp.r);
                nb(Rm.D, Rm.D * Rm.g, Rm.r);
                const int e[4] = {t.cell + kDerRZ, t.cell - kDerRZ, t.cell + 1, t.cell - 1};
                for (int k = 0; k < 4; k++) nb(sD[b][e[k]], sT[b][e[k]], sR[b][e[k]]);
                out = Rc.q - acc;
            }
            rhs[x * t.sx + t.p] = out;
        }
    };
    const int x0 = t.x0;
    V R0 = load_v(x0 - 1), R1 = load_v(x0), R2 = load_v(x0 + 1), R3 = load_v(x0 + 2), R4;
    H H0 = load_h(x0, t.hv, t.hp), H1 = load_h(x0 + 1, t.hv, t.hp), H2, H3, H4;
    for (int x = x0; x < t.x1; x += kDerRing) {
        step(x, R0, R1, R2, R4, H0, H2);
        step(x + 1, R1, R2, R3, R0, H1, H3);
        step(x + 2, R2, R3, R4, R1, H2, H4);
        step(x + 3, R3, R4, R0, R2, H3, H0);
        step(x + 4, R4, R0, R1, R3, H4, H1);
    }
}

// The coefficient gradients on the planes y = N and z = N: logmua_bar = 0
// (boundary); logD_bar from the one face to an interior neighbour j, with
// lam = 0 at the vertex itself (the other faces join boundary vertices and
// count for nothing on the tiles either).
template <bool HARM>
__device__ __forceinline__ void coef_grads_edge(const DerEdge& e, const double* __restrict__ rho,
                                                const double* __restrict__ lam, const double* __restrict__ D,
                                                double inv_h2, double* __restrict__ gD, double* __restrict__ gmu) {
    if (gmu) gmu[e.i] = 0.0;
    if (!gD) return;
    double acc = 0.0;
    if (e.jin) {
        const double Dv = D[e.i], Dj = D[e.j];
        double dcdv;
        if (HARM) {
            const double sum = Dv + Dj;
            dcdv = 2.0 * Dj * Dj * Dv / (sum * sum);
        } else {
            dcdv = 0.5 * Dv;
        }
        acc += dcdv * (0.0 - lam[e.j]) * (rho[e.i] - rho[e.j]);
    }
    gD[e.i] = -acc * inv_h2;
}

// Coefficient gradients from the adjoint state lam = qbar:
//   logmua_bar_i = -mua_i lam_i rho_i (interior, 0 on the boundary)
//   logD_bar_v   = -sum_{faces (v,j), v or j interior} dD_f/dlogD_v (lam_v - lam_j)(rho_v - rho_j) / h^2
// with lam = 0 on boundary vertices.  With data d and weights w (the
// likelihood's gradient) logmua_bar also takes the direct term of L_e =
// mua rho: w_i (mua_i rho_i - d_i) mua_i rho_i.  Neighbours in the order
// +x, -x, +y, -y, +z, -z.
// DATA: d and w are given (and gmu is not null).
template <bool HARM, bool DATA>
__global__ __launch_bounds__(kDerThreads) void k_coef_grads_col(const double* __restrict__ rho,
                                                               const double* __restrict__ lam,
                                                               const double* __restrict__ D,
                                                               const double* __restrict__ mu, int N, double inv_h2,
                                                               double* __restrict__ gD, double* __restrict__ gmu,
                                                               const double* __restrict__ d,
                                                               const double* __restrict__ w, int chunk, int cover) {
    if (der_edge_block(N, chunk, [&](const DerEdge& e) { coef_grads_edge<HARM>(e, rho, lam, D, inv_h2, gD, gmu); }))
        return;
    __shared__ double sL[2][kDerCells], sR[2][kDerCells], sD[2][kDerCells];
    DerTile t;
    der_tile(N, chunk, cover, t);
    const int n = t.n;
    struct H {
        double l, r, D;   // lam (0 on boundary vertices), rho, D
    };
    struct V : H {
        double m, w, d;   // own column only: mua, and the likelihood's weight and data
    };
    const DerSpan sp(t, n);
    const auto rL = sp.rsrc(lam), rR = sp.rsrc(rho), rD = sp.rsrc(D);
    const auto rM = sp.rsrc(gmu ? mu : nullptr), rW = sp.rsrc(DATA ? w : nullptr), rDd = sp.rsrc(DATA ? d : nullptr);
    auto load_h = [&](int x, bool valid, int y, int z, int64_t p) -> H {
        const int o = valid ? (int)(p * 8) : kOob, so = sp.off(x);
        const int ol = (valid && is_interior(N, x, y, z)) ? o : kOob;
        return H{buf_load_s(rL, ol, so), buf_load_s(rR, o, so), buf_load_s(rD, o, so)};
    };
    auto load_v = [&](int x) -> V {
        V v;
        static_cast<H&>(v) = load_h(x, t.inb, t.y, t.z, t.p);
        const int oo = (t.own && x < t.x1) ? (int)(t.p * 8) : kOob, so = sp.off(x);
        v.m = buf_load_s(rM, oo, so);
        if (DATA) {
            v.w = buf_load_s(rW, oo, so);
            v.d = buf_load_s(rDd, oo, so);
        } else {
            v.w = v.d = 0.0;
        }
        return v;
    };
    const bool yz = t.y > 0 && t.y < N && t.z > 0 && t.z < N;
    const bool zin = t.z > 0 && t.z < N, yin = t.y > 0 && t.y < N;
    const bool halo = threadIdx.x < kDerHalo;
    auto step = [&](int x, V& Rm, V& Rc, V& Rp, V& Rl, H& Hc, H& Hl) {
        const int b = x & 1;
        sL[b][t.cell] = Rc.l; sR[b][t.cell] = Rc.r; sD[b][t.cell] = Rc.D;
        if (halo) { sL[b][t.hcell] = Hc.l; sR[b][t.hcell] = Hc.r; sD[b][t.hcell] = Hc.D; }
        lds_barrier();
        Rl = load_v(x + 3);
        Hl = load_h(x + 2, t.hv, t.hy, t.hz, t.hp);
        if (t.own && x < t.x1) {
            const int64_t i = x * t.sx + t.p;
            const bool vin = yz && x > 0 && x < N;
            if (gmu) {
                double g = -Rc.m * Rc.l * Rc.r;
                if (DATA) {
                    const double Le = Rc.m * Rc.r;
                    g += Rc.w * (Le - Rc.d) * Le;
                }
                gmu[i] = vin ? g : 0.0;
            }
            if (gD) {
                // a face counts when either end is interior (which also rules
                // out neighbours beyond the grid); its terms are formed on every
                // lane and selected, without branches (a neighbour beyond the
                // grid reads D = 0, lam = rho = 0, and D_i > 0)
                double acc = 0.0;
                auto nb = [&](bool jin, double lj, double rj, double Dj) {
                    double dcdv;
                    if (HARM) {
                        const double sum = Rc.D + Dj;
                        dcdv = 2.0 * Dj * Dj * Rc.D / (sum * sum);
                    } else {
                        dcdv = 0.5 * Rc.D;
                    }
                    const double term = dcdv * (Rc.l - lj) * (Rc.r - rj);
                    acc += (vin || jin) ? term : 0.0;
                };
                const bool xin = x > 0 && x < N;
                nb(yz && x + 1 < N, Rp.l, Rp.r, Rp.D);
                nb(yz && x - 1 > 0, Rm.l, Rm.r, Rm.D);
                auto cell = [&](int e, bool jin) { nb(jin, sL[b][e], sR[b][e], sD[b][e]); };
                cell(t.cell + kDerRZ, xin && zin && t.y + 1 < N);
                cell(t.cell - kDerRZ, xin && zin && t.y - 1 > 0);
                cell(t.cell + 1, xin && yin && t.z + 1 < N);
                cell(t.cell - 1, xin && yin && t.z - 1 > 0);
                gD[i] = -acc * inv_h2;
            }
        }
    };
    const int x0 = t.x0;
    V R0 = load_v(x0 - 1), R1 = load_v(x0), R2 = load_v(x0 + 1), R3 = load_v(x0 + 2), R4;
    H H0 = load_h(x0, t.hv, t.hy, t.hz, t.hp), H1 = load_h(x0 + 1, t.hv, t.hy, t.hz, t.hp), H2, H3, H4;
    for (int x = x0; x < t.x1; x += kDerRing) {
        step(x, R0, R1, R2, R4, H0, H2);
        step(x + 1, R1, R2, R3, R0, H1, H3);
        step(x + 2, R2, R3, R4, R1, H2, H4);
        step(x + 3, R3, R4, R0, R2, H3, H0);
        step(x + 4, R4, R0, R1, R3, H4, H1);
    }
}

}  // namespace dmgs
