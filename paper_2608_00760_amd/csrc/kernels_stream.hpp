// kernels_stream.hpp -- streaming kernels for the large levels.
//
// All kernels march along x (the slowest axis) over a chunk of planes; each
// workgroup owns a (y, z) tile and each thread a pair of vertices (y, z),
// (y, z+1) of a column, z even.  A column's values on the few planes around
// the march front live in registers (a ring of named planes, so nothing
// moves between registers and loads stay in flight for several steps); only
// in-plane neighbours go through LDS.  Memory operations are buffer
// instructions with per-plane resources: loads outside the grid return 0 and
// stores outside the tile are dropped, so there are no branches around
// memory operations.
//
//  k_rb_sweep_col      one red-black Gauss-Seidel sweep, out of place.
//  k_defect_restrict_col  r = q - A u and full-weighting restriction.
//  k_ir_residual_col   float64 refinement step: x_out = x + e,
//                      r32 = float(b - A x_out), ||b - A x_out||^2;
//                      optionally the likelihood epilogue of x_out.
#pragma once
#include <type_traits>

#include "grid.hpp"

namespace dmgs {

// Barrier that waits only for this wave's LDS operations (not for global
// loads still in flight, which __syncthreads() would drain).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Buffer resources: loads at offsets outside [0, num_records) return 0 and
// stores there are dropped.  One resource per plane keeps offsets within 32
// bits for any grid.
constexpr int kOob = 0x7ffffff0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int64_t plane_bytes, int p, bool valid) {
    const char* b = reinterpret_cast<const char*>(base) + (valid ? (int64_t)p * plane_bytes : 0);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), 0, valid ? (int)plane_bytes : 0, 0x00020000);
}

// Resource over a whole field of `bytes` (< 2^31) bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

template <class T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// ... with a wave-uniform offset `soff` added to the lane's `off` (the range
// check applies to their sum, so kOob in either reads 0)
__device__ __forceinline__ double buf_load_s(__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
template <class T> __device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
template <> __device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, off,
                                          0, 0);
}

// ---------------------------------------------------------------------------
// Red-black sweep.
//
// At march step s the first colour is updated on plane s (tile plus a ring
// of 1, recomputed by neighbouring tiles) and the second colour on plane s-1
// (tile), whose first-colour neighbours are then final.  Plane s is
// published to a 3-slot LDS ring at the start of the step; the first stage
// writes its updates into that slot and the second stage reads the slot of
// plane s-1, so one barrier per step suffices.  Every pair holds one vertex
// of each colour on every plane; threads are laid out so that each wave
// covers rows of one parity, which makes the colour's position in the pair
// uniform across the wave.  The update uses the precomputed inverse
// diagonal w = 1 / (sum_j c_ij + mua_i).

template <class T>
struct SweepArgs {
    const T* u_in;   // iterate before the sweep (ignored when starting from zero)
    T* u_out;        // iterate after the sweep (tile interiors written)
    const T* q;
    const T* D;
    const T* w;      // inverse diagonal
    const T* ec;     // coarse correction added by prolongation (MODE 2)
    T* r;            // defect of the result (two-sweep passes with DEFECT)
    double* partial = nullptr;   // per-block sums of the input's squared residual (two-sweep passes with NORM)
    // layout of u_in, u_out, q, D, w and r (two-sweep passes): vertex (x, y, z)
    // at x px + y py + z; the one-sweep pass takes dense fields
    int py = 0;
    int64_t px = 0;
    int N;
    int order;       // colour of the first stage: 0 red, 1 black
    int tiles_y, tiles_z, chunk, nchunks;
    Stencil<T> st;
};

// Plane-load modes of the sweep: the iterate is read as is, starts from
// zero, or gets the trilinear prolongation I ec of a coarse correction added
// (post-smoothing after the coarse-grid correction).
enum SweepMode { kSweepPlain = 0, kSweepZero = 1, kSweepProlong = 2 };

template <class T>
struct SweepPlane {
    T u0, u1, D0, D1, q0, q1, w0, w1;
};

template <int TY, int TZ>
struct SweepShape {
    static constexpr int NP = TZ / 2 + 2, RY = TY + 4, RZ = 2 * NP, RA = RY * RZ;
    static constexpr int ROWS_HALF = RY / 2;
    static constexpr int HALF = (ROWS_HALF * NP + 63) / 64 * 64;
    static constexpr int NT = 2 * HALF;
    static_assert(TY % 2 == 0 && TZ % 2 == 0, "even tile");
};

template <class T, int TY, int TZ, int MODE, bool HARM>
__global__ __launch_bounds__((SweepShape<TY, TZ>::NT)) void k_rb_sweep_col(SweepArgs<T> a) {
    constexpr bool ZERO_INIT = MODE == kSweepZero, PROLONG = MODE == kSweepProlong;
    using Sh = SweepShape<TY, TZ>;
    constexpr int NP = Sh::NP, RY = Sh::RY, RZ = Sh::RZ, RA = Sh::RA, HALF = Sh::HALF;
    __shared__ T sU[3][RA];
    __shared__ T sD[3][RA];
    const int N = a.N, n = N + 1;
    const int64_t sx = (int64_t)n * n;
    const int64_t plane_bytes = sx * (int64_t)sizeof(T);
    const int tid = threadIdx.x;
    const int hp = tid >= HALF ? 1 : 0;                 // row parity of this wave
    const int th = tid - hp * HALF;
    const bool act = th < Sh::ROWS_HALF * NP;
    const int ly = act ? 2 * (th / NP) + hp : hp, pz = act ? th % NP : 0;
    const int nb = a.tiles_y * a.tiles_z * a.nchunks;
    const int b = xcd_tile(blockIdx.x, nb);
    const int bz = b % a.tiles_z, by = (b / a.tiles_z) % a.tiles_y, bx = b / (a.tiles_z * a.tiles_y);
    const int y0 = by * TY, z0 = bz * TZ;
    const int y = y0 - 2 + ly, zl = z0 - 2 + 2 * pz;
    const int xa = 1 + bx * a.chunk, xb = min(N, xa + a.chunk);   // output planes [xa, xb)
    const int e0 = ly * RZ + 2 * pz;
    const bool yin = act && y >= 0 && y <= N;
    const bool zin0 = zl >= 0 && zl <= N, zin1 = zl + 1 <= N;
    const int off0 = (yin && zin0) ? (int)(((int64_t)y * n + zl) * sizeof(T)) : kOob;
    const int off1 = (yin && zin1) ? (int)(((int64_t)y * n + zl + 1) * sizeof(T)) : kOob;
    const bool y_int = y >= 1 && y <= N - 1;
    const bool ring1 = act && y_int && ly >= 1 && ly <= RY - 2;
    const bool tile = act && y_int && ly >= 2 && ly < 2 + TY;
    auto z_ok = [&](int z, int ring) { return z >= max(1, z0 - ring) && z <= min(N - 1, z0 + TZ - 1 + ring); };
    const int p_lo = max(0, xa - 2), p_hi = min(N, xb + 1);
    const int soff0 = (tile && z_ok(zl, 0)) ? off0 : kOob;
    const int soff1 = (tile && z_ok(zl + 1, 0)) ? off1 : kOob;
    // the two vertices of the pair: which may be updated by each stage
    const bool r1_0 = ring1 && z_ok(zl, 1), r1_1 = ring1 && z_ok(zl + 1, 1);
    const bool t0_0 = tile && z_ok(zl, 0), t0_1 = tile && z_ok(zl + 1, 0);
    // colour parity of the wave: element of the first colour on plane s is
    // (s + hp + order) & 1 (y0 - 2 is even)
    const int wpar = __builtin_amdgcn_readfirstlane(hp + a.order);
    // prolongation: coarse vertices around the pair (Z = zl/2; the odd
    // element also uses Z+1); coarse boundary values are 0, so fine boundary
    // vertices get no correction
    const int ncv = N / 2 + 1;
    const int64_t cplane_bytes = (int64_t)ncv * ncv * (int64_t)sizeof(T);
    const int Yc0 = y >> 1, Yc1 = (y >> 1) + (y & 1), Zc = zl >> 1;
    const int co00 = (PROLONG && yin && zin0) ? (int)(((int64_t)Yc0 * ncv + Zc) * sizeof(T)) : kOob;
    const int co10 = (PROLONG && yin && zin0) ? (int)(((int64_t)Yc1 * ncv + Zc) * sizeof(T)) : kOob;
    const int co01 = (PROLONG && yin && zin1) ? (int)(((int64_t)Yc0 * ncv + Zc + 1) * sizeof(T)) : kOob;
    const int co11 = (PROLONG && yin && zin1) ? (int)(((int64_t)Yc1 * ncv + Zc + 1) * sizeof(T)) : kOob;

    auto load = [&](int p, SweepPlane<T>& P) {
        const bool pv = p >= p_lo && p <= p_hi;
        const auto rD = plane_rsrc(a.D, plane_bytes, p, pv);
        const auto rQ = plane_rsrc(a.q, plane_bytes, p, pv);
        const auto rW = plane_rsrc(a.w, plane_bytes, p, pv);
        if (ZERO_INIT) {
            P.u0 = P.u1 = T(0);
        } else {
            const auto rU = plane_rsrc(a.u_in, plane_bytes, p, pv);
            P.u0 = buf_load<T>(rU, off0);
            P.u1 = buf_load<T>(rU, off1);
        }
        if (PROLONG) {
            const auto rA = plane_rsrc(a.ec, cplane_bytes, p >> 1, pv);
            const auto rB = plane_rsrc(a.ec, cplane_bytes, (p >> 1) + (p & 1), pv);
            const T a00 = buf_load<T>(rA, co00), a10 = buf_load<T>(rA, co10), b00 = buf_load<T>(rB, co00),
                    b10 = buf_load<T>(rB, co10);
            const T a01 = buf_load<T>(rA, co01), a11 = buf_load<T>(rA, co11), b01 = buf_load<T>(rB, co01),
                    b11 = buf_load<T>(rB, co11);
            const T s0 = (a00 + a10) + (b00 + b10);
            P.u0 += s0 * T(0.25);
            P.u1 += (s0 + ((a01 + a11) + (b01 + b11))) * T(0.125);
        }
        P.D0 = buf_load<T>(rD, off0); P.D1 = buf_load<T>(rD, off1);
        P.q0 = buf_load<T>(rQ, off0); P.q1 = buf_load<T>(rQ, off1);
        P.w0 = buf_load<T>(rW, off0); P.w1 = buf_load<T>(rW, off1);
    };

    // Gauss-Seidel update of element O of the pair on a plane:
    // v = w (q + sum_j c_ij u_j); in-plane neighbours from LDS slot (U, Dl),
    // x-neighbours from the planes below (Pb) and above (Pa).
    auto update = [&](auto Oc, const T* U, const T* Dl, const SweepPlane<T>& Pb, const SweepPlane<T>& P,
                      const SweepPlane<T>& Pa) -> T {
        constexpr int O = decltype(Oc)::value;
        const int e = e0 + O;
        const T Di = O ? P.D1 : P.D0;
        const T uzl = O ? P.u0 : U[e - 1], uzr = O ? U[e + 1] : P.u1;
        const T Dzl = O ? P.D0 : Dl[e - 1], Dzr = O ? Dl[e + 1] : P.D1;
        const T cxm = face<HARM>(Di, O ? Pb.D1 : Pb.D0, a.st), cxp = face<HARM>(Di, O ? Pa.D1 : Pa.D0, a.st);
        const T cym = face<HARM>(Di, Dl[e - RZ], a.st), cyp = face<HARM>(Di, Dl[e + RZ], a.st);
        const T czl = face<HARM>(Di, Dzl, a.st), czr = face<HARM>(Di, Dzr, a.st);
        const T num = (O ? P.q1 : P.q0) + cxm * (O ? Pb.u1 : Pb.u0) + cxp * (O ? Pa.u1 : Pa.u0) + cym * U[e - RZ] +
                      cyp * U[e + RZ] + czl * uzl + czr * uzr;
        return num * (O ? P.w1 : P.w0);
    };

    auto step = [&](int s, SweepPlane<T>& Pm2, SweepPlane<T>& Pm1, SweepPlane<T>& P0, SweepPlane<T>& Pp1) {
        const int sl = (s + 3) % 3, slm = (s + 2) % 3;
        T* U = sU[sl];
        T* Dl = sD[sl];
        if (act) { U[e0] = P0.u0; U[e0 + 1] = P0.u1; Dl[e0] = P0.D0; Dl[e0 + 1] = P0.D1; }
        lds_barrier();
        const bool st1 = s >= 1 && s <= N - 1 && s >= xa - 1 && s <= xb;
        const int sm = s - 1;
        const bool st2 = sm >= xa && sm < xb;
        const T* Um = sU[slm];
        const T* Dm = sD[slm];
        if ((s + wpar) & 1) {   // first colour at element 1 on plane s (and second colour at element 1 on s-1)
            if (st1 && r1_1) { const T v = update(std::integral_constant<int, 1>(), U, Dl, Pm1, P0, Pp1); P0.u1 = v; U[e0 + 1] = v; }
            if (st2 && t0_1) Pm1.u1 = update(std::integral_constant<int, 1>(), Um, Dm, Pm2, Pm1, P0);
        } else {
            if (st1 && r1_0) { const T v = update(std::integral_constant<int, 0>(), U, Dl, Pm1, P0, Pp1); P0.u0 = v; U[e0] = v; }
            if (st2 && t0_0) Pm1.u0 = update(std::integral_constant<int, 0>(), Um, Dm, Pm2, Pm1, P0);
        }
        // output plane s-1 (both vertices of the pair are final)
        const auto rO = plane_rsrc(a.u_out, plane_bytes, sm, st2);
        buf_store<T>(Pm1.u0, rO, soff0);
        buf_store<T>(Pm1.u1, rO, soff1);
    };

    // register ring of six planes; the step loop is unrolled by six so planes
    // never move between registers and a load issued at step s is first used
    // at step s + 3.  Plane s-2 is dead after step s; its registers take s+4.
    SweepPlane<T> R0, R1, R2, R3, R4, R5;
    R0.u0 = R0.u1 = R0.D0 = R0.D1 = T(0);
    load(xa - 2, R1);
    load(xa - 1, R2);
    load(xa, R3);
    load(xa + 1, R4);
    load(xa + 2, R5);
    for (int s0 = xa - 1; s0 <= xb; s0 += 6) {
        step(s0, R0, R1, R2, R3); load(s0 + 4, R0);
        if (s0 + 1 > xb) break;
        step(s0 + 1, R1, R2, R3, R4); load(s0 + 5, R1);
        if (s0 + 2 > xb) break;
        step(s0 + 2, R2, R3, R4, R5); load(s0 + 6, R2);
        if (s0 + 3 > xb) break;
        step(s0 + 3, R3, R4, R5, R0); load(s0 + 7, R3);
        if (s0 + 4 > xb) break;
        step(s0 + 4, R4, R5, R0, R1); load(s0 + 8, R4);
        if (s0 + 5 > xb) break;
        step(s0 + 5, R5, R0, R1, R2); load(s0 + 9, R5);
    }
}

// ---------------------------------------------------------------------------
// Defect and full-weighting restriction.  Each workgroup owns a TYC x TZC
// tile of coarse interior vertices and a chunk of coarse planes; threads own
// fine column pairs of the region the tile's stencils cover (plus a ring of
// 1 for the operator).  At fine plane p the residual is formed in LDS, and
// one step later (after the next step's barrier, so one barrier per step)
// each coarse vertex of the tile sums its 3 x 3 in-plane weights
// (1,2,1) x (1,2,1) and accumulates along x with weights (1,2,1); the /64
// is applied when the coarse plane completes.

template <class T>
struct RestrictArgs {
    const T* u;
    const T* q;
    const T* D;
    const T* mu;
    T* qc;
    int py = 0;        // layout of the fine fields u, q, D, mu: vertex (x, y, z) at x px + y py + z
    int64_t px = 0;
    int N;   // fine cells per axis
    int rzero;   // FROM_R: colour ((x+y+z) mod 2) whose defect is 0 and not read
    int tiles_y, tiles_z, chunk, nchunks;
    Stencil<T> st;
};

template <class T>
struct ResPlane {
    T u0, u1, D0, D1, q0, q1, m0, m1;
};

template <int TYC, int TZC>
struct RestrictShape {
    static constexpr int NP = TZC + 2, RY = 2 * TYC + 3, RZ = 2 * NP, RA = RY * RZ;
    static constexpr int NT = (RY * NP + 63) / 64 * 64;
    static_assert(TYC * TZC <= NT, "coarse tile larger than the workgroup");
};

// FROM_R: the fine defect is given (in a.u, 0 off the interior; the colour
// a.rzero is taken as 0 and not read) and only restricted.
template <class T, int TYC, int TZC, bool HARM, bool FROM_R>
__device__ __forceinline__ void defect_restrict_body(const RestrictArgs<T>& a, const int bid) {
    using Sh = RestrictShape<TYC, TZC>;
    constexpr int NP = Sh::NP, RY = Sh::RY, RZ = Sh::RZ, RA = Sh::RA;
    __shared__ T sU[2][RA];
    __shared__ T sD[2][RA];
    __shared__ T sR[2][RA];
    const int N = a.N, Nc = N / 2, ncv = Nc + 1;
    const int64_t plane_bytes = a.px * (int64_t)sizeof(T);
    const int64_t cplane_bytes = (int64_t)ncv * ncv * (int64_t)sizeof(T);
    const int tid = threadIdx.x;
    const bool act = tid < RY * NP;
    const int ly = act ? tid / NP : 0, pz = act ? tid % NP : 0;
    const int nb = a.tiles_y * a.tiles_z * a.nchunks;
    const int b = xcd_tile(bid, nb);
    const int bz = b % a.tiles_z, by = (b / a.tiles_z) % a.tiles_y, bx = b / (a.tiles_z * a.tiles_y);
    const int Y0 = 1 + by * TYC, Z0 = 1 + bz * TZC;
    const int Xa = 1 + bx * a.chunk, Xb = min(Nc, Xa + a.chunk);   // coarse planes [Xa, Xb)
    const int y = 2 * Y0 - 2 + ly, zl = 2 * Z0 - 2 + 2 * pz;
    const int e0 = ly * RZ + 2 * pz;
    const bool yin = act && y >= 0 && y <= N;
    const int off0 = (yin && zl <= N) ? (int)(((int64_t)y * a.py + zl) * sizeof(T)) : kOob;
    const int off1 = (yin && zl + 1 <= N) ? (int)(((int64_t)y * a.py + zl + 1) * sizeof(T)) : kOob;
    // residual needed on region rows/cols 1 .. R-2 (interior vertices only)
    const bool rrow = act && ly >= 1 && ly <= RY - 2 && y >= 1 && y <= N - 1;
    const bool rc0 = rrow && 2 * pz >= 1 && zl >= 1 && zl <= N - 1;
    const bool rc1 = rrow && 2 * pz + 1 <= RZ - 2 && zl + 1 >= 1 && zl + 1 <= N - 1;
    // coarse vertex owned by this thread
    const bool cown = tid < TYC * TZC;
    const int lyc = cown ? tid / TZC : 0, lzc = cown ? tid % TZC : 0;
    const int Yc = Y0 + lyc, Zc = Z0 + lzc;
    const int coff = (cown && Yc <= Nc - 1 && Zc <= Nc - 1) ? (int)(((int64_t)Yc * ncv + Zc) * sizeof(T)) : kOob;
    const int cc = (2 * lyc + 2) * RZ + 2 * lzc + 2;   // fine centre in the region
    const int p_first = 2 * Xa - 1, p_last = 2 * Xb - 1;
    const int p_lo = p_first - 1, p_hi = p_last + 1;

    auto load = [&](int p, ResPlane<T>& P) {
        const bool pv = p >= p_lo && p <= p_hi && p >= 0 && p <= N;
        const auto rU = plane_rsrc(a.u, plane_bytes, p, pv);
        P.u0 = buf_load<T>(rU, off0); P.u1 = buf_load<T>(rU, off1);
        if (FROM_R) return;
        const auto rD = plane_rsrc(a.D, plane_bytes, p, pv);
        const auto rQ = plane_rsrc(a.q, plane_bytes, p, pv);
        const auto rM = plane_rsrc(a.mu, plane_bytes, p, pv);
        P.D0 = buf_load<T>(rD, off0); P.D1 = buf_load<T>(rD, off1);
        P.q0 = buf_load<T>(rQ, off0); P.q1 = buf_load<T>(rQ, off1);
        P.m0 = buf_load<T>(rM, off0); P.m1 = buf_load<T>(rM, off1);
    };
    auto resid = [&](auto Oc, const T* U, const T* Dl, const ResPlane<T>& Pb, const ResPlane<T>& P,
                     const ResPlane<T>& Pa) -> T {
        constexpr int O = decltype(Oc)::value;
        const int e = e0 + O;
        const T ui = O ? P.u1 : P.u0, Di = O ? P.D1 : P.D0;
        const T uzl = O ? P.u0 : U[e - 1], uzr = O ? U[e + 1] : P.u1;
        const T Dzl = O ? P.D0 : Dl[e - 1], Dzr = O ? Dl[e + 1] : P.D1;
        const T Au = (O ? P.m1 : P.m0) * ui + face<HARM>(Di, O ? Pb.D1 : Pb.D0, a.st) * (ui - (O ? Pb.u1 : Pb.u0)) +
                     face<HARM>(Di, O ? Pa.D1 : Pa.D0, a.st) * (ui - (O ? Pa.u1 : Pa.u0)) +
                     face<HARM>(Di, Dl[e - RZ], a.st) * (ui - U[e - RZ]) + face<HARM>(Di, Dl[e + RZ], a.st) * (ui - U[e + RZ]) +
                     face<HARM>(Di, Dzl, a.st) * (ui - uzl) + face<HARM>(Di, Dzr, a.st) * (ui - uzr);
        return (O ? P.q1 : P.q0) - Au;
    };

    T acc = T(0);
    // restriction of the residual of plane p (in sR[p & 1]) into the coarse accumulator
    auto restrict_plane = [&](int p) {
        const T* Rp = sR[p & 1];
        auto row = [&](int c) { return (Rp[c - 1] + T(2) * Rp[c]) + Rp[c + 1]; };
        const T w = (row(cc - RZ) + T(2) * row(cc)) + row(cc + RZ);
        if (p & 1) {   // p = 2X - 1: completes coarse plane X - 1, starts X
            if (p > p_first) {
                const int X = (p - 1) / 2;
                const auto rC = plane_rsrc(a.qc, cplane_bytes, X, true);
                buf_store<T>((acc + w) * T(1.0 / 64.0), rC, coff);
            }
            acc = w;
        } else {
            acc += T(2) * w;
        }
    };
    auto step = [&](int p, ResPlane<T>& Pm1, ResPlane<T>& P0, ResPlane<T>& Pp1) {
        const int sl = p & 1;
        T* U = sU[sl];
        T* Dl = sD[sl];
        if (act && !FROM_R) { U[e0] = P0.u0; U[e0 + 1] = P0.u1; Dl[e0] = P0.D0; Dl[e0 + 1] = P0.D1; }
        lds_barrier();
        const bool pin = p >= 1 && p <= N - 1;
        T r0, r1;
        if (FROM_R) {
            const bool z0c = ((p + y + zl) & 1) == a.rzero;   // colour of element 0 is the zero colour
            r0 = (pin && rc0 && !z0c) ? P0.u0 : T(0);
            r1 = (pin && rc1 && z0c) ? P0.u1 : T(0);
        } else {
            r0 = (pin && rc0) ? resid(std::integral_constant<int, 0>(), U, Dl, Pm1, P0, Pp1) : T(0);
            r1 = (pin && rc1) ? resid(std::integral_constant<int, 1>(), U, Dl, Pm1, P0, Pp1) : T(0);
        }
        if (act) { sR[sl][e0] = r0; sR[sl][e0 + 1] = r1; }
        // sR[sl ^ 1] was written before this step's barrier
        if (cown && p > p_first) restrict_plane(p - 1);
    };

    // register ring of four planes; plane p-1 is dead after step p and its
    // registers take plane p+3
    ResPlane<T> R0, R1, R2, R3;
    load(p_first - 1, R0);
    load(p_first, R1);
    load(p_first + 1, R2);
    load(p_first + 2, R3);
    for (int p0 = p_first; p0 <= p_last; p0 += 4) {
        step(p0, R0, R1, R2); load(p0 + 3, R0);
        if (p0 + 1 > p_last) break;
        step(p0 + 1, R1, R2, R3); load(p0 + 4, R1);
        if (p0 + 2 > p_last) break;
        step(p0 + 2, R2, R3, R0); load(p0 + 5, R2);
        if (p0 + 3 > p_last) break;
        step(p0 + 3, R3, R0, R1); load(p0 + 6, R3);
    }
    lds_barrier();
    if (cown) restrict_plane(p_last);
}

template <class T, int TYC, int TZC, bool HARM, bool FROM_R = false>
__global__ __launch_bounds__((RestrictShape<TYC, TZC>::NT)) void k_defect_restrict_col(RestrictArgs<T> a) {
    defect_restrict_body<T, TYC, TZC, HARM, FROM_R>(a, blockIdx.x);
}

template <class T, int TYC, int TZC, bool HARM, bool FROM_R = false>
__global__ __launch_bounds__((RestrictShape<TYC, TZC>::NT)) void k_defect_restrict_grp(const Group<RestrictArgs<T>>* g) {
    int bid;
    const int m = group_member(g, &bid);
    if (bid < 0) return;
    const RestrictArgs<T> a = g->a[m];
    defect_restrict_body<T, TYC, TZC, HARM, FROM_R>(a, bid);
}

// ---------------------------------------------------------------------------
// Float64 refinement step (and the plain float64 residual norm): threads own
// column pairs of the tile plus a ring of 1 in y and one pair in z.
//   x_out = x + e  (e float32; HAS_E false: no correction)     on the tile
//   r32   = float(b - A x_out)                                 on the tile
//   partial[block] = sum over the tile of (b - A x_out)^2
// x_out and r32 may be null (not written).

struct IrArgs {
    const double* x;
    const float* e;
    double* x_out;
    const double* b;
    const double* D;
    const double* mu;
    float* r32;
    double* partial;
    // likelihood epilogue of the refined iterate rho = x_out (EPI): data d,
    // weights w; rhobar = mua w (mua rho - d) on tile vertices, and block
    // sums of w (d - mua rho)^2 and of w > 0 at partial[gridDim + b] and
    // partial[2 gridDim + b]
    const double* ed = nullptr;
    const double* ew = nullptr;
    double* erhobar = nullptr;
    int py = 0;        // layout of the float32 fields e and r32: vertex (x, y, z) at x px + y py + z
    int64_t px = 0;    // (the float64 fields are dense)
    int N;
    int tiles_y, tiles_z, chunk, nchunks;
    Stencil<double> st;
};

struct IrPlane {
    double x0, x1, D0, D1, b0, b1, m0, m1;
    float e0, e1;
    double d0, d1, w0, w1;   // likelihood data and weights (EPI)
};

template <int TY, int TZ>
struct IrShape {
    static constexpr int NP = TZ / 2 + 2, RY = TY + 2, RZ = 2 * NP, RA = RY * RZ;
    static constexpr int NT = (RY * NP + 63) / 64 * 64;
};

// X_ZERO: the iterate x is 0 everywhere (not read): with e, x_out = e;
// without e, the residual is b itself.
// One workgroup (bid of nblk) of the refinement step.
template <int TY, int TZ, bool HAS_E, bool X_ZERO, bool HARM, bool EPI>
__device__ __forceinline__ void ir_residual_body(const IrArgs& a, const int bid, const int nblk) {
    using Sh = IrShape<TY, TZ>;
    constexpr int NP = Sh::NP, RY = Sh::RY, RZ = Sh::RZ, RA = Sh::RA;
    __shared__ double sU[2][RA];
    __shared__ double sD[2][RA];
    const int N = a.N, n = N + 1;
    const int64_t sx = (int64_t)n * n;
    const int64_t pb8 = sx * 8, pb4 = a.px * 4;
    const int tid = threadIdx.x;
    const bool act = tid < RY * NP;
    const int ly = act ? tid / NP : 0, pz = act ? tid % NP : 0;
    const int nb = a.tiles_y * a.tiles_z * a.nchunks;
    const int tb = xcd_tile(bid, nb);
    const int bz = tb % a.tiles_z, by = (tb / a.tiles_z) % a.tiles_y, bx = tb / (a.tiles_z * a.tiles_y);
    const int y0 = by * TY, z0 = bz * TZ;
    const int y = y0 - 1 + ly, zl = z0 - 2 + 2 * pz;
    const int xa = 1 + bx * a.chunk, xb = min(N, xa + a.chunk);   // planes [xa, xb)
    const int e0 = ly * RZ + 2 * pz;
    const bool yin = act && y >= 0 && y <= N;
    const int64_t v0 = (int64_t)y * n + zl, v4 = (int64_t)y * a.py + zl;
    const int o8_0 = (yin && zl >= 0 && zl <= N) ? (int)(v0 * 8) : kOob;
    const int o8_1 = (yin && zl + 1 <= N) ? (int)((v0 + 1) * 8) : kOob;
    const int o4_0 = (yin && zl >= 0 && zl <= N) ? (int)(v4 * 4) : kOob;
    const int o4_1 = (yin && zl + 1 <= N) ? (int)((v4 + 1) * 4) : kOob;
    const bool tile_y = act && ly >= 1 && ly <= TY && y >= 1 && y <= N - 1;
    const bool t0 = tile_y && zl >= max(1, z0) && zl <= min(N - 1, z0 + TZ - 1);
    const bool t1 = tile_y && zl + 1 >= max(1, z0) && zl + 1 <= min(N - 1, z0 + TZ - 1);
    const int s8_0 = t0 ? o8_0 : kOob, s8_1 = t1 ? o8_1 : kOob;
    const int s4_0 = t0 ? o4_0 : kOob, s4_1 = t1 ? o4_1 : kOob;
    const int p_lo = xa - 1, p_hi = xb;

    auto load = [&](int p, IrPlane& P) {
        const bool pv = p >= p_lo && p <= p_hi;
        const auto rX = plane_rsrc(a.x, pb8, p, pv);
        const auto rD = plane_rsrc(a.D, pb8, p, pv);
        const auto rB = plane_rsrc(a.b, pb8, p, pv);
        const auto rM = plane_rsrc(a.mu, pb8, p, pv);
        if (X_ZERO) {
            P.x0 = P.x1 = 0.0;
        } else {
            P.x0 = buf_load<double>(rX, o8_0); P.x1 = buf_load<double>(rX, o8_1);
        }
        P.b0 = buf_load<double>(rB, o8_0); P.b1 = buf_load<double>(rB, o8_1);
        if (X_ZERO && !HAS_E) {   // A 0 = 0: no coefficients needed
            P.D0 = P.D1 = P.m0 = P.m1 = 0.0;
        } else {
            P.D0 = buf_load<double>(rD, o8_0); P.D1 = buf_load<double>(rD, o8_1);
            P.m0 = buf_load<double>(rM, o8_0); P.m1 = buf_load<double>(rM, o8_1);
        }
        if (HAS_E) {
            const auto rE = plane_rsrc(a.e, pb4, p, pv);
            P.e0 = buf_load<float>(rE, o4_0); P.e1 = buf_load<float>(rE, o4_1);
        } else {
            P.e0 = P.e1 = 0.0f;
        }
        if (EPI) {
            const auto rDd = plane_rsrc(a.ed, pb8, p, pv);
            const auto rW = plane_rsrc(a.ew, pb8, p, pv);
            P.d0 = buf_load<double>(rDd, o8_0); P.d1 = buf_load<double>(rDd, o8_1);
            P.w0 = buf_load<double>(rW, o8_0); P.w1 = buf_load<double>(rW, o8_1);
        }
    };
    auto u0of = [&](const IrPlane& P) { return HAS_E ? P.x0 + (double)P.e0 : P.x0; };
    auto u1of = [&](const IrPlane& P) { return HAS_E ? P.x1 + (double)P.e1 : P.x1; };

    double acc = 0.0, accH = 0.0, accN = 0.0;
    auto step = [&](int p, IrPlane& Pm1, IrPlane& P0, IrPlane& Pp1) {
        const int sl = p & 1;
        double* U = sU[sl];
        double* Dl = sD[sl];
        const double u0 = u0of(P0), u1 = u1of(P0);
        if (act) { U[e0] = u0; U[e0 + 1] = u1; Dl[e0] = P0.D0; Dl[e0 + 1] = P0.D1; }
        lds_barrier();
        auto res = [&](auto Oc) -> double {
            constexpr int O = decltype(Oc)::value;
            if (X_ZERO && !HAS_E) return O ? P0.b1 : P0.b0;
            const int e = e0 + O;
            const double ui = O ? u1 : u0, Di = O ? P0.D1 : P0.D0;
            const double uzl = O ? u0 : U[e - 1], uzr = O ? U[e + 1] : u1;
            const double Dzl = O ? P0.D0 : Dl[e - 1], Dzr = O ? Dl[e + 1] : P0.D1;
            const double ub = O ? u1of(Pm1) : u0of(Pm1), ua = O ? u1of(Pp1) : u0of(Pp1);
            const double Au = (O ? P0.m1 : P0.m0) * ui + face<HARM>(Di, O ? Pm1.D1 : Pm1.D0, a.st) * (ui - ub) +
                              face<HARM>(Di, O ? Pp1.D1 : Pp1.D0, a.st) * (ui - ua) +
                              face<HARM>(Di, Dl[e - RZ], a.st) * (ui - U[e - RZ]) +
                              face<HARM>(Di, Dl[e + RZ], a.st) * (ui - U[e + RZ]) + face<HARM>(Di, Dzl, a.st) * (ui - uzl) +
                              face<HARM>(Di, Dzr, a.st) * (ui - uzr);
            return (O ? P0.b1 : P0.b0) - Au;
        };
        const bool pin = p >= xa && p < xb;
        const double r0 = (pin && t0) ? res(std::integral_constant<int, 0>()) : 0.0;
        const double r1 = (pin && t1) ? res(std::integral_constant<int, 1>()) : 0.0;
        acc += r0 * r0 + r1 * r1;
        const auto rO = plane_rsrc(a.x_out, pb8, p, pin && a.x_out != nullptr);
        buf_store<double>(u0, rO, s8_0);
        buf_store<double>(u1, rO, s8_1);
        const auto rR = plane_rsrc(a.r32, pb4, p, pin && a.r32 != nullptr);
        buf_store<float>((float)r0, rR, s4_0);
        buf_store<float>((float)r1, rR, s4_1);
        if (EPI) {
            // L_e = mua rho, the data residual and the pull-back's cotangent
            // on the tile's interior vertices (the boundary of rhobar is 0)
            auto epi = [&](double u, double m, double d, double w, bool on, double& rb) {
                const double res = m * u - d;
                rb = m * w * res;
                if (on) {
                    accH += w * res * res;
                    accN += w > 0.0 ? 1.0 : 0.0;
                }
            };
            double rb0, rb1;
            epi(u0, P0.m0, P0.d0, P0.w0, pin && t0, rb0);
            epi(u1, P0.m1, P0.d1, P0.w1, pin && t1, rb1);
            const auto rRb = plane_rsrc(a.erhobar, pb8, p, pin);
            buf_store<double>(rb0, rRb, s8_0);
            buf_store<double>(rb1, rRb, s8_1);
        }
    };

    IrPlane R0, R1, R2, R3;
    load(xa - 1, R0);
    load(xa, R1);
    load(xa + 1, R2);
    load(xa + 2, R3);
    for (int p0 = xa; p0 < xb; p0 += 4) {
        step(p0, R0, R1, R2); load(p0 + 3, R0);
        if (p0 + 1 >= xb) break;
        step(p0 + 1, R1, R2, R3); load(p0 + 4, R1);
        if (p0 + 2 >= xb) break;
        step(p0 + 2, R2, R3, R0); load(p0 + 5, R2);
        if (p0 + 3 >= xb) break;
        step(p0 + 3, R3, R0, R1); load(p0 + 6, R3);
    }
    // deterministic block sums (fixed order over waves)
    __shared__ double wsum[3][Sh::NT / 64];
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_down(acc, off, 64);
        if (EPI) {
            accH += __shfl_down(accH, off, 64);
            accN += __shfl_down(accN, off, 64);
        }
    }
    if (tid % 64 == 0) {
        wsum[0][tid / 64] = acc;
        if (EPI) {
            wsum[1][tid / 64] = accH;
            wsum[2][tid / 64] = accN;
        }
    }
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < (EPI ? 3 : 1); k++) {
            double s = 0.0;
            for (int i = 0; i < Sh::NT / 64; i++) s += wsum[k][i];
            a.partial[k * nblk + bid] = s;
        }
    }
}

template <int TY, int TZ, bool HAS_E, bool X_ZERO, bool HARM, bool EPI = false>
__global__ __launch_bounds__((IrShape<TY, TZ>::NT)) void k_ir_residual_col(IrArgs a) {
    ir_residual_body<TY, TZ, HAS_E, X_ZERO, HARM, EPI>(a, blockIdx.x, gridDim.x);
}

template <int TY, int TZ, bool HAS_E, bool X_ZERO, bool HARM, bool EPI = false>
__global__ __launch_bounds__((IrShape<TY, TZ>::NT)) void k_ir_residual_grp(const Group<IrArgs>* g) {
    int bid;
    const int m = group_member(g, &bid);
    if (bid < 0) return;
    const IrArgs a = g->a[m];
    ir_residual_body<TY, TZ, HAS_E, X_ZERO, HARM, EPI>(a, bid, g->nblk[m]);
}

// Set the boundary layer of an iterate to g (interior untouched).
template <class T>
__global__ void k_set_boundary(T* __restrict__ u, int N, T g) {
    const int n = N + 1;
    const int64_t sx = (int64_t)n * n;
    const int face_id = blockIdx.y;   // 0: x=0, 1: x=N, 2: y=0, 3: y=N, 4: z=0, 5: z=N
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * n; t += gridDim.x * blockDim.x) {
        const int i = t / n, j = t - (t / n) * n;
        const int c = (face_id & 1) ? N : 0;
        int64_t v;
        if (face_id < 2) v = (int64_t)c * sx + (int64_t)i * n + j;
        else if (face_id < 4) v = (int64_t)i * sx + (int64_t)c * n + j;
        else v = (int64_t)i * sx + (int64_t)j * n + c;
        u[v] = g;
    }
}

}  // namespace dmgs
