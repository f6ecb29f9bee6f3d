// kernels_sweep2.hpp -- two red-black Gauss-Seidel sweeps in one streaming
// pass (temporal blocking along x), for iterates with a zero Dirichlet
// boundary (the float32 corrections of the refinement solver).
//
// A V(2,2) cycle smooths twice before and twice after the coarse-grid
// correction; doing both sweeps of a phase in one pass reads the level's
// fields once instead of twice.  The four colour updates of the two sweeps
// (first colour, second colour, first, second) run as a pipeline along the
// march: at step s, stage j updates plane s - j.  Every stage sees its
// neighbours in exactly the state the sequential order gives:
//   stage 0 on plane s     first colour,  neighbours before any update;
//   stage 1 on plane s-1   second colour, neighbours after stage 0;
//   stage 2 on plane s-2   first colour,  neighbours after stage 1;
//   stage 3 on plane s-3   second colour, neighbours after stage 2.
// In y and z, stage j is applied to the tile plus a ring of 3 - j vertices
// (neighbouring tiles recompute the ring), so the tile's final values need
// nothing from other workgroups.  Along x, a chunk [xa, xb) runs steps
// xa-3 .. xb+2: the final values of its planes depend only on stage j
// applied to planes [xa-3+j, xb+2-j], which the pipeline computes from
// loaded data; what the first and last steps compute outside those ranges
// is never read by them.  Planes at or beyond the grid boundary need no
// special case: there the inverse diagonal w is 0 and loads return 0, so an
// update reproduces the zero boundary value.
//
// Threads own a column pair (y; z, z+1), z even, of the tile plus a ring of
// 4, and keep eight planes of their pair in a register ring (planes s-4 ..
// s+3; s+2 and s+3 are loads in flight).  Plane s+3 is loaded right after
// step s's barrier into the registers of plane s-5 (dead since step s-1), so
// the load is in flight while the step computes; it is first used at step
// s+2.  In-plane neighbours go through an
// eight-slot LDS ring of planes holding {u, D}, laid out by pair element so
// that consecutive lanes read consecutive 8-byte words; with eight slots
// and the march unrolled by eight, every slot address is a compile-time
// offset.  Each stage updates its colour in its plane's slot in place (it
// reads only the other colour), the four stages of a step touch four
// different slots, and a slot is republished five steps after its last
// use, so one barrier per step orders everything.  Stages are applied to
// every lane and the result is selected by the lane's ring membership.  At
// step s all four stages update the same element of the pair, (s + row
// parity + order) mod 2, uniform across a wave because waves hold rows of
// one parity.
//
// With DEFECT the pass also writes the defect r = q - A u of its result on
// the tile (the restriction of the next coarser right-hand side then reads
// r alone).  The loaded ring grows to 5 so that the final values are known
// on the tile plus a ring of 1, the stages run one step earlier and one
// step longer, the last stage publishes its values to the slot too, and at
// step s the defect of plane s - 4 is formed from the slots of planes s - 4
// and s - 5 and the registers of plane s - 3.  After a red-black sweep the
// residual of the colour updated last is zero (its update solved its own
// equation with its neighbours' final values), so only the first colour's
// residual is computed and stored; the reader takes the second colour's as
// 0.  Waves with no tile vertex skip the defect.
//
// With NORM (plain passes) the pass also sums the squared residual of its
// input over the tile's first-colour vertices: stage 0 forms q + sum_j c_ij
// u_j from the input, and the residual is that minus u_i / w_i.  When the
// input ended a red-black sweep whose last colour is this pass's second,
// the second colour's residual is 0 (up to rounding), so the block sums
// (one per workgroup, in a.partial) add up to ||q - A u||^2 of the input.
#pragma once
#include "kernels_stream.hpp"

namespace dmgs {

template <int TY, int TZ, int RING = 4>
struct Sweep2Shape {
    static constexpr int R = RING;                           // ring of loaded vertices
    static constexpr int NP = TZ / 2 + R, RY = TY + 2 * R;   // pairs per row, rows
    static constexpr int RA = RY * NP;                       // pairs per plane (per element)
    static constexpr int ROWS_HALF = RY / 2;
    static constexpr int HALF = (ROWS_HALF * NP + 63) / 64 * 64;
    static constexpr int NT = 2 * HALF;
    static constexpr int SLOTS = 8;
    static constexpr int PAD = NP + 2;                       // guard entries before and after the ring
    static constexpr int ENTRIES = SLOTS * 2 * RA + 2 * PAD;
    // coarse-correction planes (prolongation): rows and columns of the coarse
    // vertices the tile plus its ring interpolates from, four planes
    static constexpr int CRY = RY / 2 + 1, CRZ = NP + 1, CPL = CRY * CRZ, CSLOTS = 4;
    static_assert(TY % 2 == 0 && TZ % 2 == 0, "even tile");
};

template <class T>
struct UD {
    T u, D;
};

template <class T, int TY, int TZ, int RING = 4>
constexpr size_t sweep2_lds_bytes() {
    using Sh = Sweep2Shape<TY, TZ, RING>;
    return (size_t)Sh::ENTRIES * sizeof(UD<T>) + (size_t)Sh::CSLOTS * Sh::CPL * sizeof(T);
}

// Largest level the two-sweep pass takes: buffer offsets of a whole field
// of planes of px elements (plus a few planes beyond it) stay below kOob.
template <class T>
__host__ __device__ constexpr bool sweep2_fits(int N, int64_t px) {
    return (px * (N + 20) + 64) * (int64_t)sizeof(T) < (int64_t)kOob;
}

// One workgroup of the pass: tile and chunk bid of the level's grid.
template <class T, int TY, int TZ, int MODE, bool HARM, bool DEFECT, bool NORM>
__device__ __forceinline__ void rb_sweep2_body(const SweepArgs<T>& a, const int bid) {
    constexpr bool ZERO_INIT = MODE == kSweepZero, PROLONG = MODE == kSweepProlong;
    static_assert(!(DEFECT && PROLONG), "the defect is formed after pre-smoothing only");
    static_assert(!NORM || (MODE == kSweepPlain && !DEFECT), "the input's residual norm needs a plain pass");
    using Sh = Sweep2Shape<TY, TZ, DEFECT ? 5 : 4>;
    constexpr int R = Sh::R, NP = Sh::NP, RA = Sh::RA, HALF = Sh::HALF;
    // slot k, element O: ring[(k * 2 + O) * RA + ly * NP + pz]
    extern __shared__ __align__(16) unsigned char lds_raw[];
    UD<T>* const ring = reinterpret_cast<UD<T>*>(lds_raw) + Sh::PAD;
    const int N = a.N, n = N + 1;
    const int plane_bytes = (int)(a.px * (int64_t)sizeof(T));   // the level's fields: rows of a.py, planes of a.px
    const int field_bytes = n * plane_bytes;
    const int tid = threadIdx.x;
    const int hp = tid >= HALF ? 1 : 0;                 // row parity of this wave
    // lanes past the half's pairs (in its last wave) repeat the first pairs
    // of the half: they compute and write bit-identical values and store
    // nothing to memory
    const int th0 = tid - hp * HALF;
    const bool own = th0 < Sh::ROWS_HALF * NP;
    const int th = own ? th0 : th0 - Sh::ROWS_HALF * NP;
    const int ly = 2 * (th / NP) + hp, pz = th % NP;
    const int nb = a.tiles_y * a.tiles_z * a.nchunks;
    const int b = xcd_tile(bid, nb);
    const int bz = b % a.tiles_z, by = (b / a.tiles_z) % a.tiles_y, bx = b / (a.tiles_z * a.tiles_y);
    const int y0 = by * TY, z0 = bz * TZ;
    const int y = y0 - R + ly, zl = z0 - R + 2 * pz;
    const int xa = 1 + bx * a.chunk, xb = min(N, xa + a.chunk);   // output planes [xa, xb)
    const int pe = ly * NP + pz;                                   // this pair's index in a slot
    // in-plane offset of element 0 (element 1 is the next word); rows outside
    // the grid read 0, columns just outside it read finite data (the
    // neighbouring row's, or row padding) that no update of an interior
    // vertex uses
    const int off = (y >= 0 && y <= N) ? (y * a.py + zl) * (int)sizeof(T) : kOob;
    // ring membership: stage j updates a vertex within R - 1 - j of the tile
    auto in_ring = [&](int z, int r) {
        return y >= max(1, y0 - r) && y <= min(N - 1, y0 + TY - 1 + r) && z >= max(1, z0 - r) &&
               z <= min(N - 1, z0 + TZ - 1 + r);
    };
    bool m0[4], m1[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        m0[j] = in_ring(zl, R - 1 - j);
        m1[j] = in_ring(zl + 1, R - 1 - j);
    }
    const int soff0 = (own && in_ring(zl, 0)) ? off : kOob;   // tile vertices are stored
    const int soff1 = (own && in_ring(zl + 1, 0)) ? off + (int)sizeof(T) : kOob;
    const auto rR = field_rsrc(a.r, DEFECT ? field_bytes : 0);
    const auto rU = field_rsrc(a.u_in, field_bytes), rD = field_rsrc(a.D, field_bytes);
    const auto rQ = field_rsrc(a.q, field_bytes), rW = field_rsrc(a.w, field_bytes);
    const auto rO = field_rsrc(a.u_out, field_bytes);
    // prolongation: coarse vertices around the pair (the odd element also
    // uses Z+1); coarse boundary values are 0
    const int ncv = N / 2 + 1;
    const int cplane_bytes = ncv * ncv * (int)sizeof(T);
    const auto rC = field_rsrc(a.ec, PROLONG ? (int64_t)ncv * cplane_bytes : 0);
    const bool pin = PROLONG && y >= 0 && y <= N && zl >= 0 && zl <= N;
    const int Yc0 = y >> 1, Yc1 = (y >> 1) + (y & 1), Zc = zl >> 1;
    const int co0 = pin ? (Yc0 * ncv + Zc) * (int)sizeof(T) : kOob;
    const int co1 = pin ? (Yc1 * ncv + Zc) * (int)sizeof(T) : kOob;

    // zero the ring once: every value a stage reads is then finite
    for (int i = tid; i < Sh::ENTRIES; i += Sh::NT) reinterpret_cast<UD<T>*>(lds_raw)[i] = UD<T>{T(0), T(0)};
    __syncthreads();

    auto load = [&](int p, SweepPlane<T>& P) {
        const int vo = off + p * plane_bytes;   // p < 0 or p > N: outside the field
        if (ZERO_INIT) {
            P.u0 = P.u1 = T(0);
        } else {
            P.u0 = buf_load<T>(rU, vo);
            P.u1 = buf_load<T>(rU, vo + (int)sizeof(T));
        }
        P.D0 = buf_load<T>(rD, vo); P.D1 = buf_load<T>(rD, vo + (int)sizeof(T));
        P.q0 = buf_load<T>(rQ, vo); P.q1 = buf_load<T>(rQ, vo + (int)sizeof(T));
        P.w0 = buf_load<T>(rW, vo); P.w1 = buf_load<T>(rW, vo + (int)sizeof(T));
    };
    // prolongation of the coarse correction onto the pair of plane p, from
    // memory (the planes before the first step)
    struct Coarse {
        T a00, a10, b00, b10, a01, a11, b01, b11;
    };
    auto load_coarse = [&](int p, Coarse& C) {
        const int ca = co0 + (p >> 1) * cplane_bytes, cb = co1 + (p >> 1) * cplane_bytes;
        const int pa = (p & 1) * cplane_bytes;
        C.a00 = buf_load<T>(rC, ca); C.a10 = buf_load<T>(rC, cb);
        C.b00 = buf_load<T>(rC, ca + pa); C.b10 = buf_load<T>(rC, cb + pa);
        C.a01 = buf_load<T>(rC, ca + (int)sizeof(T)); C.a11 = buf_load<T>(rC, cb + (int)sizeof(T));
        C.b01 = buf_load<T>(rC, ca + pa + (int)sizeof(T)); C.b11 = buf_load<T>(rC, cb + pa + (int)sizeof(T));
    };
    auto add_coarse = [&](const Coarse& C, SweepPlane<T>& P) {
        const T s0 = (C.a00 + C.a10) + (C.b00 + C.b10);
        P.u0 += s0 * T(0.25);
        P.u1 += (s0 + ((C.a01 + C.a11) + (C.b01 + C.b11))) * T(0.125);
    };
    // ... and from the LDS planes of the coarse correction during the march:
    // coarse plane X is loaded at step 2X-4 by the first CPL threads, stored
    // at step 2X-3 and read at steps 2X-2 .. 2X (fine planes 2X-1 .. 2X+1);
    // writing a plane again stores the same values
    T* const cring = reinterpret_cast<T*>(lds_raw + Sh::ENTRIES * sizeof(UD<T>));
    const bool cloader = PROLONG && tid < Sh::CPL;
    const int cy = tid / Sh::CRZ, cz = tid % Sh::CRZ;
    const int cY = y0 / 2 - 2 + cy, cZ = z0 / 2 - 2 + cz;
    const int coff = (cloader && cY >= 0 && cY < ncv && cZ >= 0 && cZ < ncv) ? (cY * ncv + cZ) * (int)sizeof(T) : kOob;
    auto coarse_plane = [&](int X) {   // this loader thread's value of coarse plane X (0 outside the grid)
        return buf_load<T>(rC, (X >= 0 && X < ncv) ? coff + X * cplane_bytes : kOob);
    };
    const int cl0 = (ly >> 1) * Sh::CRZ + pz;   // this pair's coarse row (even y) and column in a plane
    const int cl1 = cl0 + hp * Sh::CRZ;         // the row below for odd y
    // Even fine planes (one coarse plane) and even rows (waves with hp = 0:
    // one coarse row) read fewer values; doubling is exact in floating point,
    // so every case gives the bits of the general sum.
    auto add_coarse_lds = [&](int p, SweepPlane<T>& P) {
        const int X0 = p >> 1, X1 = X0 + (p & 1);
        const T* A = cring + (X0 & 3) * Sh::CPL;
        const T* B = cring + (X1 & 3) * Sh::CPL;
        T s0, s1;
        if (hp == 0) {
            const T a0 = A[cl0], a1 = A[cl0 + 1];
            if (p & 1) {
                const T b0 = B[cl0], b1 = B[cl0 + 1];
                s0 = (a0 + a0) + (b0 + b0);
                s1 = (a1 + a1) + (b1 + b1);
            } else {
                s0 = (a0 + a0) + (a0 + a0);
                s1 = (a1 + a1) + (a1 + a1);
            }
        } else {
            if (p & 1) {
                s0 = (A[cl0] + A[cl1]) + (B[cl0] + B[cl1]);
                s1 = (A[cl0 + 1] + A[cl1 + 1]) + (B[cl0 + 1] + B[cl1 + 1]);
            } else {
                const T a0 = A[cl0] + A[cl1], a1 = A[cl0 + 1] + A[cl1 + 1];
                s0 = a0 + a0;
                s1 = a1 + a1;
            }
        }
        P.u0 += s0 * T(0.25);
        P.u1 += (s0 + s1) * T(0.125);
    };
    T cg = T(0);   // loader: coarse value in flight

    // q + sum_j c_ij u_j at element O of the pair on a plane whose slot is
    // S (the Gauss-Seidel value is w times it); x-neighbours from the planes
    // below (Pb) and above (Pa), the in-pair z-neighbour from registers, the
    // others from the slot.
    auto gs_num = [&](auto Oc, const UD<T>* S, const SweepPlane<T>& Pb, const SweepPlane<T>& P,
                      const SweepPlane<T>& Pa) -> T {
        constexpr int O = decltype(Oc)::value;
        const UD<T>* So = S + O * RA + pe;          // same element, this pair
        const UD<T> ym = So[-NP], yp = So[NP];
        // z-neighbour outside the pair: element 1 of the pair to the left
        // (O = 0) or element 0 of the pair to the right (O = 1)
        const UD<T> zo = O ? S[pe + 1] : S[RA + pe - 1];
        const T Di = O ? P.D1 : P.D0;
        const T uzl = O ? P.u0 : zo.u, uzr = O ? zo.u : P.u1;
        const T Dzl = O ? P.D0 : zo.D, Dzr = O ? zo.D : P.D1;
        const T Dxm = O ? Pb.D1 : Pb.D0, Dxp = O ? Pa.D1 : Pa.D0;
        const T uxm = O ? Pb.u1 : Pb.u0, uxp = O ? Pa.u1 : Pa.u0;
        T num;
        if (HARM) {
            // harmonic mean; the smallest normal number in the denominator
            // keeps 0/0 (outside the grid, D = 0) finite and changes no
            // rounding for D >= 1e-30
            auto hf = [&](T Da, T Db) { return (Da * Db) / ((Da + Db) + T(1.17549435e-38)) * a.st.two_inv_h2; };
            num = (O ? P.q1 : P.q0) + hf(Di, Dxm) * uxm + hf(Di, Dxp) * uxp + hf(Di, ym.D) * ym.u + hf(Di, yp.D) * yp.u +
                  hf(Di, Dzl) * uzl + hf(Di, Dzr) * uzr;
        } else {
            // arithmetic mean: c_ij = (D_i + D_j) / (2 h^2), the common factor applied once
            const T s = ((Di + Dxm) * uxm + (Di + Dxp) * uxp) + ((Di + ym.D) * ym.u + (Di + yp.D) * yp.u) +
                        ((Di + Dzl) * uzl + (Di + Dzr) * uzr);
            num = (O ? P.q1 : P.q0) + s * a.st.half_inv_h2;
        }
        return num;
    };
    auto update = [&](auto Oc, const UD<T>* S, const SweepPlane<T>& Pb, const SweepPlane<T>& P,
                      const SweepPlane<T>& Pa) -> T {
        constexpr int O = decltype(Oc)::value;
        return gs_num(Oc, S, Pb, P, Pa) * (O ? P.w1 : P.w0);
    };

    // stage j at unrolled step K updates element O of plane s - j (slot (K - j) mod 8)
    // a wave none of whose lanes is in stage j's ring skips the stage (its
    // slot entries already hold the values it would write)
    bool wact0[4], wact1[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        wact0[j] = __builtin_amdgcn_ballot_w64(m0[j]) != 0;
        wact1[j] = __builtin_amdgcn_ballot_w64(m1[j]) != 0;
    }
    double nacc = 0.0;   // NORM: this lane's squared residuals of the input
    bool step_in = false;   // NORM: the current step's plane is one of the chunk's
    auto stage = [&](auto Oc, auto Jc, auto Kc, SweepPlane<T>& Pb, SweepPlane<T>& P, SweepPlane<T>& Pa) {
        constexpr int O = decltype(Oc)::value, J = decltype(Jc)::value, K = decltype(Kc)::value;
        if (!(O ? wact1[J] : wact0[J])) return;
        UD<T>* S = ring + ((K - J + 8) & 7) * 2 * RA;
        T v;
        if constexpr (NORM && J == 0) {
            const T num = gs_num(Oc, S, Pb, P, Pa);
            const T wi = O ? P.w1 : P.w0;
            const bool on = step_in && (O ? soff1 : soff0) != kOob;
            const T r = num - (O ? P.u1 : P.u0) / (on ? wi : T(1));
            nacc += on ? (double)r * (double)r : 0.0;
            v = num * wi;
        } else {
            // from a zero iterate every neighbour of the first colour is 0: the
            // update is w q (the same value the full formula gives)
            v = (ZERO_INIT && J == 0) ? (O ? P.q1 * P.w1 : P.q0 * P.w0) : update(Oc, S, Pb, P, Pa);
        }
        if (O) {
            P.u1 = m1[J] ? v : P.u1;
            if (J < 3 || DEFECT) S[RA + pe].u = P.u1;
        } else {
            P.u0 = m0[J] ? v : P.u0;
            if (J < 3 || DEFECT) S[pe].u = P.u0;
        }
    };
    // defect of plane s - 4 (final since step s - 1) at element O, the
    // colour of the first half-sweep: x-neighbour below from the slot of
    // plane s - 5, above from the registers of plane s - 3 (final after this
    // step's last stage)
    const bool dwave = __builtin_amdgcn_ballot_w64(soff0 != kOob || soff1 != kOob) != 0;
    auto defect = [&](auto Oc, auto Kc, int s, const SweepPlane<T>& Pm4, const SweepPlane<T>& Pm3) {
        if (!dwave) return;
        constexpr int O = decltype(Oc)::value, K = decltype(Kc)::value;
        const UD<T>* S4 = ring + ((K + 4) & 7) * 2 * RA;
        const UD<T> xm = ring[((K + 3) & 7) * 2 * RA + O * RA + pe];
        SweepPlane<T> Pb;
        Pb.u0 = Pb.u1 = xm.u;
        Pb.D0 = Pb.D1 = xm.D;
        const T num = gs_num(Oc, S4, Pb, Pm4, Pm3);
        // diagonal 1/w by the hardware reciprocal (1 ulp; the difference is
        // rounded in float32 anyway)
        const T r = num - (O ? Pm4.u1 * __builtin_amdgcn_rcpf(Pm4.w1) : Pm4.u0 * __builtin_amdgcn_rcpf(Pm4.w0));
        const int po = s - 4;
        if (po >= xa && po < xb) buf_store<T>(r, rR, (O ? soff1 : soff0) + po * plane_bytes);
    };
    auto stages = [&](auto Oc, auto Kc, SweepPlane<T>& Pm4, SweepPlane<T>& Pm3, SweepPlane<T>& Pm2,
                      SweepPlane<T>& Pm1, SweepPlane<T>& P0, SweepPlane<T>& Pp1) {
        stage(Oc, std::integral_constant<int, 0>(), Kc, Pm1, P0, Pp1);
        stage(Oc, std::integral_constant<int, 1>(), Kc, Pm2, Pm1, P0);
        stage(Oc, std::integral_constant<int, 2>(), Kc, Pm3, Pm2, Pm1);
        stage(Oc, std::integral_constant<int, 3>(), Kc, Pm4, Pm3, Pm2);
    };

    // with DEFECT, final values are needed on planes xa - 1 .. xb
    const int s0 = xa - 3 - (DEFECT ? 1 : 0), s_end = xb + 2 + (DEFECT ? 1 : 0);
    const int par0 = __builtin_amdgcn_readfirstlane((s0 + hp + a.order) & 1);   // element updated at step s0
    auto step = [&](auto Kc, int s, SweepPlane<T>& Pm4, SweepPlane<T>& Pm3, SweepPlane<T>& Pm2, SweepPlane<T>& Pm1,
                    SweepPlane<T>& P0, SweepPlane<T>& Pp1, SweepPlane<T>& Pp3) {
        constexpr int K = decltype(Kc)::value;
        UD<T>* S = ring + K * 2 * RA;
        S[pe] = UD<T>{P0.u0, P0.D0};
        S[RA + pe] = UD<T>{P0.u1, P0.D1};
        if (NORM) step_in = s >= xa && s < xb;
        lds_barrier();
        load(s + 3, Pp3);   // into the registers of plane s-5
        if (PROLONG) {
            add_coarse_lds(s + 1, Pp1);   // plane s+1, first used now
            if (cloader) {
                cring[(((s + 3) >> 1) & 3) * Sh::CPL + tid] = cg;   // coarse plane loaded at step s-1
                cg = coarse_plane((s + 4) >> 1);
            }
        }
        if (par0 ^ (K & 1)) {
            stages(std::integral_constant<int, 1>(), Kc, Pm4, Pm3, Pm2, Pm1, P0, Pp1);
            if (DEFECT) defect(std::integral_constant<int, 1>(), Kc, s, Pm4, Pm3);
        } else {
            stages(std::integral_constant<int, 0>(), Kc, Pm4, Pm3, Pm2, Pm1, P0, Pp1);
            if (DEFECT) defect(std::integral_constant<int, 0>(), Kc, s, Pm4, Pm3);
        }
        const int po = s - 3;   // final
        if (po >= xa && po < xb) {
            buf_store<T>(Pm3.u0, rO, soff0 + po * plane_bytes);
            buf_store<T>(Pm3.u1, rO, soff1 + po * plane_bytes);
        }
    };

    // register ring of eight planes, the march unrolled by eight so planes
    // never move between registers; plane p lives in R(p - s0 + 4 mod 8),
    // and step s loads plane s+3 into the registers plane s-5 held.
    SweepPlane<T> R0, R1, R2, R3, R4, R5, R6, R7;
    load(s0 - 4, R0);
    load(s0 - 3, R1);
    load(s0 - 2, R2);
    load(s0 - 1, R3);
    load(s0, R4);
    load(s0 + 1, R5);
    load(s0 + 2, R6);
    if (PROLONG) {   // planes up to s0 from memory; coarse planes of steps s0 and s0+1 into LDS
        SweepPlane<T>* Ps[] = {&R0, &R1, &R2, &R3, &R4};
        for (int i = 0; i < 5; i++) {
            Coarse C;
            load_coarse(s0 - 4 + i, C);
            add_coarse(C, *Ps[i]);
        }
        if (cloader) {
            for (int X = (s0 + 1) >> 1; X <= ((s0 + 2) >> 1); X++) cring[(X & 3) * Sh::CPL + tid] = coarse_plane(X);
            cg = coarse_plane((s0 + 3) >> 1);
        }
    }
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using I6 = std::integral_constant<int, 6>;
    using I7 = std::integral_constant<int, 7>;
    for (int s = s0; s <= s_end; s += 8) {
        step(I0(), s, R0, R1, R2, R3, R4, R5, R7);
        if (s + 1 > s_end) break;
        step(I1(), s + 1, R1, R2, R3, R4, R5, R6, R0);
        if (s + 2 > s_end) break;
        step(I2(), s + 2, R2, R3, R4, R5, R6, R7, R1);
        if (s + 3 > s_end) break;
        step(I3(), s + 3, R3, R4, R5, R6, R7, R0, R2);
        if (s + 4 > s_end) break;
        step(I4(), s + 4, R4, R5, R6, R7, R0, R1, R3);
        if (s + 5 > s_end) break;
        step(I5(), s + 5, R5, R6, R7, R0, R1, R2, R4);
        if (s + 6 > s_end) break;
        step(I6(), s + 6, R6, R7, R0, R1, R2, R3, R5);
        if (s + 7 > s_end) break;
        step(I7(), s + 7, R7, R0, R1, R2, R3, R4, R6);
    }
    if constexpr (NORM) {
        const double b = block_sum(nacc);
        if (tid == 0) a.partial[bid] = b;
    }
}

template <class T, int TY, int TZ, int MODE, bool HARM, bool DEFECT = false, bool NORM = false>
__global__ __launch_bounds__((Sweep2Shape<TY, TZ, DEFECT ? 5 : 4>::NT)) void k_rb_sweep2_col(SweepArgs<T> a) {
    rb_sweep2_body<T, TY, TZ, MODE, HARM, DEFECT, NORM>(a, blockIdx.x);
}

// Grouped form (one launch for several requests' passes).
template <class T, int TY, int TZ, int MODE, bool HARM, bool DEFECT = false, bool NORM = false>
__global__ __launch_bounds__((Sweep2Shape<TY, TZ, DEFECT ? 5 : 4>::NT)) void k_rb_sweep2_grp(const Group<SweepArgs<T>>* g) {
    int bid;
    const int m = group_member(g, &bid);
    if (bid < 0) return;
    const SweepArgs<T> a = g->a[m];
    rb_sweep2_body<T, TY, TZ, MODE, HARM, DEFECT, NORM>(a, bid);
}

}  // namespace dmgs
