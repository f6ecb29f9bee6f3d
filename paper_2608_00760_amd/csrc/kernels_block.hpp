// kernels_block.hpp -- whole smoothing phases of a mid-size level in 3D
// blocks (float32 corrections, zero Dirichlet boundary, two sweeps).
//
// On levels of a few hundred thousand vertices the marching kernels have too
// little parallelism and each phase needs several launches.  Here every
// workgroup owns a B^3 block of interior vertices, loads the block plus a
// halo of R vertices into LDS and runs one whole phase of the V-cycle there:
//
//   pre   two red-black sweeps (from zero or from u_in), then the defect
//         r = q - A u on the block plus a ring of 1 and its full-weighting
//         restriction to the coarse vertices 2X inside the block (R = 6);
//   post  u_in plus the trilinear prolongation of the coarse correction,
//         then two red-black sweeps (R = 4).
//
// The four colour updates of the two sweeps are applied on shrinking
// regions -- the block plus a ring of s+3, s+2, s+1, s (s = 2 before a
// defect, 0 otherwise) -- so every value the block's output depends on is
// computed in the block (neighbouring blocks recompute the rings).  Vertices
// outside the grid are loaded as 0 and never updated; grid boundary vertices
// keep their value (0 for corrections).
#pragma once
#include "kernels_stream.hpp"

namespace dmgs {

enum BlockMode { kBlockPreZero = 0, kBlockPre = 1, kBlockPost = 2 };

template <class T>
struct BlockArgs {
    const T* u_in;   // iterate (kBlockPre, kBlockPost)
    T* u_out;        // iterate after the phase (block interiors written)
    const T* q;
    const T* D;
    const T* w;      // inverse diagonal (0 on the boundary)
    const T* ec;     // coarse correction (kBlockPost)
    T* qc;           // restricted defect (pre modes; coarse interior written)
    int N;
    int nb;          // blocks per axis
    int order;       // colour of the first half-sweep
    Stencil<T> st;
};

template <int B, int MODE>
struct BlockShape {
    static constexpr bool PRE = MODE != kBlockPost;
    static constexpr int S0 = PRE ? 2 : 0;   // ring of the last colour update
    static constexpr int R = S0 + 4;         // loaded halo
    static constexpr int S = B + 2 * R;      // box side
    static constexpr int V = S * S * S;
    static constexpr int RB = B + 2;         // defect region side (ring 1)
    static constexpr size_t lds_bytes(size_t tsize) { return (4 * (size_t)V + (PRE ? (size_t)RB * RB * RB : 0)) * tsize; }
};

constexpr int kBlockThreads = 1024;

template <class T, int B, int MODE, bool HARM>
__device__ __forceinline__ void block_pass_body(const BlockArgs<T>& a, const int bid) {
    using Sh = BlockShape<B, MODE>;
    constexpr int R = Sh::R, S = Sh::S, V = Sh::V, S0 = Sh::S0;
    extern __shared__ __align__(16) unsigned char block_smem[];
    T* const lu = reinterpret_cast<T*>(block_smem);
    T* const lD = lu + V;
    T* const lq = lu + 2 * V;
    T* const lw = lu + 3 * V;
    T* const lr = lu + 4 * V;   // defect (pre)
    const int N = a.N, n = N + 1, tid = threadIdx.x;
    const int bx = bid / (a.nb * a.nb), by = (bid / a.nb) % a.nb, bz = bid % a.nb;
    const int ox = 1 + bx * B, oy = 1 + by * B, oz = 1 + bz * B;   // block origin (grid coordinates)
    const int bxg = ox - R, byg = oy - R, bzg = oz - R;             // box origin
    const int first = a.order;

    // load the box: vertices outside [0, N]^3 read as 0 (buffer loads at an
    // offset past the field); every load of a thread is issued before its
    // first LDS write
    const int ncv = N / 2 + 1;
    const int fbytes = n * n * n * (int)sizeof(T), cbytes = ncv * ncv * ncv * (int)sizeof(T);
    const auto rU = field_rsrc(a.u_in, MODE == kBlockPreZero ? 0 : fbytes), rD = field_rsrc(a.D, fbytes);
    const auto rQ = field_rsrc(a.q, fbytes), rW = field_rsrc(a.w, fbytes);
    const auto rC = field_rsrc(a.ec, MODE == kBlockPost ? cbytes : 0);
    {
        constexpr int PER = (V + kBlockThreads - 1) / kBlockThreads;
        T ru[PER], rd[PER], rq[PER], rw[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int i = tid + k * kBlockThreads;
            const int z = i % S, y = (i / S) % S, x = i / (S * S);
            const int gx = bxg + x, gy = byg + y, gz = bzg + z;
            const bool in = i < V && gx >= 0 && gx <= N && gy >= 0 && gy <= N && gz >= 0 && gz <= N;
            const int g = in ? ((gx * n + gy) * n + gz) * (int)sizeof(T) : kOob;
            rd[k] = buf_load<T>(rD, g);
            rq[k] = buf_load<T>(rQ, g);
            rw[k] = buf_load<T>(rW, g);
            ru[k] = MODE == kBlockPreZero ? T(0) : buf_load<T>(rU, g);
            if (MODE == kBlockPost) {
                // trilinear prolongation of the coarse correction (0 on the coarse boundary;
                // fine boundary vertices get none)
                const bool ip = in && is_interior(N, gx, gy, gz);
                const int x0 = gx >> 1, y0 = gy >> 1, z0 = gz >> 1;
                const int dx = (gx & 1) * ncv * ncv, dy = (gy & 1) * ncv, dz = gz & 1;
                const int c0 = ip ? ((x0 * ncv + y0) * ncv + z0) * (int)sizeof(T) : kOob;
                constexpr int e = (int)sizeof(T);
                const T s = ((buf_load<T>(rC, c0) + buf_load<T>(rC, c0 + dz * e)) +
                             (buf_load<T>(rC, c0 + dy * e) + buf_load<T>(rC, c0 + (dy + dz) * e))) +
                            ((buf_load<T>(rC, c0 + dx * e) + buf_load<T>(rC, c0 + (dx + dz) * e)) +
                             (buf_load<T>(rC, c0 + (dx + dy) * e) + buf_load<T>(rC, c0 + (dx + dy + dz) * e)));
                ru[k] += s * T(0.125);
            }
        }
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int i = tid + k * kBlockThreads;
            if (i < V) {
                lu[i] = ru[k];
                lD[i] = rd[k];
                lq[i] = rq[k];
                lw[i] = rw[k];
            }
        }
    }
    __syncthreads();

    // one colour update on the block plus a ring of r: interior grid vertices of colour c
    auto colour_update = [&](auto Rc, int c) {
        constexpr int r = decltype(Rc)::value;
        constexpr int s = B + 2 * r, half = s / 2, cnt = s * s * half, lo = R - r;
        for (int it = tid; it < cnt; it += kBlockThreads) {
            const int zz = it % half, y = lo + (it / half) % s, x = lo + it / (half * s);
            const int gx = bxg + x, gy = byg + y;
            // z of colour c in this row: (gx + gy + gz) mod 2 = c
            const int z = lo + 2 * zz + ((gx + gy + bzg + lo + c) & 1);
            const int gz = bzg + z;
            if (!is_interior(N, gx, gy, gz) || z >= lo + s) continue;
            const int v = (x * S + y) * S + z;
            const T Di = lD[v];
            const T num = lq[v] + face<HARM>(Di, lD[v + S * S], a.st) * lu[v + S * S] +
                          face<HARM>(Di, lD[v - S * S], a.st) * lu[v - S * S] + face<HARM>(Di, lD[v + S], a.st) * lu[v + S] +
                          face<HARM>(Di, lD[v - S], a.st) * lu[v - S] + face<HARM>(Di, lD[v + 1], a.st) * lu[v + 1] +
                          face<HARM>(Di, lD[v - 1], a.st) * lu[v - 1];
            lu[v] = num * lw[v];
        }
        __syncthreads();
    };
    colour_update(std::integral_constant<int, S0 + 3>(), first);
    colour_update(std::integral_constant<int, S0 + 2>(), 1 - first);
    colour_update(std::integral_constant<int, S0 + 1>(), first);
    colour_update(std::integral_constant<int, S0>(), 1 - first);

    // block interior to memory
    for (int i = tid; i < B * B * B; i += kBlockThreads) {
        const int z = i % B, y = (i / B) % B, x = i / (B * B);
        const int gx = ox + x, gy = oy + y, gz = oz + z;
        if (gx <= N - 1 && gy <= N - 1 && gz <= N - 1)
            a.u_out[((int64_t)gx * n + gy) * n + gz] = lu[((x + R) * S + (y + R)) * S + (z + R)];
    }

    if constexpr (Sh::PRE) {
        // defect on the block plus a ring of 1 (diagonal 1/w), 0 outside the interior
        constexpr int RB = Sh::RB, lo = R - 1;
        for (int i = tid; i < RB * RB * RB; i += kBlockThreads) {
            const int z = lo + i % RB, y = lo + (i / RB) % RB, x = lo + i / (RB * RB);
            const int gx = bxg + x, gy = byg + y, gz = bzg + z;
            T r = T(0);
            if (is_interior(N, gx, gy, gz)) {
                const int v = (x * S + y) * S + z;
                const T Di = lD[v];
                const T off = face<HARM>(Di, lD[v + S * S], a.st) * lu[v + S * S] +
                              face<HARM>(Di, lD[v - S * S], a.st) * lu[v - S * S] + face<HARM>(Di, lD[v + S], a.st) * lu[v + S] +
                              face<HARM>(Di, lD[v - S], a.st) * lu[v - S] + face<HARM>(Di, lD[v + 1], a.st) * lu[v + 1] +
                              face<HARM>(Di, lD[v - 1], a.st) * lu[v - 1];
                r = lq[v] - (lu[v] / lw[v] - off);
            }
            lr[i] = r;
        }
        __syncthreads();
        // coarse vertices X with 2X in the block (block origins are odd: 2X = o + 1 + 2i)
        constexpr int BC = B / 2;
        const int Nc = N / 2;
        for (int i = tid; i < BC * BC * BC; i += kBlockThreads) {
            const int iz = i % BC, iy = (i / BC) % BC, ix = i / (BC * BC);
            const int X = (ox + 1) / 2 + ix, Y = (oy + 1) / 2 + iy, Z = (oz + 1) / 2 + iz;
            if (X > Nc - 1 || Y > Nc - 1 || Z > Nc - 1) continue;
            // fine 2X relative to the defect region origin (grid ox - 1)
            const int fx = 2 * X - (ox - 1), fy = 2 * Y - (oy - 1), fz = 2 * Z - (oz - 1);
            T sacc = T(0);
            for (int da = -1; da <= 1; da++)
                for (int db = -1; db <= 1; db++) {
                    const T wab = T((2 - abs(da)) * (2 - abs(db)));
                    const T* row = lr + ((fx + da) * RB + (fy + db)) * RB + fz;
                    sacc += wab * (row[-1] + T(2) * row[0] + row[1]);
                }
            a.qc[((int64_t)X * ncv + Y) * ncv + Z] = sacc * T(1.0 / 64.0);
        }
    }
}

template <class T, int B, int MODE, bool HARM>
__global__ __launch_bounds__(kBlockThreads) void k_block_pass(BlockArgs<T> a) {
    block_pass_body<T, B, MODE, HARM>(a, blockIdx.x);
}

template <class T, int B, int MODE, bool HARM>
__global__ __launch_bounds__(kBlockThreads) void k_block_grp(const Group<BlockArgs<T>>* g) {
    int bid;
    const int m = group_member(g, &bid);
    if (bid < 0) return;
    const BlockArgs<T> a = g->a[m];
    block_pass_body<T, B, MODE, HARM>(a, bid);
}

}  // namespace dmgs
