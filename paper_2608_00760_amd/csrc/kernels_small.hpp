// kernels_small.hpp -- the coarse end of the V-cycle in one workgroup.
//
// All levels from the first one whose arrays fit in LDS (N <= 16 in float32,
// N <= 8 in float64) down to the coarsest run inside a single workgroup: the
// iterate, right-hand side and coefficients of every such level live in LDS,
// each step of the cycle (red-black half-sweeps, defect, full-weighting
// restriction, prolongation) is one barrier-separated phase, and the coarsest
// level is solved exactly in float64 by a product with the inverse of its
// operator (formed once per coefficient set).  This replaces dozens of
// launches of a few microseconds each per cycle by one.
//
// The work of a phase is spread over the threads with power-of-two padded
// index maps (plane, row, column from shifts and masks).  The operator's
// diagonal is taken as 1/w from the inverse diagonal the smoother uses.  A
// level entered from a zero iterate starts its first half-sweep without
// neighbours (u = w q on the first colour), which is folded into the phase
// that produces q; the prolongated correction is added only to the colour
// the next half-sweep reads (the other colour is overwritten by it).
#pragma once
#include "grid.hpp"
#include "kernels_basic.hpp"

namespace dmgs {

constexpr int kSmallMaxLevels = 6;
constexpr int kSmallThreads = 1024;

template <class T>
struct SmallLevel {
    int N;
    int off;       // LDS offset (elements) of the level's arrays u, q, D, w (each nv long)
    int nv;        // (N+1)^3
    const T* D;    // level coefficient arrays, (N+1)^3
    const T* w;    // inverse diagonal
    Stencil<T> st;
};

template <class T>
struct SmallArgs {
    int nlev;                          // levels handled (first small level .. coarsest)
    SmallLevel<T> lev[kSmallMaxLevels];
    const T* q;                        // right-hand side on the first small level
    T* u;                              // result on the first small level (whole array written)
    const double* cinv;                // inverse of the coarsest operator (m x m, m = (Nc-1)^3 <= 8)
    int nu_pre, nu_post, order;
    int roff;                          // LDS offset of the defect scratch
};

// LDS layout: level i's u, q, D, w at offsets off_i + {0, 1, 2, 3} nv_i,
// levels in order, then the defect scratch (nv of the first level).
// Dynamic LDS available beside the kernel's own coarse-inverse array.
constexpr size_t kSmallLdsLimit = 160 * 1024 - 64 * sizeof(double);

template <class T>
__host__ __device__ inline size_t small_lds_bytes(const int* Ns, int nlev) {
    size_t b = 0, first = 0;
    for (int i = 0; i < nlev; i++) {
        size_t n = (size_t)Ns[i] + 1, nv = n * n * n;
        if (i == 0) first = nv;
        b += 4 * nv * sizeof(T);   // u, q, D, w
    }
    return b + first * sizeof(T);  // defect scratch
}

__device__ __forceinline__ int ilog2_ceil(int v) { return v <= 1 ? 0 : 32 - __builtin_clz(v - 1); }

template <class T, bool HARM>
__device__ __forceinline__ void small_vcycle_body(const SmallArgs<T>& a) {
    extern __shared__ __align__(16) unsigned char small_smem[];
    T* const base = reinterpret_cast<T*>(small_smem);
    // level arrays addressed from the LDS base (no pointer tables: they
    // would be indexed at run time and lose the address space)
    auto U = [&](int i) { return base + a.lev[i].off; };
    auto Q = [&](int i) { return base + a.lev[i].off + a.lev[i].nv; };
    auto D = [&](int i) { return base + a.lev[i].off + 2 * a.lev[i].nv; };
    auto W = [&](int i) { return base + a.lev[i].off + 3 * a.lev[i].nv; };
    T* const R = base + a.roff;
    const int tid = threadIdx.x;
    const int first = a.order ? 1 : 0;   // colour of the first half-sweep
    const bool pre1 = a.nu_pre > 0;        // the first half-sweep from zero is folded in

    // level arrays into LDS, with every global load issued before the first
    // LDS write (the first level has at most 17^3 vertices, the others at
    // most 9^3, one per thread); the first level starts its pre-smoothing
    // from zero, so its first half-sweep is u = w q on the first colour
    __shared__ double sinv[kCoarseMax * kCoarseMax];
    {
        constexpr int kPer = (17 * 17 * 17 + kSmallThreads - 1) / kSmallThreads;
        const int n0 = a.lev[0].N + 1, nv0 = a.lev[0].nv;
        const int Nc = a.lev[a.nlev - 1].N, mc = (Nc - 1) * (Nc - 1) * (Nc - 1);
        T d[kPer], w[kPer], q[kPer], dl[kSmallMaxLevels], wl[kSmallMaxLevels];
        double ci = 0.0;
        if (tid < mc * mc) ci = a.cinv[tid];
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const int v = tid + k * kSmallThreads;
            d[k] = v < nv0 ? a.lev[0].D[v] : T(0);
            w[k] = v < nv0 ? a.lev[0].w[v] : T(0);
            q[k] = v < nv0 ? a.q[v] : T(0);
        }
#pragma unroll
        for (int i = 1; i < kSmallMaxLevels; i++) {
            const bool in = i < a.nlev && tid < a.lev[i].nv;
            dl[i] = in ? a.lev[i].D[tid] : T(0);
            wl[i] = in ? a.lev[i].w[tid] : T(0);
        }
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const int v = tid + k * kSmallThreads;
            if (v < nv0) {
                D(0)[v] = d[k];
                W(0)[v] = w[k];
                Q(0)[v] = q[k];
                const int z = v % n0, y = (v / n0) % n0, x = v / (n0 * n0);
                U(0)[v] = (pre1 && ((x + y + z) & 1) == first) ? w[k] * q[k] : T(0);   // w = 0 on the boundary
            }
        }
#pragma unroll
        for (int i = 1; i < kSmallMaxLevels; i++) {
            if (i < a.nlev && tid < a.lev[i].nv) {
                D(i)[tid] = dl[i];
                W(i)[tid] = wl[i];
                Q(i)[tid] = T(0);
                U(i)[tid] = T(0);
            }
        }
        if (tid < mc * mc) sinv[tid] = ci;
    }
    __syncthreads();

    // thread map of the interior points of one colour: plane offset, row
    // and pair index from shifts; NP2 = pow2 >= N/2 pairs, NY2 = pow2 >= N-1 rows
    auto half_sweep = [&](int i, int colour) {
        const int N = a.lev[i].N, n = N + 1, sx = n * n;
        const int lz = ilog2_ceil(N / 2), ly = ilog2_ceil(N - 1), lp = lz + ly;
        const Stencil<T> st = a.lev[i].st;
        T* u = U(i);
        const T *q = Q(i), *Dl = D(i), *w = W(i);
        for (int it = tid; it < ((N - 1) << lp); it += kSmallThreads) {
            const int zz = it & ((1 << lz) - 1), y = 1 + ((it >> lz) & ((1 << ly) - 1)), x = 1 + (it >> lp);
            {
                const int z = 1 + ((x + y + 1 + colour) & 1) + 2 * zz;
                if (y > N - 1 || z > N - 1) continue;
                const int v = (x * n + y) * n + z;
                const T Di = Dl[v];
                const T num = q[v] + face<HARM>(Di, Dl[v + sx], st) * u[v + sx] + face<HARM>(Di, Dl[v - sx], st) * u[v - sx] +
                              face<HARM>(Di, Dl[v + n], st) * u[v + n] + face<HARM>(Di, Dl[v - n], st) * u[v - n] +
                              face<HARM>(Di, Dl[v + 1], st) * u[v + 1] + face<HARM>(Di, Dl[v - 1], st) * u[v - 1];
                u[v] = num * w[v];
            }
        }
        __syncthreads();
    };
    // r = q - A u on the interior (the restriction reads interior points only);
    // the diagonal of A is 1/w
    auto defect = [&](int i) {
        const int N = a.lev[i].N, n = N + 1, sx = n * n;
        const int lz = ilog2_ceil(N - 1), lp = 2 * lz;
        const Stencil<T> st = a.lev[i].st;
        const T *u = U(i), *q = Q(i), *Dl = D(i), *w = W(i);
        for (int it = tid; it < ((N - 1) << lp); it += kSmallThreads) {
            const int z = 1 + (it & ((1 << lz) - 1)), y = 1 + ((it >> lz) & ((1 << lz) - 1)), x = 1 + (it >> lp);
            if (y <= N - 1 && z <= N - 1) {
                const int v = (x * n + y) * n + z;
                const T Di = Dl[v];
                const T off = face<HARM>(Di, Dl[v + sx], st) * u[v + sx] + face<HARM>(Di, Dl[v - sx], st) * u[v - sx] +
                              face<HARM>(Di, Dl[v + n], st) * u[v + n] + face<HARM>(Di, Dl[v - n], st) * u[v - n] +
                              face<HARM>(Di, Dl[v + 1], st) * u[v + 1] + face<HARM>(Di, Dl[v - 1], st) * u[v - 1];
                R[v] = q[v] - (u[v] / w[v] - off);
            }
        }
        __syncthreads();
    };
    // q_{i+1} = R r on the coarse interior, and the first half-sweep of
    // level i+1 from its zero iterate (u = w q on the first colour)
    auto restrict_start = [&](int i) {
        const int N = a.lev[i].N, n = N + 1;
        const int Nc = N / 2, nc = Nc + 1;
        const int lz = ilog2_ceil(Nc - 1), lp = 2 * lz;
        T *qc = Q(i + 1), *uc = U(i + 1);
        const T* wc = W(i + 1);
        for (int it = tid; it < ((Nc - 1) << lp); it += kSmallThreads) {
            const int Z = 1 + (it & ((1 << lz) - 1)), Y = 1 + ((it >> lz) & ((1 << lz) - 1)), X = 1 + (it >> lp);
            if (Y <= Nc - 1 && Z <= Nc - 1) {
                T s = T(0);
                for (int da = -1; da <= 1; da++)
                    for (int db = -1; db <= 1; db++) {
                        const T wab = T((2 - abs(da)) * (2 - abs(db)));
                        const T* row = R + ((2 * X + da) * n + (2 * Y + db)) * n + 2 * Z;
                        s += wab * (row[-1] + T(2) * row[0] + row[1]);
                    }
                s *= T(1.0 / 64.0);
                const int V = (X * nc + Y) * nc + Z;
                qc[V] = s;
                uc[V] = (pre1 && ((X + Y + Z) & 1) == first) ? wc[V] * s : T(0);
            }
        }
        __syncthreads();
    };
    // u_i += I u_{i+1} on the interior points of one colour
    auto prolong_add = [&](int i, int colour) {
        const int N = a.lev[i].N, n = N + 1, nc = N / 2 + 1;
        const int lz = ilog2_ceil(N / 2), ly = ilog2_ceil(N - 1), lp = lz + ly;
        T* u = U(i);
        const T* ec = U(i + 1);
        for (int it = tid; it < ((N - 1) << lp); it += kSmallThreads) {
            const int zz = it & ((1 << lz) - 1), y = 1 + ((it >> lz) & ((1 << ly) - 1)), x = 1 + (it >> lp);
            {
                const int z = 1 + ((x + y + 1 + colour) & 1) + 2 * zz;
                if (y > N - 1 || z > N - 1) continue;
                const int x0 = x >> 1, y0 = y >> 1, z0 = z >> 1;
                const int x1 = x0 + (x & 1), y1 = y0 + (y & 1), z1 = z0 + (z & 1);
                auto E = [&](int X, int Y, int Z) { return ec[(X * nc + Y) * nc + Z]; };
                const T s = E(x0, y0, z0) + E(x0, y0, z1) + E(x0, y1, z0) + E(x0, y1, z1) + E(x1, y0, z0) +
                            E(x1, y0, z1) + E(x1, y1, z0) + E(x1, y1, z1);
                u[(x * n + y) * n + z] += s * T(0.125);
            }
        }
        __syncthreads();
    };
    // nu sweeps, the first half-sweep of the first one already done when skip1
    auto sweeps = [&](int i, int count, bool skip1) {
        for (int c = 0; c < count; c++) {
            if (!(skip1 && c == 0)) half_sweep(i, first);
            half_sweep(i, 1 - first);
        }
    };

    const int L = a.nlev;
    for (int i = 0; i < L - 1; i++) {   // down: every level starts from a zero iterate
        sweeps(i, a.nu_pre, pre1);
        defect(i);
        restrict_start(i);
    }
    {   // coarsest level: u = A^-1 q on the interior unknowns (x, y, z order)
        const int Nc = a.lev[L - 1].N, Nm = Nc - 1, mc = Nm * Nm * Nm, nc = Nc + 1;
        auto vid = [&](int c) { return ((1 + c / (Nm * Nm)) * nc + 1 + (c / Nm) % Nm) * nc + 1 + c % Nm; };
        if (tid < mc) {
            const T* qc = Q(L - 1);
            double acc = 0.0;
            for (int c = 0; c < mc; c++) acc += sinv[tid * mc + c] * (double)qc[vid(c)];
            U(L - 1)[vid(tid)] = (T)acc;
        }
        __syncthreads();
    }
    for (int i = L - 2; i >= 0; i--) {  // up
        // the next half-sweep updates the first colour from the second
        // colour's values; with no post-smoothing both colours are corrected
        prolong_add(i, 1 - first);
        if (a.nu_post == 0) prolong_add(i, first);
        sweeps(i, a.nu_post, false);
    }
    const int n0 = a.lev[0].N + 1, nv0 = n0 * n0 * n0;
    for (int v = tid; v < nv0; v += kSmallThreads) a.u[v] = U(0)[v];
}

template <class T, bool HARM>
__global__ __launch_bounds__(kSmallThreads) void k_small_vcycle(SmallArgs<T> a) {
    small_vcycle_body<T, HARM>(a);
}

// Grouped form: one workgroup per member.
template <class T, bool HARM>
__global__ __launch_bounds__(kSmallThreads) void k_small_grp(const Group<SmallArgs<T>>* g) {
    int bid;
    const int m = group_member(g, &bid);
    if (bid < 0) return;
    const SmallArgs<T> a = g->a[m];
    small_vcycle_body<T, HARM>(a);
}

}  // namespace dmgs
