// kernels_small.hpp -- the coarse end of the V-cycle in one workgroup.
//
// All levels from the first one whose arrays fit in LDS (N <= 16 in float32,
// N <= 8 in float64) down to the coarsest run inside a single workgroup: the
// iterate, right-hand side and coefficients of every such level live in LDS,
// each step of the cycle (red-black half-sweeps, defect, full-weighting
// restriction, prolongation) is one barrier-separated phase, and the coarsest
// level is solved exactly in float64 by one thread.  This replaces dozens of
// launches of a few microseconds each per cycle by one.
#pragma once
#include "grid.hpp"
#include "kernels_basic.hpp"

namespace dmgs {

constexpr int kSmallMaxLevels = 6;
constexpr int kSmallThreads = 1024;

template <class T>
struct SmallLevel {
    int N;
    const T* D;    // level coefficient arrays, (N+1)^3
    const T* w;    // inverse diagonal
    const T* mu;
    Stencil<T> st;
};

template <class T>
struct SmallArgs {
    int nlev;                          // levels handled (first small level .. coarsest)
    SmallLevel<T> lev[kSmallMaxLevels];
    const T* q;                        // right-hand side on the first small level
    T* u;                              // result on the first small level (whole array written)
    const double* Dc;                  // coarsest level coefficients in float64
    const double* muc;
    Stencil<double> stc;
    int nu_pre, nu_post, order;
};

template <class T>
__host__ __device__ inline size_t small_lds_bytes(const int* Ns, int nlev) {
    size_t b = 0, first = 0;
    for (int i = 0; i < nlev; i++) {
        size_t n = (size_t)Ns[i] + 1, nv = n * n * n;
        if (i == 0) first = nv;
        b += 5 * nv * sizeof(T);   // u, q, D, w, mu
    }
    return b + first * sizeof(T);  // defect scratch
}

template <class T, bool HARM>
__global__ __launch_bounds__(kSmallThreads) void k_small_vcycle(SmallArgs<T> a) {
    extern __shared__ __align__(16) unsigned char small_smem[];
    T* base = reinterpret_cast<T*>(small_smem);
    T *U[kSmallMaxLevels], *Q[kSmallMaxLevels], *D[kSmallMaxLevels], *W[kSmallMaxLevels], *M[kSmallMaxLevels];
    const int tid = threadIdx.x;
    {
        T* p = base;
        for (int i = 0; i < a.nlev; i++) {
            int n = a.lev[i].N + 1, nv = n * n * n;
            U[i] = p; p += nv;
            Q[i] = p; p += nv;
            D[i] = p; p += nv;
            W[i] = p; p += nv;
            M[i] = p; p += nv;
        }
        for (int i = a.nlev; i < kSmallMaxLevels; i++) U[i] = Q[i] = D[i] = W[i] = M[i] = nullptr;
    }
    T* R = base;   // defect scratch follows the last level
    for (int i = 0; i < a.nlev; i++) {
        const int n = a.lev[i].N + 1;
        R += 5 * n * n * n;
    }
    for (int i = 0; i < a.nlev; i++) {
        const int n = a.lev[i].N + 1, nv = n * n * n;
        for (int v = tid; v < nv; v += kSmallThreads) {
            U[i][v] = T(0);
            Q[i][v] = i == 0 ? a.q[v] : T(0);
            D[i][v] = a.lev[i].D[v];
            W[i][v] = a.lev[i].w[v];
            M[i][v] = a.lev[i].mu[v];
        }
    }
    __syncthreads();

    auto sweep_half = [&](int i, int colour) {
        const int N = a.lev[i].N, n = N + 1, Ni = N - 1, M2 = N / 2;
        const Stencil<T> st = a.lev[i].st;
        T* u = U[i];
        const T *q = Q[i], *Dl = D[i], *w = W[i];
        const int total = Ni * Ni * M2;
        for (int t = tid; t < total; t += kSmallThreads) {
            const int zz = t % M2, r = t / M2;
            const int y = 1 + r % Ni, x = 1 + r / Ni;
            const int z = 1 + ((x + y + 1 + colour) & 1) + 2 * zz;
            if (z > N - 1) continue;
            const int v = (x * n + y) * n + z, sx = n * n;
            const T Di = Dl[v];
            const T num = q[v] + face<HARM>(Di, Dl[v + sx], st) * u[v + sx] + face<HARM>(Di, Dl[v - sx], st) * u[v - sx] +
                          face<HARM>(Di, Dl[v + n], st) * u[v + n] + face<HARM>(Di, Dl[v - n], st) * u[v - n] +
                          face<HARM>(Di, Dl[v + 1], st) * u[v + 1] + face<HARM>(Di, Dl[v - 1], st) * u[v - 1];
            u[v] = num * w[v];
        }
        __syncthreads();
    };
    auto sweeps = [&](int i, int count) {
        const int first = a.order ? 1 : 0;
        for (int c = 0; c < count; c++) {
            sweep_half(i, first);
            sweep_half(i, 1 - first);
        }
    };
    auto defect_restrict = [&](int i) {
        const int N = a.lev[i].N, n = N + 1, sx = n * n;
        const Stencil<T> st = a.lev[i].st;
        const T *u = U[i], *q = Q[i], *Dl = D[i], *mu = M[i];
        const int nv = n * n * n;
        for (int v = tid; v < nv; v += kSmallThreads) {
            const int z = v % n, y = (v / n) % n, x = v / sx;
            T r = T(0);
            if (is_interior(N, x, y, z)) {
                const T Di = Dl[v], ui = u[v];
                const T Au = mu[v] * ui + face<HARM>(Di, Dl[v + sx], st) * (ui - u[v + sx]) +
                             face<HARM>(Di, Dl[v - sx], st) * (ui - u[v - sx]) + face<HARM>(Di, Dl[v + n], st) * (ui - u[v + n]) +
                             face<HARM>(Di, Dl[v - n], st) * (ui - u[v - n]) + face<HARM>(Di, Dl[v + 1], st) * (ui - u[v + 1]) +
                             face<HARM>(Di, Dl[v - 1], st) * (ui - u[v - 1]);
                r = q[v] - Au;
            }
            R[v] = r;
        }
        __syncthreads();
        const int Nc = N / 2, nc = Nc + 1, nvc = nc * nc * nc;
        T* qc = Q[i + 1];
        for (int V = tid; V < nvc; V += kSmallThreads) {
            const int Z = V % nc, Y = (V / nc) % nc, X = V / (nc * nc);
            T s = T(0);
            if (is_interior(Nc, X, Y, Z)) {
                for (int da = -1; da <= 1; da++)
                    for (int db = -1; db <= 1; db++) {
                        const T wab = T((2 - abs(da)) * (2 - abs(db)));
                        const T* row = R + ((2 * X + da) * n + (2 * Y + db)) * n + 2 * Z;
                        s += wab * (row[-1] + T(2) * row[0] + row[1]);
                    }
                s *= T(1.0 / 64.0);
            }
            qc[V] = s;
        }
        __syncthreads();
    };
    auto prolong_add = [&](int i) {
        const int N = a.lev[i].N, n = N + 1, nc = N / 2 + 1;
        T* u = U[i];
        const T* ec = U[i + 1];
        const int nv = n * n * n;
        for (int v = tid; v < nv; v += kSmallThreads) {
            const int z = v % n, y = (v / n) % n, x = v / (n * n);
            if (!is_interior(N, x, y, z)) continue;
            const int x0 = x >> 1, y0 = y >> 1, z0 = z >> 1;
            const int x1 = x0 + (x & 1), y1 = y0 + (y & 1), z1 = z0 + (z & 1);
            auto E = [&](int X, int Y, int Z) { return ec[(X * nc + Y) * nc + Z]; };
            const T s = E(x0, y0, z0) + E(x0, y0, z1) + E(x0, y1, z0) + E(x0, y1, z1) + E(x1, y0, z0) + E(x1, y0, z1) +
                        E(x1, y1, z0) + E(x1, y1, z1);
            u[v] += s * T(0.125);
        }
        __syncthreads();
    };

    const int L = a.nlev;
    for (int i = 0; i < L - 1; i++) {   // down: coarse iterates start from zero
        sweeps(i, a.nu_pre);
        defect_restrict(i);
    }
    if (tid == 0) dense_exact_solve(Q[L - 1], U[L - 1], a.Dc, a.muc, a.lev[L - 1].N, a.stc);
    __syncthreads();
    for (int i = L - 2; i >= 0; i--) {  // up
        prolong_add(i);
        sweeps(i, a.nu_post);
    }
    const int n0 = a.lev[0].N + 1, nv0 = n0 * n0 * n0;
    for (int v = tid; v < nv0; v += kSmallThreads) a.u[v] = U[0][v];
}

}  // namespace dmgs
