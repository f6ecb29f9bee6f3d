// grid.hpp -- indexing and stencil helpers shared by the HIP kernels.
//
// Vertex-centred grid with N cells per axis: (N+1)^3 vertices, x slowest,
// z fastest, v = (x*(N+1) + y)*(N+1) + z.  Interior vertices (the unknowns)
// have all coordinates in [1, N-1]; the boundary layer holds the Dirichlet
// value of the iterate (g on the finest level, 0 for coarse corrections).
//
// The operator (paper, Eq. (maineq), second-order finite differences):
//   (A u)_i = sum_{6 neighbours j} c_ij (u_i - u_j) + mua_i u_i,
//   c_ij = D_f / h^2, D_f = (D_i + D_j)/2 (or the harmonic mean).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmgs {

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
    const int kXcd = 8;
    if (nblocks % kXcd) return b;
    return (b % kXcd) * (nblocks / kXcd) + b / kXcd;
}


// The same for any block count: XCD x (blocks b = x, x + 8, ...) takes the
// contiguous range of logical blocks [x*floor(nb/8) + min(x, nb%8), ...) of
// its size, a bijection of [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int kXcd = 8;
    const int x = b % kXcd, i = b / kXcd, q = nblocks / kXcd, r = nblocks % kXcd;
    return x * q + min(x, r) + i;
}

constexpr int kWave = 64;

// Grouped launches: one launch runs the same kernel for several requests.
// Member m owns the grid's blocks [start[m], start[m+1]) and runs with its
// own arguments a[m] on the first nblk[m] of them (block index within the
// member bid = blockIdx.x - start[m]); the host starts every member at a
// multiple of 8 blocks, so a member's blocks fall on the XCDs as in a
// launch of its own, and the blocks past nblk[m] exit at once.
constexpr int kGroupMax = 16;

template <class Args>
struct Group {
    int count;
    int start[kGroupMax + 1];
    int nblk[kGroupMax];
    Args a[kGroupMax];
};

// This block's member, and its block index within the member (-1: a
// padding block, which does nothing).
template <class Args>
__device__ __forceinline__ int group_member(const Group<Args>* g, int* bid) {
    const int b = blockIdx.x;
    int m = 0;
    while (m + 1 < g->count && b >= g->start[m + 1]) m++;
    const int i = b - g->start[m];
    *bid = i < g->nblk[m] ? i : -1;
    return m;
}

__host__ __device__ inline int64_t vidx(int n, int x, int y, int z) {
    return ((int64_t)x * n + y) * n + z;
}

__host__ __device__ inline bool is_interior(int N, int x, int y, int z) {
    return x > 0 && x < N && y > 0 && y < N && z > 0 && z < N;
}

// Per-level stencil constants in the arithmetic type T.
template <class T>
struct Stencil {
    T half_inv_h2;   // 1 / (2 h^2): arithmetic face mean
    T two_inv_h2;    // 2 / h^2: harmonic face mean
    int harmonic;
};

template <class T>
__device__ __forceinline__ T face_coef(T Da, T Db, const Stencil<T>& s) {
    return s.harmonic ? (Da * Db) / (Da + Db) * s.two_inv_h2 : (Da + Db) * s.half_inv_h2;
}

// Face coefficient with the face mean fixed at compile time.
template <bool HARM, class T>
__device__ __forceinline__ T face(T Da, T Db, const Stencil<T>& s) {
    if (HARM) return (Da * Db) / (Da + Db) * s.two_inv_h2;
    return (Da + Db) * s.half_inv_h2;
}

// Deterministic block sum of a double (wave64 shuffles, then LDS); result in
// thread 0.  blockDim.x must be a multiple of 64 and at most 1024.
__device__ inline double block_sum(double v) {
    __shared__ double wsum[16];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        int nw = blockDim.x / kWave;
        for (int i = 0; i < nw; i++) s += wsum[i];
    }
    __syncthreads();
    return s;
}

}  // namespace dmgs
