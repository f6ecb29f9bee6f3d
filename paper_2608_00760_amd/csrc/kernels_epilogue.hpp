// kernels_epilogue.hpp -- the response and likelihood epilogue (Sec. 2.5).
//
// Elementwise passes over the finest level of a plan (3D or 2D): the noise
// model's weights (Eq. (noise) with the edge mask), and the fused epilogue
// of a likelihood evaluation: L_e = mua rho, the data residual, the
// partial sums of H = 1/2 sum w (d - L_e)^2 and of the number of kept
// voxels, and the cotangent dH/drho = mua w (mua rho - d) that seeds the
// pull-back.  Reductions are deterministic two-stage sums (k_sum_partials).
#pragma once
#include <cfloat>
#include "kernels_basic.hpp"

namespace dmgs {

// vertex counts per axis, fastest axis first (an axis of count 1 is absent:
// two-dimensional grids)
struct VertDims {
    int n[3];
};

// distance of vertex v to the nearest face of the grid
__device__ __forceinline__ int face_depth(int64_t v, const VertDims& g) {
    int d = 1 << 30;
    for (int a = 0; a < 3; a++) {
        const int n = g.n[a];
        if (n <= 1) continue;
        const int c = (int)(v % n);
        v /= n;
        d = min(d, min(c, n - 1 - c));
    }
    return d;
}

// block maximum (wave64 shuffles, then LDS); result in thread 0
__device__ inline double block_max(double v) {
    __shared__ double wmax[16];
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, kWave));
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) wmax[w] = v;
    __syncthreads();
    double m = -DBL_MAX;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) m = fmax(m, wmax[i]);
    __syncthreads();
    return m;
}

// partial[block] = max of a over the block's share of [0, nv)
__global__ void k_max_partials(const double* __restrict__ a, int64_t nv, double* __restrict__ partial) {
    double m = -DBL_MAX;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, a[i]);
    const double b = block_max(m);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// w = 1 / sigma^2, sigma = max(rel Le, floor_frac max Le), on vertices at
// least `mask` from every face (0 elsewhere, and where sigma <= 0).  Every
// block reduces the npart partial maxima itself.
__global__ void k_noise_weights(const double* __restrict__ Le, const double* __restrict__ partial, int npart,
                                int64_t nv, VertDims g, int mask, double rel, double floor_frac,
                                double* __restrict__ w) {
    __shared__ double smax;
    double m = -DBL_MAX;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) m = fmax(m, partial[i]);
    m = block_max(m);
    if (threadIdx.x == 0) smax = m;
    __syncthreads();
    const double floor_sigma = floor_frac * smax;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const double sigma = fmax(rel * Le[v], floor_sigma);
        w[v] = (face_depth(v, g) >= mask && sigma > 0.0) ? 1.0 / (sigma * sigma) : 0.0;
    }
}

// rhobar = mua w (mua rho - d) on interior vertices (0 on the boundary);
// partial[b] = sum of w (d - mua rho)^2 and partial[nblocks + b] = number of
// vertices with w > 0 over the block's interior vertices.
__global__ void k_likelihood_epilogue(const double* __restrict__ rho, const double* __restrict__ mu,
                                      const double* __restrict__ d, const double* __restrict__ w, int64_t nv,
                                      VertDims g, double* __restrict__ rhobar, double* __restrict__ partial) {
    double acc = 0.0, cnt = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        if (face_depth(v, g) < 1) {
            rhobar[v] = 0.0;
            continue;
        }
        const double wv = w[v], m = mu[v];
        const double res = m * rho[v] - d[v];
        rhobar[v] = m * wv * res;
        acc += wv * res * res;
        cnt += wv > 0.0 ? 1.0 : 0.0;
    }
    const double s = block_sum(acc);
    const double c = block_sum(cnt);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        partial[gridDim.x + blockIdx.x] = c;
    }
}

// gmu += w (mua rho - d) mua rho on interior vertices: log mua enters L_e
// directly as well as through the operator
__global__ void k_likelihood_direct(const double* __restrict__ rho, const double* __restrict__ mu,
                                    const double* __restrict__ d, const double* __restrict__ w, int64_t nv,
                                    VertDims g, double* __restrict__ gmu) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        if (face_depth(v, g) < 1) continue;
        const double l = mu[v] * rho[v];
        gmu[v] += w[v] * (l - d[v]) * l;
    }
}

}  // namespace dmgs
