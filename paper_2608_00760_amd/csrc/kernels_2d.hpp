// kernels_2d.hpp -- kernels of the two-dimensional (five-point) variant.
//
// Grid: N cells per axis, (N+1)^2 vertices, x slowest, y fastest,
// v = x*(N+1) + y; interior vertices have both coordinates in [1, N-1].
// The operator is the two-dimensional form of Eq. (maineq):
//   (A u)_i = sum over the 4 neighbours j of c_ij (u_i - u_j) + mua_i u_i,
//   c_ij = D_f / h^2 with the arithmetic (or harmonic) face mean,
// red = (x + y) even, restriction (1/16)(1,2,1) x (1,2,1), bilinear
// prolongation, coefficients coarsened by full weighting (injection on the
// boundary) -- the readings of the three-dimensional solver.
//
// Every kernel here is float64 and memory-bound.  Kernels that read
// neighbouring rows take one item per thread over a grid of whole blocks
// rounded up to a multiple of 8, remapped so that each XCD walks a
// contiguous band of rows (the rows it reads twice stay in its L2).
#pragma once
#include "grid.hpp"
#include "kernels_basic.hpp"

namespace dmgs {

__device__ __forceinline__ bool interior2(int N, int x, int y) { return x > 0 && x < N && y > 0 && y < N; }

__device__ __forceinline__ int64_t item_of_thread2() {
    return (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
}

// ---------------------------------------------------------------------------
// Coefficients.

__global__ void k2_validate(const double* __restrict__ D, const double* __restrict__ mu, int N, int* __restrict__ bad) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    int b = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(v / n), y = (int)(v % n);
        if (!coef_ok(D[v], mu[v], interior2(N, x, y))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

__global__ void k2_exp_validate(const double* __restrict__ logD, const double* __restrict__ logmu,
                                double* __restrict__ D, double* __restrict__ mu, int N, int* __restrict__ bad) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    int b = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(v / n), y = (int)(v % n);
        const double d = exp(logD[v]), m = exp(logmu[v]);
        D[v] = d;
        mu[v] = m;
        if (!coef_ok(d, m, interior2(N, x, y))) b = 1;
    }
    if (b) atomicOr(bad, 1);
}

// sum over a, b in {-1, 0, 1} of (2 - |a|)(2 - |b|) f[2X + a, 2Y + b] / 16
__device__ __forceinline__ double full_weight2(const double* __restrict__ f, int nf, int X, int Y) {
    double s = 0.0;
    for (int a = -1; a <= 1; a++) {
        const double* row = f + (int64_t)(2 * X + a) * nf + 2 * Y;
        s += (double)(2 - abs(a)) * (row[-1] + 2.0 * row[0] + row[1]);
    }
    return s * (1.0 / 16.0);
}

__global__ void k2_coarsen_coef(const double* __restrict__ fD, const double* __restrict__ fmu, double* __restrict__ cD,
                                double* __restrict__ cmu, int Nf) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nc * nc) return;
    const int X = (int)(v / nc), Y = (int)(v % nc);
    if (!interior2(Nc, X, Y)) {
        const int64_t i = (int64_t)(2 * X) * nf + 2 * Y;
        cD[v] = fD[i];
        cmu[v] = fmu[i];
        return;
    }
    cD[v] = full_weight2(fD, nf, X, Y);
    cmu[v] = full_weight2(fmu, nf, X, Y);
}

// ---------------------------------------------------------------------------
// The cycle.

// u = 0 on interior vertices, g on the boundary.
__global__ void k2_init_iterate(double* __restrict__ u, int N, double g) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x)
        u[v] = interior2(N, (int)(v / n), (int)(v % n)) ? 0.0 : g;
}

// One red (colour 0) or black (colour 1) half-sweep in place (Sec. 2.2):
// u_i = (q_i + sum_j c_ij u_j) / (sum_j c_ij + mua_i) on the interior
// vertices of the colour.  Item t = row (x - 1) * (N/2) + j is the j-th
// vertex of the colour in row x; N is even on every level that smooths.
template <bool HARM>
__global__ void k2_half_sweep(double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                              const double* __restrict__ mu, int N, Stencil<double> s, int colour) {
    const int S = N / 2;
    const int64_t t = item_of_thread2();
    if (t >= (int64_t)(N - 1) * S) return;
    const int x = 1 + (int)(t / S);
    const int y = (((colour - x) & 1) ? 1 : 2) + 2 * (int)(t % S);
    if (y >= N) return;
    const int n = N + 1;
    const int64_t i = (int64_t)x * n + y;
    const double Di = D[i];
    const double cxm = face<HARM>(Di, D[i - n], s), cxp = face<HARM>(Di, D[i + n], s);
    const double cym = face<HARM>(Di, D[i - 1], s), cyp = face<HARM>(Di, D[i + 1], s);
    u[i] = (q[i] + cxm * u[i - n] + cxp * u[i + n] + cym * u[i - 1] + cyp * u[i + 1]) / (cxm + cxp + cym + cyp + mu[i]);
}

// q - A u at the interior vertex i = (x, y) (row stride n).
template <bool HARM>
__device__ __forceinline__ double defect2_at(const double* __restrict__ u, const double* __restrict__ q,
                                             const double* __restrict__ D, const double* __restrict__ mu, int64_t i,
                                             int n, const Stencil<double>& s) {
    const double Di = D[i], ui = u[i];
    return q[i] - (mu[i] * ui + face<HARM>(Di, D[i - n], s) * (ui - u[i - n]) + face<HARM>(Di, D[i + n], s) * (ui - u[i + n]) +
                   face<HARM>(Di, D[i - 1], s) * (ui - u[i - 1]) + face<HARM>(Di, D[i + 1], s) * (ui - u[i + 1]));
}

// qc = R (q - A u) (Sec. 2.3.2 and Eq. (rest)): one coarse vertex per
// thread, its nine fine defects formed on the fly (0 on the coarse boundary).
template <bool HARM>
__global__ void k2_defect_restrict(const double* __restrict__ u, const double* __restrict__ q,
                                   const double* __restrict__ D, const double* __restrict__ mu, int Nf,
                                   Stencil<double> s, double* __restrict__ qc) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nc * nc) return;
    const int X = (int)(v / nc), Y = (int)(v % nc);
    if (!interior2(Nc, X, Y)) {
        qc[v] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int a = -1; a <= 1; a++) {
        const int64_t i = (int64_t)(2 * X + a) * nf + 2 * Y;
        const double row = defect2_at<HARM>(u, q, D, mu, i - 1, nf, s) + 2.0 * defect2_at<HARM>(u, q, D, mu, i, nf, s) +
                           defect2_at<HARM>(u, q, D, mu, i + 1, nf, s);
        acc += (double)(2 - abs(a)) * row;
    }
    qc[v] = acc * (1.0 / 16.0);
}

// u += I ec on fine interior vertices (Sec. 2.3.3, bilinear).
__global__ void k2_prolong_add(const double* __restrict__ ec, double* __restrict__ u, int Nf) {
    const int nf = Nf + 1, nc = Nf / 2 + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nf * nf) return;
    const int x = (int)(v / nf), y = (int)(v % nf);
    if (!interior2(Nf, x, y)) return;
    const int X0 = x >> 1, X1 = (x + 1) >> 1, Y0 = y >> 1, Y1 = (y + 1) >> 1;
    const double* r0 = ec + (int64_t)X0 * nc;
    const double* r1 = ec + (int64_t)X1 * nc;
    double e;
    if (X0 == X1) e = (Y0 == Y1) ? r0[Y0] : 0.5 * (r0[Y0] + r0[Y1]);
    else if (Y0 == Y1) e = 0.5 * (r0[Y0] + r1[Y0]);
    else e = 0.25 * (r0[Y0] + r1[Y0] + r0[Y1] + r1[Y1]);
    u[v] += e;
}

// Exact solve on the coarsest level (N in {2, 3}: at most 4 unknowns), the
// boundary values of u moved to the right-hand side; one thread, Cholesky.
template <bool HARM>
__global__ void k2_exact(const double* __restrict__ q, double* __restrict__ u, const double* __restrict__ D,
                         const double* __restrict__ mu, int N, Stencil<double> s) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int n = N + 1, m1 = N - 1, m = m1 * m1;
    double A[4][4], b[4];
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) A[r][c] = 0.0;
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++) {
            const int t = (x - 1) * m1 + (y - 1);
            const int i = x * n + y;
            A[t][t] = mu[i];
            b[t] = q[i];
            const int nb[4][2] = {{x - 1, y}, {x + 1, y}, {x, y - 1}, {x, y + 1}};
            for (int e = 0; e < 4; e++) {
                const int xa = nb[e][0], ya = nb[e][1], j = xa * n + ya;
                const double c = face<HARM>(D[i], D[j], s);
                A[t][t] += c;
                if (interior2(N, xa, ya)) A[t][(xa - 1) * m1 + (ya - 1)] -= c;
                else b[t] += c * u[j];
            }
        }
    for (int j = 0; j < m; j++) {
        double d = A[j][j];
        for (int p = 0; p < j; p++) d -= A[j][p] * A[j][p];
        d = sqrt(d);
        A[j][j] = d;
        for (int i = j + 1; i < m; i++) {
            double acc = A[i][j];
            for (int p = 0; p < j; p++) acc -= A[i][p] * A[j][p];
            A[i][j] = acc / d;
        }
    }
    for (int i = 0; i < m; i++) {
        double acc = b[i];
        for (int p = 0; p < i; p++) acc -= A[i][p] * b[p];
        b[i] = acc / A[i][i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double acc = b[i];
        for (int p = i + 1; p < m; p++) acc -= A[p][i] * b[p];
        b[i] = acc / A[i][i];
    }
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++) u[x * n + y] = b[(x - 1) * m1 + (y - 1)];
}

// partial[block] = sum over the block's interior vertices of (q - A u)^2.
template <bool HARM>
__global__ void k2_resid_sq(const double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ D,
                            const double* __restrict__ mu, int N, Stencil<double> s, double* __restrict__ partial) {
    const int n = N + 1;
    const int64_t nv = (int64_t)n * n;
    double acc = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        if (!interior2(N, (int)(v / n), (int)(v % n))) continue;
        const double r = defect2_at<HARM>(u, q, D, mu, v, n, s);
        acc += r * r;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// ---------------------------------------------------------------------------
// Derivatives (the adjoint-state formulas of the three-dimensional solver
// with four neighbours).

// rhs = dq - (dA) rho on interior vertices, 0 on the boundary; dA along
// dlogD (face values) and dlogmu (dmua = mua dlogmu).  dq, dlogD or dlogmu
// may be null (zero).
__global__ void k2_tangent_rhs(const double* __restrict__ rho, const double* __restrict__ dq,
                               const double* __restrict__ dlogD, const double* __restrict__ dlogmu,
                               const double* __restrict__ D, const double* __restrict__ mu, int N, double inv_h2,
                               int harmonic, double* __restrict__ rhs) {
    const int n = N + 1;
    const int64_t i = item_of_thread2();
    if (i >= (int64_t)n * n) return;
    const int x = (int)(i / n), y = (int)(i % n);
    if (!interior2(N, x, y)) {
        rhs[i] = 0.0;
        return;
    }
    const int off[4] = {n, -n, 1, -1};
    const double ri = rho[i], Di = D[i];
    double acc = dlogmu ? mu[i] * dlogmu[i] * ri : 0.0;
    if (dlogD) {
        const double dDi = Di * dlogD[i];
        for (int e = 0; e < 4; e++) {
            const int64_t j = i + off[e];
            const double Dj = D[j], dDj = Dj * dlogD[j];
            double dDf;
            if (harmonic) {
                const double sum = Di + Dj;
                dDf = 2.0 * (Dj * Dj * dDi + Di * Di * dDj) / (sum * sum);
            } else {
                dDf = 0.5 * (dDi + dDj);
            }
            acc += dDf * inv_h2 * (ri - rho[j]);
        }
    }
    rhs[i] = (dq ? dq[i] : 0.0) - acc;
}

// g_logmua = -mua lam rho (interior, 0 on the boundary);
// g_logD_v = -sum over faces (v, j) with an interior endpoint of
// dD_f/dlogD_v (lam_v - lam_j)(rho_v - rho_j) / h^2, lam = 0 on the boundary.
__global__ void k2_coef_grads(const double* __restrict__ rho, const double* __restrict__ lam,
                              const double* __restrict__ D, const double* __restrict__ mu, int N, double inv_h2,
                              int harmonic, double* __restrict__ gD, double* __restrict__ gmu) {
    const int n = N + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)n * n) return;
    const int x = (int)(v / n), y = (int)(v % n);
    const bool vin = interior2(N, x, y);
    const double lv = vin ? lam[v] : 0.0, rv = rho[v], Dv = D[v];
    if (gmu) gmu[v] = vin ? -mu[v] * lv * rv : 0.0;
    if (!gD) return;
    double acc = 0.0;
    const int o[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int e = 0; e < 4; e++) {
        const int xa = x + o[e][0], ya = y + o[e][1];
        if (xa < 0 || xa > N || ya < 0 || ya > N) continue;
        const bool jin = interior2(N, xa, ya);
        if (!vin && !jin) continue;
        const int64_t j = (int64_t)xa * n + ya;
        const double lj = jin ? lam[j] : 0.0, Dj = D[j];
        double dcdv;
        if (harmonic) {
            const double sum = Dv + Dj;
            dcdv = 2.0 * Dj * Dj * Dv / (sum * sum);
        } else {
            dcdv = 0.5 * Dv;
        }
        acc += dcdv * (lv - lj) * (rv - rho[j]);
    }
    gD[v] = -acc * inv_h2;
}

}  // namespace dmgs

namespace dmgs {

// ---------------------------------------------------------------------------
// Two red-black sweeps per pass, out of place (u_in -> u_out).
//
// One wave per tile of TILE interior columns [ts, ts + TILE); lane t holds
// the column pair (yb + 2t, yb + 2t + 1), yb = ts - RING, so a wave covers
// the tile and a ring of RING columns on each side (TILE = 128 - 2 RING).
// A chunk of rows [xa, xb) is marched one row per step; the four colour
// updates of the two sweeps run as a pipeline: at step s, stage j (j =
// 1..4) updates row s - j + 1, which then sees its neighbours exactly as the
// sequential order leaves them (a stage never changes the other colour).
// Stage j is applied on the tile plus a ring of RING - j columns
// (neighbouring tiles recompute these), and its rows reach RING - j beyond
// the chunk, so the output rows depend only on rows [xa - RING, xb + RING)
// of u_in.  Each lane keeps eight rows of its two columns (u, D, q, mua) in
// a register ring indexed by row & 7 (the march is unrolled by 8, so ring
// slots are compile-time); in-row neighbours of the other column come from
// the adjacent lane by a shuffle.  A row is loaded three steps before the
// first stage reads it and enters its ring slot at the end of the step.
// Only interior vertices of the tile are written; u_out's boundary keeps
// its values.  Rows: with O = RING - 1, chunk 0 is [1, O + chunk) and chunk
// c > 0 is [O + c chunk, O + (c + 1) chunk), cut at N (chunk a multiple of
// 8, so that every march starts at a multiple of 8).
//
// PROLONG (post-smoothing): the pass smooths u_in + I ec (Sec. 2.3.3,
// bilinear, ec on the next coarser level with a zero boundary); the
// correction of a row is added at the step before its first use, from
// coarse values loaded with the row.
//
// DEFECT (pre-smoothing): RING = 5, so the final values are known on the
// tile plus a ring of 1 and on one row beyond the chunk; at step s, once
// row s - 3 is final, the pass also writes the defect r = q - A u of row
// s - 4 on the tile (Sec. 2.3.2), for the restriction to read.
template <bool DEFECT> struct Sweep2Shape2 {
    static constexpr int RING = DEFECT ? 5 : 4, TILE = 2 * kWave - 2 * RING;
};
constexpr int kTile2 = Sweep2Shape2<false>::TILE, kTile2D = Sweep2Shape2<true>::TILE;

template <bool HARM, bool PROLONG, bool DEFECT = false>
__global__ __launch_bounds__(256) void k2_sweep2(const double* __restrict__ uin, double* __restrict__ uout,
                                                 const double* __restrict__ q, const double* __restrict__ D,
                                                 const double* __restrict__ mu, const double* __restrict__ ec,
                                                 double* __restrict__ rout, int N, Stencil<double> st,
                                                 int first_colour, int chunk, int ntiles, int nchunks) {
    static_assert(!(PROLONG && DEFECT), "the defect is formed after pre-smoothing only");
    constexpr int RING = Sweep2Shape2<DEFECT>::RING, TILE = Sweep2Shape2<DEFECT>::TILE, O = RING - 1;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tile = wave % ntiles, ch = wave / ntiles;
    if (ch >= nchunks) return;   // whole waves exit
    const int n = N + 1;
    const int ts = 1 + tile * TILE;
    const int yb = ts - RING;
    const int ya = yb + 2 * lane, yo = ya + 1;   // this lane's columns
    const int xa = ch == 0 ? 1 : O + ch * chunk, xb = min(N, O + (ch + 1) * chunk);
    // rows and columns outside the grid are read clamped to its edge: no
    // update that is kept reads them (an updated interior vertex has all its
    // neighbours in the grid), and unconditional loads let the compiler wait
    // for each row's loads alone
    const int yca = min(max(ya, 0), N), yco = min(max(yo, 0), N);

    double ua[8], uo[8], da[8], dd[8], qa[8], qo[8], ma[8], mo[8];
    // coarse values of the correction: rows X0 = r >> 1 and X1 = (r + 1) >> 1,
    // columns C0 = ya >> 1 and C0 + 1
    double e00[8], e01[8], e10[8], e11[8];
    const int Nc = N >> 1, nc = Nc + 1;
    // (clamped separately: on the left edge the lane of columns (-1, 0) must
    // take column 0 of ec, which is 0, for y = 0)
    const int C0 = min(max(ya >> 1, 0), Nc), C1 = min(max((ya >> 1) + 1, 0), Nc);
    struct Row {
        double ua, uo, da, dd, qa, qo, ma, mo, e00, e01, e10, e11;
    };
    // 32-bit element offsets (a grid has at most 16385^2 < 2^32 vertices)
    auto fetch_row = [&](int r) __attribute__((always_inline)) {
        Row t;
        const uint32_t b = (uint32_t)min(max(r, 0), N) * (uint32_t)n;
        t.ua = uin[b + yca];
        t.uo = uin[b + yco];
        t.da = D[b + yca];
        t.dd = D[b + yco];
        t.qa = q[b + yca];
        t.qo = q[b + yco];
        t.ma = mu[b + yca];
        t.mo = mu[b + yco];
        t.e00 = t.e01 = t.e10 = t.e11 = 0.0;
        if (PROLONG) {
            const int rc = min(max(r, 0), N);
            const uint32_t b0 = (uint32_t)(rc >> 1) * (uint32_t)nc, b1 = (uint32_t)min((rc + 1) >> 1, Nc) * (uint32_t)nc;
            t.e00 = ec[b0 + C0];
            t.e01 = ec[b0 + C1];
            t.e10 = ec[b1 + C0];
            t.e11 = ec[b1 + C1];
        }
        return t;
    };
    auto store_row = [&](const Row& t, int sl) __attribute__((always_inline)) {
        ua[sl] = t.ua; uo[sl] = t.uo; da[sl] = t.da; dd[sl] = t.dd;
        qa[sl] = t.qa; qo[sl] = t.qo; ma[sl] = t.ma; mo[sl] = t.mo;
        if (PROLONG) { e00[sl] = t.e00; e01[sl] = t.e01; e10[sl] = t.e10; e11[sl] = t.e11; }
    };
    // u += I ec on row r (the bilinear weights of k2_prolong_add; the
    // boundary gets 0, as ec vanishes there)
    auto correct_row = [&](int r, int sl) __attribute__((always_inline)) {
        if (!PROLONG) return;
        const bool rodd = r & 1;
        const double c0 = rodd ? 0.5 * (e00[sl] + e10[sl]) : e00[sl];
        const double c1 = rodd ? 0.5 * (e01[sl] + e11[sl]) : e01[sl];
        const double cm = rodd ? 0.25 * (e00[sl] + e10[sl] + e01[sl] + e11[sl]) : 0.5 * (e00[sl] + e01[sl]);
        // ya even: ya on C0, yo between C0 and C1; ya odd: the reverse
        const bool aodd = ya & 1;
        ua[sl] += aodd ? cm : c0;
        uo[sl] += aodd ? c1 : cm;
    };
    // colour c on row r (slot sl, rows r -1 / r + 1 in slots sm / sp), on the
    // tile plus a ring of `ring` columns
    auto stage = [&](int r, int sl, int sm, int sp, int c, int ring) __attribute__((always_inline)) {
        // the pair column of the colour (wave-uniform): odd -> yo, else ya;
        // every ring entry is updated through value selects, so the ring
        // stays in registers
        const bool odd = (c - r - yb) & 1;
        const double su = odd ? ua[sl] : uo[sl], sd = odd ? da[sl] : dd[sl];   // the pair's other column
        const int src = odd ? min(lane + 1, kWave - 1) : max(lane - 1, 0);
        const double un = __shfl(su, src, kWave), dn = __shfl(sd, src, kWave);   // the adjacent lane's
        const double ul = odd ? su : un, ur = odd ? un : su;
        const double dl = odd ? sd : dn, dr = odd ? dn : sd;
        const double Di = odd ? dd[sl] : da[sl];
        const double cxm = face<HARM>(Di, odd ? dd[sm] : da[sm], st), cxp = face<HARM>(Di, odd ? dd[sp] : da[sp], st);
        const double cym = face<HARM>(Di, dl, st), cyp = face<HARM>(Di, dr, st);
        const double um = odd ? uo[sm] : ua[sm], up = odd ? uo[sp] : ua[sp];
        const double qi = odd ? qo[sl] : qa[sl], mi = odd ? mo[sl] : ma[sl];
        const double v = (qi + cxm * um + cxp * up + cym * ul + cyp * ur) / (cxm + cxp + cym + cyp + mi);
        const int y = odd ? yo : ya;
        const bool act = r >= 1 && r <= N - 1 && y >= max(1, ts - ring) && y <= min(N - 1, ts + TILE - 1 + ring);
        ua[sl] = (act && !odd) ? v : ua[sl];
        uo[sl] = (act && odd) ? v : uo[sl];
    };
    // defect of row r (slot sl, final rows r -1 / r + 1 in slots sm / sp) on
    // the tile, in the order of defect2_at
    auto defect_row = [&](int r, int sl, int sm, int sp) __attribute__((always_inline)) {
        const double uL = __shfl_up(uo[sl], 1, kWave), dL = __shfl_up(dd[sl], 1, kWave);       // column ya - 1
        const double uR = __shfl_down(ua[sl], 1, kWave), dR = __shfl_down(da[sl], 1, kWave);   // column yo + 1
        if (r < xa || r >= xb) return;
        const uint32_t b = (uint32_t)r * (uint32_t)n;
        const double Da = da[sl], u_a = ua[sl];
        const double Do = dd[sl], u_o = uo[sl];
        const double ra = qa[sl] - (ma[sl] * u_a + face<HARM>(Da, da[sm], st) * (u_a - ua[sm]) +
                                    face<HARM>(Da, da[sp], st) * (u_a - ua[sp]) + face<HARM>(Da, dL, st) * (u_a - uL) +
                                    face<HARM>(Da, Do, st) * (u_a - u_o));
        const double ro = qo[sl] - (mo[sl] * u_o + face<HARM>(Do, dd[sm], st) * (u_o - uo[sm]) +
                                    face<HARM>(Do, dd[sp], st) * (u_o - uo[sp]) + face<HARM>(Do, Da, st) * (u_o - u_a) +
                                    face<HARM>(Do, dR, st) * (u_o - uR));
        if (ya >= ts && ya < ts + TILE && ya <= N - 1) rout[b + ya] = ra;
        if (yo >= ts && yo < ts + TILE && yo <= N - 1) rout[b + yo] = ro;
    };
    const int c1 = first_colour, c2 = 1 - first_colour;
    const int sb = (xa - O) & ~7;   // first step, a multiple of 8 (chunk 0 starts a few harmless steps early)
    const int se = xb + O;          // one past the last step
    // rows sb - 4 .. sb + 2 before the first step
#pragma unroll
    for (int k = -4; k <= 2; k++) store_row(fetch_row(sb + k), k & 7);
#pragma unroll
    for (int k = -4; k <= 0; k++) correct_row(sb + k, k & 7);
    for (int s8 = sb; s8 < se; s8 += 8) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int s = s8 + k;
            const Row next = fetch_row(s + 3);   // enters slot (k + 3) & 7 (row s - 5's) at the end of the step
            correct_row(s + 1, (k + 1) & 7);   // first read by stage 1 below
            stage(s, k & 7, (k - 1) & 7, (k + 1) & 7, c1, RING - 1);
            stage(s - 1, (k - 1) & 7, (k - 2) & 7, k & 7, c2, RING - 2);
            stage(s - 2, (k - 2) & 7, (k - 3) & 7, (k - 1) & 7, c1, RING - 3);
            stage(s - 3, (k - 3) & 7, (k - 4) & 7, (k - 2) & 7, c2, RING - 4);
            const int r = s - 3;
            if (r >= xa && r < xb) {
                const uint32_t b = (uint32_t)r * (uint32_t)n;
                const int sl = (k - 3) & 7;
                if (ya >= ts && ya < ts + TILE && ya <= N - 1) uout[b + ya] = ua[sl];
                if (yo >= ts && yo < ts + TILE && yo <= N - 1) uout[b + yo] = uo[sl];
            }
            if (DEFECT) defect_row(s - 4, (k - 4) & 7, (k - 5) & 7, (k - 3) & 7);
            store_row(next, (k + 3) & 7);
        }
    }
}

// qc = R r on coarse interior vertices from a fine defect r written by a
// DEFECT pass (0 on the coarse boundary): (1/16)(1,2,1) x (1,2,1), summed
// in the order of k2_defect_restrict.
__global__ void k2_restrict_r(const double* __restrict__ r, double* __restrict__ qc, int Nf) {
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int64_t v = item_of_thread2();
    if (v >= (int64_t)nc * nc) return;
    const int X = (int)(v / nc), Y = (int)(v % nc);
    if (!interior2(Nc, X, Y)) {
        qc[v] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int a = -1; a <= 1; a++) {
        const double* row = r + (int64_t)(2 * X + a) * nf + 2 * Y;
        acc += (double)(2 - abs(a)) * (row[-1] + 2.0 * row[0] + row[1]);
    }
    qc[v] = acc * (1.0 / 16.0);
}

}  // namespace dmgs

namespace dmgs {

// qc = R (q - A u) streamed along fine rows (Sec. 2.3.2 and Eq. (rest)).
// One wave per tile of kTileR = 62 coarse columns [Ys, Ys + 62): lane t
// holds the fine column pair (2Y, 2Y + 1) of coarse column Y = Ys - 1 + t
// (lanes 0 and 63 are halo lanes).  Each fine defect is formed once; a
// fine row gives the horizontal sums h_x(Y) = r(x, 2Y-1) + 2 r(x, 2Y) +
// r(x, 2Y+1) (one shuffle), and coarse row X is (h_{2X-1} + 2 h_{2X} +
// h_{2X+1}) / 16, the order in which k2_defect_restrict sums.  A chunk of
// coarse rows [Xa, Xb) (Xa = 1 + c cx, cx a multiple of 4) marches fine
// rows 2Xa - 2 ... 2Xb - 1 in steps of 8 with rows in a register ring
// (row x in slot x & 7), each loaded three steps before the step that
// forms its defect.  Only coarse interior vertices are written.
constexpr int kTileR = 62;

template <bool HARM>
__global__ __launch_bounds__(256) void k2_defect_restrict_rows(const double* __restrict__ u, const double* __restrict__ q,
                                                               const double* __restrict__ D,
                                                               const double* __restrict__ mu, int Nf,
                                                               Stencil<double> st, double* __restrict__ qc, int cx,
                                                               int ntiles, int nchunks) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tile = wave % ntiles, ch = wave / ntiles;
    if (ch >= nchunks) return;   // whole waves exit
    const int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    const int Ys = 1 + tile * kTileR;
    const int Y = Ys - 1 + lane;
    const int ye = 2 * Y, yo = ye + 1;                     // this lane's fine columns
    const int yce = min(max(ye, 0), Nf), yco = min(max(yo, 0), Nf);   // clamped reads (kept defects never need them)
    const int Xa = 1 + ch * cx, Xb = min(Nc, Xa + cx);
    const bool wr = lane >= 1 && lane <= kTileR && Y <= Nc - 1;

    double ue[8], uo[8], de[8], dd[8], qe[8], qo[8], me[8], mo[8];
    auto load_row = [&](int x, int sl) __attribute__((always_inline)) {
        const uint32_t b = (uint32_t)min(max(x, 0), Nf) * (uint32_t)nf;
        ue[sl] = u[b + yce];
        uo[sl] = u[b + yco];
        de[sl] = D[b + yce];
        dd[sl] = D[b + yco];
        qe[sl] = q[b + yce];
        qo[sl] = q[b + yco];
        me[sl] = mu[b + yce];
        mo[sl] = mu[b + yco];
    };
    // h_x for row x (slot sl; rows x -1 / x + 1 in slots sm / sp)
    auto hsum = [&](int sl, int sm, int sp) __attribute__((always_inline)) {
        const double uoL = __shfl_up(uo[sl], 1, kWave), doL = __shfl_up(dd[sl], 1, kWave);     // column 2Y - 1
        const double ueR = __shfl_down(ue[sl], 1, kWave), deR = __shfl_down(de[sl], 1, kWave); // column 2Y + 2
        const double Dei = de[sl], uei = ue[sl];
        const double re = qe[sl] - (me[sl] * uei + face<HARM>(Dei, de[sm], st) * (uei - ue[sm]) +
                                    face<HARM>(Dei, de[sp], st) * (uei - ue[sp]) + face<HARM>(Dei, doL, st) * (uei - uoL) +
                                    face<HARM>(Dei, dd[sl], st) * (uei - uo[sl]));
        const double Doi = dd[sl], uoi = uo[sl];
        const double ro = qo[sl] - (mo[sl] * uoi + face<HARM>(Doi, dd[sm], st) * (uoi - uo[sm]) +
                                    face<HARM>(Doi, dd[sp], st) * (uoi - uo[sp]) + face<HARM>(Doi, de[sl], st) * (uoi - uei) +
                                    face<HARM>(Doi, deR, st) * (uoi - ueR));
        const double roL = __shfl_up(ro, 1, kWave);   // r(x, 2Y - 1)
        return roL + 2.0 * re + ro;
    };
    const int x0 = 2 * Xa - 2;            // a multiple of 8
    const int xe = 2 * Xb;                // one past the last fine row, 2 Xb - 1
#pragma unroll
    for (int k = -1; k <= 2; k++) load_row(x0 + k, k & 7);
    double carry = 0.0, hmid = 0.0;
    for (int x8 = x0; x8 < xe; x8 += 8) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int x = x8 + k;
            load_row(x + 3, (k + 3) & 7);
            const double h = hsum(k & 7, (k - 1) & 7, (k + 1) & 7);
            if ((k & 1) == 0) {
                hmid = h;                 // x = 2X
            } else {                      // x = 2X + 1 closes coarse row X
                const int X = x >> 1;
                if (wr && X >= Xa && X < Xb) qc[(uint32_t)X * (uint32_t)nc + Y] = (carry + 2.0 * hmid + h) * (1.0 / 16.0);
                carry = h;
            }
        }
    }
}

}  // namespace dmgs

namespace dmgs {

// ---------------------------------------------------------------------------
// The coarse end of a two-dimensional V-cycle in one workgroup: levels
// ks .. L-1 (N_ks <= kSmall2MaxN), every field LDS-resident.  The correction
// of level ks starts from 0 with a zero boundary (a coarse correction), and
// the same steps as the per-level kernels run in the same order: nu_pre
// sweeps, defect and restriction, the next level, prolongation and
// correction, nu_post sweeps; the coarsest level is solved exactly (one
// thread, Cholesky).  Barriers separate the steps.
constexpr int kSmall2MaxN = 32, kSmall2MaxLevels = 6;

struct Small2Args {
    const double* q;                          // right-hand side of level ks
    double* u;                                // its correction (written on every vertex)
    const double* D[kSmall2MaxLevels];
    const double* mu[kSmall2MaxLevels];
    Stencil<double> st[kSmall2MaxLevels];
    int N[kSmall2MaxLevels];
    int nl;                                   // levels ks .. L-1
    int nu_pre, nu_post, first;               // first: colour of the first half-sweep
};

__host__ __device__ inline int small2_words(const int* Ns, int nl) {
    int w = 0;
    for (int i = 0; i < nl; i++) w += 4 * (Ns[i] + 1) * (Ns[i] + 1);
    return w;
}

template <bool HARM>
__global__ __launch_bounds__(1024) void k2_small_vcycle(Small2Args a) {
    extern __shared__ double lds2[];
    // level i holds u, q, D, mua (each (N_i + 1)^2) from lds2 + 4 sum_{j<i} (N_j + 1)^2
    auto lvl = [&](int i) __attribute__((always_inline)) {
        int off = 0;
        for (int j = 0; j < i; j++) off += 4 * (a.N[j] + 1) * (a.N[j] + 1);
        return lds2 + off;
    };
    auto nvl = [&](int i) __attribute__((always_inline)) { return (a.N[i] + 1) * (a.N[i] + 1); };
#define U(i) (lvl(i))
#define Q(i) (lvl(i) + nvl(i))
#define DD(i) (lvl(i) + 2 * nvl(i))
#define M(i) (lvl(i) + 3 * nvl(i))
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = 0; i < a.nl; i++) {
        const int nv = (a.N[i] + 1) * (a.N[i] + 1);
        for (int v = tid; v < nv; v += nt) {
            U(i)[v] = 0.0;
            Q(i)[v] = i == 0 ? a.q[v] : 0.0;
            DD(i)[v] = a.D[i][v];
            M(i)[v] = a.mu[i][v];
        }
    }
    __syncthreads();
    auto half = [&](int i, int colour) {
        const int N = a.N[i], n = N + 1, S = N / 2;
        const Stencil<double> s = a.st[i];
        double* u = U(i);
        for (int t = tid; t < (N - 1) * S; t += nt) {
            const int x = 1 + t / S;
            const int y = (((colour - x) & 1) ? 1 : 2) + 2 * (t % S);
            if (y >= N) continue;
            const int v = x * n + y;
            const double Di = DD(i)[v];
            const double cxm = face<HARM>(Di, DD(i)[v - n], s), cxp = face<HARM>(Di, DD(i)[v + n], s);
            const double cym = face<HARM>(Di, DD(i)[v - 1], s), cyp = face<HARM>(Di, DD(i)[v + 1], s);
            u[v] = (Q(i)[v] + cxm * u[v - n] + cxp * u[v + n] + cym * u[v - 1] + cyp * u[v + 1]) /
                   (cxm + cxp + cym + cyp + M(i)[v]);
        }
        __syncthreads();
    };
    auto sweeps = [&](int i, int count) {
        for (int c = 0; c < count; c++) {
            half(i, a.first);
            half(i, 1 - a.first);
        }
    };
    for (int i = 0; i + 1 < a.nl; i++) {
        sweeps(i, a.nu_pre);
        // qc = R (q - A u)
        const int Nf = a.N[i], nf = Nf + 1, Nc = a.N[i + 1], nc = Nc + 1;
        const Stencil<double> s = a.st[i];
        for (int v = tid; v < (Nc - 1) * (Nc - 1); v += nt) {
            const int X = 1 + v / (Nc - 1), Y = 1 + v % (Nc - 1);
            double acc = 0.0;
            for (int da = -1; da <= 1; da++) {
                double row = 0.0;
                for (int db = -1; db <= 1; db++) {
                    const int f = (2 * X + da) * nf + 2 * Y + db;
                    const double Di = DD(i)[f], ui = U(i)[f];
                    const double r = Q(i)[f] - (M(i)[f] * ui + face<HARM>(Di, DD(i)[f - nf], s) * (ui - U(i)[f - nf]) +
                                                face<HARM>(Di, DD(i)[f + nf], s) * (ui - U(i)[f + nf]) +
                                                face<HARM>(Di, DD(i)[f - 1], s) * (ui - U(i)[f - 1]) +
                                                face<HARM>(Di, DD(i)[f + 1], s) * (ui - U(i)[f + 1]));
                    row += (db == 0 ? 2.0 : 1.0) * r;
                }
                acc += (double)(2 - abs(da)) * row;
            }
            Q(i + 1)[X * nc + Y] = acc * (1.0 / 16.0);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // exact solve on the coarsest level (N in {2, 3}), zero boundary
        const int i = a.nl - 1, N = a.N[i], n = N + 1, m1 = N - 1, m = m1 * m1;
        const Stencil<double> s = a.st[i];
        double A[4][4], b[4];
        for (int r = 0; r < m; r++)
            for (int c = 0; c < m; c++) A[r][c] = 0.0;
        for (int x = 1; x < N; x++)
            for (int y = 1; y < N; y++) {
                const int t = (x - 1) * m1 + (y - 1), v = x * n + y;
                A[t][t] = M(i)[v];
                b[t] = Q(i)[v];
                const int nb[4][2] = {{x - 1, y}, {x + 1, y}, {x, y - 1}, {x, y + 1}};
                for (int e = 0; e < 4; e++) {
                    const int xa = nb[e][0], ya = nb[e][1];
                    const double c = face<HARM>(DD(i)[v], DD(i)[xa * n + ya], s);
                    A[t][t] += c;
                    if (xa > 0 && xa < N && ya > 0 && ya < N) A[t][(xa - 1) * m1 + (ya - 1)] -= c;
                }
            }
        for (int j = 0; j < m; j++) {
            double d = A[j][j];
            for (int p = 0; p < j; p++) d -= A[j][p] * A[j][p];
            d = sqrt(d);
            A[j][j] = d;
            for (int r = j + 1; r < m; r++) {
                double acc = A[r][j];
                for (int p = 0; p < j; p++) acc -= A[r][p] * A[j][p];
                A[r][j] = acc / d;
            }
        }
        for (int r = 0; r < m; r++) {
            double acc = b[r];
            for (int p = 0; p < r; p++) acc -= A[r][p] * b[p];
            b[r] = acc / A[r][r];
        }
        for (int r = m - 1; r >= 0; r--) {
            double acc = b[r];
            for (int p = r + 1; p < m; p++) acc -= A[p][r] * b[p];
            b[r] = acc / A[r][r];
        }
        for (int x = 1; x < N; x++)
            for (int y = 1; y < N; y++) U(i)[x * n + y] = b[(x - 1) * m1 + (y - 1)];
    }
    __syncthreads();
    for (int i = a.nl - 2; i >= 0; i--) {
        // u += I uc on fine interior vertices
        const int Nf = a.N[i], nf = Nf + 1, nc = a.N[i + 1] + 1;
        const double* ec = U(i + 1);
        for (int v = tid; v < nf * nf; v += nt) {
            const int x = v / nf, y = v % nf;
            if (x == 0 || x == Nf || y == 0 || y == Nf) continue;
            const int X0 = x >> 1, X1 = (x + 1) >> 1, Y0 = y >> 1, Y1 = (y + 1) >> 1;
            const double* r0 = ec + X0 * nc;
            const double* r1 = ec + X1 * nc;
            double e;
            if (X0 == X1) e = (Y0 == Y1) ? r0[Y0] : 0.5 * (r0[Y0] + r0[Y1]);
            else if (Y0 == Y1) e = 0.5 * (r0[Y0] + r1[Y0]);
            else e = 0.25 * (r0[Y0] + r1[Y0] + r0[Y1] + r1[Y1]);
            U(i)[v] += e;
        }
        __syncthreads();
        sweeps(i, a.nu_post);
    }
    const int nv0 = (a.N[0] + 1) * (a.N[0] + 1);
    for (int v = tid; v < nv0; v += nt) a.u[v] = U(0)[v];
#undef U
#undef Q
#undef DD
#undef M
}

}  // namespace dmgs

namespace dmgs {

// ---------------------------------------------------------------------------
// A whole smoothing phase of a mid-size level in one launch: one workgroup
// per 32 x 32 tile, the tile and a ring of kH2 = 6 vertices staged in LDS
// (u, q, D, mua), two red-black sweeps (four half-sweeps) with a barrier
// after each, half-sweep j updating the tile plus a shrinking ring.
//   MODE 0 / 1 (pre-smoothing from u_in / from zero): the sweeps leave u
//     final on the tile plus a ring of 2; the pass writes u on the tile and
//     the restricted defect qc = R (q - A u) of the tile's 16 x 16 coarse
//     vertices (each forms its nine fine defects from LDS).
//   MODE 2 (post-smoothing): u_in + I ec (bilinear, the bilinear weights of
//     k2_prolong_add) is staged, then the sweeps; the pass writes u on the
//     tile.
// Only interior grid vertices are updated or written; staged vertices
// outside the grid hold u = q = mua = 0, D = 1 and are never updated.
constexpr int kB2 = 32, kH2 = 6, kW2 = kB2 + 2 * kH2;

template <bool HARM, int MODE>
__global__ __launch_bounds__(256) void k2_block_pass(const double* __restrict__ uin, double* __restrict__ uout,
                                                     const double* __restrict__ q, const double* __restrict__ D,
                                                     const double* __restrict__ mu, const double* __restrict__ ec,
                                                     double* __restrict__ qc, int N, Stencil<double> st, int first,
                                                     int ntx) {
    __shared__ double su[kW2 * kW2], sq[kW2 * kW2], sd[kW2 * kW2], sm[kW2 * kW2];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int x0 = tx * kB2 - kH2, y0 = ty * kB2 - kH2;   // grid coordinates of LDS entry (0, 0)
    const int n = N + 1, Nc = N / 2, nc = Nc + 1;
    for (int i = tid; i < kW2 * kW2; i += nt) {
        const int gx = x0 + i / kW2, gy = y0 + i % kW2;
        const bool in = gx >= 0 && gx <= N && gy >= 0 && gy <= N;
        const int64_t g = (int64_t)gx * n + gy;
        sd[i] = in ? D[g] : 1.0;
        sm[i] = in ? mu[g] : 0.0;
        sq[i] = in ? q[g] : 0.0;
        double u = 0.0;
        if (MODE == 0 || MODE == 2) u = in ? uin[g] : 0.0;
        if (MODE == 2 && in && gx > 0 && gx < N && gy > 0 && gy < N) {
            const int X0 = gx >> 1, X1 = (gx + 1) >> 1, Y0 = gy >> 1, Y1 = (gy + 1) >> 1;
            const double* r0 = ec + (int64_t)X0 * nc;
            const double* r1 = ec + (int64_t)X1 * nc;
            double e;
            if (X0 == X1) e = (Y0 == Y1) ? r0[Y0] : 0.5 * (r0[Y0] + r0[Y1]);
            else if (Y0 == Y1) e = 0.5 * (r0[Y0] + r1[Y0]);
            else e = 0.25 * (r0[Y0] + r1[Y0] + r0[Y1] + r1[Y1]);
            u += e;
        }
        su[i] = u;
    }
    __syncthreads();
    const int ring0 = MODE == 2 ? 3 : 5;   // ring of the first half-sweep
    for (int j = 0; j < 4; j++) {
        const int colour = (j & 1) ? 1 - first : first, ring = ring0 - j;
        const int lo = kH2 - ring, hi = kH2 + kB2 + ring;   // local range [lo, hi)
        for (int i = tid; i < kW2 * kW2; i += nt) {
            const int lx = i / kW2, ly = i % kW2, gx = x0 + lx, gy = y0 + ly;
            if (lx < lo || lx >= hi || ly < lo || ly >= hi || ((gx + gy) & 1) != colour) continue;
            if (gx < 1 || gx > N - 1 || gy < 1 || gy > N - 1) continue;
            const double Di = sd[i];
            const double cxm = face<HARM>(Di, sd[i - kW2], st), cxp = face<HARM>(Di, sd[i + kW2], st);
            const double cym = face<HARM>(Di, sd[i - 1], st), cyp = face<HARM>(Di, sd[i + 1], st);
            su[i] = (sq[i] + cxm * su[i - kW2] + cxp * su[i + kW2] + cym * su[i - 1] + cyp * su[i + 1]) /
                    (cxm + cxp + cym + cyp + sm[i]);
        }
        __syncthreads();
    }
    for (int i = tid; i < kB2 * kB2; i += nt) {
        const int lx = kH2 + i / kB2, ly = kH2 + i % kB2, gx = x0 + lx, gy = y0 + ly;
        if (gx < 1 || gx > N - 1 || gy < 1 || gy > N - 1) continue;
        uout[(int64_t)gx * n + gy] = su[lx * kW2 + ly];
    }
    if (MODE == 2) return;
    // restriction of the defect to the tile's coarse vertices (one per thread)
    for (int c = tid; c < (kB2 / 2) * (kB2 / 2); c += nt) {
        const int X = tx * (kB2 / 2) + c / (kB2 / 2), Y = ty * (kB2 / 2) + c % (kB2 / 2);
        if (X < 1 || X > Nc - 1 || Y < 1 || Y > Nc - 1) continue;
        double acc = 0.0;
        for (int a = -1; a <= 1; a++) {
            double row = 0.0;
            for (int b = -1; b <= 1; b++) {
                const int i = (2 * X + a - x0) * kW2 + (2 * Y + b - y0);
                const double Di = sd[i], ui = su[i];
                const double r = sq[i] - (sm[i] * ui + face<HARM>(Di, sd[i - kW2], st) * (ui - su[i - kW2]) +
                                          face<HARM>(Di, sd[i + kW2], st) * (ui - su[i + kW2]) +
                                          face<HARM>(Di, sd[i - 1], st) * (ui - su[i - 1]) +
                                          face<HARM>(Di, sd[i + 1], st) * (ui - su[i + 1]));
                row += (b == 0 ? 2.0 : 1.0) * r;
            }
            acc += (double)(2 - abs(a)) * row;
        }
        qc[(int64_t)X * nc + Y] = acc * (1.0 / 16.0);
    }
}

}  // namespace dmgs
