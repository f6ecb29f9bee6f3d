/*
 * dmgs_ref.c -- plain, slow, FP64 CPU oracle of the differentiable multigrid
 * solver for the steady-state diffusion-absorption equation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against.  It shares no code, header, table or helper with the HIP
 * path under paper_2608_00760_amd/csrc, and only tests/, the smoke entry point
 * and the CPU-baseline leg of the benchmark may load it.
 *
 * What it computes (paper: "Variational Inference Using a Differentiable
 * Multigrid Linear Solver"):
 *   - the operator L of Eq. (maineq), -div(D grad rho) + lambda rho = q, written
 *     as a 7-point second-order finite-difference stencil on a vertex-centred
 *     grid with Dirichlet boundary (Sec. 2, Sec. 2.2);
 *   - the solver S: V-cycles of red-black Gauss-Seidel (Sec. 2.2, Sec. 2.3.1),
 *     defect (Sec. 2.3.2, Eq. (defect)), full-weighting restriction
 *     (Eq. (rest)) and prolongation I = 2^n R^T (Sec. 2.3.3), repeated a fixed
 *     number of times or until a relative residual is reached (Sec. 2.4);
 *   - the pull-back S^dagger as the reversed composition of the adjoints of
 *     every step (Eq. (EqcompT), Sec. 2.3.1-2.3.3), written as exact matrix
 *     transposes;
 *   - the push-forward in q (S itself, Sec. 2.3) and, beyond the paper (which
 *     lists it as future work in Sec. 4), the adjoint-state derivatives with
 *     respect to log D and log lambda of the discrete solution.
 *
 * Notation follows the paper: rho is the solution (fluence), q the source,
 * D the diffusion coefficient and lambda (here "mua", lambda_a of
 * Eq. (medimcoeffs)) the absorption coefficient.  Bars denote cotangents.
 *
 * Readings of passages the paper leaves open:
 *   - sign convention: L is symmetric positive definite, Au = q, defect
 *     r = q - A rho (Eq. (maineq), Eq. (defect));
 *   - face diffusivity: arithmetic mean of the two vertex values (harmonic
 *     mean on request);
 *   - grid: N cells per axis, (N+1)^3 vertices, N = c 2^m with c in {2,3};
 *     coarsening stops at N in {2,3}, where the level is solved exactly;
 *   - red = (x+y+z) even in each level's own coordinates, red first;
 *   - 3D restriction is the tensor product of the 1D stencil of Eq. (rest);
 *   - coarse coefficients: full weighting on coarse interior vertices,
 *     injection on coarse boundary vertices; coarse operators are
 *     rediscretised with h_k = 2^k h (Sec. 2.2);
 *   - coarse-level corrections start from zero (Sec. 2.3.1);
 *   - the alternative smoother, weighted Jacobi, takes the weight
 *     omega = 6/7 unless set: u <- u + omega (q - A u) / diag(A).
 *
 * Every function below is pinned by a test in tests/ (closed form, brute
 * force, transpose identities, invariants); none is "parity unpinned".
 *
 * Layout: every field is a dense C-order array of (N+1)^3 doubles, x slowest,
 * z fastest: v = (x*(N+1) + y)*(N+1) + z.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#include <stdio.h>

#define REF_MAXLEV 16

enum { REF_OK = 0, REF_ERR_INVALID = 1, REF_ERR_OOM = 2, REF_ERR_NOT_CONVERGED = 3,
       REF_ERR_NONFINITE = 4 };

typedef struct ref_hier {
    int L;                 /* number of levels */
    int N[REF_MAXLEV];     /* cells per axis on level k */
    double h[REF_MAXLEV];  /* spacing on level k */
    double *D[REF_MAXLEV];
    double *mua[REF_MAXLEV];
    int face_mean;         /* 0 arithmetic, 1 harmonic */
    double g;              /* Dirichlet value on the fine level */
    int smoother;          /* 0 red-black Gauss-Seidel, 1 weighted Jacobi */
    double omega;          /* weighted-Jacobi weight */
} ref_hier;

typedef struct ref_opts {
    int order;        /* 0: red then black (forward); 1: black then red */
    int nu1, nu2;     /* pre- and post-smoothing sweeps */
    double rtol;      /* relative residual target */
    int max_cycles;
    int fixed_cycles; /* >0: exactly this many cycles (Sec. 2.4, second mode) */
} ref_opts;

static inline size_t idx(int n, int x, int y, int z) {
    return ((size_t)x * n + y) * n + z;
}
static inline size_t nvert(int N) { size_t n = (size_t)N + 1; return n * n * n; }
static inline int interior(int N, int x, int y, int z) {
    return x > 0 && x < N && y > 0 && y < N && z > 0 && z < N;
}

/* ------------------------------------------------------------------------ */
/* Grid hierarchy (Sec. 2.2: each coarse grid halves the resolution).         */

/* Number of levels for N = c 2^m, c in {2,3}: levels N, N/2, ..., c.
 * Returns 0 when N has no such form. */
int ref_num_levels_for(int N) {
    if (N < 2) return 0;
    int L = 1;
    while (N > 3) {
        if (N % 2) return 0;
        N /= 2;
        L++;
    }
    return L;
}

/* Face coefficient c_ij = D_f / h^2 between neighbouring vertices a and b
 * (the second-order finite-difference flux of Eq. (maineq)). */
static inline double face_coef(const double *D, size_t a, size_t b, double inv_h2, int fm) {
    double Df = fm ? 2.0 * D[a] * D[b] / (D[a] + D[b]) : 0.5 * (D[a] + D[b]);
    return Df * inv_h2;
}

/* Coefficient transfer to the next coarser level: full weighting on coarse
 * interior vertices (tensor product of Eq. (rest)), injection on coarse
 * boundary vertices. */
void ref_coarsen_field(int Nf, const double *f, double *c) {
    int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    #pragma omp parallel for
    for (int X = 0; X < nc; X++)
        for (int Y = 0; Y < nc; Y++)
            for (int Z = 0; Z < nc; Z++) {
                if (!interior(Nc, X, Y, Z)) {
                    c[idx(nc, X, Y, Z)] = f[idx(nf, 2 * X, 2 * Y, 2 * Z)];
                    continue;
                }
                double s = 0.0;
                for (int a = -1; a <= 1; a++)
                    for (int b = -1; b <= 1; b++)
                        for (int d = -1; d <= 1; d++) {
                            double w = (2 - abs(a)) * (2 - abs(b)) * (2 - abs(d)) / 64.0;
                            s += w * f[idx(nf, 2 * X + a, 2 * Y + b, 2 * Z + d)];
                        }
                c[idx(nc, X, Y, Z)] = s;
            }
}

void ref_hier_destroy(ref_hier *H) {
    if (!H) return;
    for (int k = 0; k < H->L; k++) { free(H->D[k]); free(H->mua[k]); }
    free(H);
}

/* Build the hierarchy of rediscretised operators (Sec. 2.2: "finite
 * differences for each level").  D > 0, mua >= 0 and finiteness are checked. */
ref_hier *ref_hier_create(int N, double h, double g, int face_mean,
                          const double *D, const double *mua, int *status) {
    int L = ref_num_levels_for(N);
    *status = REF_OK;
    if (L == 0 || L > REF_MAXLEV || !(h > 0.0) || !isfinite(g)) { *status = REF_ERR_INVALID; return NULL; }
    size_t nv = nvert(N);
    int bad = 0;
    for (size_t v = 0; v < nv; v++)
        if (!(D[v] > 0.0) || !isfinite(D[v]) || !(mua[v] >= 0.0) || !isfinite(mua[v])) bad = 1;
    if (bad) { *status = REF_ERR_INVALID; return NULL; }
    ref_hier *H = calloc(1, sizeof(ref_hier));
    if (!H) { *status = REF_ERR_OOM; return NULL; }
    H->L = L; H->face_mean = face_mean; H->g = g;
    H->smoother = 0; H->omega = 6.0 / 7.0;
    int Nk = N; double hk = h;
    for (int k = 0; k < L; k++) {
        H->N[k] = Nk; H->h[k] = hk;
        H->D[k] = malloc(nvert(Nk) * sizeof(double));
        H->mua[k] = malloc(nvert(Nk) * sizeof(double));
        if (!H->D[k] || !H->mua[k]) { H->L = k + 1; ref_hier_destroy(H); *status = REF_ERR_OOM; return NULL; }
        if (k == 0) {
            memcpy(H->D[0], D, nv * sizeof(double));
            memcpy(H->mua[0], mua, nv * sizeof(double));
        } else {
            ref_coarsen_field(H->N[k - 1], H->D[k - 1], H->D[k]);
            ref_coarsen_field(H->N[k - 1], H->mua[k - 1], H->mua[k]);
        }
        Nk /= 2; hk *= 2.0;
    }
    return H;
}

int ref_levels(const ref_hier *H) { return H->L; }
int ref_level_N(const ref_hier *H, int k) { return H->N[k]; }
void ref_level_coef(const ref_hier *H, int k, double *D, double *mua) {
    memcpy(D, H->D[k], nvert(H->N[k]) * sizeof(double));
    memcpy(mua, H->mua[k], nvert(H->N[k]) * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Operator, smoother, defect, transfers (Sec. 2.2-2.3).                     */

/* out = A_k u on interior vertices, 0 on the boundary.  Boundary entries of u
 * are read as the Dirichlet values. */
void ref_apply(const ref_hier *H, int k, const double *u, double *out) {
    int N = H->N[k], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[k] * H->h[k]);
    const double *D = H->D[k], *mu = H->mua[k];
    const long s[6] = { (long)n * n, -(long)n * n, n, -n, 1, -1 };
    #pragma omp parallel for
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t i = idx(n, x, y, z);
                if (!interior(N, x, y, z)) { out[i] = 0.0; continue; }
                double acc = mu[i] * u[i];
                for (int t = 0; t < 6; t++) {
                    size_t j = (size_t)((long)i + s[t]);
                    acc += face_coef(D, i, j, inv_h2, fm) * (u[i] - u[j]);
                }
                out[i] = acc;
            }
}

/* One red-black Gauss-Seidel half-sweep on colour c (0 = red = (x+y+z) even):
 * rho_i <- (q_i + sum_j c_ij rho_j) / (sum_j c_ij + lambda_i)  (Sec. 2.3.1,
 * with the sign convention of Eq. (maineq)). */
void ref_gs_half(const ref_hier *H, int k, int colour, double *u, const double *q) {
    int N = H->N[k], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[k] * H->h[k]);
    const double *D = H->D[k], *mu = H->mua[k];
    const long s[6] = { (long)n * n, -(long)n * n, n, -n, 1, -1 };
    #pragma omp parallel for
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) {
                if (((x + y + z) & 1) != colour) continue;
                size_t i = idx(n, x, y, z);
                double num = q[i], den = mu[i];
                for (int t = 0; t < 6; t++) {
                    size_t j = (size_t)((long)i + s[t]);
                    double c = face_coef(D, i, j, inv_h2, fm);
                    num += c * u[j];
                    den += c;
                }
                u[i] = num / den;
            }
}

/* Select the smoother of every V-cycle: 0 red-black Gauss-Seidel, 1 weighted
 * Jacobi with weight omega. */
void ref_set_smoother(ref_hier *H, int smoother, double omega) {
    H->smoother = smoother ? 1 : 0;
    H->omega = omega;
}

/* One weighted-Jacobi sweep, every interior vertex from the old iterate:
 * rho_i <- rho_i + omega (q_i - (A rho)_i) / (sum_j c_ij + lambda_i). */
void ref_wj_sweep(const ref_hier *H, int k, double *u, const double *q) {
    int N = H->N[k], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[k] * H->h[k]);
    const double *D = H->D[k], *mu = H->mua[k];
    const long s[6] = { (long)n * n, -(long)n * n, n, -n, 1, -1 };
    size_t nv = nvert(N);
    double *Au = malloc(nv * sizeof(double));
    ref_apply(H, k, u, Au);
    #pragma omp parallel for
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) {
                size_t i = idx(n, x, y, z);
                double d = mu[i];
                for (int e = 0; e < 6; e++) d += face_coef(D, i, (size_t)((long)i + s[e]), inv_h2, fm);
                u[i] += H->omega * (q[i] - Au[i]) / d;
            }
    free(Au);
}

/* Defect e = q - A rho on interior vertices, 0 on the boundary (Eq. (defect)). */
void ref_defect(const ref_hier *H, int k, const double *u, const double *q, double *r) {
    int N = H->N[k], n = N + 1;
    ref_apply(H, k, u, r);
    #pragma omp parallel for
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t i = idx(n, x, y, z);
                r[i] = interior(N, x, y, z) ? q[i] - r[i] : 0.0;
            }
}

/* Full-weighting restriction q_{k+1} = R r (Eq. (rest), tensor product in 3D)
 * on coarse interior vertices; coarse boundary entries are set to 0. */
void ref_restrict(int Nf, const double *r, double *qc) {
    int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    #pragma omp parallel for
    for (int X = 0; X < nc; X++)
        for (int Y = 0; Y < nc; Y++)
            for (int Z = 0; Z < nc; Z++) {
                if (!interior(Nc, X, Y, Z)) { qc[idx(nc, X, Y, Z)] = 0.0; continue; }
                double s = 0.0;
                for (int a = -1; a <= 1; a++)
                    for (int b = -1; b <= 1; b++)
                        for (int d = -1; d <= 1; d++) {
                            double w = (2 - abs(a)) * (2 - abs(b)) * (2 - abs(d)) / 64.0;
                            s += w * r[idx(nf, 2 * X + a, 2 * Y + b, 2 * Z + d)];
                        }
                qc[idx(nc, X, Y, Z)] = s;
            }
}

/* Prolongation I = 2^3 R^T (Sec. 2.3.3): u += I e on fine interior vertices.
 * A fine vertex takes weight 1 from a coarse vertex it coincides with along an
 * axis and 1/2 from each of the two coarse vertices it lies between. */
void ref_prolong_add(int Nf, const double *ec, double *u) {
    int Nc = Nf / 2, nf = Nf + 1, nc = Nc + 1;
    (void)Nc;
    #pragma omp parallel for
    for (int x = 1; x < Nf; x++)
        for (int y = 1; y < Nf; y++)
            for (int z = 1; z < Nf; z++) {
                int xs[2], ys[2], zs[2], cx, cy, cz;
                double wx, wy, wz;
                if (x % 2 == 0) { xs[0] = x / 2; cx = 1; wx = 1.0; } else { xs[0] = (x - 1) / 2; xs[1] = (x + 1) / 2; cx = 2; wx = 0.5; }
                if (y % 2 == 0) { ys[0] = y / 2; cy = 1; wy = 1.0; } else { ys[0] = (y - 1) / 2; ys[1] = (y + 1) / 2; cy = 2; wy = 0.5; }
                if (z % 2 == 0) { zs[0] = z / 2; cz = 1; wz = 1.0; } else { zs[0] = (z - 1) / 2; zs[1] = (z + 1) / 2; cz = 2; wz = 0.5; }
                double s = 0.0;
                for (int a = 0; a < cx; a++)
                    for (int b = 0; b < cy; b++)
                        for (int d = 0; d < cz; d++)
                            s += wx * wy * wz * ec[idx(nc, xs[a], ys[b], zs[d])];
                u[idx(nf, x, y, z)] += s;
            }
}

/* Exact solve on a level (used on the coarsest one): assemble the dense
 * matrix of the interior unknowns and solve by Cholesky.  Boundary entries of
 * u are the Dirichlet values and move to the right-hand side.  Supports up to
 * 27 unknowns (N <= 4). */
int ref_exact_solve(const ref_hier *H, int k, const double *q, double *u) {
    int N = H->N[k], n = N + 1, fm = H->face_mean;
    int m = (N - 1) * (N - 1) * (N - 1);
    if (m > 27) return REF_ERR_INVALID;
    double inv_h2 = 1.0 / (H->h[k] * H->h[k]);
    const double *D = H->D[k], *mu = H->mua[k];
    double A[27][27], b[27];
    size_t vid[27];
    int slot[5][5][5];
    int t = 0;
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) { slot[x][y][z] = t; vid[t++] = idx(n, x, y, z); }
    memset(A, 0, sizeof(A));
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) {
                int r = slot[x][y][z];
                size_t i = vid[r];
                int nb[6][3] = { {x + 1, y, z}, {x - 1, y, z}, {x, y + 1, z}, {x, y - 1, z}, {x, y, z + 1}, {x, y, z - 1} };
                A[r][r] = mu[i];
                b[r] = q[i];
                for (int e = 0; e < 6; e++) {
                    size_t j = idx(n, nb[e][0], nb[e][1], nb[e][2]);
                    double c = face_coef(D, i, j, inv_h2, fm);
                    A[r][r] += c;
                    if (interior(N, nb[e][0], nb[e][1], nb[e][2]))
                        A[r][slot[nb[e][0]][nb[e][1]][nb[e][2]]] -= c;
                    else
                        b[r] += c * u[j];
                }
            }
    /* Cholesky A = G G^T, in place in the lower triangle. */
    for (int j = 0; j < m; j++) {
        double d = A[j][j];
        for (int p = 0; p < j; p++) d -= A[j][p] * A[j][p];
        if (!(d > 0.0)) return REF_ERR_NONFINITE;
        A[j][j] = sqrt(d);
        for (int i = j + 1; i < m; i++) {
            double s = A[i][j];
            for (int p = 0; p < j; p++) s -= A[i][p] * A[j][p];
            A[i][j] = s / A[j][j];
        }
    }
    for (int i = 0; i < m; i++) {          /* G y = b */
        double s = b[i];
        for (int p = 0; p < i; p++) s -= A[i][p] * b[p];
        b[i] = s / A[i][i];
    }
    for (int i = m - 1; i >= 0; i--) {     /* G^T x = y */
        double s = b[i];
        for (int p = i + 1; p < m; p++) s -= A[p][i] * b[p];
        b[i] = s / A[i][i];
    }
    for (int r = 0; r < m; r++) u[vid[r]] = b[r];
    return REF_OK;
}

/* ||q - A u||_2 over interior vertices. */
static double resnorm(const ref_hier *H, int k, const double *u, const double *q, double *tmp) {
    ref_defect(H, k, u, q, tmp);
    size_t nv = nvert(H->N[k]);
    double s = 0.0;
    #pragma omp parallel for reduction(+:s)
    for (size_t v = 0; v < nv; v++) s += tmp[v] * tmp[v];
    return sqrt(s);
}

static double norm2(size_t nv, const double *a) {
    double s = 0.0;
    #pragma omp parallel for reduction(+:s)
    for (size_t v = 0; v < nv; v++) s += a[v] * a[v];
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* The V-cycle (Sec. 2.2, Fig. 1) and the solver S (Eq. (Eqcomp), Sec. 2.4). */

typedef struct ref_work {
    double *u[REF_MAXLEV], *q[REF_MAXLEV], *r[REF_MAXLEV];
} ref_work;

static void work_free(const ref_hier *H, ref_work *W) {
    for (int k = 0; k < H->L; k++) {
        if (k > 0) { free(W->u[k]); free(W->q[k]); }
        free(W->r[k]);
    }
}
static int work_alloc(const ref_hier *H, ref_work *W) {
    memset(W, 0, sizeof(*W));
    for (int k = 0; k < H->L; k++) {
        size_t nv = nvert(H->N[k]);
        W->r[k] = calloc(nv, sizeof(double));
        if (k > 0) { W->u[k] = calloc(nv, sizeof(double)); W->q[k] = calloc(nv, sizeof(double)); }
        if (!W->r[k] || (k > 0 && (!W->u[k] || !W->q[k]))) { work_free(H, W); return REF_ERR_OOM; }
    }
    return REF_OK;
}

/* One V(nu1,nu2)-cycle on level k, in place on W->u[k] with right-hand side
 * W->q[k].  order 0 = red half-sweep before black, 1 = black before red. */
static void vcycle(const ref_hier *H, ref_work *W, int k, const ref_opts *o) {
    if (k == H->L - 1) { ref_exact_solve(H, k, W->q[k], W->u[k]); return; }
    int first = o->order ? 1 : 0, second = 1 - first;
    for (int s = 0; s < o->nu1; s++) {
        if (H->smoother) { ref_wj_sweep(H, k, W->u[k], W->q[k]); continue; }
        ref_gs_half(H, k, first, W->u[k], W->q[k]);
        ref_gs_half(H, k, second, W->u[k], W->q[k]);
    }
    ref_defect(H, k, W->u[k], W->q[k], W->r[k]);                 /* Eq. (defect) */
    ref_restrict(H->N[k], W->r[k], W->q[k + 1]);                  /* Eq. (rest)   */
    memset(W->u[k + 1], 0, nvert(H->N[k + 1]) * sizeof(double));   /* Sec. 2.3.1: coarse start 0 */
    vcycle(H, W, k + 1, o);
    ref_prolong_add(H->N[k], W->u[k + 1], W->u[k]);               /* Sec. 2.3.3 */
    for (int s = 0; s < o->nu2; s++) {
        if (H->smoother) { ref_wj_sweep(H, k, W->u[k], W->q[k]); continue; }
        ref_gs_half(H, k, first, W->u[k], W->q[k]);
        ref_gs_half(H, k, second, W->u[k], W->q[k]);
    }
}

/* Apply exactly n cycles to u (in place) with right-hand side q; no
 * convergence test.  Exposed for the transposition tests. */
void ref_cycles(const ref_hier *H, const double *q, double *u, int n, int order, int nu1, int nu2) {
    ref_work W;
    if (work_alloc(H, &W)) return;
    ref_opts o = { order, nu1, nu2, 0.0, n, n };
    W.u[0] = u; W.q[0] = (double *)q;
    for (int c = 0; c < n; c++) vcycle(H, &W, 0, &o);
    work_free(H, &W);
}

/* The solver S (Sec. 2.4): rho starts at 0 in the interior and at the
 * Dirichlet value bc on the boundary, then V-cycles are applied either a fixed
 * number of times or until ||q - A rho|| / ||q - A rho_0|| <= rtol.
 * history (may be NULL) receives the relative residual after each cycle. */
int ref_solve(const ref_hier *H, double bc, const double *q, double *rho, const ref_opts *o,
              int *cycles, double *relres, double *history, int history_len) {
    int N = H->N[0], n = N + 1;
    size_t nv = nvert(N);
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++)
                rho[idx(n, x, y, z)] = interior(N, x, y, z) ? 0.0 : bc;
    ref_work W;
    if (work_alloc(H, &W)) return REF_ERR_OOM;
    W.u[0] = rho; W.q[0] = (double *)q;
    double r0 = resnorm(H, 0, rho, q, W.r[0]);
    *cycles = 0; *relres = 0.0;
    int st = REF_OK;
    if (!isfinite(r0)) { work_free(H, &W); return REF_ERR_NONFINITE; }
    if (r0 == 0.0 && o->fixed_cycles <= 0) { work_free(H, &W); return REF_OK; }
    for (int c = 1;; c++) {
        vcycle(H, &W, 0, o);
        double rel = resnorm(H, 0, rho, q, W.r[0]) / (r0 > 0.0 ? r0 : 1.0);
        *cycles = c; *relres = rel;
        if (history && c <= history_len) history[c - 1] = rel;
        if (!isfinite(rel)) { st = REF_ERR_NONFINITE; break; }
        if (o->fixed_cycles > 0) { if (c == o->fixed_cycles) break; continue; }
        if (rel <= o->rtol) break;
        if (c >= o->max_cycles) { st = REF_ERR_NOT_CONVERGED; break; }
    }
    (void)nv;
    work_free(H, &W);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Adjoints of every step (Sec. 2.3.1-2.3.3), as exact transposes, and the   */
/* pull-back S^dagger as their reversed composition (Eq. (EqcompT)).         */

/* Adjoint of one half-sweep on colour c.  The forward step overwrites the
 * colour-c interior entries with (q_c + C rho_notc) / d_c.  Given the
 * cotangent ubar of its output, the cotangent of its inputs is
 *   qbar_c += ubar_c / d_c,  ubar_notc += C^T (ubar_c / d_c),  ubar_c = 0.
 * (Sec. 2.3.1; the 1D formula there factors the coefficients for the
 * constant-coefficient case, this is the exact transpose.) */
void ref_gs_half_adj(const ref_hier *H, int k, int colour, double *ubar, double *qbar) {
    int N = H->N[k], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[k] * H->h[k]);
    const double *D = H->D[k], *mu = H->mua[k];
    const long s[6] = { (long)n * n, -(long)n * n, n, -n, 1, -1 };
    size_t nv = nvert(N);
    double *t = calloc(nv, sizeof(double));
    #pragma omp parallel for
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) {
                if (((x + y + z) & 1) != colour) continue;
                size_t i = idx(n, x, y, z);
                double den = mu[i];
                for (int e = 0; e < 6; e++)
                    den += face_coef(D, i, (size_t)((long)i + s[e]), inv_h2, fm);
                t[i] = ubar[i] / den;
            }
    #pragma omp parallel for
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) {
                size_t i = idx(n, x, y, z);
                if (((x + y + z) & 1) == colour) {
                    qbar[i] += t[i];
                    ubar[i] = 0.0;
                } else {
                    double acc = 0.0;
                    for (int e = 0; e < 6; e++) {
                        size_t j = (size_t)((long)i + s[e]);
                        acc += face_coef(D, i, j, inv_h2, fm) * t[j];  /* t = 0 off colour c */
                    }
                    ubar[i] += acc;
                }
            }
    free(t);
}

/* Adjoint of the defect r = q - A rho (Sec. 2.3.2): qbar += rbar,
 * ubar -= A rbar (A is symmetric; rbar lives on interior vertices). */
void ref_defect_adj(const ref_hier *H, int k, const double *rbar, double *ubar, double *qbar) {
    int N = H->N[k], n = N + 1;
    size_t nv = nvert(N);
    double *Ar = malloc(nv * sizeof(double));
    double *rb = malloc(nv * sizeof(double));
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t i = idx(n, x, y, z);
                rb[i] = interior(N, x, y, z) ? rbar[i] : 0.0;
            }
    ref_apply(H, k, rb, Ar);
    #pragma omp parallel for
    for (size_t v = 0; v < nv; v++) { qbar[v] += rb[v]; ubar[v] -= Ar[v]; }
    free(Ar); free(rb);
}

/* Adjoint of one weighted-Jacobi sweep rho' = rho + omega D^-1 (q - A rho)
 * (D the diagonal, interior rows): with t = omega D^-1 ubar' on interior
 * vertices, qbar += t and ubar = ubar' - A t -- the adjoint of a defect
 * applied to t. */
void ref_wj_sweep_adj(const ref_hier *H, int k, double *ubar, double *qbar) {
    int N = H->N[k], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[k] * H->h[k]);
    const double *D = H->D[k], *mu = H->mua[k];
    const long s[6] = { (long)n * n, -(long)n * n, n, -n, 1, -1 };
    size_t nv = nvert(N);
    double *t = calloc(nv, sizeof(double));
    #pragma omp parallel for
    for (int x = 1; x < N; x++)
        for (int y = 1; y < N; y++)
            for (int z = 1; z < N; z++) {
                size_t i = idx(n, x, y, z);
                double d = mu[i];
                for (int e = 0; e < 6; e++) d += face_coef(D, i, (size_t)((long)i + s[e]), inv_h2, fm);
                t[i] = H->omega * ubar[i] / d;
            }
    ref_defect_adj(H, k, t, ubar, qbar);
    free(t);
}

/* Adjoint of the V-cycle on level k.  On entry ubar is the cotangent of the
 * cycle's output; on exit it is the cotangent of the cycle's input iterate,
 * and the cotangent of the right-hand side has been added to qbar. */
static void vcycle_adj(const ref_hier *H, ref_work *U, ref_work *Q, int k, const ref_opts *o) {
    double *ub = U->u[k], *qb = Q->u[k];
    size_t nv = nvert(H->N[k]);
    if (k == H->L - 1) {
        /* Forward: u = A_c^{-1} q (input iterate discarded).  Adjoint:
         * qbar += A_c^{-1} ubar, ubar = 0; A_c is symmetric. */
        double *t = calloc(nv, sizeof(double));
        ref_exact_solve(H, k, ub, t);   /* boundary of t is 0 */
        for (size_t v = 0; v < nv; v++) { qb[v] += t[v]; ub[v] = 0.0; }
        free(t);
        return;
    }
    int first = o->order ? 1 : 0, second = 1 - first;
    for (int s = 0; s < o->nu2; s++) {           /* post-smoothing, reversed */
        if (H->smoother) { ref_wj_sweep_adj(H, k, ub, qb); continue; }
        ref_gs_half_adj(H, k, second, ub, qb);
        ref_gs_half_adj(H, k, first, ub, qb);
    }
    /* prolongation u += I e_c: ebar_c = I^T ubar = 2^3 R ubar (Sec. 2.3.3) */
    size_t nvc = nvert(H->N[k + 1]);
    ref_restrict(H->N[k], ub, U->u[k + 1]);
    for (size_t v = 0; v < nvc; v++) U->u[k + 1][v] *= 8.0;
    memset(Q->u[k + 1], 0, nvc * sizeof(double));
    vcycle_adj(H, U, Q, k + 1, o);               /* coarse start-zero: ubar_c dropped */
    /* restriction q_c = R r: rbar = R^T qbar_c = 2^-3 I qbar_c (Sec. 2.3.3) */
    double *rb = U->r[k];
    memset(rb, 0, nv * sizeof(double));
    ref_prolong_add(H->N[k], Q->u[k + 1], rb);
    for (size_t v = 0; v < nv; v++) rb[v] *= 0.125;
    ref_defect_adj(H, k, rb, ub, qb);            /* Sec. 2.3.2 */
    for (int s = 0; s < o->nu1; s++) {           /* pre-smoothing, reversed */
        if (H->smoother) { ref_wj_sweep_adj(H, k, ub, qb); continue; }
        ref_gs_half_adj(H, k, second, ub, qb);
        ref_gs_half_adj(H, k, first, ub, qb);
    }
}

/* Pull-back S^dagger rhobar (Eq. (EqcompT)): the adjoint cycles applied in
 * reverse order.  Fixed mode applies exactly fixed_cycles adjoint cycles
 * (Sec. 2.4, second mode).  Otherwise adjoint cycles are applied until the
 * carried cotangent, which equals rhobar - A qbar, satisfies
 * ||ubar|| / ||rhobar|| <= rtol.  The result is qbar (interior; boundary 0). */
int ref_pullback(const ref_hier *H, const double *rhobar, double *qbar, const ref_opts *o,
                 int *cycles, double *relres) {
    int N = H->N[0], n = N + 1;
    size_t nv = nvert(N);
    ref_work U, Q;
    if (work_alloc(H, &U)) return REF_ERR_OOM;
    if (work_alloc(H, &Q)) { work_free(H, &U); return REF_ERR_OOM; }
    double *ub = malloc(nv * sizeof(double));
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t i = idx(n, x, y, z);
                ub[i] = interior(N, x, y, z) ? rhobar[i] : 0.0;
                qbar[i] = 0.0;
            }
    U.u[0] = ub; Q.u[0] = qbar;
    double w0 = norm2(nv, ub);
    int st = REF_OK;
    *cycles = 0; *relres = 0.0;
    if (!isfinite(w0)) st = REF_ERR_NONFINITE;
    else if (w0 > 0.0 || o->fixed_cycles > 0) {
        for (int c = 1;; c++) {
            vcycle_adj(H, &U, &Q, 0, o);
            double rel = norm2(nv, ub) / (w0 > 0.0 ? w0 : 1.0);
            *cycles = c; *relres = rel;
            if (!isfinite(rel)) { st = REF_ERR_NONFINITE; break; }
            if (o->fixed_cycles > 0) { if (c == o->fixed_cycles) break; continue; }
            if (rel <= o->rtol) break;
            if (c >= o->max_cycles) { st = REF_ERR_NOT_CONVERGED; break; }
        }
    }
    free(ub);
    work_free(H, &U); work_free(H, &Q);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Derivatives with respect to the coefficients (extension; the paper lists  */
/* them as future work in Sec. 4).  These are the adjoint-state derivatives  */
/* of the discrete solution of A(logD, loglambda) rho = q.                   */

/* Tangent right-hand side: rhs = dq - (dA) rho on interior vertices, where
 * dA is the derivative of A along (dlogD, dloglambda):
 *   (dA rho)_i = sum_j dc_ij (rho_i - rho_j) + lambda_i dloglambda_i rho_i,
 *   dc_ij = d(D_f)/h^2 along dlogD (arithmetic or harmonic face mean). */
void ref_tangent_rhs(const ref_hier *H, const double *rho, const double *dq, const double *dlogD,
                     const double *dlogmua, double *rhs) {
    int N = H->N[0], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[0] * H->h[0]);
    const double *D = H->D[0], *mu = H->mua[0];
    const long s[6] = { (long)n * n, -(long)n * n, n, -n, 1, -1 };
    #pragma omp parallel for
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t i = idx(n, x, y, z);
                if (!interior(N, x, y, z)) { rhs[i] = 0.0; continue; }
                double acc = mu[i] * dlogmua[i] * rho[i];
                for (int e = 0; e < 6; e++) {
                    size_t j = (size_t)((long)i + s[e]);
                    double dDa = D[i] * dlogD[i], dDb = D[j] * dlogD[j], dDf;
                    if (fm) {
                        double sum = D[i] + D[j];
                        /* d/dD_a of 2 D_a D_b/(D_a+D_b) = 2 D_b^2/(D_a+D_b)^2 */
                        dDf = 2.0 * (D[j] * D[j] * dDa + D[i] * D[i] * dDb) / (sum * sum);
                    } else {
                        dDf = 0.5 * (dDa + dDb);
                    }
                    acc += dDf * inv_h2 * (rho[i] - rho[j]);
                }
                rhs[i] = dq[i] - acc;
            }
}

/* Coefficient gradients from the adjoint state qbar = A^{-1} rhobar:
 *   logmua_bar_i = -lambda_i qbar_i rho_i                   (interior; 0 on boundary)
 *   logD_bar_v   = -sum over faces f=(a,b) containing v of
 *                  d(c_f)/d(logD_v) (qbar_a - qbar_b)(rho_a - rho_b)
 * with qbar = 0 on boundary vertices and rho = the Dirichlet value there; the
 * sum runs over faces with at least one interior end (all vertices v). */
void ref_coef_grads(const ref_hier *H, const double *rho, const double *qbar,
                    double *logD_bar, double *logmua_bar) {
    int N = H->N[0], n = N + 1, fm = H->face_mean;
    double inv_h2 = 1.0 / (H->h[0] * H->h[0]);
    const double *D = H->D[0], *mu = H->mua[0];
    int nb[6][3] = { {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1} };
    #pragma omp parallel for
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t v = idx(n, x, y, z);
                int vin = interior(N, x, y, z);
                double lv = vin ? qbar[v] : 0.0;
                if (logmua_bar) logmua_bar[v] = vin ? -mu[v] * qbar[v] * rho[v] : 0.0;
                double acc = 0.0;
                for (int e = 0; e < 6; e++) {
                    int xa = x + nb[e][0], ya = y + nb[e][1], za = z + nb[e][2];
                    if (xa < 0 || xa > N || ya < 0 || ya > N || za < 0 || za > N) continue;
                    int jin = interior(N, xa, ya, za);
                    if (!vin && !jin) continue;
                    size_t j = idx(n, xa, ya, za);
                    double lj = jin ? qbar[j] : 0.0;
                    double dcdv;   /* d(D_f)/d(log D_v) */
                    if (fm) {
                        double sum = D[v] + D[j];
                        dcdv = 2.0 * D[j] * D[j] * D[v] / (sum * sum);
                    } else {
                        dcdv = 0.5 * D[v];
                    }
                    acc += dcdv * inv_h2 * (lv - lj) * (rho[v] - rho[j]);
                }
                if (logD_bar) logD_bar[v] = -acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Convenience entry points used by the tests.                               */

/* Forward solve S(q) (Sec. 2.4). */
int ref_forward(const ref_hier *H, const double *q, double *rho, int nu1, int nu2, double rtol,
                int max_cycles, int fixed_cycles, int *cycles, double *relres) {
    ref_opts o = { 0, nu1, nu2, rtol, max_cycles, fixed_cycles };
    return ref_solve(H, H->g, q, rho, &o, cycles, relres, NULL, 0);
}

/* Forward solve with per-cycle residual history (length max_cycles). */
int ref_forward_history(const ref_hier *H, const double *q, double *rho, int nu1, int nu2, double rtol,
                        int max_cycles, int *cycles, double *relres, double *history) {
    ref_opts o = { 0, nu1, nu2, rtol, max_cycles, 0 };
    return ref_solve(H, H->g, q, rho, &o, cycles, relres, history, max_cycles);
}

/* Push-forward: drho = S(dq - dA rho) with homogeneous boundary (Sec. 2.3:
 * S is linear in q; the coefficient part is the extension above). */
int ref_jvp(const ref_hier *H, const double *rho, const double *dq, const double *dlogD,
            const double *dlogmua, double *drho, int nu1, int nu2, double rtol, int max_cycles,
            int fixed_cycles, int *cycles, double *relres) {
    size_t nv = nvert(H->N[0]);
    double *rhs = malloc(nv * sizeof(double));
    if (!rhs) return REF_ERR_OOM;
    ref_tangent_rhs(H, rho, dq, dlogD, dlogmua, rhs);
    ref_opts o = { 0, nu1, nu2, rtol, max_cycles, fixed_cycles };
    int st = ref_solve(H, 0.0, rhs, drho, &o, cycles, relres, NULL, 0);
    free(rhs);
    return st;
}

/* Pull-back: qbar = S^dagger rhobar (literal reversed composition), then the
 * coefficient gradients.  logD_bar / logmua_bar may be NULL. */
int ref_vjp(const ref_hier *H, const double *rho, const double *rhobar, double *qbar,
            double *logD_bar, double *logmua_bar, int nu1, int nu2, double rtol, int max_cycles,
            int fixed_cycles, int *cycles, double *relres) {
    ref_opts o = { 0, nu1, nu2, rtol, max_cycles, fixed_cycles };
    int st = ref_pullback(H, rhobar, qbar, &o, cycles, relres);
    if (st == REF_OK || st == REF_ERR_NOT_CONVERGED)
        ref_coef_grads(H, rho, qbar, logD_bar, logmua_bar);
    return st;
}

/* Pull-back in q computed instead by transposed V-cycles on
 * A qbar = rhobar from qbar = 0 (used to check that this equals the literal
 * reversed composition).  Reversing a cycle's steps (Eq. (EqcompT)) turns
 * its post-smoothing into the pre-smoothing, so the transposed cycle has the
 * pre- and post-smoothing counts exchanged; red-black sweeps also run black
 * before red (with weighted Jacobi the colour order has no meaning). */
int ref_pullback_br(const ref_hier *H, const double *rhobar, double *qbar, int nu1, int nu2,
                    double rtol, int max_cycles, int fixed_cycles, int *cycles, double *relres) {
    int N = H->N[0], n = N + 1;
    size_t nv = nvert(N);
    double *w = malloc(nv * sizeof(double));
    for (int x = 0; x < n; x++)
        for (int y = 0; y < n; y++)
            for (int z = 0; z < n; z++) {
                size_t i = idx(n, x, y, z);
                w[i] = interior(N, x, y, z) ? rhobar[i] : 0.0;
            }
    ref_opts o = { 1, nu2, nu1, rtol, max_cycles, fixed_cycles };
    int st = ref_solve(H, 0.0, w, qbar, &o, cycles, relres, NULL, 0);
    free(w);
    return st;
}

/* Adjoint of the exact (coarsest-level) solve applied to a cotangent:
 * qbar = A_k^{-1} ubar with homogeneous boundary. */
int ref_exact_solve_adj(const ref_hier *H, int k, const double *ubar, double *qbar) {
    size_t nv = nvert(H->N[k]);
    memset(qbar, 0, nv * sizeof(double));
    return ref_exact_solve(H, k, ubar, qbar);
}
