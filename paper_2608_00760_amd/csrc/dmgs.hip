// dmgs.hip -- host side of the solver: plan creation, coefficient hierarchy,
// V-cycle driver, float32-in-float64 iterative refinement, push-forward,
// pull-back and the C ABI declared in include/dmgs.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "kernels_basic.hpp"
#include "plan.hpp"

using namespace dmgs;

namespace {

thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_error("%s:%d %s: %s", __FILE__, __LINE__, #expr, hipGetErrorString(e_));    \
            return DMGS_ERR_HIP;                                                            \
        }                                                                                   \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

#define TRY(expr)                        \
    do {                                 \
        int s_ = (expr);                 \
        if (s_ != DMGS_OK) return s_;    \
    } while (0)

constexpr int kBlock = 256;

unsigned grid_for(int64_t work, int64_t cap = 1 << 20) {
    int64_t b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

int levels_for(int N) {
    if (N < 2) return 0;
    int L = 1;
    while (N > 3) {
        if (N % 2) return 0;
        N /= 2;
        L++;
    }
    return L;
}

int check_options(const dmgs_options* o) {
    if (!o) { set_error("options is NULL"); return DMGS_ERR_INVALID; }
    int N = o->n[0];
    if (o->n[1] != N || o->n[2] != N) { set_error("only cubic grids are supported (n = %d,%d,%d)", o->n[0], o->n[1], o->n[2]); return DMGS_ERR_INVALID; }
    if (N < 2 || N > 1024 || levels_for(N) == 0 || levels_for(N) > kMaxLevels) {
        set_error("N = %d is not c*2^m with c in {2,3}, 2 <= N <= 1024", N);
        return DMGS_ERR_INVALID;
    }
    if (o->precision != DMGS_FP64 && o->precision != DMGS_FP32_IN_FP64) { set_error("bad precision %d", o->precision); return DMGS_ERR_INVALID; }
    if (o->smoother != DMGS_RBGS) { set_error("bad smoother %d", o->smoother); return DMGS_ERR_INVALID; }
    if (o->nu_pre < 0 || o->nu_pre > 8 || o->nu_post < 0 || o->nu_post > 8 || o->nu_pre + o->nu_post == 0) {
        set_error("bad smoothing counts %d,%d", o->nu_pre, o->nu_post);
        return DMGS_ERR_INVALID;
    }
    if (o->face_mean != DMGS_FACE_ARITH && o->face_mean != DMGS_FACE_HARMONIC) { set_error("bad face_mean"); return DMGS_ERR_INVALID; }
    if (!(o->h > 0.0) || !std::isfinite(o->h) || !std::isfinite(o->bc_value)) { set_error("bad h or bc_value"); return DMGS_ERR_INVALID; }
    if (o->fixed_cycles < 0 || o->fixed_cycles > 100000) { set_error("bad fixed_cycles"); return DMGS_ERR_INVALID; }
    if (o->fixed_cycles == 0 && (!(o->rtol > 0.0) || o->max_cycles < 1)) { set_error("bad rtol or max_cycles"); return DMGS_ERR_INVALID; }
    return DMGS_OK;
}

// Byte sizes of every allocation, in allocation order (used both to allocate
// and to report the footprint).
struct Sizes {
    int L;
    int64_t nv[kMaxLevels];
};

Sizes sizes_for(const dmgs_options* o) {
    Sizes s;
    s.L = levels_for(o->n[0]);
    int N = o->n[0];
    for (int k = 0; k < s.L; k++, N /= 2) s.nv[k] = (int64_t)(N + 1) * (N + 1) * (N + 1);
    return s;
}

size_t footprint(const dmgs_options* o) {
    Sizes s = sizes_for(o);
    bool ir = o->precision == DMGS_FP32_IN_FP64;
    size_t b = 0;
    for (int k = 0; k < s.L; k++) {
        b += 2 * s.nv[k] * sizeof(double);                            // D64, mu64
        if (ir) b += 5 * s.nv[k] * sizeof(float);                     // D32, mu32, u32, q32, t32
        else b += (k > 0 ? 3 : 1) * s.nv[k] * sizeof(double);         // (u64, q64), t64
    }
    b += s.nv[0] * sizeof(double);                                    // scratch64
    b += kMaxPartials * sizeof(double) + 4 * sizeof(double) + sizeof(int);
    return b;
}

template <class T>
int dalloc(dmgs_plan P, T** p, int64_t count) {
    hipError_t e = hipMalloc((void**)p, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        set_error("hipMalloc of %lld bytes failed: %s", (long long)(count * sizeof(T)), hipGetErrorString(e));
        return DMGS_ERR_OOM;
    }
    P->bytes += (size_t)count * sizeof(T);
    return DMGS_OK;
}

void free_plan(dmgs_plan P) {
    if (!P) return;
    for (int k = 0; k < P->L; k++) {
        Level& l = P->lev[k];
        void* ps[] = {l.D64, l.mu64, l.D32, l.mu32, l.u64, l.q64, l.t64, l.u32, l.q32, l.t32};
        for (void* p : ps)
            if (p) (void)hipFree(p);
    }
    if (P->scratch64) (void)hipFree(P->scratch64);
    if (P->partial) (void)hipFree(P->partial);
    if (P->dnorm) (void)hipFree(P->dnorm);
    if (P->dflag) (void)hipFree(P->dflag);
    if (P->hnorm) (void)hipHostFree(P->hnorm);
    if (P->hflag) (void)hipHostFree(P->hflag);
    if (P->ev_start) (void)hipEventDestroy(P->ev_start);
    if (P->ev_stop) (void)hipEventDestroy(P->ev_stop);
    for (int i = 0; i < 2 * kTimerSlots; i++)
        if (P->tev[i]) (void)hipEventDestroy(P->tev[i]);
    delete P;
}

bool is_ir(dmgs_plan P) { return P->opt.precision == DMGS_FP32_IN_FP64; }
int harmonic(dmgs_plan P) { return P->opt.face_mean == DMGS_FACE_HARMONIC; }

// ---------------------------------------------------------------------------
// Kernel timing: finest-level launches bracketed by events when enabled.

int timing_flush(dmgs_plan P) {
    for (int i = 0; i < P->tpending; i++) {
        float ms = 0.f;
        HIPCHK(hipEventSynchronize(P->tev[2 * i + 1]));
        HIPCHK(hipEventElapsedTime(&ms, P->tev[2 * i], P->tev[2 * i + 1]));
        int c = P->trec[i].cls;
        P->t_count[c]++;
        P->t_ms[c] += ms;
        P->t_bytes[c] += P->trec[i].bytes;
    }
    P->tpending = 0;
    return DMGS_OK;
}

int tbeg(dmgs_plan P, int k, hipStream_t st, int* slot) {
    *slot = -1;
    if (!P->timing || k != 0) return DMGS_OK;
    if (P->tpending == kTimerSlots) TRY(timing_flush(P));
    *slot = P->tpending++;
    HIPCHK(hipEventRecord(P->tev[2 * *slot], st));
    return DMGS_OK;
}

int tend(dmgs_plan P, int slot, int cls, double bytes, hipStream_t st) {
    if (slot < 0) return DMGS_OK;
    P->trec[slot].cls = cls;
    P->trec[slot].bytes = bytes;
    HIPCHK(hipEventRecord(P->tev[2 * slot + 1], st));
    return DMGS_OK;
}

// Launch `launch` on level k; on the finest level, time it as class `cls`
// moving `bytes` algorithmic bytes.
#define TIMED(P, k, cls, bytes, st, launch)              \
    do {                                                 \
        int slot_;                                       \
        TRY(tbeg((P), (k), (st), &slot_));               \
        launch;                                          \
        LAUNCHCHK();                                     \
        TRY(tend((P), slot_, (cls), (bytes), (st)));     \
    } while (0)

// ---------------------------------------------------------------------------
// Cycle building blocks (one launch per operation).

template <class T>
int fill(T* a, int64_t nv, T val, hipStream_t st) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(nv)), dim3(kBlock), 0, st, a, nv, val);
    LAUNCHCHK();
    return DMGS_OK;
}

template <class T>
int half_sweep(dmgs_plan P, int k, T* u, const T* q, int colour, hipStream_t st) {
    const Level& l = P->lev[k];
    int64_t total = (int64_t)(l.N - 1) * (l.N - 1) * (l.N / 2);
    // reads all of u and D, the colour's q and mua, writes the colour's u
    TIMED(P, k, DMGS_K_SMOOTH, 3.5 * l.nv * sizeof(T), st,
          hipLaunchKernelGGL(k_gs_half<T>, dim3(grid_for(total, INT64_C(1) << 30)), dim3(kBlock), 0, st, u, q,
                             (const T*)Typed<T>::D(l), (const T*)Typed<T>::mu(l), l.N, l.stencil<T>(harmonic(P)), colour));
    return DMGS_OK;
}

template <class T>
int sweeps(dmgs_plan P, int k, T* u, const T* q, int count, int order, hipStream_t st) {
    int first = order ? 1 : 0;
    for (int s = 0; s < count; s++) {
        TRY(half_sweep<T>(P, k, u, q, first, st));
        TRY(half_sweep<T>(P, k, u, q, 1 - first, st));
    }
    return DMGS_OK;
}

template <class T>
int apply_or_defect(dmgs_plan P, int k, const T* u, const T* q, T* out, int apply_only, hipStream_t st) {
    const Level& l = P->lev[k];
    TIMED(P, k, DMGS_K_DEFECT_RESTRICT, 5.0 * l.nv * sizeof(T), st,
          hipLaunchKernelGGL(k_defect<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, u, q, (const T*)Typed<T>::D(l),
                             (const T*)Typed<T>::mu(l), out, l.N, l.stencil<T>(harmonic(P)), apply_only));
    return DMGS_OK;
}

// pre pass: nu_pre sweeps in place on u, then qc = R (q - A u).
template <class T>
int pre_pass(dmgs_plan P, int k, T* u, const T* q, T* qc, int order, hipStream_t st) {
    const Level& l = P->lev[k];
    TRY(sweeps<T>(P, k, u, q, P->opt.nu_pre, order, st));
    T* r = Typed<T>::t(l);
    TRY(apply_or_defect<T>(P, k, u, q, r, 0, st));
    TIMED(P, k, DMGS_K_DEFECT_RESTRICT, (double)(l.nv + P->lev[k + 1].nv) * sizeof(T), st,
          hipLaunchKernelGGL(k_restrict<T>, dim3(grid_for(P->lev[k + 1].nv)), dim3(kBlock), 0, st, (const T*)r, qc, l.N));
    return DMGS_OK;
}

// post pass: u += I ec, then nu_post sweeps in place.
template <class T>
int post_pass(dmgs_plan P, int k, T* u, const T* ec, const T* q, int order, hipStream_t st) {
    const Level& l = P->lev[k];
    TIMED(P, k, DMGS_K_PROLONG, (double)(2 * l.nv + P->lev[k + 1].nv) * sizeof(T), st,
          hipLaunchKernelGGL(k_prolong_add<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, ec, u, l.N));
    return sweeps<T>(P, k, u, q, P->opt.nu_post, order, st);
}

template <class T>
int coarsest(dmgs_plan P, const T* q, T* u, hipStream_t st) {
    const Level& l = P->lev[P->L - 1];
    hipLaunchKernelGGL(k_exact_solve<T>, dim3(1), dim3(64), 0, st, q, u, (const double*)l.D64, (const double*)l.mu64,
                       l.N, l.stencil<double>(harmonic(P)));
    LAUNCHCHK();
    return DMGS_OK;
}

// One V-cycle on level k: u[k] updated in place with right-hand side q[k];
// coarser levels use the plan's arrays of type T (start-from-zero
// corrections).
template <class T>
int vcycle(dmgs_plan P, int k, T* u, const T* q, int order, hipStream_t st) {
    if (k == P->L - 1) return coarsest<T>(P, q, u, st);
    const Level& c = P->lev[k + 1];
    T* uc = Typed<T>::u(c);
    T* qc = Typed<T>::q(c);
    TRY(pre_pass<T>(P, k, u, q, qc, order, st));
    TRY(fill<T>(uc, c.nv, T(0), st));
    TRY(vcycle<T>(P, k + 1, uc, qc, order, st));
    return post_pass<T>(P, k, u, uc, q, order, st);
}

// Squared residual norm of level 0 (float64) into dnorm[slot]; u == nullptr
// gives ||q||^2.
int resid_sq64(dmgs_plan P, const double* u, const double* q, int slot, hipStream_t st) {
    const Level& l = P->lev[0];
    unsigned nb = grid_for(l.nv, kMaxPartials);
    TIMED(P, 0, DMGS_K_RESIDUAL, 4.0 * l.nv * sizeof(double), st,
          hipLaunchKernelGGL(k_resid_sq<double>, dim3(nb), dim3(kBlock), 0, st, u, q, (const double*)l.D64,
                             (const double*)l.mu64, l.N, l.stencil<double>(harmonic(P)), P->partial));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)nb, P->dnorm, slot);
    LAUNCHCHK();
    return DMGS_OK;
}

// Iterative-refinement residual: level-0 q32 = float(b - A x), ||.||^2 into dnorm[slot].
int resid_cast(dmgs_plan P, const double* x, const double* b, int slot, hipStream_t st) {
    const Level& l = P->lev[0];
    unsigned nb = grid_for(l.nv, kMaxPartials);
    TIMED(P, 0, DMGS_K_RESIDUAL, 36.0 * l.nv, st,
          hipLaunchKernelGGL(k_resid_cast, dim3(nb), dim3(kBlock), 0, st, x, b, (const double*)l.D64, (const double*)l.mu64,
                             l.N, l.stencil<double>(harmonic(P)), l.q32, P->partial));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)nb, P->dnorm, slot);
    LAUNCHCHK();
    return DMGS_OK;
}

int read_norms(dmgs_plan P, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(P->hnorm, P->dnorm, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (P->timing) TRY(timing_flush(P));
    return DMGS_OK;
}

// Solve A x = b on the finest level from x = 0 (interior) / bc (boundary).
// order 0: red-first cycles (S); order 1: black-first cycles (S^T).
int solve(dmgs_plan P, const double* b, double* x, double bc, int order, dmgs_info* info, hipStream_t st) {
    const dmgs_options& o = P->opt;
    const Level& l0 = P->lev[0];
    const bool fixed = o.fixed_cycles > 0;
    hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, l0.N, bc);
    LAUNCHCHK();
    int cycles = 0, status = DMGS_OK;
    double r0 = 0.0, rel = 0.0;
    if (!is_ir(P)) {
        TRY(resid_sq64(P, x, b, 0, st));
        if (!fixed) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            if (!std::isfinite(r0)) { set_error("non-finite right-hand side"); status = DMGS_ERR_NONFINITE; goto done; }
            if (r0 == 0.0) goto done;
        }
        for (cycles = 1;; cycles++) {
            TRY(vcycle<double>(P, 0, x, b, order, st));
            if (fixed) {
                if (cycles == o.fixed_cycles) break;
                continue;
            }
            TRY(resid_sq64(P, x, b, 1, st));
            TRY(read_norms(P, st));
            rel = std::sqrt(P->hnorm[1]) / r0;
            if (!std::isfinite(rel)) { set_error("non-finite residual after %d cycles", cycles); status = DMGS_ERR_NONFINITE; break; }
            if (rel <= o.rtol) break;
            if (cycles >= o.max_cycles) { set_error("not converged after %d cycles (rel %.3e)", cycles, rel); status = DMGS_ERR_NOT_CONVERGED; break; }
        }
        if (fixed && info) {
            TRY(resid_sq64(P, x, b, 1, st));
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            rel = std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0);
        }
    } else {
        float* e = l0.u32;
        for (cycles = 0;; cycles++) {
            TRY(resid_cast(P, x, b, cycles == 0 ? 0 : 1, st));
            if (!fixed) {
                TRY(read_norms(P, st));
                if (cycles == 0) {
                    r0 = std::sqrt(P->hnorm[0]);
                    if (!std::isfinite(r0)) { set_error("non-finite right-hand side"); status = DMGS_ERR_NONFINITE; break; }
                    if (r0 == 0.0) break;
                    rel = 1.0;
                } else {
                    rel = std::sqrt(P->hnorm[1]) / r0;
                    if (!std::isfinite(rel)) { set_error("non-finite residual after %d steps", cycles); status = DMGS_ERR_NONFINITE; break; }
                    if (rel <= o.rtol) break;
                }
                if (cycles >= o.max_cycles) { set_error("not converged after %d steps (rel %.3e)", cycles, rel); status = DMGS_ERR_NOT_CONVERGED; break; }
            } else if (cycles == o.fixed_cycles) {
                break;
            }
            TRY(fill<float>(e, l0.nv, 0.0f, st));
            TRY(vcycle<float>(P, 0, e, l0.q32, order, st));
            TIMED(P, 0, DMGS_K_UPDATE, 20.0 * l0.nv, st,
                  hipLaunchKernelGGL(k_add_correction, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, (const float*)e, l0.nv));
        }
        if (fixed && info) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            rel = std::sqrt(P->hnorm[o.fixed_cycles > 0 ? 1 : 0]) / (r0 > 0.0 ? r0 : 1.0);
        }
    }
done:
    if (info) {
        info->cycles = cycles;
        info->rel_residual = rel;
        info->status = status;
    }
    return status;
}

int begin_call(dmgs_plan P, hipStream_t st, bool need_coef = true) {
    if (!P) { set_error("plan is NULL"); return DMGS_ERR_INVALID; }
    if (need_coef && !P->coef_set) { set_error("coefficients not set"); return DMGS_ERR_INVALID; }
    HIPCHK(hipSetDevice(P->device));
    HIPCHK(hipEventRecord(P->ev_start, st));
    return DMGS_OK;
}

int end_call(dmgs_plan P, int status, dmgs_info* info, hipStream_t st) {
    if (P->timing && P->tpending) {
        int s = timing_flush(P);
        if (s != DMGS_OK && status == DMGS_OK) status = s;
    }
    if (info) {
        info->status = status;
        info->device_ms = 0.0;
        if (hipEventRecord(P->ev_stop, st) == hipSuccess && hipEventSynchronize(P->ev_stop) == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, P->ev_start, P->ev_stop) == hipSuccess) info->device_ms = ms;
        }
    }
    return status;
}

int build_hierarchy(dmgs_plan P, hipStream_t st) {
    Level& l0 = P->lev[0];
    *P->hflag = 0;
    HIPCHK(hipMemsetAsync(P->dflag, 0, sizeof(int), st));
    TIMED(P, 0, DMGS_K_COEF, 16.0 * l0.nv, st,
          hipLaunchKernelGGL(k_validate, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, (const double*)l0.D64,
                             (const double*)l0.mu64, l0.N, P->dflag));
    HIPCHK(hipMemcpyAsync(P->hflag, P->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (*P->hflag) {
        P->coef_set = false;
        set_error("coefficients must satisfy D > 0, mua >= 0 and be finite");
        return DMGS_ERR_INVALID;
    }
    for (int k = 1; k < P->L; k++) {
        const Level& f = P->lev[k - 1];
        Level& c = P->lev[k];
        hipLaunchKernelGGL(k_coarsen_coef, dim3(grid_for(c.nv)), dim3(kBlock), 0, st, (const double*)f.D64, c.D64, f.N);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_coarsen_coef, dim3(grid_for(c.nv)), dim3(kBlock), 0, st, (const double*)f.mu64, c.mu64, f.N);
        LAUNCHCHK();
    }
    if (is_ir(P)) {
        for (int k = 0; k < P->L; k++) {
            Level& l = P->lev[k];
            hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, (const double*)l.D64, l.D32, l.nv);
            LAUNCHCHK();
            hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, (const double*)l.mu64, l.mu32, l.nv);
            LAUNCHCHK();
        }
    }
    P->coef_set = true;
    return DMGS_OK;
}

int debug_check(dmgs_plan P, int k, int fp32, bool need_coarse) {
    if (!P || !P->coef_set) { set_error("plan without coefficients"); return DMGS_ERR_INVALID; }
    if (k < 0 || k >= P->L || (need_coarse && k >= P->L - 1)) { set_error("bad level %d", k); return DMGS_ERR_INVALID; }
    if (fp32 && !is_ir(P)) { set_error("float32 arrays need a DMGS_FP32_IN_FP64 plan"); return DMGS_ERR_INVALID; }
    if (hipSetDevice(P->device) != hipSuccess) { set_error("hipSetDevice failed"); return DMGS_ERR_HIP; }
    return DMGS_OK;
}

template <class T>
int debug_pre_t(dmgs_plan P, int k, int order, const T* u_in, const T* q, T* u_out, T* qc, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(u_out, u_in, P->lev[k].nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    return pre_pass<T>(P, k, u_out, q, qc, order, st);
}

template <class T>
int debug_post_t(dmgs_plan P, int k, int order, const T* u_in, const T* ec, const T* q, T* u_out, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(u_out, u_in, P->lev[k].nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    return post_pass<T>(P, k, u_out, ec, q, order, st);
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

void dmgs_default_options(int32_t n, dmgs_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n[0] = o->n[1] = o->n[2] = n;
    o->precision = DMGS_FP64;
    o->smoother = DMGS_RBGS;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->max_cycles = 200;
    o->fixed_cycles = 0;
    o->face_mean = DMGS_FACE_ARITH;
    o->h = 1.0;
    o->bc_value = 0.0;
    o->rtol = 1e-10;
}

size_t dmgs_workspace_bytes(const dmgs_options* o) {
    if (check_options(o) != DMGS_OK) return 0;
    return footprint(o);
}

int dmgs_plan_create(const dmgs_options* o, dmgs_plan* out) {
    if (!out) { set_error("out is NULL"); return DMGS_ERR_INVALID; }
    *out = nullptr;
    TRY(check_options(o));
    dmgs_plan P = new (std::nothrow) dmgs_plan_s();
    if (!P) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
    P->opt = *o;
    if (hipGetDevice(&P->device) != hipSuccess) { delete P; set_error("hipGetDevice failed"); return DMGS_ERR_HIP; }
    Sizes s = sizes_for(o);
    P->L = s.L;
    bool ir = o->precision == DMGS_FP32_IN_FP64;
    int st = DMGS_OK;
    int N = o->n[0];
    double h = o->h;
    for (int k = 0; k < s.L && st == DMGS_OK; k++, N /= 2, h *= 2.0) {
        Level& l = P->lev[k];
        l.N = N;
        l.n = N + 1;
        l.nv = s.nv[k];
        l.h = h;
        l.inv_h2 = 1.0 / (h * h);
        if (st == DMGS_OK) st = dalloc(P, &l.D64, l.nv);
        if (st == DMGS_OK) st = dalloc(P, &l.mu64, l.nv);
        if (ir) {
            if (st == DMGS_OK) st = dalloc(P, &l.D32, l.nv);
            if (st == DMGS_OK) st = dalloc(P, &l.mu32, l.nv);
            if (st == DMGS_OK) st = dalloc(P, &l.u32, l.nv);
            if (st == DMGS_OK) st = dalloc(P, &l.q32, l.nv);
            if (st == DMGS_OK) st = dalloc(P, &l.t32, l.nv);
        } else {
            if (k > 0 && st == DMGS_OK) st = dalloc(P, &l.u64, l.nv);
            if (k > 0 && st == DMGS_OK) st = dalloc(P, &l.q64, l.nv);
            if (st == DMGS_OK) st = dalloc(P, &l.t64, l.nv);
        }
    }
    if (st == DMGS_OK) st = dalloc(P, &P->scratch64, P->lev[0].nv);
    if (st == DMGS_OK) st = dalloc(P, &P->partial, kMaxPartials);
    if (st == DMGS_OK) st = dalloc(P, &P->dnorm, 4);
    if (st == DMGS_OK) st = dalloc(P, &P->dflag, 1);
    if (st == DMGS_OK && hipHostMalloc((void**)&P->hnorm, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        st = DMGS_ERR_OOM;
    }
    if (st == DMGS_OK && hipHostMalloc((void**)&P->hflag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        st = DMGS_ERR_OOM;
    }
    if (st == DMGS_OK && (hipEventCreate(&P->ev_start) != hipSuccess || hipEventCreate(&P->ev_stop) != hipSuccess)) {
        set_error("hipEventCreate failed");
        st = DMGS_ERR_HIP;
    }
    if (st != DMGS_OK) {
        free_plan(P);
        return st;
    }
    *out = P;
    return DMGS_OK;
}

int dmgs_plan_destroy(dmgs_plan P) {
    if (!P) return DMGS_OK;
    (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    free_plan(P);
    return DMGS_OK;
}

int dmgs_plan_levels(dmgs_plan P) { return P ? P->L : 0; }
int dmgs_plan_level_n(dmgs_plan P, int k) { return (P && k >= 0 && k < P->L) ? P->lev[k].N : 0; }

int dmgs_set_coefficients(dmgs_plan P, const double* D, const double* mua, void* stream) {
    if (!P || !D || !mua) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(P->device));
    Level& l0 = P->lev[0];
    HIPCHK(hipMemcpyAsync(l0.D64, D, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(l0.mu64, mua, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    return build_hierarchy(P, st);
}

int dmgs_set_log_coefficients(dmgs_plan P, const double* logD, const double* logmua, void* stream) {
    if (!P || !logD || !logmua) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(P->device));
    Level& l0 = P->lev[0];
    hipLaunchKernelGGL(k_exp_copy, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, logD, l0.D64, l0.nv);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_exp_copy, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, logmua, l0.mu64, l0.nv);
    LAUNCHCHK();
    return build_hierarchy(P, st);
}

int dmgs_forward(dmgs_plan P, const double* q, double* rho, dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!q || !rho) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    int s = solve(P, q, rho, P->opt.bc_value, 0, info, st);
    return end_call(P, s, info, st);
}

int dmgs_jvp(dmgs_plan P, const double* rho, const double* dq, const double* dlogD, const double* dlogmua, double* drho,
             dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!rho || !drho) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    const Level& l0 = P->lev[0];
    TIMED(P, 0, DMGS_K_GRAD, 56.0 * l0.nv, st,
          hipLaunchKernelGGL(k_tangent_rhs, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, rho, dq, dlogD, dlogmua,
                             (const double*)l0.D64, (const double*)l0.mu64, l0.N, l0.inv_h2, harmonic(P), P->scratch64));
    int s = solve(P, P->scratch64, drho, 0.0, 0, info, st);
    return end_call(P, s, info, st);
}

int dmgs_vjp(dmgs_plan P, const double* rho, const double* rhobar, double* qbar, double* logD_bar, double* logmua_bar,
             dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!rho || !rhobar || !qbar) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    int s = solve(P, rhobar, qbar, 0.0, 1, info, st);
    if ((s == DMGS_OK || s == DMGS_ERR_NOT_CONVERGED) && (logD_bar || logmua_bar)) {
        const Level& l0 = P->lev[0];
        TIMED(P, 0, DMGS_K_GRAD, 48.0 * l0.nv, st,
              hipLaunchKernelGGL(k_coef_grads, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, rho, (const double*)qbar,
                                 (const double*)l0.D64, (const double*)l0.mu64, l0.N, l0.inv_h2, harmonic(P), logD_bar,
                                 logmua_bar));
    }
    return end_call(P, s, info, st);
}

int dmgs_solve_once(const dmgs_options* o, const double* D, const double* mua, const double* q, double* rho,
                    dmgs_info* info, void* stream) {
    dmgs_plan P = nullptr;
    TRY(dmgs_plan_create(o, &P));
    int s = dmgs_set_coefficients(P, D, mua, stream);
    if (s == DMGS_OK) s = dmgs_forward(P, q, rho, info, stream);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && s == DMGS_OK) s = DMGS_ERR_HIP;
    dmgs_plan_destroy(P);
    return s;
}

const char* dmgs_status_string(int s) {
    switch (s) {
        case DMGS_OK: return "ok";
        case DMGS_ERR_INVALID: return "invalid argument";
        case DMGS_ERR_OOM: return "out of device memory";
        case DMGS_ERR_NOT_CONVERGED: return "not converged";
        case DMGS_ERR_NONFINITE: return "non-finite value";
        case DMGS_ERR_HIP: return "HIP runtime error";
        case DMGS_ERR_BUDGET: return "memory budget exceeded";
        default: return "unknown status";
    }
}

const char* dmgs_last_error(void) { return g_err; }

int dmgs_timing_enable(dmgs_plan P, int enable) {
    if (!P) { set_error("plan is NULL"); return DMGS_ERR_INVALID; }
    HIPCHK(hipSetDevice(P->device));
    if (P->tpending) TRY(timing_flush(P));
    if (enable && !P->tev[0])
        for (int i = 0; i < 2 * kTimerSlots; i++) HIPCHK(hipEventCreate(&P->tev[i]));
    P->timing = enable != 0;
    for (int c = 0; c < DMGS_K_COUNT; c++) {
        P->t_count[c] = 0;
        P->t_ms[c] = 0.0;
        P->t_bytes[c] = 0.0;
    }
    return DMGS_OK;
}

int dmgs_timing_read(dmgs_plan P, int cls, int64_t* launches, double* total_ms, double* bytes) {
    if (!P || cls < 0 || cls >= DMGS_K_COUNT) { set_error("bad plan or kernel class"); return DMGS_ERR_INVALID; }
    if (P->tpending) TRY(timing_flush(P));
    if (launches) *launches = P->t_count[cls];
    if (total_ms) *total_ms = P->t_ms[cls];
    if (bytes) *bytes = P->t_bytes[cls];
    return DMGS_OK;
}

// ---------------------------------------------------------------------------
// Diagnostic entry points.

int dmgs_debug_apply(dmgs_plan P, int k, int fp32, const void* u, void* out, void* stream) {
    TRY(debug_check(P, k, fp32, false));
    hipStream_t st = (hipStream_t)stream;
    if (fp32) return apply_or_defect<float>(P, k, (const float*)u, (const float*)u, (float*)out, 1, st);
    // float64 plans have no level-0 scratch of type float; use the typed path
    return apply_or_defect<double>(P, k, (const double*)u, (const double*)u, (double*)out, 1, st);
}

int dmgs_debug_level_coefficients(dmgs_plan P, int k, double* D, double* mua, void* stream) {
    TRY(debug_check(P, k, 0, false));
    hipStream_t st = (hipStream_t)stream;
    const Level& l = P->lev[k];
    HIPCHK(hipMemcpyAsync(D, l.D64, l.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(mua, l.mu64, l.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    return DMGS_OK;
}

int dmgs_debug_pre(dmgs_plan P, int k, int fp32, int order, const void* u_in, const void* q, void* u_out, void* qc,
                   void* stream) {
    TRY(debug_check(P, k, fp32, true));
    hipStream_t st = (hipStream_t)stream;
    if (fp32) return debug_pre_t<float>(P, k, order, (const float*)u_in, (const float*)q, (float*)u_out, (float*)qc, st);
    if (!P->lev[k].t64) { set_error("no float64 scratch"); return DMGS_ERR_INVALID; }
    return debug_pre_t<double>(P, k, order, (const double*)u_in, (const double*)q, (double*)u_out, (double*)qc, st);
}

int dmgs_debug_post(dmgs_plan P, int k, int fp32, int order, const void* u_in, const void* ec, const void* q,
                    void* u_out, void* stream) {
    TRY(debug_check(P, k, fp32, true));
    hipStream_t st = (hipStream_t)stream;
    if (fp32) return debug_post_t<float>(P, k, order, (const float*)u_in, (const float*)ec, (const float*)q, (float*)u_out, st);
    return debug_post_t<double>(P, k, order, (const double*)u_in, (const double*)ec, (const double*)q, (double*)u_out, st);
}

int dmgs_debug_coarsest(dmgs_plan P, int fp32, const void* q, void* u, void* stream) {
    TRY(debug_check(P, P ? P->L - 1 : 0, fp32, false));
    hipStream_t st = (hipStream_t)stream;
    const Level& l = P->lev[P->L - 1];
    if (fp32) {
        TRY(fill<float>((float*)u, l.nv, 0.0f, st));
        return coarsest<float>(P, (const float*)q, (float*)u, st);
    }
    TRY(fill<double>((double*)u, l.nv, 0.0, st));
    return coarsest<double>(P, (const double*)q, (double*)u, st);
}

int dmgs_debug_cycles(dmgs_plan P, int order, int ncycles, const double* q, double* u, void* stream) {
    TRY(debug_check(P, 0, 0, false));
    if (is_ir(P)) { set_error("dmgs_debug_cycles needs a DMGS_FP64 plan"); return DMGS_ERR_INVALID; }
    hipStream_t st = (hipStream_t)stream;
    for (int c = 0; c < ncycles; c++) TRY(vcycle<double>(P, 0, u, q, order, st));
    return DMGS_OK;
}

}  // extern "C"
