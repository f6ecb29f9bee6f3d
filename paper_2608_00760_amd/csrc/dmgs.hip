// dmgs.hip -- host side of the solver: plan creation, coefficient hierarchy,
// V-cycle driver, float32-in-float64 iterative refinement, push-forward,
// pull-back and the C ABI declared in include/dmgs.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <algorithm>
#include <utility>
#include <new>
#include <string>
#include <thread>
#include <mutex>
#include <vector>

#include "kernels_basic.hpp"
#include "kernels_stream.hpp"
#include "kernels_sweep2.hpp"
#include "kernels_deriv.hpp"
#include "kernels_block.hpp"
#include "kernels_small.hpp"
#include "kernels_2d.hpp"
#include "kernels_epilogue.hpp"
#include "kernels_unrolled.hpp"
#include "kernels_grid.hpp"
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

// A failed HIP call is reported through the return code; HIP's per-thread
// last error is cleared as well, so that a later call on this thread (after
// an out-of-memory, say) is not failed by the next launch check.
#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            (void)hipGetLastError();                                                        \
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

// One thread per vertex in whole blocks, rounded up to a multiple of the 8
// XCDs (kernels using vertex_of_thread()).
unsigned vertex_grid(int64_t nv) { return (unsigned)(((nv + kBlock - 1) / kBlock + 7) / 8 * 8); }

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

// Spacing of axis a (h_axis[a], or h when it is 0).
double axis_h(const dmgs_options* o, int a) { return o->h_axis[a] > 0.0 ? o->h_axis[a] : o->h; }

// A three-dimensional plan with different cell counts or spacings per axis.
bool general_grid(const dmgs_options* o) {
    if (o->ndim != 3) return false;
    return o->n[0] != o->n[1] || o->n[1] != o->n[2] || axis_h(o, 0) != axis_h(o, 1) || axis_h(o, 1) != axis_h(o, 2);
}

// Levels of a general grid: every axis halves until the smallest count is 2
// or 3 (cn receives the counts of each level); 0 when the counts do not
// halve down so.
int grid_levels(const int32_t* n, int cn[][3]) {
    int c[3] = {n[0], n[1], n[2]};
    for (int a = 0; a < 3; a++)
        if (c[a] < 2) return 0;
    int L = 0;
    while (true) {
        if (L >= kMaxLevels) return 0;
        for (int a = 0; a < 3; a++) cn[L][a] = c[a];
        L++;
        const int m = std::min(c[0], std::min(c[1], c[2]));
        if (m <= 3) return (m == 2 || m == 3) ? L : 0;
        for (int a = 0; a < 3; a++) {
            if (c[a] % 2) return 0;
            c[a] /= 2;
        }
    }
}

int check_options(const dmgs_options* o) {
    if (!o) { set_error("options is NULL"); return DMGS_ERR_INVALID; }
    int N = o->n[0];
    if (o->ndim != 2 && o->ndim != 3) { set_error("bad ndim %d", o->ndim); return DMGS_ERR_INVALID; }
    const int nmax = o->ndim == 2 ? 16384 : 1024;
    for (int a = 0; a < 3 && o->ndim == 3; a++)
        if (!(o->h_axis[a] >= 0.0) || !std::isfinite(o->h_axis[a])) { set_error("bad h_axis"); return DMGS_ERR_INVALID; }
    if (general_grid(o)) {
        int cn[kMaxLevels][3];
        const int L = grid_levels(o->n, cn);
        if (L == 0 || std::max(o->n[0], std::max(o->n[1], o->n[2])) > nmax) {
            set_error("cell counts %d,%d,%d do not halve down to a smallest count of 2 or 3 (each 2..%d)", o->n[0],
                      o->n[1], o->n[2], nmax);
            return DMGS_ERR_INVALID;
        }
        if ((cn[L - 1][0] - 1) * (cn[L - 1][1] - 1) * (cn[L - 1][2] - 1) > kGridCoarseMax) {
            set_error("the coarsest level (%d,%d,%d cells) has more than %d interior vertices", cn[L - 1][0],
                      cn[L - 1][1], cn[L - 1][2], kGridCoarseMax);
            return DMGS_ERR_INVALID;
        }
        if (o->precision != DMGS_FP64 || o->smoother != DMGS_RBGS) {
            set_error("general-grid plans take DMGS_FP64 and DMGS_RBGS");
            return DMGS_ERR_INVALID;
        }
    } else if (o->n[1] != N || (o->ndim == 3 && o->n[2] != N)) {
        set_error("two-dimensional plans are square (n = %d,%d)", o->n[0], o->n[1]);
        return DMGS_ERR_INVALID;
    } else if (N < 2 || N > nmax || levels_for(N) == 0 || levels_for(N) > kMaxLevels) {
        set_error("N = %d is not c*2^m with c in {2,3}, 2 <= N <= %d", N, nmax);
        return DMGS_ERR_INVALID;
    }
    if (o->ndim == 2 && (o->precision != DMGS_FP64 || o->smoother != DMGS_RBGS)) {
        set_error("two-dimensional plans take DMGS_FP64 and DMGS_RBGS");
        return DMGS_ERR_INVALID;
    }
    if (o->precision != DMGS_FP64 && o->precision != DMGS_FP32_IN_FP64) { set_error("bad precision %d", o->precision); return DMGS_ERR_INVALID; }
    if (o->smoother != DMGS_RBGS && o->smoother != DMGS_WJACOBI) { set_error("bad smoother %d", o->smoother); return DMGS_ERR_INVALID; }
    if (o->adjoint_schedule != 0 && o->adjoint_schedule != 1) { set_error("bad adjoint_schedule %d", o->adjoint_schedule); return DMGS_ERR_INVALID; }
    if (o->nu_pre < 0 || o->nu_pre > 8 || o->nu_post < 0 || o->nu_post > 8 || o->nu_pre + o->nu_post == 0) {
        set_error("bad smoothing counts %d,%d", o->nu_pre, o->nu_post);
        return DMGS_ERR_INVALID;
    }
    if (o->face_mean != DMGS_FACE_ARITH && o->face_mean != DMGS_FACE_HARMONIC) { set_error("bad face_mean"); return DMGS_ERR_INVALID; }
    if (!(o->h > 0.0) || !std::isfinite(o->h) || !std::isfinite(o->bc_value)) { set_error("bad h or bc_value"); return DMGS_ERR_INVALID; }
    if (o->fixed_cycles < 0 || o->fixed_cycles > 100000) { set_error("bad fixed_cycles"); return DMGS_ERR_INVALID; }
    if (o->precision == DMGS_FP32_IN_FP64 && (o->ir_inner_cycles < 1 || o->ir_inner_cycles > 16)) {
        set_error("bad ir_inner_cycles %d", o->ir_inner_cycles);
        return DMGS_ERR_INVALID;
    }
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
    if (general_grid(o)) {
        int cn[kMaxLevels][3];
        s.L = grid_levels(o->n, cn);
        for (int k = 0; k < s.L; k++) s.nv[k] = (int64_t)(cn[k][0] + 1) * (cn[k][1] + 1) * (cn[k][2] + 1);
        return s;
    }
    s.L = levels_for(o->n[0]);
    int N = o->n[0];
    for (int k = 0; k < s.L; k++, N /= 2)
        s.nv[k] = (int64_t)(N + 1) * (N + 1) * (o->ndim == 2 ? 1 : (N + 1));
    return s;
}

// Tuning knobs of cubic plans that decide which kernels run on the finest
// level (environment variables; plan_init keeps them in the plan).
struct Knobs {
    int fuse_min, sweep2_min, block_max, defect;
    bool pad;
};

Knobs read_knobs(const dmgs_options* o) {
    const bool ir = o->precision == DMGS_FP32_IN_FP64;
    // float64 plans have no block passes: their two-sweep passes reach down
    // to the levels the small-level kernel leaves (one launch per phase
    // instead of two)
    Knobs k{ir ? 32 : 16, ir ? 64 : 16, 64, 2, true};
    if (const char* e = std::getenv("DMGS_FUSE_MIN")) k.fuse_min = std::max(8, std::atoi(e));
    if (const char* e = std::getenv("DMGS_SWEEP2_MIN")) k.sweep2_min = std::max(16, std::atoi(e));
    if (const char* e = std::getenv("DMGS_BLOCK_MAX")) k.block_max = std::atoi(e);
    if (const char* e = std::getenv("DMGS_SWEEP2_DEFECT")) k.defect = std::min(2, std::max(0, std::atoi(e)));
    if (const char* e = std::getenv("DMGS_PAD")) k.pad = std::atoi(e) != 0;
    return k;
}

// Row pitch of the finest level's float32 arrays.  Refinement plans pad the
// rows to a multiple of four elements (n = 257: 1040-byte rows instead of
// 1028) when every kernel that runs on that level takes a pitch: red-black
// smoothing by two-sweep passes only (even smoothing counts), no block or
// simple passes, a coarser level.  A tile's rows then fall on different
// memory channels; the two-sweep pass at 256^3 moves the same bytes about
// 12 % faster.
int fine_row_pitch(const dmgs_options* o, const Knobs& kn, int L) {
    const int N = o->n[0], n = N + 1;
    const bool ok = kn.pad && o->ndim == 3 && !general_grid(o) && o->precision == DMGS_FP32_IN_FP64 &&
                    o->smoother == DMGS_RBGS && L > 1 && o->nu_pre >= 2 && o->nu_pre % 2 == 0 && o->nu_post >= 2 &&
                    o->nu_post % 2 == 0 && N >= kn.fuse_min && N > kn.block_max && N >= kn.sweep2_min;
    if (!ok) return n;
    const int py = (n + 3) / 4 * 4;
    return sweep2_fits<float>(N, (int64_t)py * n) ? py : n;
}

// Float32 elements allocated per array on level k (padded rows on the finest).
int64_t nv32_of(const dmgs_options* o, const Sizes& s, int k, int py0) {
    if (k > 0 || o->ndim == 2) return s.nv[k];
    const int64_t n = o->n[0] + 1;
    return n * n * py0;
}

size_t footprint(const dmgs_options* o) {
    Sizes s = sizes_for(o);
    bool ir = o->precision == DMGS_FP32_IN_FP64;
    size_t b = 0;
    if (general_grid(o)) {
        // per level D64, mu64, (u64, q64 below the finest), (t64: the defect,
        // above the coarsest); the finest scratch; partials, the coarsest
        // inverse, norm slots and the flag
        for (int k = 0; k < s.L; k++)
            b += (2 + (k > 0 ? 2 : 0) + (k < s.L - 1 ? 1 : 0)) * s.nv[k] * sizeof(double);
        b += s.nv[0] * sizeof(double);
        b += kMaxPartials * sizeof(double) + kGridCoarseMax * kGridCoarseMax * sizeof(double) + 4 * sizeof(double) +
             sizeof(int);
        return b;
    }
    const int py0 = fine_row_pitch(o, read_knobs(o), s.L);
    for (int k = 0; k < s.L; k++) {
        if (o->ndim == 2) {   // D64, mu64, (u64, q64), t64, (rd64)
            b += ((k > 0 ? 5 : 3) + (k < s.L - 1 ? 1 : 0)) * s.nv[k] * sizeof(double);
            continue;
        }
        b += 2 * s.nv[k] * sizeof(double);                            // D64, mu64
        if (ir) b += (k < s.L - 1 ? 7 : 6) * nv32_of(o, s, k, py0) * sizeof(float);  // D32, mu32, w32, u32, q32, t32, (r32)
        else b += (k > 0 ? 4 : 2) * s.nv[k] * sizeof(double);         // w64, (u64, q64), t64
    }
    b += (ir ? 2 : 1) * s.nv[0] * sizeof(double);                     // scratch64 (+ xalt64)
    b += kMaxPartials * sizeof(double) + kCoarseMax * kCoarseMax * sizeof(double) + 4 * sizeof(double) + sizeof(int);
    return b;
}

// Slack of an arena plan over its footprint: each buffer starts on a 256-byte
// boundary (at most kMaxLevels * 12 + 8 buffers).
constexpr size_t kArenaSlack = 64 * 1024;

template <class T>
int dalloc(dmgs_plan P, T** p, int64_t count) {
    if (P->arena) {
        const size_t off = (P->arena_used + 255) & ~(size_t)255;
        const size_t bytes = (size_t)count * sizeof(T);
        if (off + bytes > P->arena_cap) {
            *p = nullptr;
            set_error("the plan needs more than the %zu bytes of its arena", P->arena_cap);
            return DMGS_ERR_INVALID;
        }
        *p = reinterpret_cast<T*>(P->arena + off);
        P->arena_used = off + bytes;
        P->bytes += bytes;
        return DMGS_OK;
    }
    hipError_t e = hipMalloc((void**)p, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();   // reported here; not left for the next launch check
        set_error("hipMalloc of %lld bytes failed: %s", (long long)(count * sizeof(T)), hipGetErrorString(e));
        return DMGS_ERR_OOM;
    }
    P->bytes += (size_t)count * sizeof(T);
    return DMGS_OK;
}

void free_plan(dmgs_plan P) {
    if (!P) return;
    if (P->arena) return;   // arena plans own no resources and live in static storage
    if (P->unwork && P->unwork_free) P->unwork_free(P->unwork);
    if (P->twin) free_plan(P->twin);
    if (P->twin_stream) (void)hipStreamDestroy(P->twin_stream);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    for (int k = 0; k < P->L; k++) {
        Level& l = P->lev[k];
        void* work[] = {l.u64, l.q64, l.t64, l.u32, l.q32, l.t32, l.r32, l.rd64};
        for (void* p : work)
            if (p) (void)hipFree(p);
        if (!P->owns_coef) continue;
        void* coef[] = {l.D64, l.mu64, l.w64, l.D32, l.mu32, l.w32};
        for (void* p : coef)
            if (p) (void)hipFree(p);
    }
    if (P->scratch64) (void)hipFree(P->scratch64);
    if (P->xalt64) (void)hipFree(P->xalt64);
    if (P->partial) (void)hipFree(P->partial);
    if (P->cinv && P->owns_coef) (void)hipFree(P->cinv);
    if (P->dflag) (void)hipFree(P->dflag);
    if (P->hnorm) (void)hipHostFree(P->hnorm);
    if (P->hflag) (void)hipHostFree(P->hflag);
    if (P->ev_start) (void)hipEventDestroy(P->ev_start);
    if (P->ev_stop) (void)hipEventDestroy(P->ev_stop);
    if (P->ev_norm) (void)hipEventDestroy(P->ev_norm);
    if (P->ev_flag) (void)hipEventDestroy(P->ev_flag);
    for (int i = 0; i < 2 * kTimerSlots; i++)
        if (P->tev[i]) (void)hipEventDestroy(P->tev[i]);
    delete P;
}

bool is_ir(dmgs_plan P) { return P->opt.precision == DMGS_FP32_IN_FP64; }

// Where the reductions write their norms: the pinned host slots, or the
// device slots of an arena plan (copied to the host by read_norms).
double* norm_dst(dmgs_plan P) { return P->arena ? P->dnorm : P->hnorm; }

// After the last norm reduction enqueued on st.
int mark_norms(dmgs_plan P, hipStream_t st) {
    if (P->rec) return DMGS_OK;   // a batch tick synchronises itself
    if (!P->arena) HIPCHK(hipEventRecord(P->ev_norm, st));
    P->tmark = P->tpending;
    return DMGS_OK;
}
bool is2d(dmgs_plan P) { return P->opt.ndim == 2; }
int harmonic(dmgs_plan P) { return P->opt.face_mean == DMGS_FACE_HARMONIC; }

// ---------------------------------------------------------------------------
// Kernel timing: finest-level launches bracketed by events when enabled.

// Accumulate the first `upto` pending slots (all by default); later slots
// move to the front.
int timing_flush(dmgs_plan P, int upto = -1) {
    if (upto < 0 || upto > P->tpending) upto = P->tpending;
    for (int i = 0; i < upto; i++) {
        float ms = 0.f;
        HIPCHK(hipEventSynchronize(P->tev[2 * i + 1]));
        HIPCHK(hipEventElapsedTime(&ms, P->tev[2 * i], P->tev[2 * i + 1]));
        int c = P->trec[i].cls;
        P->t_count[c]++;
        P->t_ms[c] += ms;
        P->t_bytes[c] += P->trec[i].bytes;
    }
    for (int i = upto; i < P->tpending; i++) {
        std::swap(P->tev[2 * (i - upto)], P->tev[2 * i]);
        std::swap(P->tev[2 * (i - upto) + 1], P->tev[2 * i + 1]);
        P->trec[i - upto] = P->trec[i];
    }
    P->tpending -= upto;
    return DMGS_OK;
}

// Launch of class cls on level k: times it (slot >= 0) when timing is on,
// k is the finest level and it is the class's sampled launch.
int tbeg(dmgs_plan P, int k, hipStream_t st, int* slot, int cls) {
    *slot = -1;
    if (!P->timing || k != 0 || P->rec) return DMGS_OK;
    if (P->t_seen[cls]++ % P->tstride != 0) return DMGS_OK;
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
        TRY(tbeg((P), (k), (st), &slot_, (cls)));        \
        launch;                                          \
        LAUNCHCHK();                                     \
        TRY(tend((P), slot_, (cls), (bytes), (st)));     \
    } while (0)

// ---------------------------------------------------------------------------
// Cycle building blocks.  Levels with N >= kFuseMin use the fused streaming
// passes (out of place, ping-pong between the level's two buffers); smaller
// levels use one launch per operation, in place.

// Lay `count` recorded launches of one grouped kernel out as its Group table.
template <class Args>
void write_group(unsigned char* dst, const RecOp* const* ops, int count, const int* start) {
    Group<Args>* g = reinterpret_cast<Group<Args>*>(dst);
    std::memset(g, 0, sizeof(Group<Args>));
    g->count = count;
    for (int i = 0; i <= count; i++) g->start[i] = start[i];
    for (int i = 0; i < count; i++) {
        g->nblk[i] = (int)ops[i]->nblk;
        std::memcpy(&g->a[i], ops[i]->args, sizeof(Args));
    }
}

// Launch kernel `solo` with the one argument a, or, while the plan records
// (grouped execution), append the launch of its grouped form `grp` instead.
template <class Args>
int launch_rec(dmgs_plan P, const void* solo, const void* grp, unsigned nb, unsigned threads, size_t lds, const Args& a,
               hipStream_t st) {
    if (P->rec) {
        static_assert(sizeof(Args) <= sizeof(RecOp::args), "kernel arguments exceed a recorded launch");
        if (!grp) { set_error("internal: a launch without a grouped form in grouped execution"); return DMGS_ERR_INVALID; }
        RecOp op;
        op.fn = grp;
        op.nblk = nb;
        op.threads = threads;
        op.lds = lds;
        op.table_bytes = sizeof(Group<Args>);
        op.write = write_group<Args>;
        std::memcpy(op.args, &a, sizeof(Args));
        P->rec->push_back(op);
        return DMGS_OK;
    }
    void* kargs[] = {const_cast<Args*>(&a)};
    HIPCHK(hipLaunchKernel(solo, dim3(nb), dim3(threads), kargs, lds, st));
    return DMGS_OK;
}

template <class T>
int fill(T* a, int64_t nv, T val, hipStream_t st) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(nv)), dim3(kBlock), 0, st, a, nv, val);
    LAUNCHCHK();
    return DMGS_OK;
}

template <class T>
int set_boundary(T* u, int N, T g, hipStream_t st) {
    int n = N + 1;
    hipLaunchKernelGGL(k_set_boundary<T>, dim3(grid_for((int64_t)n * n, 1024), 6), dim3(kBlock), 0, st, u, N, g);
    LAUNCHCHK();
    return DMGS_OK;
}

// Kernels that take dense fields only refuse a padded level (a plan pads its
// finest level only when none of them runs there).
template <class T>
int need_dense(dmgs_plan P, int k, const char* what) {
    if (dense<T>(P->lev[k])) return DMGS_OK;
    set_error("internal: %s on the padded level %d", what, k);
    return DMGS_ERR_INVALID;
}

template <class T>
int half_sweep(dmgs_plan P, int k, T* u, const T* q, int colour, hipStream_t st) {
    const Level& l = P->lev[k];
    TRY(need_dense<T>(P, k, "half-sweep"));
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
                             (const T*)Typed<T>::mu(l), out, l.N, l.stencil<T>(harmonic(P)), apply_only,
                             Typed<T>::py(l), Typed<T>::px(l)));
    return DMGS_OK;
}

// --- fused pass dispatch -------------------------------------------------------

// chunk of x-planes per workgroup: about 512 workgroups (two per CU), chunks
// of at least 4 planes (each chunk re-reads a few planes at its ends)
int choose_chunk(int interior, int tiles) {
    int want = 512;
    int nch = (want + tiles - 1) / tiles;
    int chunk = (interior + nch - 1) / nch;
    if (chunk < 4) chunk = 4;
    if (chunk > interior) chunk = interior;
    return chunk;
}

// Sweep-pass tiles (TY x TZ); the float32 choice is selectable for tuning
// by DMGS_SWEEP_CFG = 0 (16 x 64), 1 (8 x 64), 2 (16 x 32).
template <class T, int TY, int TZ, bool HARM>
int launch_sweep(const SweepArgs<T>& a0, int N, int mode, hipStream_t st) {
    SweepArgs<T> a = a0;
    constexpr int NT = SweepShape<TY, TZ>::NT;
    a.tiles_y = (N + TY - 1) / TY;
    a.tiles_z = (N + TZ - 1) / TZ;
    a.chunk = choose_chunk(N - 1, a.tiles_y * a.tiles_z);
    a.nchunks = (N - 1 + a.chunk - 1) / a.chunk;
    int nb = a.tiles_y * a.tiles_z * a.nchunks;
    if (mode == kSweepZero) hipLaunchKernelGGL((k_rb_sweep_col<T, TY, TZ, kSweepZero, HARM>), dim3(nb), dim3(NT), 0, st, a);
    else if (mode == kSweepProlong) hipLaunchKernelGGL((k_rb_sweep_col<T, TY, TZ, kSweepProlong, HARM>), dim3(nb), dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_rb_sweep_col<T, TY, TZ, kSweepPlain, HARM>), dim3(nb), dim3(NT), 0, st, a);
    LAUNCHCHK();
    return DMGS_OK;
}

template <class T, bool HARM>
int launch_sweep_cfg(dmgs_plan P, const SweepArgs<T>& a, int N, int mode, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        return launch_sweep<T, 8, 64, HARM>(a, N, mode, st);
    } else {
        if (N <= 64) return launch_sweep<T, 8, 32, HARM>(a, N, mode, st);
        switch (P->cfg_sweep) {
            case 1: return launch_sweep<T, 8, 64, HARM>(a, N, mode, st);
            case 2: return launch_sweep<T, 16, 32, HARM>(a, N, mode, st);
            default: return launch_sweep<T, 16, 64, HARM>(a, N, mode, st);
        }
    }
}

// One fused sweep pass: u_out = one red-black sweep applied to u_in (or to
// 0 when zero, or to u_in + I ec when ec is given).
template <class T>
int smooth_pass(dmgs_plan P, int k, const T* u_in, T* u_out, const T* q, int order, bool zero, const T* ec,
                hipStream_t st) {
    const Level& l = P->lev[k];
    TRY(need_dense<T>(P, k, "one-sweep pass"));
    SweepArgs<T> a;
    a.u_in = u_in;
    a.u_out = u_out;
    a.q = q;
    a.D = Typed<T>::D(l);
    a.w = Typed<T>::w(l);
    a.ec = ec;
    a.N = l.N;
    a.order = order;
    a.st = l.stencil<T>(harmonic(P));
    const int mode = zero ? kSweepZero : (ec ? kSweepProlong : kSweepPlain);
    // algorithmic bytes: read u (unless zero), q, D, w, (ec), write u
    double words = (zero ? 4.0 : 5.0) + (ec ? 0.125 : 0.0);
    int slot;
    TRY(tbeg(P, k, st, &slot, DMGS_K_SMOOTH));
    if (harmonic(P)) TRY((launch_sweep_cfg<T, true>(P, a, l.N, mode, st)));
    else TRY((launch_sweep_cfg<T, false>(P, a, l.N, mode, st)));
    TRY(tend(P, slot, DMGS_K_SMOOTH, words * l.nv * sizeof(T), st));
    return DMGS_OK;
}

// Grid of a two-sweep pass over level size N with TY x TZ tiles: chunks of
// x-planes sized for about cfg_sweep2_wgs workgroups, at least 8 planes (a
// chunk recomputes 3 planes at each end).  Returns the number of workgroups.
template <class T>
int sweep2_grid(dmgs_plan P, SweepArgs<T>& a, int N, int TY, int TZ) {
    a.tiles_y = (N + TY - 1) / TY;
    a.tiles_z = (N + TZ - 1) / TZ;
    const int tiles = a.tiles_y * a.tiles_z;
    const int wgs = N == P->lev[0].N ? P->cfg_sweep2_wgs : P->cfg_sweep2_wgs_coarse;
    int nch = std::max(1, (wgs + tiles - 1) / tiles);
    if (N == P->lev[0].N && P->cfg_sweep2_wgs == 256) {
        // finest level: one workgroup per CU, so pick the chunk count whose
        // workgroups fill the last round of CUs best, net of the 6 extra
        // march steps a chunk costs
        double best = 0.0;
        for (int c = 1; c <= 32; c++) {
            const int chunk = std::min(N - 1, std::max(8, (N - 1 + c - 1) / c));
            const int nb = tiles * ((N - 1 + chunk - 1) / chunk);
            const int rounds = (nb + P->ncu - 1) / P->ncu;
            const double v = (double)nb / ((double)rounds * P->ncu) * chunk / (chunk + 6.0);
            if (v > best + 1e-9) {
                best = v;
                nch = c;
            }
        }
    }
    a.chunk = std::min(N - 1, std::max(8, (N - 1 + nch - 1) / nch));
    a.nchunks = (N - 1 + a.chunk - 1) / a.chunk;
    return tiles * a.nchunks;
}

// NORM: a plain pass that also leaves the per-block sums of its input's
// squared residual in a.partial (*nb_out blocks).
template <class T, int TY, int TZ, bool HARM, bool DEFECT, bool NORM = false>
int launch_sweep2(dmgs_plan P, const SweepArgs<T>& a0, int N, int mode, hipStream_t st, unsigned* nb_out = nullptr) {
    SweepArgs<T> a = a0;
    constexpr int RING = DEFECT ? 5 : 4;
    constexpr int NT = Sweep2Shape<TY, TZ, RING>::NT;
    constexpr size_t lds = sweep2_lds_bytes<T, TY, TZ, RING>();
    const int nb = sweep2_grid<T>(P, a, N, TY, TZ);
    if (nb_out) *nb_out = (unsigned)nb;
    if constexpr (NORM) {
        if (mode != kSweepPlain || nb > kMaxPartials || !a.partial) {
            set_error("internal: two-sweep norm pass needs a plain pass of at most %d workgroups", kMaxPartials);
            return DMGS_ERR_INVALID;
        }
        if (P->rec) { set_error("internal: the float64 norm pass in grouped execution"); return DMGS_ERR_INVALID; }
        hipLaunchKernelGGL((k_rb_sweep2_col<T, TY, TZ, kSweepPlain, HARM, false, true>), dim3(nb), dim3(NT), lds, st, a);
        LAUNCHCHK();
        return DMGS_OK;
    }
    // grouped forms exist for the float32 passes (refinement plans)
    auto go = [&](auto Mc) {
        constexpr int M = decltype(Mc)::value;
        const void* grp = nullptr;
        if constexpr (sizeof(T) == 4) grp = (const void*)k_rb_sweep2_grp<T, TY, TZ, M, HARM, DEFECT>;
        return launch_rec(P, (const void*)k_rb_sweep2_col<T, TY, TZ, M, HARM, DEFECT>, grp, (unsigned)nb, NT, lds, a, st);
    };
    if (mode == kSweepZero) return go(std::integral_constant<int, kSweepZero>());
    if (mode == kSweepPlain) return go(std::integral_constant<int, kSweepPlain>());
    if constexpr (!DEFECT) return go(std::integral_constant<int, kSweepProlong>());
    set_error("internal: no defect output after prolongation");
    return DMGS_ERR_INVALID;
}

constexpr int kSweep2TY = 16, kSweep2TZ = 64;     // tiles of the two-sweep passes
constexpr int kSweep2DTY = 16, kSweep2DTZ = 64;   // ... of the passes that also write the defect
constexpr int kSweep2TZ64 = 32;                   // float64 passes: tiles of 16 x 32

// Dynamic-LDS limits of the two-sweep kernels (set once per plan).
int sweep2_attributes() {
    constexpr int lds = (int)sweep2_lds_bytes<float, kSweep2TY, kSweep2TZ>();
    constexpr int ldsd = (int)sweep2_lds_bytes<float, kSweep2DTY, kSweep2DTZ, 5>();
    constexpr int lds64 = (int)sweep2_lds_bytes<double, kSweep2TY, kSweep2TZ64>();
    static_assert(lds64 <= 160 * 1024, "float64 two-sweep ring exceeds the LDS");
    const std::pair<const void*, int> fns[] = {
        {(const void*)k_rb_sweep2_col<float, kSweep2TY, kSweep2TZ, kSweepPlain, false>, lds},
        {(const void*)k_rb_sweep2_col<float, kSweep2TY, kSweep2TZ, kSweepZero, false>, lds},
        {(const void*)k_rb_sweep2_col<float, kSweep2TY, kSweep2TZ, kSweepProlong, false>, lds},
        {(const void*)k_rb_sweep2_col<float, kSweep2TY, kSweep2TZ, kSweepPlain, true>, lds},
        {(const void*)k_rb_sweep2_col<float, kSweep2TY, kSweep2TZ, kSweepZero, true>, lds},
        {(const void*)k_rb_sweep2_col<float, kSweep2TY, kSweep2TZ, kSweepProlong, true>, lds},
        {(const void*)k_rb_sweep2_col<float, kSweep2DTY, kSweep2DTZ, kSweepPlain, false, true>, ldsd},
        {(const void*)k_rb_sweep2_col<float, kSweep2DTY, kSweep2DTZ, kSweepZero, false, true>, ldsd},
        {(const void*)k_rb_sweep2_col<float, kSweep2DTY, kSweep2DTZ, kSweepPlain, true, true>, ldsd},
        {(const void*)k_rb_sweep2_col<float, kSweep2DTY, kSweep2DTZ, kSweepZero, true, true>, ldsd},
        {(const void*)k_rb_sweep2_grp<float, kSweep2TY, kSweep2TZ, kSweepPlain, false>, lds},
        {(const void*)k_rb_sweep2_grp<float, kSweep2TY, kSweep2TZ, kSweepZero, false>, lds},
        {(const void*)k_rb_sweep2_grp<float, kSweep2TY, kSweep2TZ, kSweepProlong, false>, lds},
        {(const void*)k_rb_sweep2_grp<float, kSweep2TY, kSweep2TZ, kSweepPlain, true>, lds},
        {(const void*)k_rb_sweep2_grp<float, kSweep2TY, kSweep2TZ, kSweepZero, true>, lds},
        {(const void*)k_rb_sweep2_grp<float, kSweep2TY, kSweep2TZ, kSweepProlong, true>, lds},
        {(const void*)k_rb_sweep2_grp<float, kSweep2DTY, kSweep2DTZ, kSweepPlain, false, true>, ldsd},
        {(const void*)k_rb_sweep2_grp<float, kSweep2DTY, kSweep2DTZ, kSweepZero, false, true>, ldsd},
        {(const void*)k_rb_sweep2_grp<float, kSweep2DTY, kSweep2DTZ, kSweepPlain, true, true>, ldsd},
        {(const void*)k_rb_sweep2_grp<float, kSweep2DTY, kSweep2DTZ, kSweepZero, true, true>, ldsd},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepPlain, false>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepZero, false>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepProlong, false>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepPlain, true>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepZero, true>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepProlong, true>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepPlain, false, false, true>, lds64},
        {(const void*)k_rb_sweep2_col<double, kSweep2TY, kSweep2TZ64, kSweepPlain, true, false, true>, lds64}};
    for (const auto& f : fns)
        if (hipFuncSetAttribute(f.first, hipFuncAttributeMaxDynamicSharedMemorySize, f.second) != hipSuccess) {
            (void)hipGetLastError(); set_error("hipFuncSetAttribute failed");
            return DMGS_ERR_HIP;
        }
    return DMGS_OK;
}

// Two-sweep passes need a zero Dirichlet boundary (float32 corrections)
// and whole-field buffer offsets below kOob.
// The two-sweep pass needs a zero boundary: every float32 correction, every
// coarse level, and the float64 finest level when the solve's boundary value
// is 0 (the adjoint and tangent solves always; the forward solve when g = 0).
bool use_sweep2(dmgs_plan P, int k, size_t tsize) {
    if (P->lev[k].N < P->cfg_sweep2_min) return false;
    const Level& l = P->lev[k];
    if (tsize == 4) return sweep2_fits<float>(l.N, Typed<float>::px(l));
    return P->cfg_sweep2_fp64 && (k > 0 || P->bc_zero) && sweep2_fits<double>(l.N, Typed<double>::px(l));
}

// One two-sweep pass: u_out = two red-black sweeps applied to u_in (or to
// 0, or to u_in + I ec).
// norm_partial (float64, plain passes): also the per-block sums of the
// input's squared residual there (*nb_out blocks).
template <class T>
int smooth_pass2(dmgs_plan P, int k, const T* u_in, T* u_out, const T* q, int order, bool zero, const T* ec,
                 hipStream_t st, T* r = nullptr, double* norm_partial = nullptr, unsigned* nb_out = nullptr) {
    const Level& l = P->lev[k];
    SweepArgs<T> a;
    a.u_in = u_in;
    a.u_out = u_out;
    a.q = q;
    a.D = Typed<T>::D(l);
    a.w = Typed<T>::w(l);
    a.ec = ec;
    a.r = r;
    a.py = Typed<T>::py(l);
    a.px = Typed<T>::px(l);
    a.N = l.N;
    a.order = order;
    a.st = l.stencil<T>(harmonic(P));
    const int mode = zero ? kSweepZero : (ec ? kSweepProlong : kSweepPlain);
    if (r && ec) { set_error("two-sweep pass: defect only after pre-smoothing"); return DMGS_ERR_INVALID; }
    if (norm_partial && (sizeof(T) != 8 || zero || ec || r)) {
        set_error("internal: the two-sweep norm pass is a plain float64 pass");
        return DMGS_ERR_INVALID;
    }
    // algorithmic bytes: read u (unless zero), q, D, w, (ec), write u, (r) -- once for both sweeps
    double words = (zero ? 4.0 : 5.0) + (ec ? 0.125 : 0.0) + (r ? 1.0 : 0.0);
    int slot;
    TRY(tbeg(P, k, st, &slot, DMGS_K_SMOOTH));
    if constexpr (sizeof(T) == 4) {
        const bool h = harmonic(P);
        if (r) TRY(h ? (launch_sweep2<T, kSweep2DTY, kSweep2DTZ, true, true>(P, a, l.N, mode, st))
                     : (launch_sweep2<T, kSweep2DTY, kSweep2DTZ, false, true>(P, a, l.N, mode, st)));
        else TRY(h ? (launch_sweep2<T, kSweep2TY, kSweep2TZ, true, false>(P, a, l.N, mode, st))
                   : (launch_sweep2<T, kSweep2TY, kSweep2TZ, false, false>(P, a, l.N, mode, st)));
    } else {
        // float64: half-width tiles (the LDS ring holds twice the bytes);
        // no defect-writing variant
        if (r) { set_error("two-sweep pass: no defect output in float64"); return DMGS_ERR_INVALID; }
        if (norm_partial) {
            a.partial = norm_partial;
            TRY(harmonic(P) ? (launch_sweep2<T, kSweep2TY, kSweep2TZ64, true, false, true>(P, a, l.N, mode, st, nb_out))
                            : (launch_sweep2<T, kSweep2TY, kSweep2TZ64, false, false, true>(P, a, l.N, mode, st, nb_out)));
        } else {
            TRY(harmonic(P) ? (launch_sweep2<T, kSweep2TY, kSweep2TZ64, true, false>(P, a, l.N, mode, st))
                            : (launch_sweep2<T, kSweep2TY, kSweep2TZ64, false, false>(P, a, l.N, mode, st)));
        }
    }
    TRY(tend(P, slot, DMGS_K_SMOOTH, words * l.nv * sizeof(T), st));
    return DMGS_OK;
}

// Chunks of coarse planes sized for about cfg_dr_wgs workgroups (each
// chunk re-reads the fine planes at its ends), at least 4.
template <class T, int TYC, int TZC, bool HARM, bool FROM_R>
int launch_restrict(dmgs_plan P, const RestrictArgs<T>& a0, int Nc, hipStream_t st) {
    RestrictArgs<T> a = a0;
    constexpr int NT = RestrictShape<TYC, TZC>::NT;
    a.tiles_y = (Nc - 1 + TYC - 1) / TYC;
    a.tiles_z = (Nc - 1 + TZC - 1) / TZC;
    const int tiles = a.tiles_y * a.tiles_z;
    const int nch = std::max(1, (P->cfg_dr_wgs + tiles - 1) / tiles);
    a.chunk = std::max(4, (Nc - 1 + nch - 1) / nch);
    if (a.chunk > Nc - 1) a.chunk = Nc - 1;
    a.nchunks = (Nc - 1 + a.chunk - 1) / a.chunk;
    int nb = a.tiles_y * a.tiles_z * a.nchunks;
    const void* grp = nullptr;
    if constexpr (sizeof(T) == 4) grp = (const void*)k_defect_restrict_grp<T, TYC, TZC, HARM, FROM_R>;
    return launch_rec(P, (const void*)k_defect_restrict_col<T, TYC, TZC, HARM, FROM_R>, grp, (unsigned)nb, NT, 0, a, st);
}

// qc = R (q - A u); from_r: u holds the defect itself after pre-smoothing
// whose first colour was `order` (the other colour's defect is 0), qc = R u.
template <class T>
int defect_restrict(dmgs_plan P, int k, const T* u, const T* q, T* qc, hipStream_t st, bool from_r = false,
                    int order = 0) {
    const Level& l = P->lev[k];
    const Level& c = P->lev[k + 1];
    RestrictArgs<T> a;
    a.u = u;
    a.q = q;
    a.D = Typed<T>::D(l);
    a.mu = Typed<T>::mu(l);
    a.qc = qc;
    a.py = Typed<T>::py(l);
    a.px = Typed<T>::px(l);
    a.N = l.N;
    a.rzero = order ? 0 : 1;
    a.st = l.stencil<T>(harmonic(P));
    constexpr int TYC = 8, TZC = sizeof(T) == 4 ? 32 : 16;
    int slot;
    TRY(tbeg(P, k, st, &slot, DMGS_K_DEFECT_RESTRICT));
    if (from_r) TRY((launch_restrict<T, TYC, TZC, false, true>(P, a, c.N, st)));
    else if (harmonic(P)) TRY((launch_restrict<T, TYC, TZC, true, false>(P, a, c.N, st)));
    else TRY((launch_restrict<T, TYC, TZC, false, false>(P, a, c.N, st)));
    TRY(tend(P, slot, DMGS_K_DEFECT_RESTRICT, ((from_r ? 1.0 : 4.0) * l.nv + c.nv) * sizeof(T), st));
    return DMGS_OK;
}

// Smoothing phase of `nsweeps` red-black sweeps on level k starting from
// *cur (zero: from 0; ec: add I ec first, fused into the first sweep).
// Result left in *cur, which swaps between the level's two buffers.
// rout: when the phase ends with a two-sweep pass, that pass also writes
// the defect of the result to rout and *rdone is set.
template <class T>
int smooth_phase(dmgs_plan P, int k, T** cur, T** other, const T* q, int nsweeps, int order, bool zero, const T* ec,
                 hipStream_t st, T* rout = nullptr, bool* rdone = nullptr) {
    if (rdone) *rdone = false;
    const Level& l = P->lev[k];
    if (nsweeps == 0) {
        TRY(need_dense<T>(P, k, "smoothing phase without sweeps"));
        if (zero) TRY(fill<T>(*cur, l.nv, T(0), st));
        if (ec) {
            TIMED(P, k, DMGS_K_PROLONG, (double)(2 * l.nv + P->lev[k + 1].nv) * sizeof(T), st,
                  hipLaunchKernelGGL(k_prolong_add<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, ec, *cur, l.N));
        }
        return DMGS_OK;
    }
    for (int i = 0; i < nsweeps;) {
        const bool z = i == 0 && zero;
        const T* e = i == 0 ? ec : nullptr;
        if (nsweeps - i >= 2 && use_sweep2(P, k, sizeof(T))) {
            const bool want = P->cfg_defect == 2 || (P->cfg_defect == 1 && z);
            T* r = (want && nsweeps - i == 2 && !e && rout && rdone) ? rout : nullptr;
            TRY(smooth_pass2<T>(P, k, *cur, *other, q, order, z, e, st, r));
            if (r) *rdone = true;
            i += 2;
        } else {
            TRY(smooth_pass<T>(P, k, *cur, *other, q, order, z, e, st));
            i += 1;
        }
        std::swap(*cur, *other);
    }
    return DMGS_OK;
}

template <class T>
int coarsest(dmgs_plan P, const T* q, T* u, hipStream_t st) {
    const Level& l = P->lev[P->L - 1];
    hipLaunchKernelGGL(k_exact_solve<T>, dim3(1), dim3(64), 0, st, q, u, (const double*)l.D64, (const double*)l.mu64,
                       l.N, l.stencil<double>(harmonic(P)));
    LAUNCHCHK();
    return DMGS_OK;
}

bool fused_level(dmgs_plan P, int k) { return P->lev[k].N >= P->cfg_fuse_min && k < P->L - 1; }

// Mid-size float32 levels run each smoothing phase as one block launch
// (zero boundary: the refinement corrections; two sweeps each way).
template <class T>
bool block_level(dmgs_plan P, int k) {
    const int N = P->lev[k].N;
    return sizeof(T) == 4 && is_ir(P) && k < P->L - 1 && N > 16 && N <= P->cfg_block_max && P->opt.nu_pre == 2 &&
           P->opt.nu_post == 2;
}

constexpr int kBlockB = 8;

template <class T, int MODE, bool HARM>
int launch_block_t(dmgs_plan P, const BlockArgs<T>& a, hipStream_t st) {
    const int nb3 = a.nb * a.nb * a.nb;
    const size_t lds = BlockShape<kBlockB, MODE>::lds_bytes(sizeof(T));
    return launch_rec(P, (const void*)k_block_pass<T, kBlockB, MODE, HARM>, (const void*)k_block_grp<T, kBlockB, MODE, HARM>,
                      (unsigned)nb3, kBlockThreads, lds, a, st);
}

// One block phase on level k: pre (from *cur or from zero; qc written) or
// post (*cur + I ec); the result goes to *other and the buffers swap.
template <class T>
int block_phase(dmgs_plan P, int k, T** cur, T** other, const T* q, T* qc, const T* ec, int order, bool zero,
                bool post, hipStream_t st) {
    const Level& l = P->lev[k];
    TRY(need_dense<T>(P, k, "block pass"));
    BlockArgs<T> a;
    a.u_in = *cur;
    a.u_out = *other;
    a.q = q;
    a.D = Typed<T>::D(l);
    a.w = Typed<T>::w(l);
    a.ec = ec;
    a.qc = qc;
    a.N = l.N;
    a.nb = (l.N - 1 + kBlockB - 1) / kBlockB;
    a.order = order;
    a.st = l.stencil<T>(harmonic(P));
    const int mode = post ? kBlockPost : (zero ? kBlockPreZero : kBlockPre);
    const double words = (zero ? 4.0 : 5.0) + 0.125;
    int slot;
    TRY(tbeg(P, k, st, &slot, DMGS_K_SMOOTH));
    if constexpr (sizeof(T) == 4) {
        const bool h = harmonic(P);
        if (mode == kBlockPost) TRY(h ? (launch_block_t<T, kBlockPost, true>(P, a, st)) : (launch_block_t<T, kBlockPost, false>(P, a, st)));
        else if (mode == kBlockPre) TRY(h ? (launch_block_t<T, kBlockPre, true>(P, a, st)) : (launch_block_t<T, kBlockPre, false>(P, a, st)));
        else TRY(h ? (launch_block_t<T, kBlockPreZero, true>(P, a, st)) : (launch_block_t<T, kBlockPreZero, false>(P, a, st)));
    } else {
        set_error("block passes are float32 only");
        return DMGS_ERR_INVALID;
    }
    TRY(tend(P, slot, DMGS_K_SMOOTH, words * l.nv * sizeof(T), st));
    std::swap(*cur, *other);
    return DMGS_OK;
}

// Dynamic-LDS limits of the block kernels (set once per plan).
int block_attributes() {
    const void* fns[] = {
        (const void*)k_block_pass<float, kBlockB, kBlockPreZero, false>, (const void*)k_block_pass<float, kBlockB, kBlockPreZero, true>,
        (const void*)k_block_pass<float, kBlockB, kBlockPre, false>, (const void*)k_block_pass<float, kBlockB, kBlockPre, true>,
        (const void*)k_block_pass<float, kBlockB, kBlockPost, false>, (const void*)k_block_pass<float, kBlockB, kBlockPost, true>,
        (const void*)k_block_grp<float, kBlockB, kBlockPreZero, false>, (const void*)k_block_grp<float, kBlockB, kBlockPreZero, true>,
        (const void*)k_block_grp<float, kBlockB, kBlockPre, false>, (const void*)k_block_grp<float, kBlockB, kBlockPre, true>,
        (const void*)k_block_grp<float, kBlockB, kBlockPost, false>, (const void*)k_block_grp<float, kBlockB, kBlockPost, true>};
    const int lims[] = {(int)BlockShape<kBlockB, kBlockPreZero>::lds_bytes(4), (int)BlockShape<kBlockB, kBlockPreZero>::lds_bytes(4),
                        (int)BlockShape<kBlockB, kBlockPre>::lds_bytes(4), (int)BlockShape<kBlockB, kBlockPre>::lds_bytes(4),
                        (int)BlockShape<kBlockB, kBlockPost>::lds_bytes(4), (int)BlockShape<kBlockB, kBlockPost>::lds_bytes(4)};
    for (int i = 0; i < 12; i++)
        if (hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, lims[i % 6]) != hipSuccess) {
            (void)hipGetLastError(); set_error("hipFuncSetAttribute failed");
            return DMGS_ERR_HIP;
        }
    return DMGS_OK;
}

// Smoothing counts of a cycle: the transposed cycle (order 1) reverses the
// cycle's steps, so it pre-smooths with the forward cycle's post-smoothing
// count and post-smooths with its pre-smoothing count.
int nu_pre_of(dmgs_plan P, int order) { return order ? P->opt.nu_post : P->opt.nu_pre; }
int nu_post_of(dmgs_plan P, int order) { return order ? P->opt.nu_pre : P->opt.nu_post; }

// Pre-smoothing pass on level k: nu_pre_of sweeps from *cur (or from 0), then
// qc = R (q - A u).  Simple levels work in place.
template <class T>
int pre_pass(dmgs_plan P, int k, T** cur, T** other, const T* q, T* qc, int order, bool zero, hipStream_t st) {
    const Level& l = P->lev[k];
    if (block_level<T>(P, k)) return block_phase<T>(P, k, cur, other, q, qc, (const T*)nullptr, order, zero, false, st);
    if (fused_level(P, k)) {
        bool rdone;
        T* r = Typed<T>::r(l);
        TRY(smooth_phase<T>(P, k, cur, other, q, nu_pre_of(P, order), order, zero, (const T*)nullptr, st, r, &rdone));
        return rdone ? defect_restrict<T>(P, k, r, q, qc, st, true, order) : defect_restrict<T>(P, k, *cur, q, qc, st);
    }
    TRY(need_dense<T>(P, k, "simple pre-smoothing"));
    if (zero) TRY(fill<T>(*cur, l.nv, T(0), st));
    TRY(sweeps<T>(P, k, *cur, q, nu_pre_of(P, order), order, st));
    T* r = *other;   // scratch for the defect
    TRY(apply_or_defect<T>(P, k, *cur, q, r, 0, st));
    hipLaunchKernelGGL(k_restrict<T>, dim3(grid_for(P->lev[k + 1].nv)), dim3(kBlock), 0, st, (const T*)r, qc, l.N);
    LAUNCHCHK();
    // the simple path used the other buffer as scratch: restore its boundary
    return DMGS_OK;
}

// Post-smoothing pass on level k: u = *cur + I ec, then nu_post_of sweeps.
template <class T>
int post_pass(dmgs_plan P, int k, T** cur, T** other, const T* ec, const T* q, int order, hipStream_t st) {
    const Level& l = P->lev[k];
    if (block_level<T>(P, k)) return block_phase<T>(P, k, cur, other, q, (T*)nullptr, ec, order, false, true, st);
    if (fused_level(P, k)) return smooth_phase<T>(P, k, cur, other, q, nu_post_of(P, order), order, false, ec, st);
    TRY(need_dense<T>(P, k, "simple post-smoothing"));
    TIMED(P, k, DMGS_K_PROLONG, (double)(2 * l.nv + P->lev[k + 1].nv) * sizeof(T), st,
          hipLaunchKernelGGL(k_prolong_add<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, ec, *cur, l.N));
    return sweeps<T>(P, k, *cur, q, nu_post_of(P, order), order, st);
}

template <class T, bool HARM>
int launch_small_t(dmgs_plan P, int k, const T* q, T* u, int order, hipStream_t st) {
    SmallArgs<T> a;
    int Ns[kSmallMaxLevels];
    a.nlev = P->L - k;
    int off = 0;
    for (int i = 0; i < a.nlev; i++) {
        const Level& l = P->lev[k + i];
        a.lev[i].N = Ns[i] = l.N;
        a.lev[i].nv = (int)l.nv;
        a.lev[i].off = off;
        off += 4 * (int)l.nv;
        a.lev[i].D = Typed<T>::D(l);
        a.lev[i].w = Typed<T>::w(l);
        a.lev[i].st = l.stencil<T>(HARM);
    }
    a.q = q;
    a.u = u;
    a.cinv = P->cinv;
    a.nu_pre = nu_pre_of(P, order);
    a.nu_post = nu_post_of(P, order);
    a.order = order;
    a.roff = off;
    size_t bytes = small_lds_bytes<T>(Ns, a.nlev);
    const void* grp = nullptr;
    if constexpr (sizeof(T) == 4) grp = (const void*)k_small_grp<T, HARM>;
    return launch_rec(P, (const void*)k_small_vcycle<T, HARM>, grp, 1u, kSmallThreads, bytes, a, st);
}

template <class T>
int small_level(dmgs_plan P) { return sizeof(T) == 4 ? P->small32 : P->small64; }

// --- weighted-Jacobi cycles -----------------------------------------------------

bool wjacobi(dmgs_plan P) { return P->opt.smoother == DMGS_WJACOBI; }
constexpr double kWjOmega = 6.0 / 7.0;

// count weighted-Jacobi sweeps on level k, ping-ponging *cur and *other;
// zero: the first starts from a zero iterate
template <class T>
int wj_sweeps(dmgs_plan P, int k, T** cur, T** other, const T* q, int count, bool zero, hipStream_t st) {
    const Level& l = P->lev[k];
    TRY(need_dense<T>(P, k, "weighted-Jacobi sweep"));
    for (int i = 0; i < count; i++) {
        const bool z = zero && i == 0;
        // reads u, q, D, mu, w and writes u (from zero: reads q, w)
        TIMED(P, k, DMGS_K_SMOOTH, (z ? 3.0 : 6.0) * l.nv * sizeof(T), st,
              hipLaunchKernelGGL(k_wj_sweep<T>, dim3(vertex_grid(l.nv)), dim3(kBlock), 0, st, (const T*)*cur, *other,
                                 q, (const T*)Typed<T>::D(l), (const T*)Typed<T>::mu(l), (const T*)Typed<T>::w(l), l.N,
                                 l.stencil<T>(harmonic(P)), (T)kWjOmega, z ? 1 : 0));
        std::swap(*cur, *other);
    }
    return DMGS_OK;
}

// One V(nu_pre, nu_post)-cycle with weighted-Jacobi smoothing; order 1 (the
// transposed cycle) exchanges the pre- and post-smoothing counts.
template <class T>
int vcycle_wj(dmgs_plan P, int k, T** cur, T** other, const T* q, int order, bool zero, hipStream_t st) {
    const Level& l = P->lev[k];
    const int nu1 = nu_pre_of(P, order), nu2 = nu_post_of(P, order);
    TRY(need_dense<T>(P, k, "weighted-Jacobi cycle"));
    if (zero && (k == P->L - 1 || nu1 == 0)) TRY(fill<T>(*cur, l.nv, T(0), st));
    if (k == P->L - 1) return coarsest<T>(P, q, *cur, st);
    TRY(wj_sweeps<T>(P, k, cur, other, q, nu1, zero && nu1 > 0, st));
    const Level& c = P->lev[k + 1];
    T* qc = Typed<T>::q(c);
    TRY(defect_restrict<T>(P, k, *cur, q, qc, st));
    T* ccur = Typed<T>::u(c);
    T* coth = Typed<T>::t(c);
    TRY(vcycle_wj<T>(P, k + 1, &ccur, &coth, qc, order, true, st));
    TIMED(P, k, DMGS_K_PROLONG, (double)(2 * l.nv + c.nv) * sizeof(T), st,
          hipLaunchKernelGGL(k_prolong_add<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, (const T*)ccur, *cur, l.N));
    return wj_sweeps<T>(P, k, cur, other, q, nu2, false, st);
}

// One V-cycle on level k with right-hand side q, iterate in *cur (the
// level's other buffer is *other).  zero: the iterate starts from 0 (coarse
// corrections, refinement corrections).  On return *cur holds the result.
// smoothed: the pre-smoothing of level k has already been enqueued (level k
// uses the streaming passes); the cycle continues with the defect, which
// that pre-smoothing already wrote to the level's r buffer when rdone.
template <class T>
int vcycle(dmgs_plan P, int k, T** cur, T** other, const T* q, int order, bool zero, hipStream_t st,
           bool smoothed = false, bool rdone = false) {
    if (wjacobi(P)) return vcycle_wj<T>(P, k, cur, other, q, order, zero, st);
    if (k > 0 && k == small_level<T>(P) && zero) {
        if (harmonic(P)) return launch_small_t<T, true>(P, k, q, *cur, order, st);
        return launch_small_t<T, false>(P, k, q, *cur, order, st);
    }
    if (k == P->L - 1) {
        TRY(need_dense<T>(P, k, "coarsest solve"));
        if (zero) TRY(fill<T>(*cur, P->lev[k].nv, T(0), st));
        return coarsest<T>(P, q, *cur, st);
    }
    const Level& c = P->lev[k + 1];
    T* qc = Typed<T>::q(c);
    if (smoothed) TRY(rdone ? defect_restrict<T>(P, k, Typed<T>::r(P->lev[k]), q, qc, st, true, order)
                            : defect_restrict<T>(P, k, *cur, q, qc, st));
    else TRY(pre_pass<T>(P, k, cur, other, q, qc, order, zero, st));
    T* ccur = Typed<T>::u(c);
    T* coth = Typed<T>::t(c);
    TRY(vcycle<T>(P, k + 1, &ccur, &coth, qc, order, true, st));
    return post_pass<T>(P, k, cur, other, ccur, q, order, st);
}

// ||b - A x||^2 into the plan's host norm slot `slot` (fused float64 kernel); with e, also
// x_out = x + e and r32 = float(b - A x_out).
constexpr int kIrTY = 16, kIrTZ = 64;

// Blocks of the refinement kernel at level size N when each block leaves
// `sums` partial sums (kMaxPartials bounds them all); 0 if no chunking fits.
IrArgs ir_shape(int N, int sums) {
    IrArgs a;
    a.tiles_y = (N + kIrTY - 1) / kIrTY;
    a.tiles_z = (N + kIrTZ - 1) / kIrTZ;
    a.chunk = choose_chunk(N - 1, a.tiles_y * a.tiles_z);
    a.nchunks = (N - 1 + a.chunk - 1) / a.chunk;
    while (a.nchunks > 1 && a.tiles_y * a.tiles_z * a.nchunks * sums > kMaxPartials) {
        a.chunk *= 2;
        a.nchunks = (N - 1 + a.chunk - 1) / a.chunk;
    }
    if (a.tiles_y * a.tiles_z * a.nchunks * sums > kMaxPartials) a.nchunks = 0;
    return a;
}

template <bool HAS_E, bool X_ZERO, bool HARM, bool EPI>
int launch_ir(dmgs_plan P, const IrArgs& a0, int N, hipStream_t st, unsigned* nb_out) {
    IrArgs a = a0;
    const IrArgs sh = ir_shape(N, EPI ? 3 : 1);
    a.tiles_y = sh.tiles_y;
    a.tiles_z = sh.tiles_z;
    a.chunk = sh.chunk;
    a.nchunks = sh.nchunks;
    unsigned nb = (unsigned)(a.tiles_y * a.tiles_z * a.nchunks);
    *nb_out = nb;
    const void* grp = nullptr;   // the epilogue does not run in grouped execution
    if constexpr (!EPI) grp = (const void*)k_ir_residual_grp<kIrTY, kIrTZ, HAS_E, X_ZERO, HARM>;
    return launch_rec(P, (const void*)k_ir_residual_col<kIrTY, kIrTZ, HAS_E, X_ZERO, HARM, EPI>, grp, nb,
                      IrShape<kIrTY, kIrTZ>::NT, 0, a, st);
}

template <bool HAS_E, bool X_ZERO, bool EPI>
int launch_ir_h(dmgs_plan P, const IrArgs& a, int N, bool h, hipStream_t st, unsigned* nb) {
    return h ? launch_ir<HAS_E, X_ZERO, true, EPI>(P, a, N, st, nb) : launch_ir<HAS_E, X_ZERO, false, EPI>(P, a, N, st, nb);
}

// Sum `count` partials into norm slot `slot` (recorded in grouped execution).
int sum_partials(dmgs_plan P, const double* partial, int count, int slot, hipStream_t st) {
    if (P->rec) {
        SumArgs s{partial, count, norm_dst(P), slot};
        return launch_rec(P, nullptr, (const void*)k_sum_grp, 1u, 1024u, 0, s, st);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, partial, count, norm_dst(P), slot);
    LAUNCHCHK();
    return DMGS_OK;
}

// x_zero: x is 0 everywhere (the boundary value is 0 and nothing has been
// added yet); x is not read.  epi: also the likelihood epilogue of x + e
// (the plan's epi_* buffers), its sums into norm slots 2 and 3.
int ir_step(dmgs_plan P, const double* x, const float* e, double* x_out, const double* b, float* r32, int slot,
            hipStream_t st, bool x_zero = false, bool epi = false) {
    const Level& l = P->lev[0];
    IrArgs a;
    a.x = x;
    a.e = e;
    a.x_out = x_out;
    a.b = b;
    a.D = l.D64;
    a.mu = l.mu64;
    a.r32 = r32;
    a.py = l.py;
    a.px = l.px;
    a.partial = P->partial;
    a.N = l.N;
    a.st = l.stencil<double>(harmonic(P));
    if (epi) {
        if ((x_zero && !e) || !P->epi_d || !P->epi_w || !P->epi_rhobar || ir_shape(l.N, 3).nchunks == 0) {
            set_error("internal: refinement step cannot take the likelihood epilogue");
            return DMGS_ERR_INVALID;
        }
        a.ed = P->epi_d;
        a.ew = P->epi_w;
        a.erhobar = P->epi_rhobar;
    }
    double bytes = (x_zero ? (e ? 24.0 : 8.0) : 32.0) * l.nv + (e ? 4.0 * l.nv : 0.0) + (x_out ? 8.0 * l.nv : 0.0) +
                   (r32 ? 4.0 * l.nv : 0.0) + (epi ? 24.0 * l.nv : 0.0);
    unsigned nb = 0;
    int tslot;
    TRY(tbeg(P, 0, st, &tslot, DMGS_K_RESIDUAL));
    const bool h = harmonic(P);
    if (epi && P->rec) { set_error("internal: the likelihood epilogue in grouped execution"); return DMGS_ERR_INVALID; }
    if (epi) {
        if (!e) TRY((launch_ir_h<false, false, true>(P, a, l.N, h, st, &nb)));
        else if (x_zero) TRY((launch_ir_h<true, true, true>(P, a, l.N, h, st, &nb)));
        else TRY((launch_ir_h<true, false, true>(P, a, l.N, h, st, &nb)));
    } else if (e) {
        if (x_zero) TRY((launch_ir_h<true, true, false>(P, a, l.N, h, st, &nb)));
        else TRY((launch_ir_h<true, false, false>(P, a, l.N, h, st, &nb)));
    } else {
        if (x_zero) TRY((launch_ir_h<false, true, false>(P, a, l.N, h, st, &nb)));
        else TRY((launch_ir_h<false, false, false>(P, a, l.N, h, st, &nb)));
    }
    TRY(tend(P, tslot, DMGS_K_RESIDUAL, bytes, st));
    // the final sums go straight to the plan's pinned host slots
    TRY(sum_partials(P, (const double*)P->partial, (int)nb, slot, st));
    if (epi) {
        TRY(sum_partials(P, (const double*)P->partial + nb, (int)nb, 2, st));
        TRY(sum_partials(P, (const double*)P->partial + 2 * nb, (int)nb, 3, st));
    }
    return mark_norms(P, st);
}

// The reduction kernels write the norms into pinned host memory; waiting for
// the event after the last of them makes them readable (work enqueued after
// it may still be running).  An arena plan copies its device slots to the
// host and waits for the stream.
int read_norms(dmgs_plan P, hipStream_t st) {
    if (P->arena) {
        HIPCHK(hipMemcpyAsync(P->hnorm, P->dnorm, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return DMGS_OK;
    }
    HIPCHK(hipEventSynchronize(P->ev_norm));
    if (P->timing) TRY(timing_flush(P, P->tmark));
    return DMGS_OK;
}

// ---------------------------------------------------------------------------
// Two-dimensional plans (ndim = 2): float64 V-cycles, in place, one launch
// per half-sweep, the defect restricted as it is formed.

template <bool HARM>
int half_sweep2(dmgs_plan P, int k, double* u, const double* q, int colour, hipStream_t st) {
    const Level& l = P->lev[k];
    const int64_t items = (int64_t)(l.N - 1) * (l.N / 2);
    // reads u and D on every vertex, q and mua on one colour; writes one colour
    TIMED(P, k, DMGS_K_SMOOTH, 28.0 * l.nv, st,
          hipLaunchKernelGGL(k2_half_sweep<HARM>, dim3(vertex_grid(items)), dim3(kBlock), 0, st, u, q,
                             (const double*)l.D64, (const double*)l.mu64, l.N, l.stencil<double>(HARM), colour));
    return DMGS_OK;
}

// count red-black sweeps on level k (first colour `first`): pairs of sweeps
// as out-of-place passes from *cur to *other (swapping them) on levels with
// N >= cfg_2d_sweep2_min, the rest as in-place half-sweeps on *cur.  ec:
// first add the prolongated coarse correction I ec to *cur (fused into the
// first pass when there is one).
template <bool HARM>
int sweeps2(dmgs_plan P, int k, double** cur, double** other, const double* q, int count, int first, hipStream_t st,
            const double* ec = nullptr, double* rout = nullptr, bool* rdone = nullptr) {
    if (rdone) *rdone = false;
    const Level& l = P->lev[k];
    int i = 0;
    const bool pass = l.N >= P->cfg_2d_sweep2_min;
    if (ec && !(pass && count >= 2)) {
        const Level& c = P->lev[k + 1];
        TIMED(P, k, DMGS_K_PROLONG, 16.0 * l.nv + 8.0 * c.nv, st,
              hipLaunchKernelGGL(k2_prolong_add, dim3(vertex_grid(l.nv)), dim3(kBlock), 0, st, ec, *cur, l.N));
        ec = nullptr;
    }
    if (pass) {
        const int ntiles = (l.N - 1 + kTile2 - 1) / kTile2;
        // about 4096 waves on the largest grids; chunks of 32..512 rows, a
        // multiple of 8 (the kernel's row ring); chunk 0 takes 2 more rows
        int chunk = (int)std::min<int64_t>(512, std::max<int64_t>(32, ((int64_t)(l.N - 1) * ntiles / 4096 + 7) / 8 * 8));
        if (P->cfg_2d_chunk > 0) chunk = P->cfg_2d_chunk;
        const int nchunks = std::max(1, (l.N - 3 + chunk - 1) / chunk);
        const unsigned blocks = (unsigned)((ntiles * nchunks + 3) / 4);
        for (; count - i >= 2; i += 2) {
            // reads u, q, D, mua (and the coarse correction); writes u
            if (rout && count - i == 2 && !ec) {
                // the phase's last pass also writes the defect of its result
                const int ntd = (l.N - 1 + kTile2D - 1) / kTile2D;
                const int ncd = std::max(1, (l.N - 4 + chunk - 1) / chunk);
                TIMED(P, k, DMGS_K_SMOOTH, 48.0 * l.nv, st,
                      hipLaunchKernelGGL((k2_sweep2<HARM, false, true>), dim3((unsigned)((ntd * ncd + 3) / 4)), dim3(256),
                                         0, st, (const double*)*cur, *other, q, (const double*)l.D64,
                                         (const double*)l.mu64, (const double*)nullptr, rout, l.N,
                                         l.stencil<double>(HARM), first, chunk, ntd, ncd));
                *rdone = true;
            } else if (ec) {
                TIMED(P, k, DMGS_K_SMOOTH, 40.0 * l.nv + 8.0 * P->lev[k + 1].nv, st,
                      hipLaunchKernelGGL((k2_sweep2<HARM, true>), dim3(blocks), dim3(256), 0, st, (const double*)*cur,
                                         *other, q, (const double*)l.D64, (const double*)l.mu64, ec, (double*)nullptr,
                                         l.N, l.stencil<double>(HARM), first, chunk, ntiles, nchunks));
                ec = nullptr;
            } else {
                TIMED(P, k, DMGS_K_SMOOTH, 40.0 * l.nv, st,
                      hipLaunchKernelGGL((k2_sweep2<HARM, false>), dim3(blocks), dim3(256), 0, st, (const double*)*cur,
                                         *other, q, (const double*)l.D64, (const double*)l.mu64, (const double*)nullptr,
                                         (double*)nullptr, l.N, l.stencil<double>(HARM), first, chunk, ntiles, nchunks));
            }
            std::swap(*cur, *other);
        }
    }
    for (; i < count; i++) {
        TRY(half_sweep2<HARM>(P, k, *cur, q, first, st));
        TRY(half_sweep2<HARM>(P, k, *cur, q, 1 - first, st));
    }
    return DMGS_OK;
}

// One V-cycle on level k of a two-dimensional plan with iterate *cur (from 0
// when zero; the level's other buffer is *other, whose boundary holds the
// same values); order 1 is the transposed cycle.  On return *cur holds the
// result.
template <bool HARM>
int vcycle2(dmgs_plan P, int k, double** cur, double** other, const double* q, int order, bool zero, hipStream_t st) {
    const Level& l = P->lev[k];
    if (zero && k == P->small2) {
        // this level and every coarser one in one LDS-resident workgroup
        Small2Args a;
        a.q = q;
        a.u = *cur;
        a.nl = P->L - k;
        for (int i = 0; i < a.nl; i++) {
            const Level& li = P->lev[k + i];
            a.D[i] = li.D64;
            a.mu[i] = li.mu64;
            a.st[i] = li.stencil<double>(HARM);
            a.N[i] = li.N;
        }
        a.nu_pre = nu_pre_of(P, order);
        a.nu_post = nu_post_of(P, order);
        a.first = order ? 1 : 0;
        const size_t lds = (size_t)small2_words(a.N, a.nl) * sizeof(double);
        hipLaunchKernelGGL(k2_small_vcycle<HARM>, dim3(1), dim3(1024), lds, st, a);
        LAUNCHCHK();
        return DMGS_OK;
    }
    const int first = order ? 1 : 0;
    // block passes run two workgroups per CU: take them where the tiles fill
    // whole rounds (a nearly empty last round costs more than they save)
    const int btiles = ((l.N + kB2 - 1) / kB2) * ((l.N + kB2 - 1) / kB2);
    const bool bfits = btiles <= 2 * P->ncu || btiles % (2 * P->ncu) == 0;
    if (k < P->L - 1 && l.N >= P->cfg_2d_block_min && l.N < P->cfg_2d_sweep2_min && bfits && nu_pre_of(P, order) == 2 &&
        nu_post_of(P, order) == 2) {
        // mid-size level: each smoothing phase in one launch of LDS tiles,
        // the defect restricted by the pre-smoothing one
        const Level& c = P->lev[k + 1];
        const int ntx = (l.N + kB2 - 1) / kB2;
        const dim3 grid(ntx * ntx), block(256);
        const Stencil<double> s = l.stencil<double>(HARM);
        TIMED(P, k, DMGS_K_SMOOTH, (zero ? 32.0 : 40.0) * l.nv + 8.0 * c.nv, st,
              if (zero) hipLaunchKernelGGL((k2_block_pass<HARM, 1>), grid, block, 0, st, (const double*)*cur, *other,
                                           q, (const double*)l.D64, (const double*)l.mu64, (const double*)nullptr,
                                           c.q64, l.N, s, first, ntx);
              else hipLaunchKernelGGL((k2_block_pass<HARM, 0>), grid, block, 0, st, (const double*)*cur, *other, q,
                                      (const double*)l.D64, (const double*)l.mu64, (const double*)nullptr, c.q64, l.N,
                                      s, first, ntx));
        std::swap(*cur, *other);
        double* ccur = c.u64;
        double* coth = c.t64;
        TRY(vcycle2<HARM>(P, k + 1, &ccur, &coth, c.q64, order, true, st));
        TIMED(P, k, DMGS_K_SMOOTH, 40.0 * l.nv + 8.0 * c.nv, st,
              hipLaunchKernelGGL((k2_block_pass<HARM, 2>), grid, block, 0, st, (const double*)*cur, *other, q,
                                 (const double*)l.D64, (const double*)l.mu64, (const double*)ccur, (double*)nullptr,
                                 l.N, s, first, ntx));
        std::swap(*cur, *other);
        return DMGS_OK;
    }
    if (zero) TRY(fill<double>(*cur, l.nv, 0.0, st));
    if (k == P->L - 1) {
        hipLaunchKernelGGL(k2_exact<HARM>, dim3(1), dim3(64), 0, st, q, *cur, (const double*)l.D64,
                           (const double*)l.mu64, l.N, l.stencil<double>(HARM));
        LAUNCHCHK();
        return DMGS_OK;
    }
    bool rdone = false;
    TRY(sweeps2<HARM>(P, k, cur, other, q, nu_pre_of(P, order), first, st, nullptr,
                      P->cfg_2d_defect ? l.rd64 : nullptr, &rdone));
    const Level& c = P->lev[k + 1];
    if (rdone) {
        // restrict the defect the last pass wrote
        TIMED(P, k, DMGS_K_DEFECT_RESTRICT, 8.0 * l.nv + 8.0 * c.nv, st,
              hipLaunchKernelGGL(k2_restrict_r, dim3(vertex_grid(c.nv)), dim3(kBlock), 0, st, (const double*)l.rd64,
                                 c.q64, l.N));
    } else if (l.N >= P->cfg_2d_sweep2_min) {
        // row-streaming form: coarse rows in chunks of cx (a multiple of 4)
        const int ntiles = (c.N - 1 + kTileR - 1) / kTileR;
        const int cx = (int)std::min<int64_t>(256, std::max<int64_t>(16, ((int64_t)(c.N - 1) * ntiles / 4096 + 3) / 4 * 4));
        const int nchunks = (c.N - 1 + cx - 1) / cx;
        TIMED(P, k, DMGS_K_DEFECT_RESTRICT, 32.0 * l.nv + 8.0 * c.nv, st,
              hipLaunchKernelGGL(k2_defect_restrict_rows<HARM>, dim3((ntiles * nchunks + 3) / 4), dim3(256), 0, st,
                                 (const double*)*cur, q, (const double*)l.D64, (const double*)l.mu64, l.N,
                                 l.stencil<double>(HARM), c.q64, cx, ntiles, nchunks));
    } else {
        TIMED(P, k, DMGS_K_DEFECT_RESTRICT, 32.0 * l.nv + 8.0 * c.nv, st,
              hipLaunchKernelGGL(k2_defect_restrict<HARM>, dim3(vertex_grid(c.nv)), dim3(kBlock), 0, st,
                                 (const double*)*cur, q, (const double*)l.D64, (const double*)l.mu64, l.N,
                                 l.stencil<double>(HARM), c.q64));
    }
    double* ccur = c.u64;
    double* coth = c.t64;
    TRY(vcycle2<HARM>(P, k + 1, &ccur, &coth, c.q64, order, true, st));
    return sweeps2<HARM>(P, k, cur, other, q, nu_post_of(P, order), first, st, ccur);
}

// ||b - A x||^2 of the finest level into the host norm slot `slot`.
template <bool HARM>
int resid2(dmgs_plan P, const double* x, const double* b, int slot, hipStream_t st) {
    const Level& l = P->lev[0];
    const unsigned nb = grid_for(l.nv, kMaxPartials);
    TIMED(P, 0, DMGS_K_RESIDUAL, 32.0 * l.nv, st,
          hipLaunchKernelGGL(k2_resid_sq<HARM>, dim3(nb), dim3(kBlock), 0, st, x, b, (const double*)l.D64,
                             (const double*)l.mu64, l.N, l.stencil<double>(HARM), P->partial));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)nb, norm_dst(P), slot);
    LAUNCHCHK();
    return mark_norms(P, st);
}

// solve() for two-dimensional plans (same modes, schedule record and replay).
// DMGS_TRACE: one point of a solve's residual history
void trace_point(dmgs_plan P, int order, int steps, int vcycles, double rel) {
    if (P->cfg_trace) P->trace[order].push_back({steps, vcycles, rel});
}

template <bool HARM>
int solve2d(dmgs_plan P, const double* b, double* x, double bc, int order, dmgs_info* info, hipStream_t st,
            const std::vector<int>* replay, bool record) {
    const dmgs_options& o = P->opt;
    const Level& l0 = P->lev[0];
    const bool fixed = o.fixed_cycles > 0 || replay;
    const int nfix = replay ? (int)replay->size() : o.fixed_cycles;
    std::vector<int> sched;
    // the iterate alternates between x and the level's other buffer; both
    // hold the boundary value
    double* cur = x;
    double* oth = l0.t64;
    hipLaunchKernelGGL(k2_init_iterate, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, l0.N, bc);
    LAUNCHCHK();
    hipLaunchKernelGGL(k2_init_iterate, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, oth, l0.N, bc);
    LAUNCHCHK();
    int cycles = 0, status = DMGS_OK;
    double r0 = 0.0, rel = 0.0;
    TRY(resid2<HARM>(P, x, b, 0, st));
    do {
        if (!fixed) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            if (!std::isfinite(r0)) { set_error("non-finite right-hand side"); status = DMGS_ERR_NONFINITE; break; }
            if (r0 == 0.0) break;
        } else if (P->cfg_trace) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
        }
        for (cycles = 1; !(fixed && nfix == 0); cycles++) {
            TRY(vcycle2<HARM>(P, 0, &cur, &oth, b, order, false, st));
            sched.push_back(1);
            if (fixed) {
                if (P->cfg_trace) {
                    TRY(resid2<HARM>(P, cur, b, 1, st));
                    TRY(read_norms(P, st));
                    trace_point(P, order, cycles, cycles, std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0));
                }
                if (cycles == nfix) break;
                continue;
            }
            TRY(resid2<HARM>(P, cur, b, 1, st));
            TRY(read_norms(P, st));
            rel = std::sqrt(P->hnorm[1]) / r0;
            trace_point(P, order, cycles, cycles, rel);
            if (!std::isfinite(rel)) { set_error("non-finite residual after %d cycles", cycles); status = DMGS_ERR_NONFINITE; break; }
            if (rel <= o.rtol) break;
            if (cycles >= o.max_cycles) { set_error("not converged after %d cycles (rel %.3e)", cycles, rel); status = DMGS_ERR_NOT_CONVERGED; break; }
        }
        if (fixed && nfix == 0) cycles = 0;
        if (fixed && info) {
            TRY(resid2<HARM>(P, cur, b, 1, st));
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            rel = std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0);
        }
    } while (false);
    if (cur != x) HIPCHK(hipMemcpyAsync(x, cur, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (record && !fixed) {
        P->fwd_recorded = status == DMGS_OK || status == DMGS_ERR_NOT_CONVERGED;
        P->fwd_schedule = sched;
    }
    if (info) {
        info->cycles = cycles;
        info->vcycles = cycles;
        info->rel_residual = rel;
        info->status = status;
    }
    return status;
}

// Solve A x = b on the finest level from x = 0 (interior) / bc (boundary).
// order 0: red-first cycles (S); order 1: black-first cycles (S^T).
// replay: run exactly this V-cycle schedule (float64 plans: one entry per
// cycle; refinement plans: the float32 V-cycles of each step) with no
// convergence test.  record: a tolerance-mode solve stores its schedule in
// P->fwd_schedule.
// ---------------------------------------------------------------------------
// General-grid plans: float64 V-cycles, in place, one operation per launch.

GridDims gdims(dmgs_plan P, int k);

// One V(nu1, nu2)-cycle on level k (order 0: red before black; order 1, the
// transposed cycle: black before red with the counts exchanged); u on the
// coarser levels starts at 0.
// epi (finest level): the last post-smoothing half-sweep also takes the
// likelihood epilogue of the cycle's result (the plan's epi_* buffers, sums
// into norm slots 2 and 3); *epi_done reports whether it ran.
int vcycle_grid(dmgs_plan P, int k, double* u, const double* q, int order, hipStream_t st, bool epi = false,
                bool* epi_done = nullptr) {
    const Level& l = P->lev[k];
    const GridDims G = gdims(P, k);
    if (k == P->L - 1) {
        hipLaunchKernelGGL(k_g_exact, dim3(1), dim3(kGridCoarseMax), 0, st, q, u, (const double*)l.D64,
                           (const double*)P->cinv, G);
        LAUNCHCHK();
        return DMGS_OK;
    }
    const int first = order ? 1 : 0;
    const unsigned g = grid_for(l.nv);
    auto sweeps = [&](int count) -> int {
        for (int i = 0; i < count; i++)
            for (int c = 0; c < 2; c++) {
                TIMED(P, k, DMGS_K_SMOOTH, 40.0 * l.nv, st,
                      hipLaunchKernelGGL(k_g_half, dim3(g), dim3(kBlock), 0, st, u, q, (const double*)l.D64,
                                         (const double*)l.mu64, G, c ? 1 - first : first));
            }
        return DMGS_OK;
    };
    TRY(sweeps(nu_pre_of(P, order)));
    const Level& c = P->lev[k + 1];
    TIMED(P, k, DMGS_K_DEFECT_RESTRICT, 40.0 * l.nv, st,
          hipLaunchKernelGGL(k_g_defect, dim3(g), dim3(kBlock), 0, st, (const double*)u, q, (const double*)l.D64,
                             (const double*)l.mu64, G, l.t64));
    hipLaunchKernelGGL(k_g_restrict, dim3(grid_for(c.nv)), dim3(kBlock), 0, st, (const double*)l.t64, G, c.q64);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_g_fill<double>, dim3(grid_for(c.nv)), dim3(kBlock), 0, st, c.u64, gdims(P, k + 1), 0.0);
    LAUNCHCHK();
    TRY(vcycle_grid(P, k + 1, c.u64, c.q64, order, st));
    TIMED(P, k, DMGS_K_PROLONG, 17.0 * l.nv, st,
          hipLaunchKernelGGL(k_g_prolong_add, dim3(g), dim3(kBlock), 0, st, (const double*)c.u64, G, u));
    const int npost = nu_post_of(P, order);
    if (!(epi && k == 0 && npost > 0 && P->epi_d)) return sweeps(npost);
    TRY(sweeps(npost - 1));
    TIMED(P, k, DMGS_K_SMOOTH, 40.0 * l.nv, st,
          hipLaunchKernelGGL(k_g_half, dim3(g), dim3(kBlock), 0, st, u, q, (const double*)l.D64,
                             (const double*)l.mu64, G, first));
    const unsigned ge = grid_for(l.nv, kMaxPartials / 2);
    TIMED(P, k, DMGS_K_SMOOTH, 72.0 * l.nv, st,
          hipLaunchKernelGGL(k_g_half_epi, dim3(ge), dim3(kBlock), 0, st, u, q, (const double*)l.D64,
                             (const double*)l.mu64, G, 1 - first, P->epi_d, P->epi_w, P->epi_rhobar, P->partial));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)ge, norm_dst(P), 2);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial + ge, (int)ge, norm_dst(P),
                       3);
    LAUNCHCHK();
    if (epi_done) *epi_done = true;
    return mark_norms(P, st);
}

// ||b - A x||^2 of the finest level into the norm slot `slot`.
int resid_grid(dmgs_plan P, const double* x, const double* b, int slot, hipStream_t st) {
    const Level& l = P->lev[0];
    const unsigned nb = grid_for(l.nv, kMaxPartials);
    TIMED(P, 0, DMGS_K_RESIDUAL, 32.0 * l.nv, st,
          hipLaunchKernelGGL(k_g_resid_sq, dim3(nb), dim3(kBlock), 0, st, x, b, (const double*)l.D64,
                             (const double*)l.mu64, gdims(P, 0), P->partial));
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)nb, norm_dst(P), slot);
    LAUNCHCHK();
    return mark_norms(P, st);
}

// solve() for general-grid plans (same modes, schedule record and replay).
int solve_grid(dmgs_plan P, const double* b, double* x, double bc, int order, dmgs_info* info, hipStream_t st,
               const std::vector<int>* replay, bool record) {
    const dmgs_options& o = P->opt;
    const Level& l0 = P->lev[0];
    const bool fixed = o.fixed_cycles > 0 || replay;
    const int nfix = replay ? (int)replay->size() : o.fixed_cycles;
    hipLaunchKernelGGL(k_g_init, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, gdims(P, 0), bc);
    LAUNCHCHK();
    int cycles = 0, status = DMGS_OK;
    double r0 = 0.0, rel = 0.0;
    // the initial residual into slot 0 (read in fixed mode only with info)
    TRY(resid_grid(P, x, b, 0, st));
    if (!fixed) {
        TRY(read_norms(P, st));
        r0 = std::sqrt(P->hnorm[0]);
        if (!std::isfinite(r0)) {
            set_error("non-finite right-hand side");
            status = DMGS_ERR_NONFINITE;
        }
    } else if (P->cfg_trace) {
        TRY(read_norms(P, st));
        r0 = std::sqrt(P->hnorm[0]);
    }
    // A requested likelihood epilogue rides on the last half-sweep of the
    // cycle expected to be the last (in tolerance mode: the one the
    // contraction of the last cycle predicts to come within 4 rtol; a cycle
    // that takes it and is not the last costs one more read of d and w).
    const bool want_epi = P->epi_d && order == 0;
    P->epi_fused = false;
    double rel_prev = 1.0;
    bool epi_next = false;
    if (status == DMGS_OK && (fixed || r0 > 0.0)) {
        for (cycles = 1; !(fixed && nfix == 0); cycles++) {
            bool done = false;
            TRY(vcycle_grid(P, 0, x, b, order, st, want_epi && (fixed ? cycles == nfix : epi_next), &done));
            P->epi_fused = done;
            if (fixed) {
                if (P->cfg_trace) {
                    TRY(resid_grid(P, x, b, 1, st));
                    TRY(read_norms(P, st));
                    trace_point(P, order, cycles, cycles, std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0));
                }
                if (cycles == nfix) break;
                continue;
            }
            TRY(resid_grid(P, x, b, 1, st));
            TRY(read_norms(P, st));
            rel_prev = cycles == 1 ? 1.0 : rel;
            rel = std::sqrt(P->hnorm[1]) / r0;
            trace_point(P, order, cycles, cycles, rel);
            epi_next = rel < rel_prev && rel * (rel / rel_prev) <= 4.0 * o.rtol;
            if (!std::isfinite(rel)) { set_error("non-finite residual after %d cycles", cycles); status = DMGS_ERR_NONFINITE; break; }
            if (rel <= o.rtol) break;
            if (cycles >= o.max_cycles) { set_error("not converged after %d cycles (rel %.3e)", cycles, rel); status = DMGS_ERR_NOT_CONVERGED; break; }
        }
        if (fixed && nfix == 0) cycles = 0;
    } else {
        cycles = 0;
    }
    if (fixed && info) {
        TRY(resid_grid(P, x, b, 1, st));
        TRY(read_norms(P, st));
        r0 = std::sqrt(P->hnorm[0]);
        rel = std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0);
    }
    if (record && !fixed) {
        P->fwd_recorded = status == DMGS_OK || status == DMGS_ERR_NOT_CONVERGED;
        P->fwd_schedule.assign(cycles, 1);
    }
    if (info) {
        info->cycles = cycles;
        info->vcycles = cycles;
        info->rel_residual = rel;
        info->status = status;
    }
    return status;
}

int solve(dmgs_plan P, const double* b, double* x, double bc, int order, dmgs_info* info, hipStream_t st,
          const std::vector<int>* replay = nullptr, bool record = false) {
    P->trace[order].clear();
    if (P->grid) return solve_grid(P, b, x, bc, order, info, st, replay, record);
    if (is2d(P))
        return harmonic(P) ? solve2d<true>(P, b, x, bc, order, info, st, replay, record)
                           : solve2d<false>(P, b, x, bc, order, info, st, replay, record);
    P->bc_zero = bc == 0.0;
    const dmgs_options& o = P->opt;
    const Level& l0 = P->lev[0];
    const bool fixed = o.fixed_cycles > 0 || replay;
    const int nfix = replay ? (int)replay->size() : o.fixed_cycles;
    std::vector<int> sched;
    // with a zero boundary value the refinement's first steps treat the
    // zero iterate implicitly (x is neither cleared nor read; only its
    // boundary is set, and it is cleared if no correction is applied)
    const bool x_zero = is_ir(P) && bc == 0.0;
    if (x_zero) {
        TRY(set_boundary<double>(x, l0.N, 0.0, st));
    } else {
        hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, l0.N, bc);
        LAUNCHCHK();
    }
    int cycles = 0, vcycles = 0, status = DMGS_OK;
    double r0 = 0.0, rel = 0.0;
    if (!is_ir(P)) {
        double* cur = x;
        double* oth = l0.t64;
        TRY(set_boundary<double>(oth, l0.N, bc, st));
        TRY(ir_step(P, cur, nullptr, nullptr, b, nullptr, 0, st));
        if (!fixed) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            if (!std::isfinite(r0)) { set_error("non-finite right-hand side"); status = DMGS_ERR_NONFINITE; goto done; }
            if (r0 == 0.0) goto done;
        } else if (P->cfg_trace) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
        }
        // A requested likelihood epilogue rides on the residual pass after
        // the cycle expected to be the last (the contraction of the last
        // cycle predicts a residual within 4 rtol), or on the final residual
        // pass of fixed-cycle mode.
        const bool want_epi = P->epi_d && order == 0 && ir_shape(l0.N, 3).nchunks > 0;
        P->epi_fused = false;
        double rel_prev = 1.0;
        // In tolerance mode the residual norm of each iterate comes with the
        // first pre-smoothing pass of the next cycle (free_norm): after a
        // cycle whose post-smoothing ended with the second colour, the
        // second colour's residual is 0 and the first colour's is what that
        // pass's first stage forms anyway.  The pass, the defect and the
        // coarse levels of the next cycle are enqueued before the host reads
        // the norm; when it meets the tolerance, the iterate (still in the
        // pass's input buffer) is returned and the rest of that cycle is
        // dropped.
        SweepArgs<double> probe;
        const bool free_norm = !fixed && !want_epi && !wjacobi(P) && P->L > 1 && fused_level(P, 0) &&
                               use_sweep2(P, 0, sizeof(double)) && nu_pre_of(P, order) >= 2 &&
                               nu_post_of(P, order) >= 1 && sweep2_grid<double>(P, probe, l0.N, kSweep2TY, kSweep2TZ64) <= kMaxPartials;
        for (cycles = 1; !(fixed && nfix == 0); cycles++) {
            if (free_norm && cycles >= 2) {
                // cycle `cycles` from u_{cycles-1} (in cur)
                double* prev = cur;
                unsigned nb = 0;
                TRY(smooth_pass2<double>(P, 0, cur, oth, b, order, false, nullptr, st, nullptr, P->partial, &nb));
                std::swap(cur, oth);
                hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)nb,
                                   norm_dst(P), 1);
                LAUNCHCHK();
                TRY(mark_norms(P, st));
                if (nu_pre_of(P, order) > 2)
                    TRY(smooth_phase<double>(P, 0, &cur, &oth, b, nu_pre_of(P, order) - 2, order, false, (const double*)nullptr, st));
                const Level& c1 = P->lev[1];
                TRY(defect_restrict<double>(P, 0, cur, b, c1.q64, st));
                double* ccur = c1.u64;
                double* coth = c1.t64;
                TRY(vcycle<double>(P, 1, &ccur, &coth, c1.q64, order, true, st));
                TRY(read_norms(P, st));
                rel_prev = cycles == 2 ? 1.0 : rel;
                rel = std::sqrt(P->hnorm[1]) / r0;
                trace_point(P, order, cycles - 1, cycles - 1, rel);
                bool stop = false;
                if (!std::isfinite(rel)) { set_error("non-finite residual after %d cycles", cycles - 1); status = DMGS_ERR_NONFINITE; stop = true; }
                else if (rel <= o.rtol) stop = true;
                else if (cycles - 1 >= o.max_cycles) { set_error("not converged after %d cycles (rel %.3e)", cycles - 1, rel); status = DMGS_ERR_NOT_CONVERGED; stop = true; }
                if (stop) {
                    // the result is the cycle's input; prev may be x itself
                    cur = prev;
                    oth = prev == x ? l0.t64 : x;
                    cycles--;
                    break;
                }
                TRY(post_pass<double>(P, 0, &cur, &oth, ccur, b, order, st));
                sched.push_back(1);
                continue;
            }
            TRY(vcycle<double>(P, 0, &cur, &oth, b, order, false, st));
            sched.push_back(1);
            if (fixed) {
                if (P->cfg_trace) {
                    TRY(ir_step(P, cur, nullptr, nullptr, b, nullptr, 1, st));
                    TRY(read_norms(P, st));
                    trace_point(P, order, cycles, cycles, std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0));
                }
                if (cycles == nfix) break;
                continue;
            }
            if (free_norm) continue;   // the norm of this iterate comes with the next cycle
            const bool epi = want_epi && cycles > 1 && rel < rel_prev && rel * (rel / rel_prev) <= 4.0 * o.rtol;
            TRY(ir_step(P, cur, nullptr, nullptr, b, nullptr, 1, st, false, epi));
            P->epi_fused = epi;
            TRY(read_norms(P, st));
            rel_prev = cycles == 1 ? 1.0 : rel;
            rel = std::sqrt(P->hnorm[1]) / r0;
            trace_point(P, order, cycles, cycles, rel);
            if (!std::isfinite(rel)) { set_error("non-finite residual after %d cycles", cycles); status = DMGS_ERR_NONFINITE; break; }
            if (rel <= o.rtol) break;
            if (cycles >= o.max_cycles) { set_error("not converged after %d cycles (rel %.3e)", cycles, rel); status = DMGS_ERR_NOT_CONVERGED; break; }
        }
        if (fixed && nfix == 0) cycles = 0;
        if (cur != x) HIPCHK(hipMemcpyAsync(x, cur, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
        if (fixed && info) {
            TRY(ir_step(P, x, nullptr, nullptr, b, nullptr, 1, st, false, want_epi));
            P->epi_fused = want_epi;
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            rel = std::sqrt(P->hnorm[1]) / (r0 > 0.0 ? r0 : 1.0);
        }
    } else {
        double* xc = x;
        double* xo = P->xalt64;
        TRY(set_boundary<double>(xo, l0.N, bc, st));
        TRY(ir_step(P, xc, nullptr, nullptr, b, l0.q32, 0, st, x_zero));
        double r0t = 0.0;   // DMGS_TRACE in fixed mode: the initial residual norm
        if (fixed && P->cfg_trace) {
            TRY(read_norms(P, st));
            r0t = std::sqrt(P->hnorm[0]);
        }
        // While the host waits for a step's residual norm, the first
        // smoothing pass of the next step is already enqueued when the
        // residual is not expected to meet the tolerance yet.  The pass
        // writes only the correction buffers, so a step that does converge
        // discards it.  With ir_adaptive, a step after the first runs the
        // number of V-cycles the per-cycle contraction factor observed so
        // far predicts the tolerance needs (at most ir_inner_cycles).
        const bool can_speculate = !fixed && !wjacobi(P) && P->L > 1 && fused_level(P, 0) && !block_level<float>(P, 0);
        const bool adaptive = !fixed && o.ir_adaptive;
        double rel1 = 1.0;     // relative residual before the last step
        double rate = 0.0;     // per-V-cycle contraction factor (0: not known yet)
        int inner = o.ir_inner_cycles;
        // A requested likelihood epilogue rides on the refinement step that
        // is expected to be the last (in tolerance mode: the contraction
        // seen so far predicts the tolerance met); epi_step names the step
        // whose iterate it was computed for.
        const bool want_epi = P->epi_d && order == 0 && ir_shape(l0.N, 3).nchunks > 0;
        int epi_step = -1;
        P->epi_fused = false;
        for (cycles = 0;; cycles++) {
            float* e = l0.u32;
            float* eo = l0.t32;
            bool smoothed = false, rdone = false;
            if (!fixed) {
                // residual the last step is expected to reach
                const double pred = cycles == 0 ? 1.0 : rel1 * std::pow(rate > 0.0 ? rate : 0.5, inner);
                if (can_speculate && cycles < o.max_cycles && pred > o.rtol) {
                    TRY(smooth_phase<float>(P, 0, &e, &eo, l0.q32, nu_pre_of(P, order), order, true, (const float*)nullptr, st,
                                            l0.r32, &rdone));
                    smoothed = true;
                }
                TRY(read_norms(P, st));
                if (cycles == 0) {
                    r0 = std::sqrt(P->hnorm[0]);
                    if (!std::isfinite(r0)) { set_error("non-finite right-hand side"); status = DMGS_ERR_NONFINITE; break; }
                    if (r0 == 0.0) break;
                    rel = 1.0;
                } else {
                    rel = std::sqrt(P->hnorm[1]) / r0;
                    trace_point(P, order, cycles, vcycles, rel);
                    if (!std::isfinite(rel)) { set_error("non-finite residual after %d steps", cycles); status = DMGS_ERR_NONFINITE; break; }
                    if (rel <= o.rtol) break;
                    rate = rel < rel1 ? std::pow(rel / rel1, 1.0 / inner) : 0.0;
                }
                if (cycles >= o.max_cycles) { set_error("not converged after %d steps (rel %.3e)", cycles, rel); status = DMGS_ERR_NOT_CONVERGED; break; }
                rel1 = rel;
                inner = o.ir_inner_cycles;
                if (adaptive && rate > 0.0) {
                    const double need = std::ceil(std::log(o.rtol / rel) / std::log(rate) - 1e-6);
                    inner = (int)std::min<double>(inner, std::max(1.0, need));
                }
            } else if (cycles == nfix) {
                break;
            }
            if (replay) inner = (*replay)[cycles];
            sched.push_back(inner);
            for (int ic = 0; ic < inner; ic++)
                TRY(vcycle<float>(P, 0, &e, &eo, l0.q32, order, ic == 0, st, ic == 0 && smoothed, rdone));
            vcycles += inner;
            bool epi = false;
            if (want_epi) {
                epi = fixed ? cycles == nfix - 1
                            : rate > 0.0 && rel * std::pow(rate, inner) <= o.rtol * (1.0 + 1e-6);
                if (epi) epi_step = cycles + 1;
            }
            if (x_zero && cycles == 0 && ((replay ? nfix : P->ir_steps[order]) & 1)) {
                // the first update reads no iterate, so it may write x in
                // place: with an odd number of steps (as a replayed schedule
                // has, or the last solve of this kind took) the result then
                // ends in x, not in xalt64
                TRY(ir_step(P, xc, e, xc, b, l0.q32, 1, st, true, epi));
            } else {
                TRY(ir_step(P, xc, e, xo, b, l0.q32, 1, st, x_zero && cycles == 0, epi));
                std::swap(xc, xo);
            }
            if (fixed && P->cfg_trace) {
                TRY(read_norms(P, st));
                trace_point(P, order, cycles + 1, vcycles, std::sqrt(P->hnorm[1]) / (r0t > 0.0 ? r0t : 1.0));
            }
        }
        P->ir_steps[order] = cycles;
        P->epi_fused = want_epi && epi_step == cycles && cycles > 0;
        if (x_zero && cycles == 0) {
            hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, l0.N, 0.0);
            LAUNCHCHK();
        }
        if (xc != x) HIPCHK(hipMemcpyAsync(x, xc, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
        if (fixed && info) {
            TRY(read_norms(P, st));
            r0 = std::sqrt(P->hnorm[0]);
            rel = std::sqrt(P->hnorm[nfix > 0 ? 1 : 0]) / (r0 > 0.0 ? r0 : 1.0);
        }
    }
done:
    if (record && !fixed) {
        P->fwd_recorded = status == DMGS_OK || status == DMGS_ERR_NOT_CONVERGED;
        P->fwd_schedule = sched;
    }
    if (info) {
        info->cycles = cycles;
        info->vcycles = is_ir(P) ? vcycles : cycles;
        info->rel_residual = rel;
        info->status = status;
    }
    return status;
}

int begin_call(dmgs_plan P, hipStream_t st, bool need_coef = true) {
    if (!P) { set_error("plan is NULL"); return DMGS_ERR_INVALID; }
    if (need_coef && !P->coef_set) { set_error("coefficients not set"); return DMGS_ERR_INVALID; }
    HIPCHK(hipSetDevice(P->device));
    if (P->ev_start) HIPCHK(hipEventRecord(P->ev_start, st));
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
        if (P->ev_stop && hipEventRecord(P->ev_stop, st) == hipSuccess && hipEventSynchronize(P->ev_stop) == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, P->ev_start, P->ev_stop) == hipSuccess) info->device_ms = ms;
        }
    }
    return status;
}

// Coefficient hierarchy from the finest level's D64 and mu64.  from_log:
// they are formed here from logD and logmu (exp and validation in one pass).
GridDims gdims(dmgs_plan P, int k) {
    const Level& l = P->lev[k];
    GridDims g;
    g.nx = l.nc[0];
    g.ny = l.nc[1];
    g.nz = l.nc[2];
    for (int a = 0; a < 3; a++) g.ih2[a] = 1.0 / (l.h3[a] * l.h3[a]);
    g.harmonic = harmonic(P);
    return g;
}

// Vertex counts per axis, fastest first, of a plan's finest level.
VertDims vdims(dmgs_plan P) {
    const Level& l = P->lev[0];
    VertDims d;
    if (P->grid) {
        d.n[0] = l.nc[2] + 1;
        d.n[1] = l.nc[1] + 1;
        d.n[2] = l.nc[0] + 1;
    } else {
        d.n[0] = d.n[1] = l.N + 1;
        d.n[2] = P->opt.ndim == 2 ? 1 : l.N + 1;
    }
    return d;
}

// Coefficient hierarchy of a general-grid plan (see build_hierarchy).
int build_hierarchy_grid(dmgs_plan P, hipStream_t st, const double* logD, const double* logmu) {
    Level& l0 = P->lev[0];
    *P->hflag = 0;
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, st, P->dflag, (int64_t)1, 0);
    LAUNCHCHK();
    TIMED(P, 0, DMGS_K_COEF, (logD ? 32.0 : 16.0) * l0.nv, st,
          hipLaunchKernelGGL(k_g_coef_in, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, logD, logmu, l0.D64,
                             l0.mu64, gdims(P, 0), P->dflag));
    HIPCHK(hipMemcpyAsync(P->hflag, P->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    if (!P->arena) HIPCHK(hipEventRecord(P->ev_flag, st));
    for (int k = 1; k < P->L; k++) {
        const Level& f = P->lev[k - 1];
        Level& c = P->lev[k];
        hipLaunchKernelGGL(k_g_coarsen, dim3(grid_for(c.nv)), dim3(kBlock), 0, st, (const double*)f.D64,
                           (const double*)f.mu64, gdims(P, k - 1), c.D64, c.mu64);
        LAUNCHCHK();
    }
    const Level& c = P->lev[P->L - 1];
    const int m = (c.nc[0] - 1) * (c.nc[1] - 1) * (c.nc[2] - 1);
    hipLaunchKernelGGL(k_g_inverse, dim3(1), dim3(64), (size_t)(2 * m * m * sizeof(double)), st, (const double*)c.D64,
                       (const double*)c.mu64, gdims(P, P->L - 1), P->cinv);
    LAUNCHCHK();
    if (P->arena) HIPCHK(hipStreamSynchronize(st));
    else HIPCHK(hipEventSynchronize(P->ev_flag));
    if (*P->hflag) {
        P->coef_set = false;
        set_error("coefficients must satisfy D > 0, mua >= 0 and be finite");
        return DMGS_ERR_INVALID;
    }
    P->coef_set = true;
    return DMGS_OK;
}

int build_hierarchy(dmgs_plan P, hipStream_t st, const double* logD = nullptr, const double* logmu = nullptr) {
    if (P->grid) return build_hierarchy_grid(P, st, logD, logmu);
    Level& l0 = P->lev[0];
    *P->hflag = 0;
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, st, P->dflag, (int64_t)1, 0);
    LAUNCHCHK();
    if (is2d(P)) {
        if (logD) {
            TIMED(P, 0, DMGS_K_COEF, 32.0 * l0.nv, st,
                  hipLaunchKernelGGL(k2_exp_validate, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, logD, logmu,
                                     l0.D64, l0.mu64, l0.N, P->dflag));
        } else {
            TIMED(P, 0, DMGS_K_COEF, 16.0 * l0.nv, st,
                  hipLaunchKernelGGL(k2_validate, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st,
                                     (const double*)l0.D64, (const double*)l0.mu64, l0.N, P->dflag));
        }
    } else if (logD) {
        TIMED(P, 0, DMGS_K_COEF, 32.0 * l0.nv, st,
              hipLaunchKernelGGL(k_exp_validate, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, logD, logmu, l0.D64,
                                 l0.mu64, l0.N, P->dflag));
    } else {
        TIMED(P, 0, DMGS_K_COEF, 16.0 * l0.nv, st,
              hipLaunchKernelGGL(k_validate, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, (const double*)l0.D64,
                                 (const double*)l0.mu64, l0.N, P->dflag));
    }
    HIPCHK(hipMemcpyAsync(P->hflag, P->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    if (!P->arena) HIPCHK(hipEventRecord(P->ev_flag, st));
    // the hierarchy is built while the host waits for the flag (on invalid
    // coefficients it is garbage, and the plan is marked unset)
    for (int k = 1; k < P->L; k++) {
        const Level& f = P->lev[k - 1];
        Level& c = P->lev[k];
        if (is2d(P))
            hipLaunchKernelGGL(k2_coarsen_coef, dim3(vertex_grid(c.nv)), dim3(kBlock), 0, st, (const double*)f.D64,
                               (const double*)f.mu64, c.D64, c.mu64, f.N);
        else
            hipLaunchKernelGGL(k_coarsen_coef, dim3(vertex_grid(c.nv)), dim3(kBlock), 0, st, (const double*)f.D64,
                               (const double*)f.mu64, c.D64, c.mu64, f.N);
        LAUNCHCHK();
    }
    if (!is2d(P)) {
        const Level& c = P->lev[P->L - 1];
        hipLaunchKernelGGL(k_coarse_inverse, dim3(1), dim3(64), 0, st, (const double*)c.D64, (const double*)c.mu64, c.N,
                           c.stencil<double>(harmonic(P)), P->cinv);
        LAUNCHCHK();
    }
    for (int k = 0; k < P->L && !is2d(P); k++) {
        Level& l = P->lev[k];
        if (is_ir(P)) {
            hipLaunchKernelGGL(k_level_prep<float>, dim3(vertex_grid(l.nv)), dim3(kBlock), 0, st, (const double*)l.D64,
                               (const double*)l.mu64, l.N, l.stencil<double>(harmonic(P)), l.w32, l.D32, l.mu32, l.py,
                               l.px);
        } else {
            hipLaunchKernelGGL(k_level_prep<double>, dim3(vertex_grid(l.nv)), dim3(kBlock), 0, st, (const double*)l.D64,
                               (const double*)l.mu64, l.N, l.stencil<double>(harmonic(P)), l.w64, (float*)nullptr,
                               (float*)nullptr, l.n, (int64_t)l.n * l.n);
        }
        LAUNCHCHK();
    }
    if (P->arena) HIPCHK(hipStreamSynchronize(st));
    else HIPCHK(hipEventSynchronize(P->ev_flag));
    if (*P->hflag) {
        P->coef_set = false;
        set_error("coefficients must satisfy D > 0, mua >= 0 and be finite");
        return DMGS_ERR_INVALID;
    }
    P->coef_set = true;
    return DMGS_OK;
}

int debug_check(dmgs_plan P, int k, int fp32, bool need_coarse) {
    if (!P || !P->coef_set) { set_error("plan without coefficients"); return DMGS_ERR_INVALID; }
    if (is2d(P) || P->grid) { set_error("the diagnostic entry points take cubic three-dimensional plans"); return DMGS_ERR_INVALID; }
    if (k < 0 || k >= P->L || (need_coarse && k >= P->L - 1)) { set_error("bad level %d", k); return DMGS_ERR_INVALID; }
    if (fp32 && !is_ir(P)) { set_error("float32 arrays need a DMGS_FP32_IN_FP64 plan"); return DMGS_ERR_INVALID; }
    if (hipSetDevice(P->device) != hipSuccess) { (void)hipGetLastError(); set_error("hipSetDevice failed"); return DMGS_ERR_HIP; }
    return DMGS_OK;
}

// Scratch of level k with the element type T (float64 plans: t64;
// refinement plans: t32).
template <class T>
T* level_scratch(dmgs_plan P, int k) { return Typed<T>::t(P->lev[k]); }

// Copy a field of level k between the dense layout (to_level false: dst)
// and the level's layout of T arrays (to_level true: dst).
template <class T>
int repitch(dmgs_plan P, int k, const T* src, T* dst, bool to_level, hipStream_t st) {
    const Level& l = P->lev[k];
    const int n = l.n, py = Typed<T>::py(l);
    const int64_t px = Typed<T>::px(l), dpx = (int64_t)n * n;
    if (to_level) hipLaunchKernelGGL(k_repitch<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, src, n, dpx, dst, py, px, n);
    else hipLaunchKernelGGL(k_repitch<T>, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, src, py, px, dst, n, dpx, n);
    LAUNCHCHK();
    return DMGS_OK;
}

// The diagnostic passes on a level whose T arrays have padded rows: the
// dense inputs are copied into the level's own iterate, partner and
// right-hand-side buffers (their previous contents are lost), the passes run
// there, and the result is copied back out.
template <class T>
int debug_pre_padded(dmgs_plan P, int k, int order, const T* u_in, const T* q, T* u_out, T* qc, hipStream_t st) {
    const Level& l = P->lev[k];
    T* cur = Typed<T>::u(l);
    T* oth = Typed<T>::t(l);
    T* ql = Typed<T>::q(l);
    if (u_in) {
        TRY(repitch<T>(P, k, u_in, cur, true, st));
        TRY(repitch<T>(P, k, u_in, oth, true, st));
    } else {
        TRY(fill<T>(cur, l.nv32, T(0), st));
        TRY(fill<T>(oth, l.nv32, T(0), st));
    }
    TRY(repitch<T>(P, k, q, ql, true, st));
    TRY(fill<T>(qc, P->lev[k + 1].nv, T(0), st));
    TRY(pre_pass<T>(P, k, &cur, &oth, ql, qc, order, u_in == nullptr, st));
    return repitch<T>(P, k, cur, u_out, false, st);
}

template <class T>
int debug_post_padded(dmgs_plan P, int k, int order, const T* u_in, const T* ec, const T* q, T* u_out, hipStream_t st) {
    const Level& l = P->lev[k];
    T* cur = Typed<T>::u(l);
    T* oth = Typed<T>::t(l);
    T* ql = Typed<T>::q(l);
    TRY(repitch<T>(P, k, u_in, cur, true, st));
    TRY(repitch<T>(P, k, u_in, oth, true, st));
    TRY(repitch<T>(P, k, q, ql, true, st));
    TRY(post_pass<T>(P, k, &cur, &oth, ec, ql, order, st));
    return repitch<T>(P, k, cur, u_out, false, st);
}

template <class T>
int debug_pre_t(dmgs_plan P, int k, int order, const T* u_in, const T* q, T* u_out, T* qc, hipStream_t st) {
    const Level& l = P->lev[k];
    if (!dense<T>(l)) return debug_pre_padded<T>(P, k, order, u_in, q, u_out, qc, st);
    T* scratch = level_scratch<T>(P, k);
    if (!scratch) { set_error("no scratch of this type on level %d", k); return DMGS_ERR_INVALID; }
    if (u_in) {
        HIPCHK(hipMemcpyAsync(u_out, u_in, l.nv * sizeof(T), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(scratch, u_in, l.nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    } else {   // zero iterate: both buffers get a zero boundary
        TRY(fill<T>(u_out, l.nv, T(0), st));
        TRY(fill<T>(scratch, l.nv, T(0), st));
    }
    TRY(fill<T>(qc, P->lev[k + 1].nv, T(0), st));   // coarse boundary entries are 0
    T* cur = u_out;
    T* oth = scratch;
    TRY(pre_pass<T>(P, k, &cur, &oth, q, qc, order, u_in == nullptr, st));
    if (cur != u_out) HIPCHK(hipMemcpyAsync(u_out, cur, l.nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    return DMGS_OK;
}

template <class T>
int debug_post_t(dmgs_plan P, int k, int order, const T* u_in, const T* ec, const T* q, T* u_out, hipStream_t st) {
    const Level& l = P->lev[k];
    if (!dense<T>(l)) return debug_post_padded<T>(P, k, order, u_in, ec, q, u_out, st);
    T* scratch = level_scratch<T>(P, k);
    if (!scratch) { set_error("no scratch of this type on level %d", k); return DMGS_ERR_INVALID; }
    HIPCHK(hipMemcpyAsync(u_out, u_in, l.nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(scratch, u_in, l.nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    T* cur = u_out;
    T* oth = scratch;
    TRY(post_pass<T>(P, k, &cur, &oth, ec, q, order, st));
    if (cur != u_out) HIPCHK(hipMemcpyAsync(u_out, cur, l.nv * sizeof(T), hipMemcpyDeviceToDevice, st));
    return DMGS_OK;
}

}  // namespace

// ===========================================================================
// C ABI

namespace {

// Grid of the column-tile kernels (derivatives, unrolled adjoint): (tile, chunk) blocks of kDerThreads; the
// chunk count is chosen so that the blocks, one per CU, fill the last round
// of CUs best, net of the two extra planes each chunk reads.  Chunks are
// whole multiples of the kernels' unrolled march.
// Levels from this size on leave the boundary planes y = N, z = N to extra
// grid rows of the same launch (at most two vertices per thread); smaller
// ones tile every vertex.
constexpr int kDerSplitMin = 128;

// Levels of the unrolled adjoint from this size on run the column-tile
// kernels (whole sweeps per pass), smaller ones the x-march kernels.
constexpr int kUnTileMin = 96;

dim3 der_grid(dmgs_plan P, int N, int* chunk, int* cover) {
    const int n = N + 1;
    *cover = N >= kDerSplitMin ? N : n;
    const int tiles = ((*cover + kDerTY - 1) / kDerTY) * ((*cover + kDerTZ - 1) / kDerTZ);   // y, z < cover
    int best_c = 1;
    double best = 0.0;
    auto chunk_of = [&](int c) { return ((n + c - 1) / c + kDerRing - 1) / kDerRing * kDerRing; };
    const int64_t pb = (int64_t)n * n * 8;
    for (int c = 1; c <= 64 && c <= n; c++) {
        const int ch = chunk_of(c);
        if ((int64_t)(ch + 5) * pb >= (int64_t)kOob) continue;   // the kernels' 32-bit span of planes
        const int nb = tiles * ((n + ch - 1) / ch);
        const int rounds = (nb + P->ncu - 1) / P->ncu;
        const double v = (double)nb / ((double)rounds * P->ncu) * ch / (ch + 2.0);
        if (v > best + 1e-9) {
            best = v;
            best_c = c;
        }
    }
    *chunk = chunk_of(best_c);
    const int nch = (n + *chunk - 1) / *chunk;
    const int64_t per_row = (int64_t)tiles * kDerThreads * 2;
    const int erows = *cover == N ? (int)((der_edge_count(N) + per_row - 1) / per_row) : 0;
    return dim3((unsigned)tiles, (unsigned)(nch + erows));
}

// tangent right-hand side q' - A' rho of the push-forward (Sec. 2.3)
int tangent_rhs(dmgs_plan P, const double* rho, const double* dq, const double* dlogD, const double* dlogmua,
                double* out, hipStream_t st) {
    const Level& l0 = P->lev[0];
    if (P->grid) {
        TIMED(P, 0, DMGS_K_GRAD, 56.0 * l0.nv, st,
              hipLaunchKernelGGL(k_g_tangent_rhs, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, rho, dq, dlogD, dlogmua,
                                 (const double*)l0.D64, (const double*)l0.mu64, gdims(P, 0), out));
        return DMGS_OK;
    }
    if (is2d(P)) {
        TIMED(P, 0, DMGS_K_GRAD, 56.0 * l0.nv, st,
              hipLaunchKernelGGL(k2_tangent_rhs, dim3(vertex_grid(l0.nv)), dim3(kBlock), 0, st, rho, dq, dlogD,
                                 dlogmua, (const double*)l0.D64, (const double*)l0.mu64, l0.N, l0.inv_h2,
                                 harmonic(P), out));
        return DMGS_OK;
    }
    int chunk = 1, cover = 0;
    const dim3 g = der_grid(P, l0.N, &chunk, &cover);
    auto launch = [&](auto harm) {
        hipLaunchKernelGGL(k_tangent_rhs_col<decltype(harm)::value>, g, dim3(kDerThreads), 0, st, rho, dq, dlogD,
                           dlogmua, (const double*)l0.D64, (const double*)l0.mu64, l0.N, l0.inv_h2, out, chunk, cover);
    };
    TIMED(P, 0, DMGS_K_GRAD, 56.0 * l0.nv, st,
          (harmonic(P) ? launch(std::true_type()) : launch(std::false_type())));
    return DMGS_OK;
}

// coefficient gradients from the adjoint state lam (the derivative of the discrete solution); with data d and
// weights w, also the likelihood's direct log mua term
int coef_grads(dmgs_plan P, const double* rho, const double* lam, double* gD, double* gmu, const double* d,
               const double* w, hipStream_t st) {
    const Level& l0 = P->lev[0];
    if (P->grid) {
        TIMED(P, 0, DMGS_K_GRAD, 48.0 * l0.nv, st,
              hipLaunchKernelGGL(k_g_coef_grads, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, rho, lam,
                                 (const double*)l0.D64, (const double*)l0.mu64, gdims(P, 0), gD, gmu, d, w));
        return DMGS_OK;
    }
    if (is2d(P)) {
        TIMED(P, 0, DMGS_K_GRAD, 48.0 * l0.nv, st,
              hipLaunchKernelGGL(k2_coef_grads, dim3(vertex_grid(l0.nv)), dim3(kBlock), 0, st, rho, lam,
                                 (const double*)l0.D64, (const double*)l0.mu64, l0.N, l0.inv_h2, harmonic(P), gD,
                                 gmu));
        if (d && gmu) {
            hipLaunchKernelGGL(k_likelihood_direct, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, rho,
                               (const double*)l0.mu64, d, w, l0.nv, vdims(P), gmu);
            LAUNCHCHK();
        }
        return DMGS_OK;
    }
    int chunk = 1, cover = 0;
    const dim3 g = der_grid(P, l0.N, &chunk, &cover);
    const double bytes = (gD ? 40.0 : 24.0) + (gmu ? 8.0 : 0.0) + (d && gmu ? 16.0 : 0.0);
    const bool data = d && w && gmu;
    auto launch = [&](auto harm, auto dat) {
        hipLaunchKernelGGL((k_coef_grads_col<decltype(harm)::value, decltype(dat)::value>), g, dim3(kDerThreads), 0, st,
                           rho, lam, (const double*)l0.D64, (const double*)l0.mu64, l0.N, l0.inv_h2, gD, gmu, d, w,
                           chunk, cover);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    TIMED(P, 0, DMGS_K_GRAD, bytes * l0.nv, st,
          (harmonic(P) ? (data ? launch(T_(), T_()) : launch(T_(), F_())) : (data ? launch(F_(), T_()) : launch(F_(), F_()))));
    return DMGS_OK;
}

}  // namespace

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
    o->ir_inner_cycles = 8;
    o->ir_adaptive = 1;
    o->adjoint_schedule = 0;
    o->ndim = 3;
}

size_t dmgs_workspace_bytes(const dmgs_options* o) {
    if (check_options(o) != DMGS_OK) return 0;
    return footprint(o);
}

size_t dmgs_forward_vjp_workspace_bytes(const dmgs_options* o) {
    if (check_options(o) != DMGS_OK) return 0;
    if (general_grid(o)) return footprint(o);   // the two solves share the plan's buffers
    // the twin's work buffers (make_twin): per level the iterate, right-hand
    // side and partner (+ the defect buffer below the coarsest) in IR plans,
    // or partner (+ iterate and right-hand side below the finest) in float64
    // plans; the float64 scratch (+ alternate iterate) and the partials
    Sizes s = sizes_for(o);
    const bool ir = o->precision == DMGS_FP32_IN_FP64;
    const int py0 = fine_row_pitch(o, read_knobs(o), s.L);
    size_t b = 0;
    for (int k = 0; k < s.L; k++) {
        if (ir) b += (k < s.L - 1 ? 4 : 3) * nv32_of(o, s, k, py0) * sizeof(float);
        else b += ((k > 0 ? 3 : 1) + (o->ndim == 2 && k < s.L - 1 ? 1 : 0)) * s.nv[k] * sizeof(double);
    }
    b += (ir ? 2 : 1) * s.nv[0] * sizeof(double);
    b += kMaxPartials * sizeof(double) + 4 * sizeof(double);
    return footprint(o) + b;
}

}  // extern "C"

namespace {

// Dynamic-LDS limits of the kernels that take more than the default, set
// once per device (the attributes are process-wide, and plans may be created
// by several host threads while others launch those kernels).
int kernel_attributes(int device) {
    constexpr int kDevices = 64;
    static std::mutex lock;
    static bool done[kDevices] = {};
    std::lock_guard<std::mutex> guard(lock);
    if (device >= 0 && device < kDevices && done[device]) return DMGS_OK;
    const int lim = (int)kSmallLdsLimit;
    const void* fns[] = {(const void*)k_small_vcycle<float, false>, (const void*)k_small_vcycle<float, true>,
                         (const void*)k_small_vcycle<double, false>, (const void*)k_small_vcycle<double, true>,
                         (const void*)k_small_grp<float, false>, (const void*)k_small_grp<float, true>};
    for (const void* f : fns)
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) {
            (void)hipGetLastError(); set_error("hipFuncSetAttribute failed");
            return DMGS_ERR_HIP;
        }
    // the general-grid coarsest inverse: a plan's own size would lower the
    // limit for plans with a larger coarsest level, so the largest is set
    if (hipFuncSetAttribute((const void*)k_g_inverse, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(2 * kGridCoarseMax * kGridCoarseMax * sizeof(double))) != hipSuccess) {
        (void)hipGetLastError(); set_error("hipFuncSetAttribute failed");
        return DMGS_ERR_HIP;
    }
    TRY(sweep2_attributes());
    TRY(block_attributes());
    if (device >= 0 && device < kDevices) done[device] = true;
    return DMGS_OK;
}

// Levels, buffers and configuration of a new plan on the current device.
// Ordinary plans allocate every buffer (hipMalloc, pinned host slots,
// events) and clear the work buffers synchronously; arena plans (P->arena
// set) carve the buffers from the arena and clear them with fill kernels on
// stream zst.  On failure the caller frees what was allocated (free_plan).
// Levels and buffers of a general-grid plan (see plan_init): per level
// D64, mu64, below the finest u64 and q64, above the coarsest t64 (the
// defect); the finest scratch, partials, the coarsest inverse, the flag.
int grid_plan_init(dmgs_plan P, const dmgs_options* o, hipStream_t zst) {
    P->grid = true;
    // the one tuning knob that applies to general grids
    if (const char* e = std::getenv("DMGS_EPI_FUSE")) P->cfg_epi_fuse = std::atoi(e) != 0;
    int cn[kMaxLevels][3];
    P->L = grid_levels(o->n, cn);
    int st = DMGS_OK;
    for (int k = 0; k < P->L && st == DMGS_OK; k++) {
        Level& l = P->lev[k];
        for (int a = 0; a < 3; a++) {
            l.nc[a] = cn[k][a];
            l.h3[a] = axis_h(o, a) * (double)(1 << k);
        }
        l.N = cn[k][0];
        l.n = l.N + 1;
        l.nv = (int64_t)(cn[k][0] + 1) * (cn[k][1] + 1) * (cn[k][2] + 1);
        l.h = l.h3[0];
        l.inv_h2 = 1.0 / (l.h * l.h);
        l.py = l.n;   // no float32 arrays
        l.px = (int64_t)l.n * l.n;
        l.nv32 = 0;
        if (st == DMGS_OK) st = dalloc(P, &l.D64, l.nv);
        if (st == DMGS_OK) st = dalloc(P, &l.mu64, l.nv);
        if (k > 0 && st == DMGS_OK) st = dalloc(P, &l.u64, l.nv);
        if (k > 0 && st == DMGS_OK) st = dalloc(P, &l.q64, l.nv);
        if (k < P->L - 1 && st == DMGS_OK) st = dalloc(P, &l.t64, l.nv);
    }
    if (st == DMGS_OK) st = dalloc(P, &P->scratch64, P->lev[0].nv);
    if (st == DMGS_OK) st = dalloc(P, &P->partial, kMaxPartials);
    if (st == DMGS_OK) st = dalloc(P, &P->cinv, kGridCoarseMax * kGridCoarseMax);
    if (st == DMGS_OK) st = dalloc(P, &P->dflag, 1);
    if (P->arena) {
        if (st == DMGS_OK) st = dalloc(P, &P->dnorm, 4);
        P->hnorm = P->hnorm_buf;
        P->hflag = &P->hflag_buf;
    } else {
        if (st == DMGS_OK && hipHostMalloc((void**)&P->hnorm, 4 * sizeof(double), hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc failed");
            st = DMGS_ERR_OOM;
        }
        if (st == DMGS_OK && hipHostMalloc((void**)&P->hflag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc failed");
            st = DMGS_ERR_OOM;
        }
        if (st == DMGS_OK && (hipEventCreate(&P->ev_start) != hipSuccess || hipEventCreate(&P->ev_stop) != hipSuccess ||
                              hipEventCreateWithFlags(&P->ev_norm, hipEventDisableTiming) != hipSuccess ||
                              hipEventCreateWithFlags(&P->ev_flag, hipEventDisableTiming) != hipSuccess)) {
            (void)hipGetLastError();
            set_error("hipEventCreate failed");
            st = DMGS_ERR_HIP;
        }
    }
    // the coarse iterates and right-hand sides start at 0 (their boundaries
    // stay 0), and so do the defects' boundaries
    for (int k = 0; k < P->L && st == DMGS_OK; k++) {
        Level& l = P->lev[k];
        for (double* p : {l.u64, l.q64, l.t64}) {
            if (!p) continue;
            hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(l.nv)), dim3(kBlock), 0, zst, p, l.nv, 0.0);
            if (hipGetLastError() != hipSuccess) { set_error("fill kernel launch failed"); st = DMGS_ERR_HIP; }
        }
    }
    if (st == DMGS_OK && !P->arena && hipStreamSynchronize(zst) != hipSuccess) {
        set_error("stream synchronisation failed");
        st = DMGS_ERR_HIP;
    }
    if (st == DMGS_OK) st = kernel_attributes(P->device);
    return st;
}

int plan_init(dmgs_plan P, const dmgs_options* o, hipStream_t zst) {
    P->opt = *o;
    if (hipGetDevice(&P->device) != hipSuccess) { (void)hipGetLastError(); set_error("hipGetDevice failed"); return DMGS_ERR_HIP; }
    if (general_grid(o)) return grid_plan_init(P, o, zst);
    // cubic and square plans: one spacing (h_axis, when all three are given and equal, is it)
    if (o->ndim == 3) P->opt.h = axis_h(o, 0);
    o = &P->opt;
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && ncu > 0)
            P->ncu = ncu;
    }
    Sizes s = sizes_for(o);
    P->L = s.L;
    bool ir = o->precision == DMGS_FP32_IN_FP64;
    const Knobs kn = read_knobs(o);
    const int py0 = fine_row_pitch(o, kn, s.L);
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
        l.py = k == 0 && o->ndim == 3 ? py0 : l.n;
        l.px = (int64_t)l.py * l.n;
        l.nv32 = nv32_of(o, s, k, py0);
        if (st == DMGS_OK) st = dalloc(P, &l.D64, l.nv);
        if (st == DMGS_OK) st = dalloc(P, &l.mu64, l.nv);
        if (ir) {
            if (st == DMGS_OK) st = dalloc(P, &l.D32, l.nv32);
            if (st == DMGS_OK) st = dalloc(P, &l.mu32, l.nv32);
            if (st == DMGS_OK) st = dalloc(P, &l.w32, l.nv32);
            if (st == DMGS_OK) st = dalloc(P, &l.u32, l.nv32);
            if (st == DMGS_OK) st = dalloc(P, &l.q32, l.nv32);
            if (st == DMGS_OK) st = dalloc(P, &l.t32, l.nv32);
            if (k < s.L - 1 && st == DMGS_OK) st = dalloc(P, &l.r32, l.nv32);
        } else {
            // two-dimensional cycles take no inverse diagonal (t64 is the
            // partner buffer of the out-of-place passes)
            if (o->ndim != 2 && st == DMGS_OK) st = dalloc(P, &l.w64, l.nv);
            if (k > 0 && st == DMGS_OK) st = dalloc(P, &l.u64, l.nv);
            if (k > 0 && st == DMGS_OK) st = dalloc(P, &l.q64, l.nv);
            if (st == DMGS_OK) st = dalloc(P, &l.t64, l.nv);
            if (o->ndim == 2 && k < s.L - 1 && st == DMGS_OK) st = dalloc(P, &l.rd64, l.nv);
        }
    }
    if (st == DMGS_OK) st = dalloc(P, &P->scratch64, P->lev[0].nv);
    if (ir && st == DMGS_OK) st = dalloc(P, &P->xalt64, P->lev[0].nv);
    if (st == DMGS_OK) st = dalloc(P, &P->partial, kMaxPartials);
    if (st == DMGS_OK) st = dalloc(P, &P->cinv, kCoarseMax * kCoarseMax);

    if (st == DMGS_OK) st = dalloc(P, &P->dflag, 1);
    if (P->arena) {
        if (st == DMGS_OK) st = dalloc(P, &P->dnorm, 4);
        P->hnorm = P->hnorm_buf;
        P->hflag = &P->hflag_buf;
    } else {
        if (st == DMGS_OK && hipHostMalloc((void**)&P->hnorm, 4 * sizeof(double), hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc failed");
            st = DMGS_ERR_OOM;
        }
        if (st == DMGS_OK && hipHostMalloc((void**)&P->hflag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc failed");
            st = DMGS_ERR_OOM;
        }
        if (st == DMGS_OK && (hipEventCreate(&P->ev_start) != hipSuccess || hipEventCreate(&P->ev_stop) != hipSuccess ||
                              hipEventCreateWithFlags(&P->ev_norm, hipEventDisableTiming) != hipSuccess ||
                              hipEventCreateWithFlags(&P->ev_flag, hipEventDisableTiming) != hipSuccess)) {
            (void)hipGetLastError();
            set_error("hipEventCreate failed");
            st = DMGS_ERR_HIP;
        }
    }
    // every work buffer starts at 0: the passes never write boundary layers
    // or row padding, and coarse corrections have homogeneous boundaries (an
    // arena keeps the last call's contents, so its buffers are cleared on the
    // stream); the coefficient arrays' row padding is 0 as well
    for (int k = 0; k < P->L && st == DMGS_OK; k++) {
        Level& l = P->lev[k];
        void* ps[] = {l.u64, l.q64, l.t64, l.u32, l.q32, l.t32, l.r32, l.rd64, l.D32, l.mu32, l.w32};
        size_t sz[] = {8, 8, 8, 4, 4, 4, 4, 8, 4, 4, 4};
        for (int j = 0; j < 11 && st == DMGS_OK; j++) {
            if (!ps[j] || (j >= 8 && dense<float>(l))) continue;
            const int64_t cnt = sz[j] == 8 ? l.nv : l.nv32;
            if (P->arena) {
                if (sz[j] == 8) hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(cnt)), dim3(kBlock), 0, zst, (double*)ps[j], cnt, 0.0);
                else hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(cnt)), dim3(kBlock), 0, zst, (float*)ps[j], cnt, 0.0f);
                if (hipGetLastError() != hipSuccess) { set_error("fill kernel launch failed"); st = DMGS_ERR_HIP; }
            } else if (hipMemset(ps[j], 0, cnt * sz[j]) != hipSuccess) {
                (void)hipGetLastError(); set_error("hipMemset failed");
                st = DMGS_ERR_HIP;
            }
        }
    }
    P->cfg_sweep = 0;
    P->cfg_fuse_min = kn.fuse_min;
    // first level handled by the single-workgroup kernel (N <= 16 in float32,
    // N <= 8 in float64, all remaining levels within the LDS budget)
    P->small32 = P->small64 = -1;
    P->small2 = -1;
    int small2_max = kSmall2MaxN;
    if (const char* e = std::getenv("DMGS_2D_SMALL_MAX")) small2_max = std::min(kSmall2MaxN, std::atoi(e));
    for (int k = 1; k < P->L - 1 && o->ndim == 2; k++)
        if (P->lev[k].N <= small2_max && P->L - k <= kSmall2MaxLevels) {
            P->small2 = k;
            break;
        }
    for (int k = 1; k < P->L && st == DMGS_OK && o->ndim != 2; k++) {
        int Ns[kSmallMaxLevels];
        int nl = P->L - k;
        if (nl > kSmallMaxLevels) continue;
        for (int i = 0; i < nl; i++) Ns[i] = P->lev[k + i].N;
        if (P->small32 < 0 && P->lev[k].N <= 16 && small_lds_bytes<float>(Ns, nl) <= kSmallLdsLimit) P->small32 = k;
        if (P->small64 < 0 && P->lev[k].N <= 8 && small_lds_bytes<double>(Ns, nl) <= kSmallLdsLimit) P->small64 = k;
    }
    if (st == DMGS_OK) st = kernel_attributes(P->device);
    P->cfg_block_max = kn.block_max;
    // float64 plans: twice the workgroups (each moves twice the bytes of a
    // float32 one; 20.76 -> 20.52 ms per 256^3 forward + VJP step)
    P->cfg_dr_wgs = o->precision == DMGS_FP64 ? 1024 : 512;
    if (const char* e = std::getenv("DMGS_DR_WGS")) P->cfg_dr_wgs = std::max(16, std::atoi(e));
    P->cfg_defect = kn.defect;
    P->cfg_sweep2_min = kn.sweep2_min;
    P->cfg_sweep2_wgs = 256;
    if (const char* e = std::getenv("DMGS_SWEEP2_WGS")) P->cfg_sweep2_wgs = std::max(16, std::atoi(e));
    // below the finest level the passes are latency-bound: longer chunks on
    // half as many workgroups take less CU time, which the concurrent solves
    // of dmgs_forward_vjp use
    P->cfg_sweep2_wgs_coarse = std::max(16, P->cfg_sweep2_wgs / 2);
    if (const char* e = std::getenv("DMGS_SWEEP2_WGS_COARSE")) P->cfg_sweep2_wgs_coarse = std::max(16, std::atoi(e));
    if (const char* e = std::getenv("DMGS_SWEEP_CFG")) P->cfg_sweep = std::min(2, std::max(0, std::atoi(e)));
    if (const char* e = std::getenv("DMGS_2D_SWEEP2_MIN")) P->cfg_2d_sweep2_min = std::max(4, std::atoi(e));
    if (const char* e = std::getenv("DMGS_SWEEP2_FP64")) P->cfg_sweep2_fp64 = std::atoi(e) != 0;
    if (const char* e = std::getenv("DMGS_2D_BLOCK_MIN")) P->cfg_2d_block_min = std::max(4, std::atoi(e));
    if (const char* e = std::getenv("DMGS_2D_DEFECT")) P->cfg_2d_defect = std::atoi(e) != 0;
    if (const char* e = std::getenv("DMGS_EPI_FUSE")) P->cfg_epi_fuse = std::atoi(e) != 0;
    if (const char* e = std::getenv("DMGS_2D_CHUNK")) P->cfg_2d_chunk = std::max(8, std::atoi(e) / 8 * 8);
    return st;
}

}  // namespace

extern "C" {

int dmgs_plan_create(const dmgs_options* o, dmgs_plan* out) {
    if (!out) { set_error("out is NULL"); return DMGS_ERR_INVALID; }
    *out = nullptr;
    TRY(check_options(o));
    dmgs_plan P = new (std::nothrow) dmgs_plan_s();
    if (!P) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
    int st = plan_init(P, o, nullptr);
    if (st == DMGS_OK) {
        // tracing aid: residual history of every solve (dmgs_trace_read) and
        // per-class kernel timing of every finest-level launch
        if (const char* e = std::getenv("DMGS_TRACE")) P->cfg_trace = std::atoi(e) != 0;
        if (P->cfg_trace) st = dmgs_timing_enable(P, 1);
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

int dmgs_plan_level_shape(dmgs_plan P, int k, int32_t* n3) {
    if (!P || !n3 || k < 0 || k >= P->L) { set_error("bad plan, pointer or level"); return DMGS_ERR_INVALID; }
    const Level& l = P->lev[k];
    for (int a = 0; a < 3; a++) n3[a] = P->grid ? l.nc[a] : (a == 2 && is2d(P) ? 0 : l.N);
    return DMGS_OK;
}

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
    return build_hierarchy(P, st, logD, logmua);
}

int dmgs_forward(dmgs_plan P, const double* q, double* rho, dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!q || !rho) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    int s = solve(P, q, rho, P->opt.bc_value, 0, info, st, nullptr, true);
    return end_call(P, s, info, st);
}

int dmgs_jvp(dmgs_plan P, const double* rho, const double* dq, const double* dlogD, const double* dlogmua, double* drho,
             dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!rho || !drho) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    TRY(tangent_rhs(P, rho, dq, dlogD, dlogmua, P->scratch64, st));
    int s = solve(P, P->scratch64, drho, 0.0, 0, info, st);
    return end_call(P, s, info, st);
}

int dmgs_vjp(dmgs_plan P, const double* rho, const double* rhobar, double* qbar, double* logD_bar, double* logmua_bar,
             dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!rho || !rhobar || !qbar) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    const std::vector<int>* replay = nullptr;
    if (P->opt.adjoint_schedule && P->opt.fixed_cycles <= 0) {
        if (!P->fwd_recorded) { set_error("adjoint_schedule: no forward solve recorded on this plan"); return DMGS_ERR_INVALID; }
        replay = &P->fwd_schedule;
    }
    int s = solve(P, rhobar, qbar, 0.0, 1, info, st, replay);
    if ((s == DMGS_OK || s == DMGS_ERR_NOT_CONVERGED) && (logD_bar || logmua_bar)) {
        TRY(coef_grads(P, rho, qbar, logD_bar, logmua_bar, nullptr, nullptr, st));
    }
    return end_call(P, s, info, st);
}

namespace {
// The twin of a plan: the same options, levels and coefficient hierarchy
// (aliased, not owned) with work buffers, reductions, events and a stream of
// its own, so that a second solve can run beside one on the plan.
int make_twin(dmgs_plan P) {
    if (P->twin) return DMGS_OK;
    dmgs_plan T = new (std::nothrow) dmgs_plan_s();
    if (!T) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
    T->opt = P->opt;
    T->L = P->L;
    T->device = P->device;
    T->owns_coef = false;
    T->cfg_sweep = P->cfg_sweep;
    T->cfg_fuse_min = P->cfg_fuse_min;
    T->cfg_sweep2_min = P->cfg_sweep2_min;
    T->cfg_sweep2_wgs = P->cfg_sweep2_wgs;
    T->cfg_sweep2_wgs_coarse = P->cfg_sweep2_wgs_coarse;
    T->cfg_block_max = P->cfg_block_max;
    T->cfg_dr_wgs = P->cfg_dr_wgs;
    T->cfg_defect = P->cfg_defect;
    T->cfg_2d_sweep2_min = P->cfg_2d_sweep2_min;
    T->cfg_sweep2_fp64 = P->cfg_sweep2_fp64;
    T->cfg_2d_block_min = P->cfg_2d_block_min;
    T->cfg_trace = P->cfg_trace;
    T->cfg_2d_defect = P->cfg_2d_defect;
    T->ncu = P->ncu;
    T->small2 = P->small2;
    T->cfg_2d_chunk = P->cfg_2d_chunk;
    T->small32 = P->small32;
    T->small64 = P->small64;
    T->cinv = P->cinv;
    const bool ir = is_ir(P);
    int st = DMGS_OK;
    for (int k = 0; k < P->L && st == DMGS_OK; k++) {
        const Level& pl = P->lev[k];
        Level& l = T->lev[k];
        l = pl;   // geometry and coefficient arrays
        l.u64 = l.q64 = l.t64 = l.rd64 = nullptr;
        l.u32 = l.q32 = l.t32 = l.r32 = nullptr;
        if (ir) {
            if (st == DMGS_OK) st = dalloc(T, &l.u32, l.nv32);
            if (st == DMGS_OK) st = dalloc(T, &l.q32, l.nv32);
            if (st == DMGS_OK) st = dalloc(T, &l.t32, l.nv32);
            if (k < P->L - 1 && st == DMGS_OK) st = dalloc(T, &l.r32, l.nv32);
        } else {
            if (k > 0 && st == DMGS_OK) st = dalloc(T, &l.u64, l.nv);
            if (k > 0 && st == DMGS_OK) st = dalloc(T, &l.q64, l.nv);
            if (st == DMGS_OK) st = dalloc(T, &l.t64, l.nv);
            if (is2d(P) && k < P->L - 1 && st == DMGS_OK) st = dalloc(T, &l.rd64, l.nv);
        }
        void* ps[] = {l.u64, l.q64, l.t64, l.u32, l.q32, l.t32, l.r32};
        size_t sz[] = {8, 8, 8, 4, 4, 4, 4};
        for (int j = 0; j < 7 && st == DMGS_OK; j++)
            if (ps[j] && hipMemset(ps[j], 0, (sz[j] == 8 ? l.nv : l.nv32) * sz[j]) != hipSuccess) {
                (void)hipGetLastError(); set_error("hipMemset failed");
                st = DMGS_ERR_HIP;
            }
    }
    if (st == DMGS_OK) st = dalloc(T, &T->scratch64, T->lev[0].nv);
    if (ir && st == DMGS_OK) st = dalloc(T, &T->xalt64, T->lev[0].nv);
    if (st == DMGS_OK) st = dalloc(T, &T->partial, kMaxPartials);
    if (st == DMGS_OK && hipHostMalloc((void**)&T->hnorm, 4 * sizeof(double), hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc failed");
        st = DMGS_ERR_OOM;
    }
    if (st == DMGS_OK && (hipEventCreate(&T->ev_start) != hipSuccess || hipEventCreate(&T->ev_stop) != hipSuccess ||
                          hipEventCreateWithFlags(&T->ev_norm, hipEventDisableTiming) != hipSuccess ||
                          hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
                          hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess ||
                          hipStreamCreateWithFlags(&P->twin_stream, hipStreamNonBlocking) != hipSuccess)) {
        (void)hipGetLastError(); set_error("hipEventCreate / hipStreamCreate failed");
        st = DMGS_ERR_HIP;
    }
    if (st == DMGS_OK) st = hipDeviceSynchronize() == hipSuccess ? DMGS_OK : DMGS_ERR_HIP;
    if (st != DMGS_OK) {
        free_plan(T);
        return st;
    }
    P->twin = T;
    P->bytes += T->bytes;
    return DMGS_OK;
}
}  // namespace

int dmgs_forward_vjp(dmgs_plan P, const double* q, const double* rhobar, double* rho, double* qbar, double* logD_bar,
                     double* logmua_bar, dmgs_info* info_fwd, dmgs_info* info_vjp, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!q || !rhobar || !rho || !qbar) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    if (P->grid) {
        // general grids: the two solves one after the other on `stream`
        const bool replay = P->opt.adjoint_schedule && P->opt.fixed_cycles <= 0;
        const int sf = solve(P, q, rho, P->opt.bc_value, 0, info_fwd, st, nullptr, true);
        if (sf != DMGS_OK && sf != DMGS_ERR_NOT_CONVERGED) return end_call(P, sf, info_fwd, st);
        const int sa = solve(P, rhobar, qbar, 0.0, 1, info_vjp, st, replay ? &P->fwd_schedule : nullptr);
        if ((sa == DMGS_OK || sa == DMGS_ERR_NOT_CONVERGED) && (logD_bar || logmua_bar))
            TRY(coef_grads(P, rho, qbar, logD_bar, logmua_bar, nullptr, nullptr, st));
        const int s = end_call(P, sf != DMGS_OK ? sf : sa, info_fwd, st);
        if (info_vjp) info_vjp->status = sa;
        return s;
    }
    TRY(make_twin(P));
    dmgs_plan T = P->twin;
    T->coef_set = true;
    // the adjoint solve starts after the work already enqueued on `stream`
    // (the coefficients) and runs on the twin's stream from a second host
    // thread; `stream` waits for it before the gradients
    // With adjoint_schedule (tolerance mode) the adjoint solve repeats the
    // forward solve's schedule, so it starts once the forward one has run
    // on the host (its kernels may still be in flight).
    const bool replay = P->opt.adjoint_schedule && P->opt.fixed_cycles <= 0;
    int sa = DMGS_OK, sf = DMGS_OK;
    std::string err_a;
    auto adjoint = [&] {
        if (hipSetDevice(P->device) != hipSuccess) { sa = DMGS_ERR_HIP; err_a = "hipSetDevice failed"; return; }
        sa = solve(T, rhobar, qbar, 0.0, 1, info_vjp, P->twin_stream, replay ? &T->fwd_schedule : nullptr);
        if (sa != DMGS_OK) err_a = dmgs_last_error();
    };
    if (replay) {
        sf = solve(P, q, rho, P->opt.bc_value, 0, info_fwd, st, nullptr, true);
        if (sf != DMGS_OK && sf != DMGS_ERR_NOT_CONVERGED) return end_call(P, sf, info_fwd, st);
        T->fwd_schedule = P->fwd_schedule;
        HIPCHK(hipEventRecord(P->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(P->twin_stream, P->ev_fork, 0));
        adjoint();
    } else {
        HIPCHK(hipEventRecord(P->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(P->twin_stream, P->ev_fork, 0));
        std::thread adj(adjoint);
        sf = solve(P, q, rho, P->opt.bc_value, 0, info_fwd, st, nullptr, true);
        adj.join();
    }
    if (hipEventRecord(P->ev_join, P->twin_stream) != hipSuccess || hipStreamWaitEvent(st, P->ev_join, 0) != hipSuccess) {
        set_error("event join failed");
        return DMGS_ERR_HIP;
    }
    P->trace[1] = T->trace[1];   // the pull-back ran on the twin
    const bool ok_f = sf == DMGS_OK || sf == DMGS_ERR_NOT_CONVERGED;
    const bool ok_a = sa == DMGS_OK || sa == DMGS_ERR_NOT_CONVERGED;
    if (ok_f && ok_a && (logD_bar || logmua_bar)) {
        TRY(coef_grads(P, rho, qbar, logD_bar, logmua_bar, nullptr, nullptr, st));
    }
    int s = sf != DMGS_OK ? sf : sa;
    if (sf == DMGS_OK && sa != DMGS_OK) set_error("adjoint solve: %s", err_a.c_str());
    s = end_call(P, s, info_fwd, st);
    if (info_vjp) {
        info_vjp->status = sa;
        if (info_fwd) info_vjp->device_ms = info_fwd->device_ms;
    }
    return s;
}

}  // extern "C"

namespace {
// Work buffers of the unrolled reverse pass, owned by the plan once its
// first call has allocated them (hipFree waits for the device).
// Grid of the column-march kernels: blocks of kBlock threads over a plane
// times chunks of planes, about 2048 blocks on large levels (each chunk
// re-reads one plane on either side).
dim3 un_col_grid(int N, int* chunk) {
    const int n = N + 1;
    const int64_t bx = ((int64_t)n * n + kBlock - 1) / kBlock;
    int nch = (int)std::min<int64_t>(n, std::max<int64_t>(1, (2048 + bx - 1) / bx));
    *chunk = (n + nch - 1) / nch;
    nch = (n + *chunk - 1) / *chunk;
    return dim3((unsigned)bx, (unsigned)nch);
}

struct UnWork {
    std::vector<void*> bufs;
    std::vector<size_t> sizes;
    size_t bytes = 0;
    bool store_all = false;                       // every cycle's states kept (no checkpoints, no recompute)
    std::vector<double*> sets;                    // the tape pointers of each kept cycle: [c][k][h]
    double* ckpt = nullptr;                       // the finest iterate at the start of every cycle
    double* u0 = nullptr;                         // the finest working iterate
    double* tape[kMaxLevels][33] = {};            // per level: the state after each half-sweep (pre, then post)
                                                  // and, last, the state the defect reads; the coarsest: its solution
    double *uc[kMaxLevels] = {}, *qc[kMaxLevels] = {}, *r[kMaxLevels] = {};
    double *ubar[kMaxLevels] = {}, *qbar[kMaxLevels] = {}, *Dbar[kMaxLevels] = {}, *mbar[kMaxLevels] = {},
           *V[kMaxLevels] = {};
    int alloc(double** p, int64_t n) {
        if (hipMalloc((void**)p, (size_t)n * sizeof(double)) != hipSuccess) {
            *p = nullptr;
            // the failure is returned here; clear HIP's last error so that the
            // next launch check does not report it again (the caller may fall
            // back to a smaller layout and go on)
            (void)hipGetLastError();
            set_error("hipMalloc of %lld bytes failed (unrolled reverse pass)", (long long)(n * sizeof(double)));
            return DMGS_ERR_OOM;
        }
        bufs.push_back(*p);
        sizes.push_back((size_t)n * sizeof(double));
        bytes += (size_t)n * sizeof(double);
        return DMGS_OK;
    }
    // [p, p + count doubles) lies inside one of the buffers
    bool holds(const double* p, int64_t count) const {
        const char* a = reinterpret_cast<const char*>(p);
        for (size_t i = 0; i < bufs.size(); i++) {
            const char* b = static_cast<const char*>(bufs[i]);
            if (a >= b && a + (size_t)count * sizeof(double) <= b + sizes[i]) return true;
        }
        return false;
    }
    // point the tape slots at cycle c's states
    void use_cycle(int c) {
        for (int k = 0; k < kMaxLevels; k++)
            for (int h = 0; h < 33; h++) tape[k][h] = sets[((size_t)c * kMaxLevels + k) * 33 + h];
    }
    ~UnWork() {
        for (void* p : bufs) (void)hipFree(p);
    }
};

// Whether the unrolled adjoint keeps the recorded states of every cycle
// (bytes: their size).  DMGS_UNROLLED_STORE = 0 checkpoints the finest
// iterate per cycle and records each cycle again in the reverse pass, 1
// keeps every cycle's states; unset, they are kept when they take at most a
// quarter of the device's memory.
bool unrolled_store_all(size_t bytes, bool* forced) {
    *forced = false;
    if (const char* e = std::getenv("DMGS_UNROLLED_STORE")) {
        *forced = true;
        return std::atoi(e) != 0;
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
    return bytes <= tot / 4;
}

unsigned un_grid(int64_t nv) { return (unsigned)((nv + kBlock - 1) / kBlock); }

// Every work buffer a launch or copy of the unrolled pass touches is checked
// on the host against the buffers allocated for it (and the count of values
// the launch or copy covers) before it is enqueued.
#define UNCHK(W, ptr, count, what)                                                                       \
    do {                                                                                                 \
        if (!(W).holds((ptr), (count))) {                                                                \
            set_error("unrolled pass: %s (level %d) is not an allocated work buffer of %lld values", what, k, \
                      (long long)(count));                                                              \
            return DMGS_ERR_INVALID;                                                                     \
        }                                                                                                \
    } while (0)

// The state the defect of level k reads in a recorded cycle: the last
// pre-smoothing half-sweep's slot, or (without pre-smoothing) the slot the
// cycle's input is copied to.
const double* pre_state(dmgs_plan P, UnWork& W, int k) {
    const int nu1 = P->opt.nu_pre, nu2 = P->opt.nu_post;
    return nu1 > 0 ? W.tape[k][2 * nu1 - 1] : W.tape[k][2 * (nu1 + nu2)];
}

// One V-cycle of the fixed-cycle solver with the per-operator kernels,
// recording the states the reverse pass needs: each half-sweep writes its
// result out of place into its tape slot and the next one reads it there.
// u is the cycle's input (overwritten on levels below the finest: it holds
// the input of the post-smoothing); *fin receives the cycle's result.
int vcycle_taped(dmgs_plan P, UnWork& W, int k, double* u, const double* q, const double** fin, hipStream_t st) {
    const Level& l = P->lev[k];
    const int nu1 = P->opt.nu_pre, nu2 = P->opt.nu_post;
    const size_t bytes = l.nv * sizeof(double);
    const Stencil<double> s = l.stencil<double>(harmonic(P));
    UNCHK(W, u, l.nv, "the cycle's iterate");
    if (k > 0) UNCHK(W, q, l.nv, "the coarse right-hand side");
    if (k == P->L - 1) {
        UNCHK(W, W.tape[k][0], l.nv, "the coarsest tape slot");
        hipLaunchKernelGGL(k_exact_solve<double>, dim3(1), dim3(64), 0, st, q, u, (const double*)l.D64,
                           (const double*)l.mu64, l.N, s);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(W.tape[k][0], u, bytes, hipMemcpyDeviceToDevice, st));
        *fin = u;
        return DMGS_OK;
    }
    int chunk = 1, cover = 0;
    const dim3 g = der_grid(P, l.N, &chunk, &cover);
    const bool tiled = l.N >= kUnTileMin;   // smaller levels: the x-march forms
    int uchunk = 1;
    const dim3 ug = un_col_grid(l.N, &uchunk);
    // one recorded half-sweep on an x-march level
    auto half = [&](const double* in, int h, int colour) -> int {
        UNCHK(W, in, l.nv, "a half-sweep input");
        UNCHK(W, W.tape[k][h], l.nv, "a tape slot");
        hipLaunchKernelGGL(k_un_gs_half, ug, dim3(kBlock), 0, st, in, W.tape[k][h], q, (const double*)l.D64,
                           (const double*)l.mu64, l.N, s, colour, uchunk);
        LAUNCHCHK();
        return DMGS_OK;
    };
    // a whole sweep (first colour, then second): on tiled levels one pass
    // writing both tape slots
    auto sweep = [&](const double* in, int h) -> int {
        if (!tiled) {
            TRY(half(in, h, 0));
            return half(W.tape[k][h], h + 1, 1);
        }
        UNCHK(W, in, l.nv, "a sweep input");
        UNCHK(W, W.tape[k][h], l.nv, "a tape slot");
        UNCHK(W, W.tape[k][h + 1], l.nv, "a tape slot");
        auto launch = [&](auto harm) {
            hipLaunchKernelGGL(k_un_gs_sweep_t<decltype(harm)::value>, g, dim3(kDerThreads), 0, st, in, W.tape[k][h],
                               W.tape[k][h + 1], q, (const double*)l.D64, (const double*)l.w64, l.N, s, 0, chunk,
                               cover);
        };
        if (s.harmonic) launch(std::true_type());
        else launch(std::false_type());
        LAUNCHCHK();
        return DMGS_OK;
    };
    const double* src = u;
    int h = 0;
    for (int i = 0; i < nu1; i++, h += 2) {
        TRY(sweep(src, h));
        src = W.tape[k][h + 1];
    }
    if (nu1 == 0) {
        // u itself becomes the post-smoothing input below: keep the state
        UNCHK(W, W.tape[k][2 * (nu1 + nu2)], l.nv, "the input's tape slot");
        HIPCHK(hipMemcpyAsync(W.tape[k][2 * (nu1 + nu2)], u, bytes, hipMemcpyDeviceToDevice, st));
        src = W.tape[k][2 * (nu1 + nu2)];
    }
    const Level& c = P->lev[k + 1];
    UNCHK(W, W.qc[k + 1], c.nv, "the coarse right-hand side");
    UNCHK(W, W.uc[k + 1], c.nv, "the coarse iterate");
    // qc = R (q - A u) in one streaming pass, the defect at every fine vertex
    // (coarse boundary entries are not written; no step reads them)
    TRY(defect_restrict<double>(P, k, src, q, W.qc[k + 1], st));
    TRY(fill<double>(W.uc[k + 1], c.nv, 0.0, st));
    const double* ec = nullptr;
    TRY(vcycle_taped(P, W, k + 1, W.uc[k + 1], W.qc[k + 1], &ec, st));
    // the post-smoothing input: the pre-smoothed state plus the correction,
    // out of place
    hipLaunchKernelGGL(k_un_prolong_to, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, ec, src, u, l.N);
    LAUNCHCHK();
    src = u;
    for (int i = 0; i < nu2; i++, h += 2) {
        TRY(sweep(src, h));
        src = W.tape[k][h + 1];
    }
    *fin = src;
    return DMGS_OK;
}

// Reverse of the recorded cycle on level k: W.ubar[k] holds the cotangent of
// the level's iterate after the cycle and is left holding the one before it;
// qbar, Dbar and mubar of the level accumulate.
int vcycle_rev(dmgs_plan P, UnWork& W, int k, hipStream_t st) {
    const Level& l = P->lev[k];
    const Stencil<double> s = l.stencil<double>(harmonic(P));
    const int nu1 = P->opt.nu_pre, nu2 = P->opt.nu_post;
    int chunk = 1, cover = 0;
    const dim3 g = der_grid(P, l.N, &chunk, &cover);
    const bool tiled = l.N >= kUnTileMin;   // smaller levels: the x-march forms
    int uchunk = 1;
    const dim3 ug = un_col_grid(l.N, &uchunk);
    const double *D = l.D64, *mu = l.mu64;
    // the defect's (or the coarsest solve's) reverse
    auto defect_rev = [&](double* ubar, const double* rb, double scale, const double* u) {
        if (!tiled) {
            hipLaunchKernelGGL(k_un_defect, ug, dim3(kBlock), 0, st, ubar, rb, scale, u, D, mu, l.N, s, W.qbar[k],
                               W.Dbar[k], W.mbar[k], uchunk);
            return;
        }
        auto launch = [&](auto harm) {
            hipLaunchKernelGGL(k_un_defect_t<decltype(harm)::value>, g, dim3(kDerThreads), 0, st, ubar, rb, scale, u,
                               D, mu, l.N, s, W.qbar[k], W.Dbar[k], W.mbar[k], chunk, cover);
        };
        if (s.harmonic) launch(std::true_type());
        else launch(std::false_type());
    };
    UNCHK(W, W.ubar[k], l.nv, "ubar");
    UNCHK(W, W.qbar[k], l.nv, "qbar");
    UNCHK(W, W.Dbar[k], l.nv, "Dbar");
    UNCHK(W, W.mbar[k], l.nv, "mubar");
    UNCHK(W, W.V[k], l.nv, "V");
    if (k == P->L - 1) {
        UNCHK(W, W.tape[k][0], l.nv, "the coarsest tape slot");
        // lam = A^-1 ubar (zero boundary), then the solve's coefficient terms
        TRY(fill<double>(W.V[k], l.nv, 0.0, st));
        hipLaunchKernelGGL(k_exact_solve<double>, dim3(1), dim3(64), 0, st, (const double*)W.ubar[k], W.V[k], D, mu, l.N, s);
        LAUNCHCHK();
        defect_rev(nullptr, (const double*)W.V[k], 1.0, (const double*)W.tape[k][0]);
        LAUNCHCHK();
        return DMGS_OK;
    }
    // x-march levels: V = ubar / d into W.V[k], then the gather updates ubar
    // in place
    auto half_rev = [&](const double* state, int colour) -> int {
        UNCHK(W, state, l.nv, "a recorded state");
        hipLaunchKernelGGL(k_un_half_v, ug, dim3(kBlock), 0, st, (const double*)W.ubar[k], state, D, mu, l.N, s,
                           colour, W.V[k], W.qbar[k], W.mbar[k], uchunk);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_un_half_gather, ug, dim3(kBlock), 0, st, W.ubar[k], (const double*)W.V[k], state, D,
                           l.N, s, colour, W.Dbar[k], uchunk);
        LAUNCHCHK();
        return DMGS_OK;
    };
    // a whole sweep's reverse (its second colour first): on tiled levels one
    // pass, ubar ping-ponging once
    auto sweep_rev = [&](const double* sa, const double* sb) -> int {
        if (!tiled) {
            TRY(half_rev(sa, 1));
            return half_rev(sb, 0);
        }
        UNCHK(W, sa, l.nv, "a recorded state");
        UNCHK(W, sb, l.nv, "a recorded state");
        auto launch = [&](auto harm) {
            hipLaunchKernelGGL(k_un_sweep_rev_t<decltype(harm)::value>, g, dim3(kDerThreads), 0, st,
                               (const double*)W.ubar[k], W.V[k], sa, sb, D, (const double*)l.w64, l.N, s, 1,
                               W.qbar[k], W.mbar[k], W.Dbar[k], chunk, cover);
        };
        if (s.harmonic) launch(std::true_type());
        else launch(std::false_type());
        LAUNCHCHK();
        std::swap(W.ubar[k], W.V[k]);
        return DMGS_OK;
    };
    for (int h = 2 * nu2 - 1; h >= 1; h -= 2) TRY(sweep_rev(W.tape[k][2 * nu1 + h], W.tape[k][2 * nu1 + h - 1]));
    // prolongation u += I ec: ecbar = I^T ubar = 8 R ubar
    const Level& c = P->lev[k + 1];
    UNCHK(W, W.ubar[k + 1], c.nv, "the coarse ubar");
    UNCHK(W, W.qbar[k + 1], c.nv, "the coarse qbar");
    UNCHK(W, W.r[k], l.nv, "rbar");
    UNCHK(W, pre_state(P, W, k), l.nv, "the defect's recorded state");
    hipLaunchKernelGGL(k_un_restrict8, dim3(grid_for(c.nv)), dim3(kBlock), 0, st, (const double*)W.ubar[k],
                       W.ubar[k + 1], l.N);
    LAUNCHCHK();
    TRY(fill<double>(W.qbar[k + 1], c.nv, 0.0, st));
    TRY(vcycle_rev(P, W, k + 1, st));
    // restriction qc = R r: rbar = R^T qcbar = I qcbar / 8; then the defect
    hipLaunchKernelGGL(k_un_prolong_to, dim3(grid_for(l.nv)), dim3(kBlock), 0, st, (const double*)W.qbar[k + 1],
                       (const double*)nullptr, W.r[k], l.N);
    LAUNCHCHK();
    defect_rev(W.ubar[k], (const double*)W.r[k], 0.125, pre_state(P, W, k));
    LAUNCHCHK();
    for (int h = 2 * nu1 - 1; h >= 1; h -= 2) TRY(sweep_rev(W.tape[k][h], W.tape[k][h - 1]));
    return DMGS_OK;
}
}  // namespace

extern "C" {

int dmgs_vjp_unrolled(dmgs_plan P, const double* q, const double* rhobar, double* rho, double* qbar, double* logD_bar,
                      double* logmua_bar, dmgs_info* info, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!q || !rhobar || !rho || !qbar) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    const dmgs_options& o = P->opt;
    if (is2d(P) || P->grid || o.precision != DMGS_FP64 || o.smoother != DMGS_RBGS || o.fixed_cycles <= 0) {
        set_error("dmgs_vjp_unrolled takes three-dimensional DMGS_FP64, DMGS_RBGS plans with fixed_cycles > 0");
        return DMGS_ERR_INVALID;
    }
    const int n = o.fixed_cycles, L = P->L, nstate = 2 * (o.nu_pre + o.nu_post) + 1;
    const Level& l0 = P->lev[0];
    if (!P->unwork) {
        // first call: allocate the work buffers; the plan keeps them
        UnWork* w = new (std::nothrow) UnWork();
        if (!w) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
        // the tapes of one cycle: one buffer, slots starting on 512-byte boundaries
        auto up = [](int64_t v) { return (v + 63) / 64 * 64; };
        int64_t per = 0;
        for (int k = 0; k < L; k++) per += (int64_t)(k == L - 1 ? 1 : nstate) * up(P->lev[k].nv);
        bool forced = false;
        const bool all = n > 1 && unrolled_store_all((size_t)n * per * sizeof(double), &forced);
        auto build = [&](UnWork& W, bool keep_all) -> int {
            W.store_all = keep_all;
            if (!keep_all) TRY(W.alloc(&W.ckpt, (int64_t)n * l0.nv));
            TRY(W.alloc(&W.u0, l0.nv));
            for (int k = 0; k < L; k++) {
                const int64_t nv = P->lev[k].nv;
                if (k < L - 1) TRY(W.alloc(&W.r[k], nv));
                if (k > 0) {
                    TRY(W.alloc(&W.uc[k], nv));
                    TRY(W.alloc(&W.qc[k], nv));
                }
                TRY(W.alloc(&W.ubar[k], nv));
                TRY(W.alloc(&W.qbar[k], nv));
                TRY(W.alloc(&W.Dbar[k], nv));
                TRY(W.alloc(&W.mbar[k], nv));
                TRY(W.alloc(&W.V[k], nv));
            }
            const int nsets = keep_all ? n : 1;
            W.sets.assign((size_t)nsets * kMaxLevels * 33, nullptr);
            for (int c = 0; c < nsets; c++) {
                double* b = nullptr;
                TRY(W.alloc(&b, per));
                int64_t off = 0;
                for (int k = 0; k < L; k++) {
                    const int ns = k == L - 1 ? 1 : nstate;
                    for (int h = 0; h < ns; h++, off += up(P->lev[k].nv))
                        W.sets[((size_t)c * kMaxLevels + k) * 33 + h] = b + off;
                }
            }
            W.use_cycle(0);
            return DMGS_OK;
        };
        int sb = build(*w, all);
        if (sb == DMGS_ERR_OOM && all && !forced) {
            // keeping every cycle did not fit after all: checkpoint instead
            delete w;
            w = new (std::nothrow) UnWork();
            if (!w) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
            sb = build(*w, false);
        }
        if (sb != DMGS_OK) {
            delete w;
            return sb;
        }
        P->unwork = w;
        P->unwork_free = [](void* p) { delete static_cast<UnWork*>(p); };
        P->bytes += w->bytes;
    }
    UnWork& W = *static_cast<UnWork*>(P->unwork);
    {
        const int k = 0;
        if (!W.store_all) UNCHK(W, W.ckpt, (int64_t)n * l0.nv, "the checkpoints");
        UNCHK(W, W.u0, l0.nv, "the working iterate");
    }
    for (int k = 0; k < L; k++) {
        const int64_t nv = P->lev[k].nv;
        TRY(fill<double>(W.Dbar[k], nv, 0.0, st));
        TRY(fill<double>(W.mbar[k], nv, 0.0, st));
        TRY(fill<double>(W.qbar[k], nv, 0.0, st));
        TRY(fill<double>(W.ubar[k], nv, 0.0, st));
        TRY(fill<double>(W.V[k], nv, 0.0, st));   // the partner of ubar in the reverse half-sweeps
    }
    const size_t b0 = l0.nv * sizeof(double);
    if (W.store_all) {
        // forward: n recorded cycles, each into its own tapes
        hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, W.u0, l0.N, o.bc_value);
        LAUNCHCHK();
        for (int c = 0; c < n; c++) {
            W.use_cycle(c);
            const double* fin = nullptr;
            TRY(vcycle_taped(P, W, 0, W.u0, q, &fin, st));
            double* next = c + 1 < n ? W.u0 : rho;   // without post-smoothing fin is W.u0 itself
            if (fin != next) HIPCHK(hipMemcpyAsync(next, fin, b0, hipMemcpyDeviceToDevice, st));
        }
    } else {
        // forward: n cycles of the solver's own (fused) V-cycle, keeping the
        // iterate at the start of each; the reverse pass records each cycle
        // again with its own kernels, whose states agree to rounding
        double* cur = rho;
        double* oth = l0.t64;
        P->bc_zero = o.bc_value == 0.0;
        hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, cur, l0.N, o.bc_value);
        LAUNCHCHK();
        TRY(set_boundary<double>(oth, l0.N, o.bc_value, st));
        for (int c = 0; c < n; c++) {
            HIPCHK(hipMemcpyAsync(W.ckpt + (int64_t)c * l0.nv, cur, b0, hipMemcpyDeviceToDevice, st));
            TRY(vcycle<double>(P, 0, &cur, &oth, q, 0, false, st));
        }
        if (cur != rho) HIPCHK(hipMemcpyAsync(rho, cur, b0, hipMemcpyDeviceToDevice, st));
    }
    // reverse: the cotangent of the last iterate is rhobar (interior)
    HIPCHK(hipMemcpyAsync(W.ubar[0], rhobar, b0, hipMemcpyDeviceToDevice, st));
    TRY(set_boundary<double>(W.ubar[0], l0.N, 0.0, st));
    for (int c = n - 1; c >= 0; c--) {
        if (W.store_all) {
            W.use_cycle(c);
        } else {
            HIPCHK(hipMemcpyAsync(W.u0, W.ckpt + (int64_t)c * l0.nv, b0, hipMemcpyDeviceToDevice, st));
            const double* fin = nullptr;
            TRY(vcycle_taped(P, W, 0, W.u0, q, &fin, st));
        }
        TRY(vcycle_rev(P, W, 0, st));
    }
    // coarse coefficient cotangents to the finest level
    for (int k = L - 1; k >= 1; k--) {
        const Level& f = P->lev[k - 1];
        hipLaunchKernelGGL(k_un_coarsen_T, dim3(un_grid(f.nv)), dim3(kBlock), 0, st, (const double*)W.Dbar[k], W.Dbar[k - 1], f.N);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_un_coarsen_T, dim3(un_grid(f.nv)), dim3(kBlock), 0, st, (const double*)W.mbar[k], W.mbar[k - 1], f.N);
        LAUNCHCHK();
    }
    HIPCHK(hipMemcpyAsync(qbar, W.qbar[0], b0, hipMemcpyDeviceToDevice, st));
    if (logD_bar) {
        hipLaunchKernelGGL(k_un_mul, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, (const double*)W.Dbar[0],
                           (const double*)l0.D64, logD_bar, l0.nv);
        LAUNCHCHK();
    }
    if (logmua_bar) {
        hipLaunchKernelGGL(k_un_mul, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, (const double*)W.mbar[0],
                           (const double*)l0.mu64, logmua_bar, l0.nv);
        LAUNCHCHK();
    }
    // the call returns with its work done (the plan's work buffers are then
    // free for the next call, on any stream)
    HIPCHK(hipStreamSynchronize(st));
    if (info) {
        info->cycles = n;
        info->vcycles = n;
        info->rel_residual = 0.0;
    }
    return end_call(P, DMGS_OK, info, st);
}

int dmgs_noise_weights(dmgs_plan P, const double* Le, int32_t mask, double rel, double floor_frac, double* w,
                       void* stream) {
    if (!P || !Le || !w) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    if (mask < 1 || !(rel >= 0.0) || !(floor_frac >= 0.0) || !std::isfinite(rel) || !std::isfinite(floor_frac)) {
        set_error("bad noise-model parameters (mask %d, rel %g, floor %g)", mask, rel, floor_frac);
        return DMGS_ERR_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(P->device));
    const Level& l0 = P->lev[0];
    const unsigned nb = grid_for(l0.nv, kMaxPartials);
    hipLaunchKernelGGL(k_max_partials, dim3(nb), dim3(kBlock), 0, st, Le, l0.nv, P->partial);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_noise_weights, dim3(grid_for(l0.nv, 4096)), dim3(kBlock), 0, st, Le, (const double*)P->partial,
                       (int)nb, l0.nv, vdims(P), (int)mask, rel, floor_frac, w);
    LAUNCHCHK();
    return DMGS_OK;
}

int dmgs_likelihood_grad(dmgs_plan P, const double* q, const double* d, const double* w, double* rho, double* qbar,
                         double* logD_bar, double* logmua_bar, double* value, dmgs_info* info_fwd, dmgs_info* info_vjp,
                         void* stream) {
    hipStream_t st = (hipStream_t)stream;
    TRY(begin_call(P, st));
    if (!q || !d || !w || !rho || !qbar || !value) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    const Level& l0 = P->lev[0];
    // the epilogue (residual, sums of H and of the kept voxels, and the
    // pull-back's cotangent into the finest-level scratch) is fused into the
    // forward solve's last refinement step where the plan refines; the
    // cotangent's boundary is 0
    const bool fuse = !is2d(P) && P->cfg_epi_fuse;
    if (fuse) {
        if (!P->grid) TRY(set_boundary<double>(P->scratch64, l0.N, 0.0, st));
        P->epi_d = d;
        P->epi_w = w;
        P->epi_rhobar = P->scratch64;
    }
    P->epi_fused = false;
    int sf = solve(P, q, rho, P->opt.bc_value, 0, info_fwd, st, nullptr, true);
    P->epi_d = P->epi_w = nullptr;
    P->epi_rhobar = nullptr;
    if (sf != DMGS_OK && sf != DMGS_ERR_NOT_CONVERGED) return end_call(P, sf, info_fwd, st);
    if (!(fuse && P->epi_fused)) {
        const unsigned nb = grid_for(l0.nv, kMaxPartials / 2);
        TIMED(P, 0, DMGS_K_GRAD, 40.0 * l0.nv, st,
              hipLaunchKernelGGL(k_likelihood_epilogue, dim3(nb), dim3(kBlock), 0, st, (const double*)rho,
                                 (const double*)l0.mu64, d, w, l0.nv, vdims(P), P->scratch64, P->partial));
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial, (int)nb, norm_dst(P), 2);
        LAUNCHCHK();
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, (const double*)P->partial + nb, (int)nb,
                           norm_dst(P), 3);
        LAUNCHCHK();
    }
    const std::vector<int>* replay = (P->opt.adjoint_schedule && P->opt.fixed_cycles <= 0) ? &P->fwd_schedule : nullptr;
    const int sa = solve(P, P->scratch64, qbar, 0.0, 1, info_vjp, st, replay);
    const bool ok_a = sa == DMGS_OK || sa == DMGS_ERR_NOT_CONVERGED;
    if (ok_a && (logD_bar || logmua_bar)) TRY(coef_grads(P, rho, qbar, logD_bar, logmua_bar, d, w, st));
    TRY(mark_norms(P, st));
    TRY(read_norms(P, st));
    const double H = 0.5 * P->hnorm[2], nvox = P->hnorm[3];
    value[0] = H;
    value[1] = nvox > 0.0 ? 2.0 * H / nvox : 0.0;
    value[2] = nvox;
    int s = sf != DMGS_OK ? sf : sa;
    s = end_call(P, s, info_fwd, st);
    if (info_vjp) info_vjp->status = sa;
    return s;
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

}  // extern "C"

// Static scratch of dmgs_solve_once_noalloc: every device the library runs
// on holds one copy until the process ends.  In host code the name stands
// for a host-side object; the device address of each device's copy comes
// from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) unsigned char scratch[DMGS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kNoallocDevices = 16;
struct NoallocSlot {
    std::mutex lock;                // serialises the calls on this device
    unsigned char* ptr = nullptr;   // this device's address of `scratch`
    dmgs_plan_s plan;               // host side of the arena plan, reset by each call
};
NoallocSlot g_noalloc[kNoallocDevices];
}  // namespace

extern "C" {

int dmgs_solve_once_noalloc(const dmgs_options* o, const double* D, const double* mua, const double* q, double* rho,
                            dmgs_info* info, void* stream) {
    TRY(check_options(o));
    if (!D || !mua || !q || !rho) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    const size_t need = footprint(o) + kArenaSlack;
    if (need > (size_t)DMGS_NOALLOC_SCRATCH_BYTES) {
        set_error("dmgs_solve_once_noalloc: the plan needs %zu bytes (workspace %zu plus alignment), more than the "
                  "%zu bytes of the static scratch", need, footprint(o), (size_t)DMGS_NOALLOC_SCRATCH_BYTES);
        return DMGS_ERR_INVALID;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocDevices) {
        set_error("dmgs_solve_once_noalloc: device %d beyond the %d the library keeps scratch addresses for", dev,
                  kNoallocDevices);
        return DMGS_ERR_INVALID;
    }
    NoallocSlot& S = g_noalloc[dev];
    std::lock_guard<std::mutex> guard(S.lock);
    if (!S.ptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError(); set_error("hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
            return DMGS_ERR_HIP;
        }
        S.ptr = static_cast<unsigned char*>(p);
    }
    hipStream_t st = (hipStream_t)stream;
    dmgs_plan P = &S.plan;
    *P = dmgs_plan_s();
    P->arena = S.ptr;
    P->arena_cap = (size_t)DMGS_NOALLOC_SCRATCH_BYTES;
    TRY(plan_init(P, o, st));
    int s = dmgs_set_coefficients(P, D, mua, stream);
    if (s == DMGS_OK) s = dmgs_forward(P, q, rho, info, stream);
    // the call returns with its work done: the next call may reuse the array
    if (hipStreamSynchronize(st) != hipSuccess && s == DMGS_OK) s = DMGS_ERR_HIP;
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
    P->tstride = enable > 1 ? enable : 1;
    for (int c = 0; c < DMGS_K_COUNT; c++) {
        P->t_count[c] = 0;
        P->t_seen[c] = 0;
        P->t_ms[c] = 0.0;
        P->t_bytes[c] = 0.0;
    }
    return DMGS_OK;
}

int dmgs_trace_read(dmgs_plan P, int32_t order, int32_t cap, int32_t* steps, int32_t* vcycles, double* rel,
                    int32_t* count) {
    if (!P || !count || (order != 0 && order != 1) || cap < 0 || (cap > 0 && (!steps || !vcycles || !rel))) {
        set_error("bad plan, order or buffers");
        return DMGS_ERR_INVALID;
    }
    if (!P->cfg_trace) {
        set_error("tracing is off (set DMGS_TRACE=1 before creating the plan)");
        return DMGS_ERR_INVALID;
    }
    const auto& tr = P->trace[order];
    *count = (int32_t)tr.size();
    for (int32_t i = 0; i < cap && i < (int32_t)tr.size(); i++) {
        steps[i] = tr[i].steps;
        vcycles[i] = tr[i].vcycles;
        rel[i] = tr[i].rel;
    }
    return DMGS_OK;
}

int dmgs_timing_read(dmgs_plan P, int cls, int64_t* launches, double* total_ms, double* bytes) {
    if (!P || cls < 0 || cls >= DMGS_K_COUNT) { set_error("bad plan or kernel class"); return DMGS_ERR_INVALID; }
    if (P->tpending) TRY(timing_flush(P));
    // sampled classes: totals scaled from the timed launches to all of them
    const double scale = P->t_count[cls] ? (double)P->t_seen[cls] / (double)P->t_count[cls] : 0.0;
    if (launches) *launches = P->t_seen[cls];
    if (total_ms) *total_ms = P->t_ms[cls] * scale;
    if (bytes) *bytes = P->t_bytes[cls] * scale;
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
    if (!q || !u_out || !qc) { set_error("q, u_out and qc are required"); return DMGS_ERR_INVALID; }
    hipStream_t st = (hipStream_t)stream;
    if (fp32) return debug_pre_t<float>(P, k, order, (const float*)u_in, (const float*)q, (float*)u_out, (float*)qc, st);
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

int dmgs_debug_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || bytes % 16) { set_error("stream copy needs 16-byte multiples"); return DMGS_ERR_INVALID; }
    hipLaunchKernelGGL(k_stream_copy, dim3(4096), dim3(256), 0, (hipStream_t)stream, (const float4*)src, (float4*)dst,
                       (int64_t)(bytes / 16));
    HIPCHK(hipGetLastError());
    return DMGS_OK;
}

int dmgs_debug_cycles(dmgs_plan P, int order, int ncycles, const double* q, double* u, void* stream) {
    TRY(debug_check(P, 0, 0, false));
    if (is_ir(P)) { set_error("dmgs_debug_cycles needs a DMGS_FP64 plan"); return DMGS_ERR_INVALID; }
    hipStream_t st = (hipStream_t)stream;
    const Level& l0 = P->lev[0];
    HIPCHK(hipMemcpyAsync(l0.t64, u, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    double* cur = u;
    double* oth = l0.t64;
    for (int c = 0; c < ncycles; c++) TRY(vcycle<double>(P, 0, &cur, &oth, q, order, false, st));
    if (cur != u) HIPCHK(hipMemcpyAsync(u, cur, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    return DMGS_OK;
}

}  // extern "C"

#include "batch.hpp"
