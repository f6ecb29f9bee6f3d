// plan.hpp -- the resident level hierarchy of a solver plan.
#pragma once
#include <vector>
#include <hip/hip_runtime.h>

#include "../../include/dmgs.h"
#include "grid.hpp"

namespace dmgs {

constexpr int kMaxLevels = 16;
constexpr int kMaxPartials = 2048;   // blocks of the first reduction stage

struct Level {
    int N = 0, n = 0;
    int64_t nv = 0;
    double h = 1.0, inv_h2 = 1.0;
    int nc[3] = {0, 0, 0};        // cells per axis (general grids; N, N, N on cubic levels)
    double h3[3] = {1.0, 1.0, 1.0};   // spacing per axis
    // coefficient hierarchy (float64 on every level; float32 copies in
    // iterative-refinement plans)
    double *D64 = nullptr, *mu64 = nullptr, *w64 = nullptr;   // w: inverse diagonal
    float *D32 = nullptr, *mu32 = nullptr, *w32 = nullptr;
    // iterate, right-hand side and scratch of the cycle on this level
    double *u64 = nullptr, *q64 = nullptr, *t64 = nullptr;
    float *u32 = nullptr, *q32 = nullptr, *t32 = nullptr;
    float* r32 = nullptr;   // fine defect written by pre-smoothing passes (iterative-refinement plans, not the coarsest)
    double* rd64 = nullptr; // ... two-dimensional plans (not the coarsest)
    // layout of the float32 arrays: vertex (x, y, z) at x px + y py + z, nv32
    // elements allocated.  Dense (py = n, px = n^2) except on the finest
    // level of refinement plans whose passes all take a pitch, where rows
    // are padded (py > n) to spread a tile's rows over the memory channels.
    int py = 0;
    int64_t px = 0, nv32 = 0;

    template <class T> Stencil<T> stencil(int harmonic) const {
        Stencil<T> s;
        s.half_inv_h2 = (T)(0.5 * inv_h2);
        s.two_inv_h2 = (T)(2.0 * inv_h2);
        s.harmonic = harmonic;
        return s;
    }
};

template <class T> struct Typed;
template <> struct Typed<double> {
    static double* D(const Level& l) { return l.D64; }
    static double* mu(const Level& l) { return l.mu64; }
    static double* w(const Level& l) { return l.w64; }
    static double* u(const Level& l) { return l.u64; }
    static double* q(const Level& l) { return l.q64; }
    static double* t(const Level& l) { return l.t64; }
    static double* r(const Level&) { return nullptr; }
    static int py(const Level& l) { return l.n; }
    static int64_t px(const Level& l) { return (int64_t)l.n * l.n; }
};
template <> struct Typed<float> {
    static float* D(const Level& l) { return l.D32; }
    static float* mu(const Level& l) { return l.mu32; }
    static float* w(const Level& l) { return l.w32; }
    static float* u(const Level& l) { return l.u32; }
    static float* q(const Level& l) { return l.q32; }
    static float* t(const Level& l) { return l.t32; }
    static float* r(const Level& l) { return l.r32; }
    static int py(const Level& l) { return l.py; }
    static int64_t px(const Level& l) { return l.px; }
};

// The level's arrays of type T are dense (every kernel takes them).
template <class T> bool dense(const Level& l) { return Typed<T>::py(l) == l.n; }

}  // namespace dmgs

namespace dmgs {
// A launch recorded for grouped execution (a plan records instead of
// launching while it takes part in a batch tick): the grouped kernel, the
// member's block count, block size and dynamic LDS, and its arguments;
// write() lays a group of such launches of one kernel out as that kernel's
// Group table (start[] holds count + 1 block offsets).
struct RecOp {
    const void* fn;
    unsigned nblk, threads;
    size_t lds;
    size_t table_bytes;
    void (*write)(unsigned char* dst, const RecOp* const* ops, int count, const int* start);
    alignas(16) unsigned char args[512];
};

constexpr int kTimerSlots = 512;
struct TimerRec {
    int cls;
    double bytes;
};
}  // namespace dmgs

struct dmgs_plan_s {
    dmgs_options opt;
    int L = 0;
    dmgs::Level lev[dmgs::kMaxLevels];
    double* scratch64 = nullptr;   // finest-level float64 scratch (tangent right-hand side)
    double* xalt64 = nullptr;      // second finest-level float64 iterate (refinement ping-pong)
    // fused-pass configuration
    int cfg_sweep = 0, cfg_fuse_min = 32;
    int cfg_sweep2_min = 64, cfg_sweep2_wgs = 256;   // two-sweep passes: smallest N, target workgroups
    int cfg_sweep2_wgs_coarse = 128;                 // ... on levels below the finest
    int cfg_block_max = 64;                         // block passes: largest N
    int cfg_dr_wgs = 512;                           // defect-restriction passes: target workgroups
    int cfg_defect = 2;   // two-sweep pre-smoothing writes the defect: 0 never, 1 from a zero iterate, 2 always
    int cfg_2d_sweep2_min = 1536;  // two-dimensional plans: smallest N of the two-sweep passes
    bool cfg_sweep2_fp64 = true;   // float64 levels use the two-sweep passes (zero boundaries only)
    int cfg_2d_block_min = 64;     // two-dimensional plans: smallest N of the LDS block passes
    bool cfg_2d_defect = true;     // ... the last pre-smoothing pass writes the defect
    bool cfg_epi_fuse = true;      // the likelihood epilogue rides on the last refinement step
    bool cfg_trace = false;        // DMGS_TRACE: record each solve's residual history
    bool bc_zero = true;           // the current solve's boundary value is 0
    int ncu = 256;                 // compute units of the plan's device
    int cfg_2d_chunk = 0;          // ... rows per chunk (0: chosen from the grid size)
    int small32 = -1, small64 = -1;   // first level of the single-workgroup coarse kernel
    int small2 = -1;                  // ... of two-dimensional plans
    double* partial = nullptr;     // first-stage reduction partials
    double* cinv = nullptr;        // inverse of the coarsest operator (kCoarseMax^2 entries)
    double* hnorm = nullptr;       // pinned host memory the reductions write their norms to (4 slots)
    int* dflag = nullptr;          // device validation flag
    int* hflag = nullptr;          // pinned host mirror
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    hipEvent_t ev_norm = nullptr;  // recorded after the last norm reduction
    hipEvent_t ev_flag = nullptr;  // recorded after the validation flag's copy to the host
    int tmark = 0;                 // timer slots recorded before ev_norm
    int ir_steps[2] = {0, 0};      // refinement steps of the last solve, by cycle order
    std::vector<int> fwd_schedule; // V-cycle schedule of the last tolerance-mode forward solve
    struct TracePoint {
        int32_t steps, vcycles;    // cycles (refinement steps) and V-cycles applied so far
        double rel;                // relative residual of the iterate then
    };
    std::vector<TracePoint> trace[2];   // residual history of the last solve of each cycle order
    // likelihood epilogue requested from the next forward solve (data, weights,
    // cotangent output); epi_fused reports whether its last refinement step
    // computed it for the returned iterate
    const double* epi_d = nullptr;
    const double* epi_w = nullptr;
    double* epi_rhobar = nullptr;
    bool epi_fused = false;
    bool fwd_recorded = false;
    bool coef_set = false;
    // kernel timing (profiling aid)
    bool timing = false;
    hipEvent_t tev[2 * dmgs::kTimerSlots] = {};
    dmgs::TimerRec trec[dmgs::kTimerSlots];
    int tpending = 0;
    int64_t t_count[DMGS_K_COUNT] = {};   // timed launches
    int64_t t_seen[DMGS_K_COUNT] = {};    // all finest-level launches
    int tstride = 1;                      // one launch in tstride of each class is timed
    double t_ms[DMGS_K_COUNT] = {};
    double t_bytes[DMGS_K_COUNT] = {};
    size_t bytes = 0;
    int device = 0;
    bool grid = false;             // general grid: per-axis cell counts and spacings
    // concurrent forward + VJP: a second plan that shares this plan's
    // coefficient hierarchy (not owned) and has its own work buffers, and
    // the stream its solves run on
    bool owns_coef = true;
    dmgs_plan_s* twin = nullptr;
    hipStream_t twin_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // work buffers of the unrolled reverse pass, allocated by its first call
    // and kept for later ones (freed with the plan through unwork_free)
    void* unwork = nullptr;
    void (*unwork_free)(void*) = nullptr;
    // allocation-free plans: every device buffer is carved from an arena of
    // device memory the plan does not own; the norms and the validation flag
    // are read back by copies and stream synchronisation instead of pinned
    // host memory and events
    // grouped execution: while set, the launches of the refinement cycle are
    // appended here instead of being issued
    std::vector<dmgs::RecOp>* rec = nullptr;
    unsigned char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    double* dnorm = nullptr;     // device norm slots the reductions write (arena plans)
    double hnorm_buf[4] = {};    // host copies of the norms (arena plans)
    int hflag_buf = 0;           // host copy of the validation flag (arena plans)
};
