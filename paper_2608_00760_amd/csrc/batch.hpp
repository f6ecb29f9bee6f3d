// batch.hpp -- grouped execution of many requests' solves (continuous
// batching of forward + push-forward and forward + pull-back requests).
//
// Included at the end of dmgs.hip: it drives the same host code as the
// single-request entry points (ir_step, vcycle<float>, tangent_rhs,
// coef_grads), so a request computes exactly what dmgs_forward followed by
// dmgs_jvp or dmgs_vjp computes on its plan.
//
// A tick advances every active request by one refinement step.  Its
// float64 residual norms from the previous tick decide, as in the single
// solve, whether the solve stops and how many float32 V-cycles the next
// step takes.  The plan then records the step's launches instead of
// issuing them.  Work a request needs at a stage change runs at once: the
// iterate's set-up, the push-forward's right-hand side, copies of results,
// the coefficient gradients.
//
// The recorded launches of all requests are merged greedily.  Each round
// takes the grouped kernel that the most requests launch next and runs it
// once for all of them, each request keeping its own launch order.  The
// group tables go to the device in one copy, and the tick ends with one
// synchronisation, after which every request's norms are in its plan's
// pinned host slots.  Requests whose last solve finished are reported at
// the end of the tick in which their final work ran.

namespace {

struct BatchSolve {
    const double* b = nullptr;   // right-hand side
    double* x = nullptr;         // result (caller's array)
    double bc = 0.0;
    int order = 0;
    double* xc = nullptr;        // current iterate (x or the plan's alternate)
    double* xo = nullptr;
    bool x_zero = false;
    int cycles = 0, vcycles = 0, inner = 0;
    double r0 = 0.0, rel = 0.0, rel1 = 1.0, rate = 0.0;
};

struct BatchReq {
    dmgs_plan P = nullptr;
    int mode = 0;
    int64_t tag = 0;
    const double *q = nullptr, *in0 = nullptr, *in1 = nullptr, *in2 = nullptr;
    double *rho = nullptr, *out0 = nullptr, *out1 = nullptr, *out2 = nullptr;
    int stage = 0;       // 0: forward solve, 1: second solve, 2: finished (to be reported)
    bool begun = false;  // the current stage's solve has been set up
    BatchSolve s;
    dmgs_info info[2] = {};
    int status = DMGS_OK;
    std::vector<RecOp> ops;   // this tick's recorded launches
    size_t next = 0;          // first of them not yet grouped
};

// While alive, the plan records its launches into ops.
struct Recording {
    dmgs_plan P;
    Recording(dmgs_plan p, std::vector<RecOp>* ops) : P(p) { P->rec = ops; }
    ~Recording() { P->rec = nullptr; }
};

// A plan takes part in grouped execution when every launch of its
// refinement step has a grouped form: a float32-in-float64 cubic 3D plan
// with V(2,2) red-black cycles whose levels above the single-workgroup
// coarse kernel run two-sweep passes or block passes.
int batch_eligible(dmgs_plan P) {
    if (!P || !P->coef_set) { set_error("dmgs_batch_add: plan without coefficients"); return DMGS_ERR_INVALID; }
    const dmgs_options& o = P->opt;
    if (!is_ir(P) || P->grid || is2d(P) || o.smoother != DMGS_RBGS || o.nu_pre != 2 || o.nu_post != 2 ||
        o.adjoint_schedule != 0 || P->small32 < 1) {
        set_error("dmgs_batch_add: grouped execution takes cubic 3D DMGS_FP32_IN_FP64 plans with V(2,2) red-black "
                  "cycles, adjoint_schedule 0 and a coarse end of at most 16 cells per axis");
        return DMGS_ERR_INVALID;
    }
    for (int k = 0; k < P->small32; k++)
        if (!block_level<float>(P, k) && !(fused_level(P, k) && use_sweep2(P, k, sizeof(float)))) {
            set_error("dmgs_batch_add: level %d (N = %d) runs passes without a grouped form", k, P->lev[k].N);
            return DMGS_ERR_INVALID;
        }
    return DMGS_OK;
}

// Set up solve s of request r: the iterate's boundary (launched now) and the
// initial residual (recorded), as the single solve does.
int batch_begin(BatchReq& r, const double* b, double* x, double bc, int order, hipStream_t st) {
    dmgs_plan P = r.P;
    const Level& l0 = P->lev[0];
    BatchSolve& s = r.s;
    s = BatchSolve();
    s.b = b;
    s.x = x;
    s.bc = bc;
    s.order = order;
    P->trace[order].clear();
    P->bc_zero = bc == 0.0;
    s.x_zero = bc == 0.0;
    if (s.x_zero) {
        TRY(set_boundary<double>(x, l0.N, 0.0, st));
    } else {
        hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, x, l0.N, bc);
        LAUNCHCHK();
    }
    s.xc = x;
    s.xo = P->xalt64;
    TRY(set_boundary<double>(s.xo, l0.N, bc, st));
    r.begun = true;
    Recording rec(P, &r.ops);
    return ir_step(P, s.xc, nullptr, nullptr, b, l0.q32, 0, st, s.x_zero);
}

// After the tick that ran the solve's last recorded work: the stopping
// decision of the single solve on the norms now in the plan's host slots.
// Not finished: the next refinement step is recorded.
int batch_advance(BatchReq& r, hipStream_t st, bool* finished, int* status) {
    dmgs_plan P = r.P;
    const dmgs_options& o = P->opt;
    const Level& l0 = P->lev[0];
    BatchSolve& s = r.s;
    *finished = false;
    *status = DMGS_OK;
    auto stop = [&](int code) {
        *finished = true;
        *status = code;
    };
    if (o.fixed_cycles <= 0) {
        if (s.cycles == 0) {
            s.r0 = std::sqrt(P->hnorm[0]);
            if (!std::isfinite(s.r0)) stop(DMGS_ERR_NONFINITE);
            else if (s.r0 == 0.0) stop(DMGS_OK);
            else s.rel = 1.0;
        } else {
            s.rel = std::sqrt(P->hnorm[1]) / s.r0;
            trace_point(P, s.order, s.cycles, s.vcycles, s.rel);
            if (!std::isfinite(s.rel)) stop(DMGS_ERR_NONFINITE);
            else if (s.rel <= o.rtol) stop(DMGS_OK);
            else s.rate = s.rel < s.rel1 ? std::pow(s.rel / s.rel1, 1.0 / s.inner) : 0.0;
        }
        if (!*finished && s.cycles >= o.max_cycles) stop(DMGS_ERR_NOT_CONVERGED);
        if (*finished) return DMGS_OK;
        s.rel1 = s.rel;
        s.inner = o.ir_inner_cycles;
        if (o.ir_adaptive && s.rate > 0.0) {
            const double need = std::ceil(std::log(o.rtol / s.rel) / std::log(s.rate) - 1e-6);
            s.inner = (int)std::min<double>(s.inner, std::max(1.0, need));
        }
    } else {
        if (s.cycles == 0) s.r0 = std::sqrt(P->hnorm[0]);
        else if (P->cfg_trace)
            trace_point(P, s.order, s.cycles, s.vcycles, std::sqrt(P->hnorm[1]) / (s.r0 > 0.0 ? s.r0 : 1.0));
        if (s.cycles == o.fixed_cycles) {
            stop(DMGS_OK);
            return DMGS_OK;
        }
        s.inner = o.ir_inner_cycles;
    }
    float* e = l0.u32;
    float* eo = l0.t32;
    {
        Recording rec(P, &r.ops);
        for (int ic = 0; ic < s.inner; ic++) TRY(vcycle<float>(P, 0, &e, &eo, l0.q32, s.order, ic == 0, st));
        TRY(ir_step(P, s.xc, e, s.xo, s.b, l0.q32, 1, st, s.x_zero && s.cycles == 0));
    }
    std::swap(s.xc, s.xo);
    s.vcycles += s.inner;
    s.cycles++;
    return DMGS_OK;
}

// The solve has stopped with `status`: its result into the caller's array
// (launched now) and its info.
int batch_end_solve(BatchReq& r, int status, dmgs_info* info, hipStream_t st) {
    dmgs_plan P = r.P;
    const Level& l0 = P->lev[0];
    BatchSolve& s = r.s;
    P->ir_steps[s.order] = s.cycles;
    if (s.x_zero && s.cycles == 0) {
        hipLaunchKernelGGL(k_init_iterate<double>, dim3(grid_for(l0.nv)), dim3(kBlock), 0, st, s.x, l0.N, 0.0);
        LAUNCHCHK();
    }
    if (s.xc != s.x) HIPCHK(hipMemcpyAsync(s.x, s.xc, l0.nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    double rel = s.rel;
    if (P->opt.fixed_cycles > 0) {
        const double r0 = std::sqrt(P->hnorm[0]);
        rel = std::sqrt(P->hnorm[P->opt.fixed_cycles > 0 ? 1 : 0]) / (r0 > 0.0 ? r0 : 1.0);
    }
    info->cycles = s.cycles;
    info->vcycles = s.vcycles;
    info->rel_residual = rel;
    info->status = status;
    info->device_ms = 0.0;
    return DMGS_OK;
}

// A stage's solve has stopped: end it, then begin the next stage or finish.
int batch_next_stage(BatchReq& r, int status, hipStream_t st) {
    dmgs_plan P = r.P;
    TRY(batch_end_solve(r, status, &r.info[r.stage], st));
    if (r.stage == 0) {
        if (status != DMGS_OK) {
            r.status = status;
            r.stage = 2;
            return DMGS_OK;
        }
        r.stage = 1;
        if (r.mode == DMGS_BATCH_JVP) {
            TRY(tangent_rhs(P, r.rho, r.in0, r.in1, r.in2, P->scratch64, st));
            return batch_begin(r, P->scratch64, r.out0, 0.0, 0, st);
        }
        return batch_begin(r, r.in0, r.out0, 0.0, 1, st);
    }
    if (r.mode == DMGS_BATCH_VJP && (status == DMGS_OK || status == DMGS_ERR_NOT_CONVERGED) && (r.out1 || r.out2))
        TRY(coef_grads(P, r.rho, r.out0, r.out1, r.out2, nullptr, nullptr, st));
    r.status = status;
    r.stage = 2;
    return DMGS_OK;
}

}  // namespace

struct dmgs_batch_s {
    int device = 0;
    std::vector<BatchReq*> reqs;    // in order of addition
    unsigned char* htab = nullptr;  // group tables: pinned host staging ...
    unsigned char* dtab = nullptr;  // ... and their device copy
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    int64_t ticks = 0, launches = 0, recorded = 0;
};

namespace {

struct BatchGroup {
    const void* fn;
    std::vector<const RecOp*> ops;
    size_t off;
};

// Merge the requests' recorded launches into grouped launches and issue them.
int batch_launch(dmgs_batch B, hipStream_t st) {
    std::vector<BatchReq*> live;
    for (BatchReq* r : B->reqs)
        if (r->next < r->ops.size()) live.push_back(r);
    std::vector<BatchGroup> groups;
    size_t bytes = 0;
    while (true) {
        // the grouped kernel most requests launch next (ties: the first request's)
        const void* best = nullptr;
        int best_n = 0;
        for (BatchReq* r : live) {
            if (r->next >= r->ops.size()) continue;
            const void* f = r->ops[r->next].fn;
            int n = 0;
            for (BatchReq* o : live)
                if (o->next < o->ops.size() && o->ops[o->next].fn == f) n++;
            if (n > best_n) {
                best_n = n;
                best = f;
            }
        }
        if (!best) break;
        BatchGroup g;
        g.fn = best;
        for (BatchReq* r : live)
            if (r->next < r->ops.size() && r->ops[r->next].fn == best && (int)g.ops.size() < kGroupMax)
                g.ops.push_back(&r->ops[r->next++]);
        g.off = bytes;
        bytes += (g.ops[0]->table_bytes + 255) & ~(size_t)255;
        groups.push_back(std::move(g));
    }
    if (groups.empty()) return DMGS_OK;
    if (bytes > B->cap) {
        // the previous tick has synchronised: the old tables are free
        if (B->htab) (void)hipHostFree(B->htab);
        if (B->dtab) (void)hipFree(B->dtab);
        B->htab = B->dtab = nullptr;
        B->cap = 0;
        const size_t cap = std::max<size_t>(bytes, (size_t)1 << 20);
        HIPCHK(hipHostMalloc((void**)&B->htab, cap, hipHostMallocDefault));
        HIPCHK(hipMalloc((void**)&B->dtab, cap));
        B->cap = cap;
    }
    std::vector<int> start;
    std::vector<unsigned> blocks(groups.size());
    std::vector<size_t> lds(groups.size());
    for (size_t i = 0; i < groups.size(); i++) {
        const BatchGroup& g = groups[i];
        const int n = (int)g.ops.size();
        start.assign(n + 1, 0);
        size_t l = 0;
        for (int m = 0; m < n; m++) {
            start[m + 1] = start[m] + (int)((g.ops[m]->nblk + 7) / 8 * 8);
            l = std::max(l, g.ops[m]->lds);
        }
        g.ops[0]->write(B->htab + g.off, g.ops.data(), n, start.data());
        blocks[i] = (unsigned)start[n];
        lds[i] = l;
    }
    HIPCHK(hipMemcpyAsync(B->dtab, B->htab, bytes, hipMemcpyHostToDevice, st));
    for (size_t i = 0; i < groups.size(); i++) {
        void* table = B->dtab + groups[i].off;
        void* kargs[] = {&table};
        HIPCHK(hipLaunchKernel(groups[i].fn, dim3(blocks[i]), dim3(groups[i].ops[0]->threads), kargs, lds[i], st));
        B->recorded += (int64_t)groups[i].ops.size();
    }
    B->launches += (int64_t)groups.size();
    return DMGS_OK;
}

}  // namespace

extern "C" {

int dmgs_batch_create(dmgs_batch* out) {
    if (!out) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    *out = nullptr;
    dmgs_batch B = new (std::nothrow) dmgs_batch_s();
    if (!B) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
    if (hipGetDevice(&B->device) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev, hipEventDisableTiming) != hipSuccess) {
        delete B;
        (void)hipGetLastError(); set_error("hipEventCreate failed");
        return DMGS_ERR_HIP;
    }
    *out = B;
    return DMGS_OK;
}

int dmgs_batch_destroy(dmgs_batch B) {
    if (!B) return DMGS_OK;
    for (BatchReq* r : B->reqs) delete r;
    if (B->htab) (void)hipHostFree(B->htab);
    if (B->dtab) (void)hipFree(B->dtab);
    if (B->ev) (void)hipEventDestroy(B->ev);
    delete B;
    return DMGS_OK;
}

int dmgs_batch_add(dmgs_batch B, dmgs_plan P, int32_t mode, const double* q, const double* in0, const double* in1,
                   const double* in2, double* rho, double* out0, double* out1, double* out2, int64_t tag) {
    if (!B) { set_error("batch is NULL"); return DMGS_ERR_INVALID; }
    TRY(batch_eligible(P));
    if (P->device != B->device) { set_error("dmgs_batch_add: the plan lives on another device"); return DMGS_ERR_INVALID; }
    if (mode != DMGS_BATCH_JVP && mode != DMGS_BATCH_VJP) { set_error("dmgs_batch_add: bad mode %d", mode); return DMGS_ERR_INVALID; }
    if (!q || !rho || !out0 || (mode == DMGS_BATCH_VJP && !in0)) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    for (BatchReq* r : B->reqs)
        if (r->P == P) { set_error("dmgs_batch_add: the plan already serves a request of this batch"); return DMGS_ERR_INVALID; }
    BatchReq* r = new (std::nothrow) BatchReq();
    if (!r) { set_error("host allocation failed"); return DMGS_ERR_OOM; }
    r->P = P;
    r->mode = mode;
    r->tag = tag;
    r->q = q;
    r->in0 = in0;
    r->in1 = in1;
    r->in2 = in2;
    r->rho = rho;
    r->out0 = out0;
    r->out1 = out1;
    r->out2 = out2;
    B->reqs.push_back(r);
    return DMGS_OK;
}

int dmgs_batch_pending(dmgs_batch B) { return B ? (int)B->reqs.size() : 0; }

int dmgs_batch_tick(dmgs_batch B, void* stream, int32_t cap, int64_t* tags, int32_t* status, dmgs_info* info_fwd,
                    dmgs_info* info_second, int32_t* count) {
    if (!B || !count || (cap > 0 && (!tags || !status))) { set_error("NULL argument"); return DMGS_ERR_INVALID; }
    *count = 0;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(B->device));
    // 1. every request: set-up, stopping decision, stage change (work needed
    //    at once is launched now, the refinement step is recorded)
    for (BatchReq* r : B->reqs) {
        r->ops.clear();
        r->next = 0;
        if (r->stage == 2) continue;
        int s = DMGS_OK;
        if (!r->begun) {
            s = batch_begin(*r, r->q, r->rho, r->P->opt.bc_value, 0, st);
        } else {
            bool fin = false;
            int code = DMGS_OK;
            s = batch_advance(*r, st, &fin, &code);
            if (s == DMGS_OK && fin) s = batch_next_stage(*r, code, st);
        }
        if (s != DMGS_OK) {   // the request ends with the error; nothing of it is launched
            r->ops.clear();
            r->status = s;
            r->stage = 2;
        }
    }
    // 2. grouped launches, 3. one synchronisation
    TRY(batch_launch(B, st));
    HIPCHK(hipEventRecord(B->ev, st));
    HIPCHK(hipEventSynchronize(B->ev));
    B->ticks++;
    // 4. finished requests, in order of addition
    std::vector<BatchReq*> keep;
    for (BatchReq* r : B->reqs) {
        if (r->stage == 2 && *count < cap) {
            tags[*count] = r->tag;
            status[*count] = r->status;
            if (info_fwd) info_fwd[*count] = r->info[0];
            if (info_second) info_second[*count] = r->info[1];
            (*count)++;
            delete r;
        } else {
            keep.push_back(r);
        }
    }
    B->reqs.swap(keep);
    return DMGS_OK;
}

int dmgs_batch_stats(dmgs_batch B, int64_t* ticks, int64_t* launches, int64_t* recorded) {
    if (!B) { set_error("batch is NULL"); return DMGS_ERR_INVALID; }
    if (ticks) *ticks = B->ticks;
    if (launches) *launches = B->launches;
    if (recorded) *recorded = B->recorded;
    return DMGS_OK;
}

}  // extern "C"
