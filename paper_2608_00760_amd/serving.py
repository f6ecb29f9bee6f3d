"""Continuous-batching request loop for forward + JVP / forward + VJP solves.

Requests of different grid sizes arrive over time (as posterior samples of a
variational inference run do).  A dispatcher admits them in arrival order
whenever a slot is free and their device-memory footprint (the plan's
hierarchy and workspace, from dmgs_workspace_bytes, plus the request's
fields) fits in the HBM budget; idle pooled plans are evicted to make room.
Freed blocks that torch's caching allocator keeps count against the budget
too: when they would take the resident total past it, they are released
before the next admission.  Admitted requests run on worker threads, each
driving the native library on its own HIP stream, so the work of requests
that arrived while others were running overlaps on the device.  Hierarchies stay resident: plans are pooled
per grid size and reused.  Per-request arithmetic does not depend on what
else is running (every kernel and reduction is deterministic), so a result
is bitwise the same alone and in the mix.

The admission policy (class Admission) is separate from execution so that
it can be exercised without a GPU.
"""
import collections
import threading
import time
import traceback
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    id: int
    N: int
    mode: str                 # "jvp" | "vjp"
    seed: int
    arrival: float = 0.0      # seconds after the stream starts
    # filled in by the server
    status: str = "pending"   # pending | done | rejected | error
    t_admit: float = None
    t_done: float = None
    cycles: tuple = None
    result: dict = field(default_factory=dict)
    error: str = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


class Admission:
    """FIFO admission by slots and memory footprint.

    footprint(req) -> bytes the request needs while it runs (its plan if none
    is pooled for its size, plus its fields).  idle_plans is the memory held
    by pooled plans not in use; evict(bytes) frees idle plans (oldest first)
    and returns the bytes freed.  A request larger than the whole budget is
    rejected; otherwise it waits at the head of the queue until it fits.
    """

    def __init__(self, budget_bytes, max_slots):
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.in_use = 0          # bytes of running requests (plans in use + fields)
        self.idle = 0            # bytes of pooled idle plans
        self.active = 0
        self.peak = 0
        self.queue = collections.deque()
        self.max_queue = 0

    def resident(self):
        return self.in_use + self.idle

    def offer(self, req):
        self.queue.append(req)
        self.max_queue = max(self.max_queue, len(self.queue))

    def next_admissible(self, need_of, evict):
        """Pop and return (req, need) for the head request if it can start
        now, ('reject', req) if it can never fit, or None."""
        if not self.queue or self.active >= self.max_slots:
            return None
        req = self.queue[0]
        need, reuse = need_of(req)     # reuse: bytes of an idle pooled plan it would take over
        if need > self.budget:
            self.queue.popleft()
            return ("reject", req, need)
        extra = need - reuse
        if self.resident() + extra > self.budget:
            freed = evict(self.resident() + extra - self.budget)
            self.idle -= freed
            need, reuse = need_of(req)   # eviction may have taken the plan it would reuse
            extra = need - reuse
        if self.resident() + extra > self.budget:
            return None
        self.queue.popleft()
        self.idle -= reuse
        self.in_use += need
        self.active += 1
        self.peak = max(self.peak, self.resident())
        return ("run", req, need)

    def finish(self, need, plan_bytes_kept):
        self.in_use -= need
        self.idle += plan_bytes_kept
        self.active -= 1


def request_fields(req, device):
    """The request's own seeded fields, drawn on the device: GRF log D and
    log mua (as the 128^3 workload), a 16-blob source and an N(0,1)
    tangent (dq, dlogD, dlogmua) or cotangent rhobar."""
    import math
    import torch
    from . import synth
    N = req.N
    g = torch.Generator(device=device)
    g.manual_seed(int(req.seed))
    logD = synth.grf_torch(N, g, device).clamp_(-math.log(100.0), math.log(100.0))
    logmua = math.log(0.05) + synth.grf_torch(N, g, device)
    q = synth.blob_source_torch(N, g, device)
    out = {"logD": logD, "logmua": logmua, "q": q}
    if req.mode == "jvp":
        out["dq"] = synth.zero_boundary_torch(torch.randn(q.shape, generator=g, device=device, dtype=q.dtype))
        out["dlogD"] = torch.randn(q.shape, generator=g, device=device, dtype=q.dtype)
        out["dlogmua"] = synth.zero_boundary_torch(torch.randn(q.shape, generator=g, device=device, dtype=q.dtype))
    else:
        out["rhobar"] = synth.zero_boundary_torch(torch.randn(q.shape, generator=g, device=device, dtype=q.dtype))
    return out


def field_bytes(N, mode):
    """Device bytes a request's own tensors take while it runs: inputs (log D,
    log mua, q, and the tangent's three fields or the cotangent), outputs
    (rho and rho', or rho and three gradients) and the generator's
    transient FFT fields (at most 5), each rounded up to the caching
    allocator's 2 MiB granularity."""
    nv = (N + 1) ** 3
    field = -(-nv * 8 // (2 << 20)) * (2 << 20)
    nfields = (6 + 2) if mode == "jvp" else (4 + 4)
    return (nfields + 5) * field


class Server:
    """Continuous-batching server for DMGS solves on one GPU."""

    def __init__(self, budget_bytes=64 << 30, max_slots=8, precision="fp32-in-fp64", rtol=1e-10, device="cuda:0",
                 keep_results=True, ir_inner_cycles=8, ir_adaptive=True):
        import torch
        from .solver import Options, workspace_bytes
        self.device = torch.device(device)
        self.opts = dict(precision=precision, rtol=rtol, max_cycles=200, ir_inner_cycles=ir_inner_cycles,
                         ir_adaptive=ir_adaptive)
        self.adm = Admission(budget_bytes, max_slots)
        self.keep = keep_results
        self.pool = collections.defaultdict(list)   # N -> idle plans
        self.pool_order = collections.deque()       # (N, plan) oldest first
        self.plan_bytes = {}
        # every pooled plan may serve forward + VJP requests, whose two
        # solves run concurrently on a second work set of the plan
        self._ws = lambda N: workspace_bytes(Options(N, **self.opts), forward_vjp=True)
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        # device bytes of the plans that exist (running or pooled) and their
        # peak, each counted as dmgs_forward_vjp_workspace_bytes (exact once
        # the plan has run a forward + VJP request, an upper bound before)
        self.plan_live = 0
        self.plan_peak = 0
        self.cache_releases = 0

    # -- plan pool (called with the lock held) ---------------------------------
    def _need_of(self, req):
        pb = self.plan_bytes.setdefault(req.N, self._ws(req.N))
        reuse = pb if self.pool[req.N] else 0
        return pb + field_bytes(req.N, req.mode), reuse

    def _evict(self, nbytes):
        freed = 0
        while freed < nbytes and self.pool_order:
            N, plan = self.pool_order.popleft()
            self.pool[N].remove(plan)
            plan.close()
            self.plan_live -= self.plan_bytes[N]
            freed += self.plan_bytes[N]
        return freed

    def _release_cache_if_needed(self):
        """Freed blocks that torch's caching allocator keeps are device memory
        the accounting does not see.  When they and the next request's need
        would take the resident total past the budget, return them to the
        device (torch.cuda.empty_cache) before admitting it."""
        import torch
        if not self.adm.queue or self.adm.active >= self.adm.max_slots:
            return
        cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        if cached <= 0:
            return
        need, reuse = self._need_of(self.adm.queue[0])
        if self.adm.resident() + (need - reuse) + cached > self.adm.budget:
            torch.cuda.empty_cache()
            self.cache_releases += 1

    def _take_plan(self, N):
        from .solver import Options, Plan
        if self.pool[N]:
            plan = self.pool[N].pop()
            self.pool_order.remove((N, plan))
            return plan
        return None

    def _new_plan(self, N):
        from .solver import Options, Plan
        return Plan(Options(N, **self.opts), device=self.device)

    # -- execution -------------------------------------------------------------
    def _execute(self, req, plan, stream):
        import torch
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            f = request_fields(req, self.device)
            plan.set_log_coefficients(f["logD"], f["logmua"])
            if req.mode == "jvp":
                rho, fi = plan.forward(f["q"])
                drho, ji = plan.jvp(rho, f["dq"], f["dlogD"], f["dlogmua"])
                out = {"rho": rho, "drho": drho}
                cyc = (fi["cycles"], ji["cycles"])
            else:
                # the adjoint solve does not need rho: both solves at once
                (rho, (qbar, gD, gmu)), fi, vi = plan.forward_vjp(f["q"], f["rhobar"])
                out = {"rho": rho, "qbar": qbar, "logD_bar": gD, "logmua_bar": gmu}
                cyc = (fi["cycles"], vi["cycles"])
            stream.synchronize()
        return out, cyc

    def run(self, requests, realtime=True):
        """Serve `requests` (sorted by arrival).  realtime: arrivals are
        honoured on the wall clock; otherwise all arrive at t = 0."""
        import torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        if not realtime:
            for r in reqs:
                r.arrival = 0.0
        work = collections.deque()
        done_count = [0]
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        stop = [False]

        def worker():
            stream = torch.cuda.Stream(device=self.device)
            while True:
                with self.cv:
                    while not work and not stop[0]:
                        self.cv.wait()
                    if not work:
                        return
                    req, need, plan = work.popleft()
                try:
                    if plan is None:
                        with self.cv:
                            self.plan_live += self.plan_bytes[req.N]
                            self.plan_peak = max(self.plan_peak, self.plan_live)
                        plan = self._new_plan(req.N)
                    out, cyc = self._execute(req, plan, stream)
                    req.cycles = cyc
                    req.result = out if self.keep else {}
                    req.status = "done"
                except Exception:     # a failed request is retired with its status and traceback
                    req.status = "error"
                    req.error = traceback.format_exc()
                    with self.cv:
                        self.plan_live -= self.plan_bytes[req.N]
                    if plan is not None:
                        plan.close()
                        plan = None
                req.t_done = clock()
                with self.cv:
                    kept = 0
                    if plan is not None:
                        self.pool[req.N].append(plan)
                        self.pool_order.append((req.N, plan))
                        kept = self.plan_bytes[req.N]
                    self.adm.finish(need, kept)
                    done_count[0] += 1
                    self.cv.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.adm.max_slots)]
        for th in threads:
            th.start()
        i = 0
        with self.cv:
            while done_count[0] < len(reqs):
                now = clock()
                while i < len(reqs) and reqs[i].arrival <= now:
                    self.adm.offer(reqs[i])
                    i += 1
                while True:
                    self._release_cache_if_needed()
                    got = self.adm.next_admissible(self._need_of, self._evict)
                    if got is None:
                        break
                    kind, req, need = got
                    if kind == "reject":
                        req.status = "rejected"
                        req.error = "footprint %d bytes exceeds the budget %d" % (need, self.adm.budget)
                        req.t_done = clock()
                        done_count[0] += 1
                        continue
                    req.t_admit = clock()
                    work.append((req, need, self._take_plan(req.N)))
                    self.cv.notify_all()
                timeout = 0.05
                if i < len(reqs):
                    timeout = max(0.0, min(timeout, reqs[i].arrival - clock()))
                self.cv.wait(timeout=timeout)
            stop[0] = True
            self.cv.notify_all()
        for th in threads:
            th.join()
        return reqs

    def close(self):
        with self.lock:
            self._evict(1 << 62)


class TickServer(Server):
    """The same admission, plan pool and request fields as Server, executed
    as grouped ticks (dmgs_batch_*).  Admitted requests join the batch of
    their size class (the classes are split at the bounds in `split`), and
    each class's batch is ticked by its own host thread on its own HIP
    stream.  A tick advances every request of the batch by one refinement
    step in grouped launches and synchronises that stream once.  The classes
    tick concurrently, so a small request's steps do not wait for a large
    request's.  A forward +
    VJP request runs its two solves one after the other (plans need no
    second work set), so plans are accounted with dmgs_workspace_bytes.
    Results are bitwise those of Server."""

    def __init__(self, *args, split=(64, 96, 128), **kw):
        super().__init__(*args, **kw)
        from .solver import Options, workspace_bytes
        self._ws = lambda N: workspace_bytes(Options(N, **self.opts))
        self.split = tuple(split)
        self.ticks = 0
        self.batch_stats = None

    def run(self, requests, realtime=True):
        import torch
        from .solver import Batch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        if not realtime:
            for r in reqs:
                r.arrival = 0.0
        by_id = {r.id: r for r in reqs}
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        classes = []
        for _ in range(len(self.split) + 1):
            classes.append({"stream": torch.cuda.Stream(device=self.device), "batch": Batch(self.device),
                            "lock": threading.Lock(), "running": {}})
        state = {"done": 0, "stop": False}

        def retire(cls, d):   # called with self.cv held
            req = by_id[d["tag"]]
            need, plan = cls["running"].pop(req.id)
            req.t_done = clock()
            req.cycles = (d["info_fwd"]["cycles"], d["info_second"]["cycles"])
            if d["status"] == 0:
                req.status = "done"
                keys = ("rho", "drho") if d["mode"] == "jvp" else ("rho", "qbar", "logD_bar", "logmua_bar")
                req.result = {k: d[k] for k in keys} if self.keep else {}
                self.pool[req.N].append(plan)
                self.pool_order.append((req.N, plan))
                self.adm.finish(need, self.plan_bytes[req.N])
            else:   # a failed request is retired with its status, and its plan closed
                req.status = "error"
                req.error = "status %d" % d["status"]
                plan.close()
                self.plan_live -= self.plan_bytes[req.N]
                self.adm.finish(need, 0)
            state["done"] += 1

        def pending(cls):
            with cls["lock"]:
                return cls["batch"].pending()

        def fail_all(cls, err):   # called with self.cv and cls["lock"] held
            # a tick that fails ends every request of its batch, whose plans
            # are closed, and the batch is replaced
            for rid, (need, plan) in list(cls["running"].items()):
                req = by_id[rid]
                req.status = "error"
                req.error = err
                req.t_done = clock()
                plan.close()
                self.plan_live -= self.plan_bytes[req.N]
                self.adm.finish(need, 0)
                state["done"] += 1
            cls["running"].clear()
            cls["batch"].close()
            cls["batch"] = Batch(self.device)

        def worker(cls):
            with torch.cuda.device(self.device):
                while True:
                    with self.cv:
                        while not state["stop"] and not pending(cls):
                            self.cv.wait()
                        if state["stop"]:
                            return
                    err = None
                    with cls["lock"]:
                        try:
                            finished = cls["batch"].tick(cls["stream"])
                        except Exception:
                            finished, err = [], traceback.format_exc()
                    with self.cv:
                        self.ticks += 1
                        for d in finished:
                            retire(cls, d)
                        if err is not None:
                            with cls["lock"]:
                                fail_all(cls, err)
                        self.cv.notify_all()

        threads = [threading.Thread(target=worker, args=(c,), daemon=True) for c in classes]
        for th in threads:
            th.start()
        i = 0
        try:
            with torch.cuda.device(self.device), self.cv:
                while state["done"] < len(reqs):
                    now = clock()
                    while i < len(reqs) and reqs[i].arrival <= now:
                        self.adm.offer(reqs[i])
                        i += 1
                    while True:
                        self._release_cache_if_needed()
                        got = self.adm.next_admissible(self._need_of, self._evict)
                        if got is None:
                            break
                        kind, req, need = got
                        if kind == "reject":
                            req.status = "rejected"
                            req.error = "footprint %d bytes exceeds the budget %d" % (need, self.adm.budget)
                            req.t_done = clock()
                            state["done"] += 1
                            continue
                        req.t_admit = clock()
                        plan = self._take_plan(req.N)
                        if plan is None:
                            self.plan_live += self.plan_bytes[req.N]
                            self.plan_peak = max(self.plan_peak, self.plan_live)
                            plan = self._new_plan(req.N)
                        cls = classes[sum(req.N > b for b in self.split)]
                        with torch.cuda.stream(cls["stream"]):
                            f = request_fields(req, self.device)
                            plan.set_log_coefficients(f["logD"], f["logmua"])
                        with cls["lock"]:
                            if req.mode == "jvp":
                                cls["batch"].add(plan, "jvp", f["q"], dq=f["dq"], dlogD=f["dlogD"],
                                                 dlogmua=f["dlogmua"], tag=req.id)
                            else:
                                cls["batch"].add(plan, "vjp", f["q"], rhobar=f["rhobar"], tag=req.id)
                        cls["running"][req.id] = (need, plan)
                        self.cv.notify_all()
                    timeout = 0.05
                    if i < len(reqs):
                        timeout = max(0.0, min(timeout, reqs[i].arrival - clock()))
                    self.cv.wait(timeout=timeout)
                state["stop"] = True
                self.cv.notify_all()
        finally:
            with self.cv:
                state["stop"] = True
                self.cv.notify_all()
            for th in threads:
                th.join()
            st = [c["batch"].stats() for c in classes]
            self.batch_stats = {k: sum(x[k] for x in st) for k in st[0]}
            for c in classes:
                c["batch"].close()
        return reqs


def summarize(reqs, wall=None):
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    t_end = max(r.t_done for r in reqs)
    t_begin = min(r.arrival for r in reqs)
    span = wall if wall is not None else max(t_end - t_begin, 1e-9)
    return {"requests": len(reqs), "done": len(done), "rejected": sum(r.status == "rejected" for r in reqs),
            "errors": sum(r.status == "error" for r in reqs),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "requests_per_s": len(done) / span, "solves_per_s": 2 * len(done) / span, "span_s": span}
