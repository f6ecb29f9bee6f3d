"""Continuous-batching serving loop: every result is bitwise the same alone
and in the mix, the memory budget is never exceeded, and requests queue when
it is tight."""
import copy

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def stream(n=16, sizes=(32, 48, 64, 96)):
    from paper_2608_00760_amd.serving import Request
    return [Request(id=i, N=sizes[i % len(sizes)], mode=("jvp", "vjp")[(i // 2) % 2], seed=7000 + i)
            for i in range(n)]


def test_alone_equals_in_the_mix_and_budget_holds():
    import torch
    from paper_2608_00760_amd.serving import Server, field_bytes, summarize
    from paper_2608_00760_amd.solver import Options, workspace_bytes
    say("serving: mixed stream")
    reqs = stream()
    need = max(workspace_bytes(Options(r.N, precision="fp32-in-fp64"), forward_vjp=True) + field_bytes(r.N, r.mode)
               for r in reqs)
    budget = int(2.5 * need)         # tight: forces queueing
    srv = Server(budget_bytes=budget, max_slots=4)
    mixed = srv.run(copy.deepcopy(reqs), realtime=False)
    s = summarize(mixed)
    say("serving summary", s, "peak", srv.adm.peak, "budget", budget, "max queue", srv.adm.max_queue)
    assert s["done"] == len(reqs)
    assert srv.adm.peak <= budget
    assert srv.adm.max_queue > 1
    srv.close()
    say("serving: each request alone")
    for r in reqs:
        alone = Server(budget_bytes=1 << 40, max_slots=1).run([copy.deepcopy(r)], realtime=False)[0]
        m = next(x for x in mixed if x.id == r.id)
        assert alone.status == "done" and alone.cycles == m.cycles
        for k, v in alone.result.items():
            assert torch.equal(v, m.result[k]), (r.id, k)


def test_poisson_arrivals_and_rejection():
    from paper_2608_00760_amd.serving import Request, Server, summarize
    say("serving: Poisson arrivals")
    reqs = stream(8, sizes=(32, 64))
    for i, r in enumerate(reqs):
        r.arrival = 0.002 * i
    big = Request(id=99, N=192, mode="vjp", seed=1)
    srv = Server(budget_bytes=600 << 20, max_slots=3, keep_results=False)
    out = srv.run(reqs + [big], realtime=True)
    s = summarize(out)
    assert s["done"] == 8 and s["rejected"] == 1
    assert next(r for r in out if r.id == 99).status == "rejected"
    assert srv.adm.peak <= 600 << 20
    srv.close()
