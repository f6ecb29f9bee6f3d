"""Host-side admission policy of the serving loop (no GPU)."""
from paper_2608_00760_amd.serving import Admission, Request


def make(n, N=64):
    return [Request(id=i, N=N, mode="vjp", seed=i) for i in range(n)]


def test_fifo_and_slots():
    adm = Admission(budget_bytes=1000, max_slots=2)
    for r in make(4):
        adm.offer(r)
    need_of = lambda r: (100, 0)
    evict = lambda b: 0
    got = [adm.next_admissible(need_of, evict) for _ in range(3)]
    assert [g[1].id for g in got[:2]] == [0, 1] and got[2] is None   # slots full
    adm.finish(100, 0)
    g = adm.next_admissible(need_of, evict)
    assert g[0] == "run" and g[1].id == 2                            # FIFO order kept


def test_budget_never_exceeded_and_head_of_line():
    adm = Admission(budget_bytes=250, max_slots=8)
    reqs = make(3)
    for r in reqs:
        adm.offer(r)
    need_of = lambda r: (100, 0)
    assert adm.next_admissible(need_of, lambda b: 0)[1].id == 0
    assert adm.next_admissible(need_of, lambda b: 0)[1].id == 1
    assert adm.next_admissible(need_of, lambda b: 0) is None          # 300 > 250: waits
    assert adm.peak <= 250
    adm.finish(100, 0)
    assert adm.next_admissible(need_of, lambda b: 0)[1].id == 2
    assert adm.peak <= 250


def test_oversize_request_rejected():
    adm = Admission(budget_bytes=100, max_slots=4)
    adm.offer(make(1)[0])
    kind, req, need = adm.next_admissible(lambda r: (101, 0), lambda b: 0)
    assert kind == "reject" and need == 101 and not adm.queue


def test_eviction_of_idle_plans_and_reuse():
    adm = Admission(budget_bytes=300, max_slots=4)
    # one request finished and left a 150-byte plan idle in the pool
    adm.in_use, adm.active = 0, 0
    adm.idle = 150
    pool = {"plans": 1}

    def need_of(r):
        return (200, 150 if pool["plans"] else 0)

    def evict(b):
        freed = 150 if pool["plans"] else 0
        pool["plans"] = 0
        return freed

    adm.offer(make(1)[0])
    kind, _, need = adm.next_admissible(need_of, evict)   # reuses the idle plan: 150 + 50 fits
    assert kind == "run" and adm.idle == 0 and adm.in_use == 200 and pool["plans"] == 1
    adm.finish(200, 150)
    adm.idle = 150
    adm.offer(make(1, N=128)[0])
    need_of2 = lambda r: (280, 0)        # a different size: the idle plan must go
    kind, _, _ = adm.next_admissible(need_of2, evict)
    assert kind == "run" and adm.resident() == 280 <= 300
