"""The batch schedule (reach_plan_batch), computed on the host: no GPU.

Every query runs exactly once.  A batch with more queries than twice the
resident waves (4096 without a context) packs, and then every item is a
segment pack: 1..64 queries of one kind with identical constants, step counts
within 1/16 octave and one cells-per-lane E in {2, 4, 8, 16}, each on
ceil(n / E) lanes in the balanced layout (n >= (E - 1) ceil(n / E)), at most
64 lanes.  A smaller batch runs every query alone (E = 0).  Items come longest
first; the plan is deterministic.  Results of packed queries are compared with single runs bit
for bit in the GPU batch tests."""
import math

import numpy as np
import pytest

import workloads

R = pytest.importorskip("paper_2001_10635_amd")

FAKE = 1 << 20     # device addresses are never dereferenced by the planner
PACK_MIN = 2 * 8 * 256 + 1   # smallest batch that packs without a context


def queries_of(stream):
    out = []
    for k, q in enumerate(stream):
        p = q.problem
        base = FAKE + 4096 * k
        out.append(R.make_query(p.kind, p.n, p.prm, R.REACH_F64, base, base + 8, base + 16,
                                base + 24, p.dt, p.nsteps, base + 32 if p.n_in else None,
                                base + 40 if p.n_in else None, n_in=p.n_in))
    return out


def bucket(cost):
    """1/16-octave class of a wave time (larger = longer)."""
    c = cost + 1
    msb = c.bit_length() - 1
    frac = (c >> (msb - 4)) & 15 if msb >= 4 else (c << (4 - msb)) & 15
    return msb * 16 + frac


def check_plan(qs, plan):
    """plan: (E, members) pairs."""
    seen = sorted(i for _, item in plan for i in item)
    assert seen == list(range(len(qs))), "every query exactly once"
    costs = []
    for E, item in plan:
        if E:
            assert E in (2, 4, 8, 16)
            assert 1 <= len(item) <= 64
            lanes = [math.ceil(qs[i].sys.n / E) for i in item]
            assert sum(lanes) <= 64
            lead = qs[item[0]]
            for i, L in zip(item, lanes):
                q = qs[i]
                assert q.sys.n >= (E - 1) * L, "balanced layout exists"
                assert (q.sys.kind, q.dt, tuple(q.sys.prm)) == \
                    (lead.sys.kind, lead.dt, tuple(lead.sys.prm))
                assert bucket(q.nsteps) == bucket(lead.nsteps), "step counts within 1/16 octave"
            costs.append(bucket(E * max(qs[i].nsteps for i in item)))
        else:
            assert len(item) == 1
            q = qs[item[0]]
            costs.append(bucket(math.ceil(q.sys.n / 64) * q.nsteps))
    assert all(a >= b for a, b in zip(costs, costs[1:])), "longest item first"


@pytest.mark.parametrize("nq", [1, 7, 400, 20000])
def test_plan_covers_every_query_once_and_packs_validly(nq):
    qs = queries_of(workloads.query_stream(nq, 5.0e4, seed=4242 + nq))
    plan = R.reach_plan_batch(None, qs, with_E=True)
    check_plan(qs, plan)
    assert plan == R.reach_plan_batch(None, qs, with_E=True), "deterministic"
    if nq < PACK_MIN:
        assert all(E == 0 for E, _ in plan), "small batches do not pack"
    else:
        assert all(E for E, _ in plan), "a packed batch runs packs only"


def test_queries_are_packed_densely():
    """In a large mix the packs fill most of their wave's lanes and cell
    slots (at 16 cells per lane a 20000-query mix has fewer queries per pack
    key than at 8, so the lane bound is a little lower than the cell bound
    suggests)."""
    qs = queries_of(workloads.query_stream(20000, 5.0e4, seed=99))
    plan = R.reach_plan_batch(None, qs, with_E=True)
    packs = [(E, it) for E, it in plan if E]
    assert len(packs) == len(plan)
    lanes = [sum(math.ceil(qs[i].sys.n / E) for i in it) for E, it in packs]
    assert np.mean(lanes) > 52
    cells = sum(qs[i].sys.n for _, it in packs for i in it)
    slots = sum(64 * E for E, _ in packs)
    assert cells > 0.8 * slots


def test_only_identical_constants_share_a_wave():
    p = workloads.small_problem(workloads.KIND_CTM, 10, 3, 50)
    qs = []
    for k in range(PACK_MIN):
        dt = 0.01 if k % 3 else 0.02          # two step sizes
        steps = 50 if k % 4 else 49           # two step counts, same 1/16 octave
        qs.append(R.make_query(p.kind, 10, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, dt, steps))
    lin = R.make_query(R.REACH_LIN3, 8, (0.1, -0.5, 0.2, 1.0), R.REACH_F64, FAKE, FAKE, FAKE,
                       FAKE, 0.01, 50)
    qs.append(lin)
    plan = R.reach_plan_batch(None, qs, with_E=True)
    check_plan(qs, plan)
    assert [len(it) for _, it in plan if len(qs) - 1 in it] == [1], "one LIN3 query runs alone"
    for _, it in plan:
        assert len({qs[i].dt for i in it}) == 1
    assert any(len({qs[i].nsteps for i in it}) == 2 for _, it in plan), \
        "49 and 50 steps share packs"


def test_more_constant_classes_than_a_chunk_keeps():
    """40 step sizes in one packed batch: a work unit keeps 16 constant classes
    in its table and runs queries of further classes in packs of their own, so
    the plan still covers every query once, never mixes constants in a pack,
    and packs the tabled classes densely."""
    p = workloads.small_problem(workloads.KIND_RD, 12, 3, 40)
    qs = [R.make_query(p.kind, 12, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE,
                       0.01 * (1 + k % 40), 40, FAKE, FAKE, n_in=1) for k in range(20000)]
    plan = R.reach_plan_batch(None, qs, with_E=True)
    check_plan(qs, plan)
    for _, it in plan:
        assert len({qs[i].dt for i in it}) == 1
    sizes = [len(it) for _, it in plan]
    assert max(sizes) > 1 and min(sizes) == 1, "shared packs and packs of their own"
    assert len(plan) < len(qs), "the tabled classes pack"


def test_cells_per_lane_follow_the_cost_rule():
    """At the default cap of 16 cells per lane: n = 10 packs at E = 4 (3
    lanes), n = 5 at E = 2 (no balanced 4-cell layout), n = 100 at E = 8 (13
    lanes; 7 lanes of 16 would need 105 cells), n = 512 at E = 16 (half the
    wave), n = 320 at E = 16 (20 lanes)."""
    qs, want = [], {}
    for n, E in ((10, 4), (5, 2), (100, 8), (512, 16), (320, 16)):
        p = workloads.small_problem(workloads.KIND_RD, n, 5, 20)
        for _ in range(1000):
            want[len(qs)] = E
            qs.append(R.make_query(p.kind, n, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, p.dt,
                                   20, FAKE, FAKE, n_in=1))
    plan = R.reach_plan_batch(None, qs, with_E=True)
    check_plan(qs, plan)
    for E, it in plan:
        for i in it:
            assert want[i] == E


def test_plan_rejects_what_the_batch_rejects():
    p = workloads.small_problem(workloads.KIND_CTM, 600, 3, 10)
    bad = R.make_query(p.kind, 600, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, p.dt, 10)
    with pytest.raises(R.ReachError) as e:
        R.reach_plan_batch(None, [bad])
    assert e.value.status == R.REACH_E_UNSUPPORTED
    neg = R.make_query(p.kind, 20, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, -0.1, 10)
    with pytest.raises(R.ReachError) as e:
        R.reach_plan_batch(None, [neg])
    assert e.value.status == R.REACH_E_INVAL
    assert R.reach_plan_batch(None, []) == []


def test_large_plan_without_context_rejects_a_bad_query_deep_inside():
    """20000 queries are planned by several host threads (a pool of the
    call's own when there is no context); one bad query anywhere fails the
    whole plan with that query's status."""
    qs = queries_of(workloads.query_stream(20000, 5.0e4, seed=99))
    p = workloads.small_problem(workloads.KIND_CTM, 20, 3, 10)
    qs[15001] = R.make_query(p.kind, 20, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, -0.1, 10)
    with pytest.raises(R.ReachError) as e:
        R.reach_plan_batch(None, qs)
    assert e.value.status == R.REACH_E_INVAL
