"""Batched small queries (persistent kernel, captured hipGraph) and the
one-launch-per-query baseline: every result equals the query run alone."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")


@pytest.fixture(scope="module")
def rc():
    r = R.Reach(0)
    yield r
    r.close()


class Batch:
    """Device buffers for a list of workload queries."""

    def __init__(self, queries):
        self.items = []
        for q in queries:
            p = q.problem
            lo, hi = p.box()
            pl, ph = p.inputs()
            d = dict(p=p, lo=lo, hi=hi, pl=pl, ph=ph, x_lo=to_dev(lo), x_hi=to_dev(hi),
                     r_lo=torch.full((p.n,), np.nan, dtype=torch.float64, device="cuda"),
                     r_hi=torch.full((p.n,), np.nan, dtype=torch.float64, device="cuda"),
                     p_lo=None if pl is None else to_dev(pl), p_hi=None if ph is None else to_dev(ph))
            self.items.append(d)

    def queries(self):
        out = []
        for d in self.items:
            p = d["p"]
            out.append(R.make_query(p.kind, p.n, p.prm, R.REACH_F64, d["x_lo"], d["x_hi"],
                                    d["r_lo"], d["r_hi"], p.dt, p.nsteps, d["p_lo"], d["p_hi"],
                                    n_in=p.n_in))
        return out

    def results(self):
        return [(to_host(d["r_lo"]), to_host(d["r_hi"])) for d in self.items]

    def clear(self):
        for d in self.items:
            d["r_lo"].fill_(np.nan)
            d["r_hi"].fill_(np.nan)


def alone(rc, d):
    p = d["p"]
    r_lo, r_hi = rc.embed(p.kind, p.prm, d["x_lo"], d["x_hi"], p.dt, p.nsteps, p_lo=d["p_lo"],
                          p_hi=d["p_hi"])
    assert rc.sync() == R.REACH_OK
    return to_host(r_lo), to_host(r_hi)


@pytest.fixture(scope="module")
def mix():
    return Batch(workloads.query_stream(400, 5.0e4, seed=4242))


# batch modes: every query alone over a wave, segment packs (capped at E cells
# per lane), one side per wave
MODES = {"alone": {"batch.pack": 2}, "packed": {"batch.pack": 1},
         "packed_E16": {"batch.pack": 1, "batch.E": 16}, "packed_E4": {"batch.pack": 1, "batch.E": 4}, "packed_E2": {"batch.pack": 1, "batch.E": 2},
         "split": {"batch.split": 1}}


class options:
    """Context options set for a block and reset to their defaults after it."""

    def __init__(self, rc, opts):
        self.rc, self.opts = rc, opts

    def __enter__(self):
        for k, v in self.opts.items():
            self.rc.set_option(k, v)

    def __exit__(self, *exc):
        for k in self.opts:
            self.rc.set_option(k, 0)


@pytest.mark.parametrize("mode", list(MODES))
def test_batch_equals_alone_and_oracle(rc, mix, mode):
    qs = mix.queries()
    nb = R.reach_batch_workspace_bytes(len(qs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    mix.clear()
    say(f"batch 400 queries {mode}")
    with options(rc, MODES[mode]):
        plan = R.reach_plan_batch(rc.ctx, qs, with_E=True)
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
        assert rc.sync() == R.REACH_OK
    cap = MODES[mode].get("batch.E", 16)
    if mode.startswith("packed"):
        assert any(E == cap for E, _ in plan), "packs at the cap"
        # wider than the cap only for queries too long for 64 lanes at it
        assert all(E <= cap or all(qs[i].sys.n > 64 * cap for i in it) for E, it in plan)
    else:
        assert all(E == 0 for E, _ in plan)
    got = mix.results()
    for k, d in enumerate(mix.items):
        a = alone(rc, d)
        assert np.array_equal(got[k][0], a[0]) and np.array_equal(got[k][1], a[1]), f"query {k}"
    for k in range(0, len(mix.items), 23):
        d = mix.items[k]
        p = d["p"]
        o_lo, o_hi = oracle.embed_rk4(p.kind, p.prm, d["lo"], d["hi"], d["pl"], d["ph"], dt=p.dt,
                                      nsteps=p.nsteps)
        assert_rel(got[k][0], o_lo, 1e-12, f"query {k} lower")
        assert_rel(got[k][1], o_hi, 1e-12, f"query {k} upper")


@pytest.mark.parametrize("mode", ["alone", "packed", "packed_E4"])
def test_batch_graph_replays_match_eager(rc, mix, mode):
    """The captured graph (counter reset kernel and worker; the descriptors
    and the work items are copied on the stream before it) is replayed
    with eager work and synchronisation in between; every replay equals the
    eager result, with the wide, the narrow and the one-query kernel."""
    qs = mix.queries()
    nb = R.reach_batch_workspace_bytes(len(qs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    mix.clear()
    with options(rc, MODES[mode]):
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)    # eager (default stream, no graph)
        assert rc.sync() == R.REACH_OK
    ref = mix.results()
    s = torch.cuda.Stream()
    for rep in range(4):
        mix.clear()
        torch.cuda.synchronize()
        say(f"graph replay {rep} {mode}")
        with options(rc, MODES[mode]):
            with torch.cuda.stream(s):
                R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, s)
            assert rc.sync(s) == R.REACH_OK
        x = torch.randn(1000, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        got = mix.results()
        for k in range(len(ref)):
            assert np.array_equal(got[k][0], ref[k][0]) and np.array_equal(got[k][1], ref[k][1])


def test_each_equals_batch(rc, mix):
    qs = mix.queries()
    nb = R.reach_batch_workspace_bytes(len(qs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    mix.clear()
    R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert rc.sync() == R.REACH_OK
    ref = mix.results()
    mix.clear()
    say("one launch per query")
    R.reach_embed_rk4_each(rc.ctx, qs, 8)
    assert rc.sync() == R.REACH_OK
    got = mix.results()
    for k in range(len(ref)):
        assert np.array_equal(got[k][0], ref[k][0]) and np.array_equal(got[k][1], ref[k][1])


@pytest.mark.parametrize("mode", ["alone", "packed", "split"])
@pytest.mark.parametrize("waves", [1, 3, 64])
def test_batch_wave_count_invariance(rc, mix, waves, mode):
    qs = mix.queries()[:60]
    nb = R.reach_batch_workspace_bytes(len(qs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    mix.clear()
    say(f"batch 60 queries waves={waves} {mode}")
    with options(rc, {"batch.waves": waves, **MODES[mode]}):
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
        assert rc.sync() == R.REACH_OK
    got = mix.results()[:60]
    for k in range(60):
        a = alone(rc, mix.items[k])
        assert np.array_equal(got[k][0], a[0]) and np.array_equal(got[k][1], a[1])


def test_batch_rejections_and_flags(rc):
    p = workloads.small_problem(workloads.KIND_CTM, 600, 3, 10)
    lo, hi = p.box()
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    r = torch.empty(600, dtype=torch.float64, device="cuda")
    q = R.make_query(p.kind, 600, p.prm, R.REACH_F64, x_lo, x_hi, r, r, p.dt, p.nsteps)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.ReachError) as e:
        R.reach_embed_rk4_batch(rc.ctx, [q], ws, 1 << 20, 0)
    assert e.value.status == R.REACH_E_UNSUPPORTED
    q32 = R.make_query(p.kind, 100, p.prm, R.REACH_F32, x_lo, x_hi, r, r, p.dt, p.nsteps)
    with pytest.raises(R.ReachError) as e:
        R.reach_embed_rk4_batch(rc.ctx, [q32], ws, 1 << 20, 0)
    assert e.value.status == R.REACH_E_UNSUPPORTED
    good = R.make_query(p.kind, 100, p.prm, R.REACH_F64, x_lo, x_hi, r, r, p.dt, p.nsteps)
    with pytest.raises(R.ReachError) as e:
        R.reach_embed_rk4_batch(rc.ctx, [good] * 10, ws, 16, 0)
    assert e.value.status == R.REACH_E_NOMEM
    bad = lo.copy()
    bad[7] = np.inf
    xb = to_dev(bad)
    r2 = torch.empty(600, dtype=torch.float64, device="cuda")
    qb = R.make_query(p.kind, 100, p.prm, R.REACH_F64, xb, x_hi, r2, r2[300:], p.dt, p.nsteps)
    R.reach_embed_rk4_batch(rc.ctx, [good, qb], ws, 1 << 20, 0)
    assert rc.sync() == R.REACH_E_NONFINITE
    assert rc.sync() == R.REACH_OK
    # an empty batch launches nothing and succeeds, with or without a workspace
    assert R.reach_embed_rk4_batch(rc.ctx, [], ws, 1 << 20, 0) == R.REACH_OK
    assert R.reach_embed_rk4_batch(rc.ctx, [], None, 0, 0) == R.REACH_OK
    assert R.reach_embed_rk4_each(rc.ctx, []) == R.REACH_OK
    assert rc.sync() == R.REACH_OK


def packed_ctm_batch(nq, seed):
    """nq CTM queries (n in [4, 512], 1-40 steps) packed in shared device buffers."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(4, 513, nq)
    ks = rng.integers(1, 41, nq)
    offs = np.concatenate([[0], np.cumsum(ns)])
    lo = rng.uniform(12.0, 24.0, offs[-1])
    hi = lo + rng.uniform(0.0, 2.0, offs[-1])
    d = dict(ns=ns, ks=ks, offs=offs, lo=lo, hi=hi, x_lo=to_dev(lo), x_hi=to_dev(hi),
             r_lo=torch.full((int(offs[-1]),), np.nan, dtype=torch.float64, device="cuda"),
             r_hi=torch.full((int(offs[-1]),), np.nan, dtype=torch.float64, device="cuda"))

    def q(i, dtype=R.REACH_F64, dt=0.01, n=None):
        o = 8 * int(offs[i])
        return R.make_query(R.REACH_CTM, int(ns[i]) if n is None else n, workloads.CTM_PRM, dtype,
                            d["x_lo"].data_ptr() + o, d["x_hi"].data_ptr() + o,
                            d["r_lo"].data_ptr() + o, d["r_hi"].data_ptr() + o, dt, int(ks[i]))
    d["q"] = q
    return d


def test_batch_of_20000_queries_equals_one_launch_per_query(rc):
    """Large batches prepare their descriptors on several host threads: the
    results still equal one launch per query, bit for bit, and the oracle."""
    b = packed_ctm_batch(20000, 77)
    qs = R.query_array([b["q"](i) for i in range(20000)])
    nb = R.reach_batch_workspace_bytes(20000)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    say("batch 20000 queries")
    R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert rc.sync() == R.REACH_OK
    got_lo, got_hi = to_host(b["r_lo"]), to_host(b["r_hi"])
    assert not np.isnan(got_lo).any() and not np.isnan(got_hi).any()
    b["r_lo"].fill_(np.nan)
    b["r_hi"].fill_(np.nan)
    say("each 20000 queries")
    R.reach_embed_rk4_each(rc.ctx, qs, 8)
    assert rc.sync() == R.REACH_OK
    assert np.array_equal(to_host(b["r_lo"]), got_lo)
    assert np.array_equal(to_host(b["r_hi"]), got_hi)
    offs = b["offs"]
    for i in (0, 1, 9999, 15001, 19999):
        a, e = int(offs[i]), int(offs[i + 1])
        o_lo, o_hi = oracle.embed_rk4(R.REACH_CTM, workloads.CTM_PRM, b["lo"][a:e], b["hi"][a:e],
                                      dt=0.01, nsteps=int(b["ks"][i]))
        assert_rel(got_lo[a:e], o_lo, 1e-12, f"query {i} lower")
        assert_rel(got_hi[a:e], o_hi, 1e-12, f"query {i} upper")


def test_back_to_back_batches_on_two_streams_share_a_workspace(rc):
    """Batches issued without waiting, alternately on two streams with one
    workspace, then on one stream, then with a smaller batch between: a call
    plans while the previous batch's kernel runs, its uploads wait on the
    device for the kernel that used their workspace block (and for the
    previous kernel when the block layout moves), and its kernel for the
    previous kernel, so every box equals the query's own launch bit for bit."""
    A = packed_ctm_batch(20000, 11)
    B = packed_ctm_batch(20000, 12)
    qa = R.query_array([A["q"](i) for i in range(20000)])
    qb = R.query_array([B["q"](i) for i in range(20000)])
    nb = R.reach_batch_workspace_bytes(20000)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    say("back-to-back batches on two streams, then on one")
    for rep in range(3):
        R.reach_embed_rk4_batch(rc.ctx, qa, ws, nb, s1)
        R.reach_embed_rk4_batch(rc.ctx, qb, ws, nb, s2)
    for rep in range(3):
        R.reach_embed_rk4_batch(rc.ctx, qb, ws, nb, s1)
        R.reach_embed_rk4_batch(rc.ctx, qa, ws, nb, s1)
    # a smaller batch (B's first 7000 queries) in the same workspace moves the
    # blocks: its uploads also wait for the batch before it
    qc = R.query_array([B["q"](i) for i in range(7000)])
    for rep in range(3):
        R.reach_embed_rk4_batch(rc.ctx, qc, ws, nb, s1)
        R.reach_embed_rk4_batch(rc.ctx, qa, ws, nb, s2)
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    got = [(to_host(X["r_lo"]), to_host(X["r_hi"])) for X in (A, B)]
    for X, q in ((A, qa), (B, qb)):
        X["r_lo"].fill_(np.nan)
        X["r_hi"].fill_(np.nan)
        R.reach_embed_rk4_each(rc.ctx, q, 8)
    assert rc.sync() == R.REACH_OK
    for (g_lo, g_hi), X in zip(got, (A, B)):
        assert not np.isnan(g_lo).any()
        assert np.array_equal(to_host(X["r_lo"]), g_lo)
        assert np.array_equal(to_host(X["r_hi"]), g_hi)


def test_batch_of_20000_reports_the_first_bad_query(rc):
    b = packed_ctm_batch(20000, 78)
    qs = [b["q"](i) for i in range(20000)]
    qs[17000] = b["q"](17000, n=600)            # too long for the batch path
    qs[3000] = b["q"](3000, dt=-1.0)             # the lower index wins
    nb = R.reach_batch_workspace_bytes(20000)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(R.ReachError) as e:
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert e.value.status == R.REACH_E_INVAL and "dt" in str(e.value)
    qs[3000] = b["q"](3000)
    with pytest.raises(R.ReachError) as e:
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert e.value.status == R.REACH_E_UNSUPPORTED and "512" in str(e.value)
    assert rc.sync() == R.REACH_OK


def test_packed_queries_report_nonfinite_and_order_and_match_alone(rc):
    """Twelve 10-cell CTM queries with 30 steps share waves (reach_plan_batch
    packs them); one starts from an infinite state, one with lower > upper.
    Both conditions reach the status word, and the clean packed queries equal
    their single runs bit for bit."""
    n, steps, nqs = 10, 30, 12
    rng = np.random.default_rng(5)
    lo = rng.uniform(12.0, 24.0, n * nqs)
    hi = lo + rng.uniform(0.0, 2.0, n * nqs)
    lo[3 * n + 4] = np.inf                     # query 3: non-finite
    lo[7 * n + 2], hi[7 * n + 2] = 30.0, 20.0  # query 7: lower > upper
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    r_lo = torch.full((n * nqs,), np.nan, dtype=torch.float64, device="cuda")
    r_hi = torch.full_like(r_lo, np.nan)
    qs = [R.make_query(R.REACH_CTM, n, workloads.CTM_PRM, R.REACH_F64, x_lo.data_ptr() + 8 * n * k,
                       x_hi.data_ptr() + 8 * n * k, r_lo.data_ptr() + 8 * n * k,
                       r_hi.data_ptr() + 8 * n * k, 0.01, steps) for k in range(nqs)]
    rc.set_option("batch.pack", 1)
    plan = R.reach_plan_batch(rc.ctx, qs)
    assert any(len(it) > 1 for it in plan) and any(3 in it and len(it) > 1 for it in plan)
    assert any(7 in it and len(it) > 1 for it in plan)
    nb = R.reach_batch_workspace_bytes(nqs)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    say("packed batch with a non-finite and a crossed query")
    R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert rc.sync() == R.REACH_E_NONFINITE
    got_lo, got_hi = to_host(r_lo), to_host(r_hi)
    for k in range(nqs):
        if k in (3, 7):
            continue
        a_lo, a_hi = rc.embed(R.REACH_CTM, workloads.CTM_PRM, x_lo[n * k:n * (k + 1)].contiguous(),
                              x_hi[n * k:n * (k + 1)].contiguous(), 0.01, steps)
        assert rc.sync() == R.REACH_OK
        assert np.array_equal(got_lo[n * k:n * (k + 1)], to_host(a_lo)), f"query {k}"
        assert np.array_equal(got_hi[n * k:n * (k + 1)], to_host(a_hi)), f"query {k}"
    # the crossed query alone in a batch of packs raises the order flag
    qs2 = [q for k, q in enumerate(qs) if k != 3]
    R.reach_embed_rk4_batch(rc.ctx, qs2, ws, nb, 0)
    rc.set_option("batch.pack", 0)
    assert rc.sync() == R.REACH_E_ORDER
    assert rc.sync() == R.REACH_OK


def test_packs_with_unequal_steps_and_sizes_equal_alone(rc):
    """Packs whose members have different step counts (49 and 50: one 1/16
    octave) and sizes (every cells-per-lane layout: n = 2..64 at E = 2, 4, 8,
    short lanes included): finished members' lanes stay masked while the
    others step, and every box equals its single run bit for bit."""
    rng = np.random.default_rng(11)
    ns = [int(v) for v in rng.integers(2, 65, 90)]
    offs = np.concatenate([[0], np.cumsum(ns)])
    lo = rng.uniform(-0.5, 0.5, offs[-1])
    hi = lo + rng.uniform(0.0, 0.05, offs[-1])
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    p_lo, p_hi = to_dev(np.array([-0.1])), to_dev(np.array([0.1]))
    r_lo = torch.full((int(offs[-1]),), np.nan, dtype=torch.float64, device="cuda")
    r_hi = torch.full_like(r_lo, np.nan)
    steps = [49 if k % 3 else 50 for k in range(len(ns))]
    qs = [R.make_query(R.REACH_RD, ns[k], (1.0,), R.REACH_F64, x_lo.data_ptr() + 8 * int(offs[k]),
                       x_hi.data_ptr() + 8 * int(offs[k]), r_lo.data_ptr() + 8 * int(offs[k]),
                       r_hi.data_ptr() + 8 * int(offs[k]), 0.1, steps[k], p_lo, p_hi, n_in=1)
          for k in range(len(ns))]
    nb = R.reach_batch_workspace_bytes(len(qs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for cap in (2, 4, 8, 16):
        r_lo.fill_(np.nan)
        r_hi.fill_(np.nan)
        with options(rc, {"batch.pack": 1, "batch.E": cap}):
            plan = R.reach_plan_batch(rc.ctx, qs, with_E=True)
            assert any(E == cap and len({steps[i] for i in it}) == 2 for E, it in plan)
            say(f"packs with unequal steps, E cap {cap}")
            R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
            assert rc.sync() == R.REACH_OK
        got_lo, got_hi = to_host(r_lo), to_host(r_hi)
        for k in range(len(ns)):
            a, e = int(offs[k]), int(offs[k + 1])
            a_lo, a_hi = rc.embed(R.REACH_RD, (1.0,), x_lo[a:e].contiguous(),
                                  x_hi[a:e].contiguous(), 0.1, steps[k], p_lo=p_lo, p_hi=p_hi)
            assert rc.sync() == R.REACH_OK
            assert np.array_equal(got_lo[a:e], to_host(a_lo)), f"query {k} n={ns[k]} cap {cap}"
            assert np.array_equal(got_hi[a:e], to_host(a_hi)), f"query {k} n={ns[k]} cap {cap}"


def test_many_constant_classes_equal_alone(rc):
    """3000 reaction-diffusion queries with 40 step sizes in one packed batch:
    classes past a work unit's table of 16 run in packs of their own, and
    every box equals its single run bit for bit."""
    rng = np.random.default_rng(5)
    nq = 3000
    ns = [int(v) for v in rng.integers(8, 80, nq)]
    offs = np.concatenate([[0], np.cumsum(ns)])
    lo = rng.uniform(-0.5, 0.5, offs[-1])
    hi = lo + rng.uniform(0.0, 0.05, offs[-1])
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    p_lo, p_hi = to_dev(np.array([-0.1])), to_dev(np.array([0.1]))
    r_lo = torch.full((int(offs[-1]),), np.nan, dtype=torch.float64, device="cuda")
    r_hi = torch.full_like(r_lo, np.nan)
    dts = [0.01 * (1 + k % 40) for k in range(nq)]
    qs = [R.make_query(R.REACH_RD, ns[k], (1.0,), R.REACH_F64, x_lo.data_ptr() + 8 * int(offs[k]),
                       x_hi.data_ptr() + 8 * int(offs[k]), r_lo.data_ptr() + 8 * int(offs[k]),
                       r_hi.data_ptr() + 8 * int(offs[k]), dts[k], 30, p_lo, p_hi, n_in=1)
          for k in range(nq)]
    nb = R.reach_batch_workspace_bytes(nq)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with options(rc, {"batch.pack": 1}):
        plan = R.reach_plan_batch(rc.ctx, qs, with_E=True)
        assert all(len({dts[i] for i in it}) == 1 for _, it in plan)
        assert any(len(it) > 1 for _, it in plan)
        say("packed batch of 40 constant classes")
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
        assert rc.sync() == R.REACH_OK
    got_lo, got_hi = to_host(r_lo), to_host(r_hi)
    for k in range(0, nq, 7):
        a, e = int(offs[k]), int(offs[k + 1])
        a_lo, a_hi = rc.embed(R.REACH_RD, (1.0,), x_lo[a:e].contiguous(), x_hi[a:e].contiguous(),
                              dts[k], 30, p_lo=p_lo, p_hi=p_hi)
        assert rc.sync() == R.REACH_OK
        assert np.array_equal(got_lo[a:e], to_host(a_lo)), f"query {k}"
        assert np.array_equal(got_hi[a:e], to_host(a_hi)), f"query {k}"


@pytest.mark.parametrize("cap", [16, 2])
def test_packs_with_zero_and_few_steps_equal_alone(rc, cap):
    """Packed queries of 1-512 cells with 0, 1, 2 or 5 steps: a zero-step
    query returns its box, every box equals its single run bit for bit."""
    rng = np.random.default_rng(17 + cap)
    nq = 600
    ns = [int(v) for v in rng.integers(1, 513, nq)]
    steps = [int(v) for v in rng.choice([0, 1, 2, 5], nq)]
    offs = np.concatenate([[0], np.cumsum(ns)])
    lo = rng.uniform(-0.5, 0.5, offs[-1])
    hi = lo + rng.uniform(0.0, 0.05, offs[-1])
    x_lo, x_hi = to_dev(lo), to_dev(hi)
    p_lo, p_hi = to_dev(np.array([-0.1])), to_dev(np.array([0.1]))
    r_lo = torch.full((int(offs[-1]),), np.nan, dtype=torch.float64, device="cuda")
    r_hi = torch.full_like(r_lo, np.nan)
    qs = [R.make_query(R.REACH_RD, ns[k], (1.0,), R.REACH_F64, x_lo.data_ptr() + 8 * int(offs[k]),
                       x_hi.data_ptr() + 8 * int(offs[k]), r_lo.data_ptr() + 8 * int(offs[k]),
                       r_hi.data_ptr() + 8 * int(offs[k]), 0.1, steps[k], p_lo, p_hi, n_in=1)
          for k in range(nq)]
    nb = R.reach_batch_workspace_bytes(nq)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with options(rc, {"batch.pack": 1, "batch.E": cap}):
        plan = R.reach_plan_batch(rc.ctx, qs, with_E=True)
        assert all(E for E, _ in plan)
        say(f"packs with 0-5 steps, cap {cap}")
        R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
        assert rc.sync() == R.REACH_OK
    got_lo, got_hi = to_host(r_lo), to_host(r_hi)
    for k in range(nq):
        a, e = int(offs[k]), int(offs[k + 1])
        if steps[k] == 0:
            assert np.array_equal(got_lo[a:e], lo[a:e]) and np.array_equal(got_hi[a:e], hi[a:e])
            continue
        if k % 5:
            continue
        a_lo, a_hi = rc.embed(R.REACH_RD, (1.0,), x_lo[a:e].contiguous(), x_hi[a:e].contiguous(),
                              0.1, steps[k], p_lo=p_lo, p_hi=p_hi)
        assert rc.sync() == R.REACH_OK
        assert np.array_equal(got_lo[a:e], to_host(a_lo)), f"query {k} n={ns[k]}"
        assert np.array_equal(got_hi[a:e], to_host(a_hi)), f"query {k} n={ns[k]}"


def test_plan_follows_the_split_option(rc, mix):
    """With batch.split = 1 the batch runs one side per wave: no packs."""
    qs = mix.queries()
    with options(rc, {"batch.pack": 1}):
        packed = R.reach_plan_batch(rc.ctx, qs)
        assert any(len(it) > 1 for it in packed)
    with options(rc, {"batch.pack": 1, "batch.split": 1}):
        plan = R.reach_plan_batch(rc.ctx, qs)
    assert all(len(it) == 1 for it in plan)
    assert sorted(it[0] for it in plan) == list(range(len(qs)))


def test_batch_autotune_keeps_results_bitwise(rc, tmp_path, monkeypatch):
    """reach_autotune_batch times every (kind, size) bucket of a 6000-query mix
    at each pack width and the whole batch at two or three wave counts; the batch after
    tuning gives the same boxes bit for bit, its plan keeps to the tuned
    widths, and a context created later reads the widths back from
    REACH_AUTOTUNE_CACHE and plans the same packs."""
    b = Batch(workloads.query_stream(6000, 5.0e4, seed=31))
    qs = b.queries()
    nb = R.reach_batch_workspace_bytes(len(qs))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    say("batch 6000 before tuning")
    R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert rc.sync() == R.REACH_OK
    ref = b.results()
    say("batch autotune")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("REACH_AUTOTUNE_CACHE", str(cache))
    tuner = R.Reach(0)
    try:
        best = R.reach_autotune_batch(tuner.ctx, qs, ws, nb, 0)
        assert tuner.sync() == R.REACH_OK
        tuned_plan = R.reach_plan_batch(tuner.ctx, qs, with_E=True)
    finally:
        tuner.close()
    assert any(l.startswith("reach2 batch ") for l in cache.read_text().splitlines())
    later = R.Reach(0)
    try:
        assert R.reach_plan_batch(later.ctx, qs, with_E=True) == tuned_plan
    finally:
        later.close()
    monkeypatch.delenv("REACH_AUTOTUNE_CACHE")
    best = R.reach_autotune_batch(rc.ctx, qs, ws, nb, 0)
    assert rc.sync() == R.REACH_OK
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert best["waves"] in (12 * cus, 8 * cus, 4 * cus) and best["batch_ns"] > 0
    plan = R.reach_plan_batch(rc.ctx, qs, with_E=True)
    assert any(E for E, _ in plan), "a 6000-query batch packs"
    b.clear()
    say("batch 6000 after tuning")
    R.reach_embed_rk4_batch(rc.ctx, qs, ws, nb, 0)
    assert rc.sync() == R.REACH_OK
    got = b.results()
    for k in range(len(ref)):
        assert np.array_equal(got[k][0], ref[k][0]) and np.array_equal(got[k][1], ref[k][1]), k
