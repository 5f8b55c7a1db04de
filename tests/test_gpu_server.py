"""Served refinement (qm_server_*): jobs admitted against a device-memory
budget and run by worker threads on their own streams.  Every served result
must be bit-identical to the same instance refined alone; admission,
collection and shutdown follow the documented rules."""
import numpy as np
import pytest

import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def canon(t):
    t = np.sort(np.asarray(t), axis=1)
    return t[np.lexsort(t.T[::-1])]


def same(a, b):
    return (a.rounds == b.rounds and np.array_equal(a.rstats, b.rstats)
            and np.array_equal(a.xyz.view(np.uint64), b.xyz.view(np.uint64))
            and np.array_equal(canon(a.tets), canon(b.tets))
            and np.array_equal(canon(a.sf), canon(b.sf)) and np.array_equal(canon(a.ss), canon(b.ss)))


def ellipsoid_instance(seed, n, B=2.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = rng.uniform(0.15, 0.40, size=3)
    rot = qi.quat_rotation(rng.standard_normal(4))
    return qi.make_workload(f"srv_{seed}_{n}", qi.uniform_interior(rng, n), B,
                            [qi.ellipsoid_inside(axes, rot)])


@pytest.fixture(scope="module")
def jobs():
    spec = [(7000, 2.0), (400, 1.4), (2500, 2.0), (1200, 1.4), (150, 2.0), (3500, 1.4)]
    return [ellipsoid_instance(300 + i, n, B) for i, (n, B) in enumerate(spec)]


@pytest.fixture(scope="module")
def big():
    return ellipsoid_instance(399, 30000, 1.5)


def test_served_jobs_match_single_instances(jobs):
    with qm.Server(8 * GiB, nworkers=3) as srv:
        tickets = [srv.submit(w) for w in jobs]
        assert all(t is not None for t in tickets)
        got = [srv.result(t) for t in tickets]
        info = srv.info()
    assert info["admitted"] == len(jobs) and info["completed"] == len(jobs)
    assert info["resident"] == 0 and info["queued"] == 0 and info["running"] == 0
    for w, g in zip(jobs, got):
        s = qm.refine_workload(w)
        print(f"[server] {w.name}: rounds={g.rounds} steiner={g.steiner}", flush=True)
        assert same(g, s), w.name


def test_admission_against_the_budget(big, jobs):
    small = jobs[4]
    with qm.Server(GiB, nworkers=2) as srv:
        t_big = srv.submit(big, est_bytes=GiB)          # fills the budget
        assert t_big is not None
        assert srv.submit(small, est_bytes=1) is None   # no room until it ends
        assert srv.poll(t_big, wait_ms=0) is None       # still refining
        info = srv.info()
        assert info["refused"] == 1 and info["resident"] == GiB
        r_big = srv.result(t_big)
        assert srv.info()["resident"] == 0
        t_small = srv.submit(small, est_bytes=1)
        assert t_small is not None
        r_small = srv.result(t_small)
        with pytest.raises(qm.QmError, match="ENOMEM"):
            srv.submit(small, est_bytes=GiB + 1)         # never fits
    assert same(r_big, qm.refine_workload(big))
    assert same(r_small, qm.refine_workload(small))


def test_estimate_covers_the_job(jobs):
    """Every served job's own peak of device memory (its buffers, including
    the larger grow tiers' slab tiles, which shrink to the job's budget)
    stays within the estimate it was admitted with, also for a clustered job
    whose regions are large for its size."""
    rng = np.random.Generator(np.random.PCG64(77))
    pts = np.concatenate([qi.gaussmix_interior(rng, 9000), qi.uniform_interior(rng, 1000)])
    clustered = qi.make_workload("srv_clustered10k", pts, 1.4, [qi.sphere_inside(r) for r in (0.15, 0.30, 0.45)])
    with qm.Server(64 * GiB, nworkers=2) as srv:
        for w in jobs + [clustered]:
            est = srv.estimate_bytes(w)
            got = srv.result(srv.submit(w))
            print(f"[server] {w.name}: peak {got.device_bytes_peak >> 20} MiB, estimate {est >> 20} MiB",
                  flush=True)
            assert 0 < got.device_bytes_peak <= est, w.name
            assert same(got, qm.refine_workload(w)), w.name


def test_job_errors_and_tickets(jobs):
    w = jobs[4]
    bad = qi.Workload(w.name, w.xyz.copy(), w.tets, w.adj, w.ftri, w.ftri_facet, w.seg, w.B)
    bad.xyz[9, 0] = 0.1                                  # off the 2^-53 lattice
    with qm.Server(4 * GiB, nworkers=2) as srv:
        t = srv.submit(bad)
        res, code, msg, wait_s, total_s = srv.poll(t, wait_ms=-1)
        assert res is None and code == -1 and "lattice" in msg
        assert 0.0 <= wait_s <= total_s
        with pytest.raises(qm.QmError, match="EINVAL"):
            srv.poll(t)                                  # collected once
        with pytest.raises(qm.QmError, match="EINVAL"):
            srv.poll(12345)
        t2 = srv.submit(w)                               # the server still serves
        assert same(srv.result(t2), qm.refine_workload(w))


def test_shutdown_with_pending_jobs(jobs):
    srv = qm.Server(8 * GiB, nworkers=1)
    for w in jobs:
        assert srv.submit(w) is not None
    srv.close()                                          # drops queued, joins running
    with qm.Server(8 * GiB, nworkers=2) as srv2:
        t = srv2.submit(jobs[1])
        assert same(srv2.result(t), qm.refine_workload(jobs[1]))


def test_admission_under_pressure(jobs):
    """More jobs than the budget holds at once: submissions are refused
    while it is full and admitted as jobs finish; every job completes with
    the result it has alone, and the budget drains to zero."""
    budget = 3 * GiB
    order = [jobs[k % len(jobs)] for k in range(12)]
    done, pending, refused = {}, {}, 0
    with qm.Server(budget, nworkers=4) as srv:
        nxt = 0
        while nxt < len(order) or pending:
            while nxt < len(order):
                t = srv.submit(order[nxt], est_bytes=GiB)
                if t is None:
                    refused += 1
                    break
                assert srv.info()["resident"] <= budget
                pending[t] = nxt
                nxt += 1
            for t in list(pending):
                got = srv.poll(t, wait_ms=5)
                if got is not None:
                    res, code, _, _, _ = got
                    assert code in (0, -4)
                    done[pending.pop(t)] = res
        info = srv.info()
    assert refused > 0 and info["refused"] == refused
    assert info["admitted"] == len(order) == info["completed"] and info["resident"] == 0
    alone = {id(w): qm.refine_workload(w) for w in jobs}
    for k, w in enumerate(order):
        assert same(done[k], alone[id(w)]), (k, w.name)


def test_stepped_server_advances_one_round_per_step(jobs):
    """With no workers the server is stepped (qm_server_step): resident jobs
    stay on the device and each step runs one round of every one of them,
    so the jobs finish after as many steps as their rounds (plus the last
    classification, which finds no work), with the results they have alone.
    A job submitted between steps joins at the next one; a server destroyed
    with resident jobs stops them."""
    first, late = jobs[1:4], jobs[4]
    alone = {w.name: qm.refine_workload(w) for w in first + [late]}
    with qm.Server(8 * GiB, nworkers=0) as srv:
        tickets = {srv.submit(w): w for w in first}
        steps, t_late = 0, None
        while True:
            n = srv.step()
            steps += 1
            if steps == 3:
                t_late = srv.submit(late)
                tickets[t_late] = late
            if n == 0 and steps > 3:
                break
        got = {w.name: srv.result(t) for t, w in tickets.items()}
        with pytest.raises(qm.QmError, match="EINVAL"):
            qm.Server(GiB, nworkers=1).step()
    for name, g in got.items():
        assert same(g, alone[name]), name
    want = max(max(alone[w.name].rounds + 1 for w in first), 3 + alone[late.name].rounds + 1)
    print(f"[server] stepped: {steps} steps, expected {want}", flush=True)
    assert steps == want
    srv = qm.Server(8 * GiB, nworkers=0)
    srv.submit(jobs[0])
    srv.step()
    srv.step()
    srv.close()                                          # stops the resident job
    with qm.Server(8 * GiB, nworkers=0) as srv2:         # the device is usable afterwards
        t = srv2.submit(jobs[4])
        while srv2.step():
            pass
        assert same(srv2.result(t), alone[jobs[4].name])


def test_pipelined_server_matches_single_runs(jobs):
    """PipelinedServer: inputs built on host threads while others refine;
    each result equals the job refined alone, and a failing preparation
    ends only its own job."""
    specs = [(300 + i, n, B) for i, (n, B) in enumerate([(7000, 2.0), (400, 1.4), (2500, 2.0), (1200, 1.4)])]

    def bad():
        raise ValueError("no input")

    with qm.PipelinedServer(8 * GiB, nworkers=2, prep_threads=3) as srv:
        hs = [srv.submit(ellipsoid_instance, *sp) for sp in specs]
        hb = srv.submit(bad)
        got = [srv.result(h) for h in hs]
        res, code, msg, prep_s, total_s = srv.poll(hb, wait_ms=-1)
        assert res is None and "no input" in msg
    for g, w in zip(got, jobs[:4]):
        assert same(g, qm.refine_workload(w)), w.name
