"""Eviction of served jobs (qm_server_evict, qm_server_readmit): a job taken
off the device at a round boundary keeps its mesh and refinement state on the
host, frees its share of the budget, and resumes when admitted again.  The
result it finally gives (round records of every segment, mesh, statistics)
must equal the instance refined alone, in the worker and the stepped form."""
import time

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
    return (a.rounds == b.rounds and a.status == b.status and np.array_equal(a.rstats, b.rstats)
            and np.array_equal(a.xyz.view(np.uint64), b.xyz.view(np.uint64))
            and np.array_equal(canon(a.tets), canon(b.tets))
            and np.array_equal(canon(a.sf), canon(b.sf)) and np.array_equal(canon(a.ss), canon(b.ss))
            and tuple(a.inserted) == tuple(b.inserted) and a.candidates == b.candidates
            and a.mis_passes == b.mis_passes)


def ellipsoid_instance(seed, n, B=2.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = rng.uniform(0.15, 0.40, size=3)
    rot = qi.quat_rotation(rng.standard_normal(4))
    return qi.make_workload(f"ev_{seed}_{n}", qi.uniform_interior(rng, n), B, [qi.ellipsoid_inside(axes, rot)])


@pytest.fixture(scope="module")
def big():
    w = ellipsoid_instance(399, 30000, 1.5)
    return w, qm.refine_workload(w)


@pytest.fixture(scope="module")
def small():
    ws = [ellipsoid_instance(500 + i, n, B) for i, (n, B) in enumerate([(400, 1.4), (1500, 2.0), (150, 2.0)])]
    return ws, [qm.refine_workload(w) for w in ws]


def wait_running(srv, n=1, limit=60.0):
    t0 = time.time()
    while srv.info()["running"] < n:
        assert time.time() - t0 < limit, "the job never started"
        time.sleep(0.002)


def test_worker_form_evicts_a_running_job_and_resumes_it(big, small):
    w, alone = big
    print(f"[evict] {w.name}: alone {alone.rounds} rounds, {alone.seconds_refine:.3f}s", flush=True)
    with qm.Server(8 * GiB, nworkers=2) as srv:
        t = srv.submit(w)
        evictions = 0
        for pause in (0.03, 0.05):
            wait_running(srv)
            time.sleep(pause)
            if not srv.evict(t):
                break                                  # it finished first
            evictions += 1
            info = srv.info()
            assert info["parked"] == 1 and info["resident"] == 0
            assert srv.poll(t) is None                 # an evicted job has no result
            ws, ref = small
            ts = srv.submit(ws[0])                     # another job runs meanwhile
            assert same(srv.result(ts), ref[0])
            assert srv.readmit(t)
        got = srv.result(t)
        info = srv.info()
    print(f"[evict] {w.name}: {evictions} evictions, {got.rounds} rounds", flush=True)
    assert evictions >= 1 and info["evictions"] == evictions and info["parked"] == 0
    assert same(got, alone)


def test_worker_form_evicts_a_queued_job(big, small):
    w, alone = big
    ws, ref = small
    with qm.Server(8 * GiB, nworkers=1) as srv:
        ta = srv.submit(w)
        tb = srv.submit(ws[1])                         # waits behind the big job
        assert srv.evict(tb)
        assert srv.info()["parked"] == 1
        got_a = srv.result(ta)
        assert srv.readmit(tb)
        got_b = srv.result(tb)
    assert same(got_a, alone) and same(got_b, ref[1])


def test_eviction_frees_the_budget(big, small):
    """Stepped form, so that nothing finishes between the calls: the big
    job's estimate leaves the budget when it is evicted, and it is admitted
    again only when there is room."""
    w, alone = big
    ws, ref = small
    est_big = qm.estimate_bytes(w)
    est_small = qm.estimate_bytes(ws[1])
    with qm.Server(est_big + est_small // 2, nworkers=0) as srv:
        t = srv.submit(w)
        srv.step()
        srv.step()
        assert srv.submit(ws[1]) is None               # no room beside the big job
        assert srv.evict(t)
        assert srv.info()["resident"] == 0
        ts = srv.submit(ws[1])
        assert ts is not None
        assert not srv.readmit(t)                      # no room beside the small job
        while srv.step() > 0:
            pass
        got_s = srv.result(ts)
        assert srv.readmit(t)
        while srv.step() > 0:
            pass
        got = srv.result(t)
    assert same(got_s, ref[1]) and same(got, alone)


def test_stepped_form_eviction(big, small):
    w, alone = big
    ws, ref = small
    with qm.Server(8 * GiB, nworkers=0) as srv:
        tb = srv.submit(w)
        ts = [srv.submit(x) for x in ws]
        tq = ts[2]
        assert srv.evict(tq)                           # admitted, not yet in a batch
        for _ in range(5):
            srv.step()
        assert srv.evict(tb)                           # resident: taken out between steps
        info = srv.info()
        assert info["parked"] == 2
        for _ in range(3):
            srv.step()                                 # the others go on meanwhile
        assert srv.readmit(tb) and srv.readmit(tq)
        steps = 0
        while srv.step() > 0:
            steps += 1
        got = [srv.result(t) for t in ts]
        got_b = srv.result(tb)
        print(f"[evict] stepped: {steps} steps after the readmission", flush=True)
    for g, r in zip(got, ref):
        assert same(g, r)
    assert same(got_b, alone)


def test_eviction_errors(small):
    ws, ref = small
    with qm.Server(8 * GiB, nworkers=1) as srv:
        with pytest.raises(qm.QmError, match="EINVAL"):
            srv.evict(12345)
        t = srv.submit(ws[2])
        with pytest.raises(qm.QmError, match="EINVAL"):
            srv.readmit(t)                             # not evicted
        g = srv.result(t)
        with pytest.raises(qm.QmError, match="EINVAL"):
            srv.evict(t)                               # collected
        t2 = srv.submit(ws[2])
        if srv.evict(t2):                              # queued or running; else it finished first
            with pytest.raises(qm.QmError, match="EINVAL"):
                srv.evict(t2)                          # already evicted
            assert srv.readmit(t2)
        g2 = srv.result(t2)
    assert same(g, ref[2]) and same(g2, ref[2])
