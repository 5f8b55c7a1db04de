"""Batched refinement (qm_refine_batch): instances of uneven size run
concurrently on several streams; each result must be bit-identical to the
same instance refined alone (and, for small ones, to the oracle)."""
import numpy as np
import pytest

import oracle
import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu


def canon(t):
    t = np.sort(np.asarray(t), axis=1)
    return t[np.lexsort(t.T[::-1])]


def same(a, b):
    return (a.rounds == b.rounds and np.array_equal(a.rstats, b.rstats)
            and np.array_equal(a.xyz.view(np.uint64), b.xyz.view(np.uint64))
            and np.array_equal(canon(a.tets), canon(b.tets)))


def ellipsoid_instance(seed, n):
    """An instance of the batched workload's generator at a chosen size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = rng.uniform(0.15, 0.40, size=3)
    rot = qi.quat_rotation(rng.standard_normal(4))
    return qi.make_workload(f"ellipsoid_{seed}_{n}", qi.uniform_interior(rng, n), 2.0,
                            [qi.ellipsoid_inside(axes, rot)])


@pytest.fixture(scope="module")
def instances():
    sizes = [300, 2500, 800, 6000, 150, 1200, 4000, 500]
    return [ellipsoid_instance(100 + i, n) for i, n in enumerate(sizes)]


def test_batch_matches_single_instances(instances):
    got = qm.refine_batch(instances, nstreams=4)
    for w, g in zip(instances, got):
        s = qm.refine_workload(w)
        print(f"[batch] {w.name}: rounds={g.rounds} steiner={g.steiner}", flush=True)
        assert same(g, s), w.name


def test_batch_small_instances_match_oracle(instances):
    small = [w for w in instances if len(w.xyz) <= 900]
    got = qm.refine_batch(small, nstreams=3)
    for w, g in zip(small, got):
        o = oracle.refine(w)
        assert same(g, o), w.name


def test_batch_reports_failing_instance(instances):
    w = instances[0]
    bad = qi.Workload(w.name, w.xyz.copy(), w.tets, w.adj, w.ftri, w.ftri_facet, w.seg, w.B)
    bad.xyz[9, 0] = 0.1                 # off the 2^-53 lattice
    with pytest.raises(qm.QmError, match="EINVAL"):
        qm.refine_batch([instances[1], bad, instances[2]], nstreams=2)
    # the library is still usable afterwards
    g = qm.refine_batch([instances[4]], nstreams=1)[0]
    assert same(g, qm.refine_workload(instances[4]))


def test_error_word_is_per_call(instances):
    """A call whose device error word is raised (test flag) fails alone: the
    next call in the process, and instances running beside it in a batch,
    return QM_OK with their normal output."""
    w = instances[0]
    with pytest.raises(qm.QmError, match="EINTERNAL"):
        qm.refine_workload(w, extra_flags=qm.QM_TEST_ERROR_WORD)
    assert same(qm.refine_workload(w), oracle.refine(w))
    trio = [instances[1], instances[2], instances[3]]
    got, codes = qm.refine_batch(trio, nstreams=3, extra_flags=[0, qm.QM_TEST_ERROR_WORD, 0],
                                 return_codes=True)
    print(f"[batch] error word: codes={codes}", flush=True)
    assert codes == [0, -6, 0] and got[1] is None
    assert same(got[0], qm.refine_workload(trio[0])) and same(got[2], qm.refine_workload(trio[2]))
