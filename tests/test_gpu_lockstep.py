"""Lockstep batched refinement (qm_refine_lockstep): instances of uneven size
and of different classes per round advance together, one launch per phase
per round over all of them.  Each result must be bit-identical to the same
instance refined alone (and, for small ones, to the oracle); per-instance
options and failures stay per instance."""
import numpy as np
import pytest

import oracle
import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu


def canon(t):
    t = np.sort(np.asarray(t), axis=1)
    return t[np.lexsort(t.T[::-1])]


def canon_tri(tri, fid):
    a = np.concatenate([np.sort(np.asarray(tri), axis=1), np.asarray(fid).reshape(-1, 1)], axis=1)
    return a[np.lexsort(a.T[::-1])]


def same(a, b):
    ok = (a.rounds == b.rounds and a.status == b.status and np.array_equal(a.rstats, b.rstats)
          and np.array_equal(a.xyz.view(np.uint64), b.xyz.view(np.uint64))
          and np.array_equal(canon(a.tets), canon(b.tets))
          and np.array_equal(canon_tri(a.sf, a.sf_facet), canon_tri(b.sf, b.sf_facet))
          and np.array_equal(canon_tri(a.ss, a.ss_seg), canon_tri(b.ss, b.ss_seg)))
    if ok and a.last_cands is not None and b.last_cands is not None:
        ok = np.array_equal(a.last_cands, b.last_cands)
    return ok


def ellipsoid_instance(seed, n, B=2.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = rng.uniform(0.15, 0.40, size=3)
    rot = qi.quat_rotation(rng.standard_normal(4))
    return qi.make_workload(f"ls_{seed}_{n}", qi.uniform_interior(rng, n), B, [qi.ellipsoid_inside(axes, rot)])


@pytest.fixture(scope="module")
def mix():
    spec = [(300, 2.0), (2500, 1.4), (800, 2.0), (6000, 2.0), (150, 1.4), (1200, 2.0), (4000, 1.4), (500, 2.0),
            (9000, 1.4), (60, 2.0)]
    ws = [ellipsoid_instance(700 + i, n, B) for i, (n, B) in enumerate(spec)]
    ws.append(qi.uniform_cube(1000, seed=1, B=2.0))                 # hull-only instance
    ws.append(qi.uniform_cube(900, seed=4, B=1.5, spheres=(0.3,)))
    return ws


def test_lockstep_matches_single_instances(mix):
    print(f"[lockstep] {len(mix)} instances", flush=True)
    got = qm.refine_lockstep(mix)
    for w, g in zip(mix, got):
        s = qm.refine_workload(w)
        print(f"[lockstep] {w.name}: rounds={g.rounds} steiner={g.steiner} | alone rounds={s.rounds}", flush=True)
        assert same(g, s), w.name


def test_lockstep_groups_match_single_instances(mix):
    """The batch split into lockstep groups on streams of their own."""
    for groups in (3, 12):
        got = qm.refine_lockstep(mix, groups=groups)
        for w, g in zip(mix, got):
            assert same(g, qm.refine_workload(w)), (groups, w.name)
    got, codes = qm.refine_lockstep(mix[:4], groups=2, extra_flags=[0, qm.QM_PROFILE, 0, 0], return_codes=True)
    assert codes == [0, -1, 0, 0] and got[1] is None


def test_lockstep_knobs_do_not_change_results(mix):
    """Launch-shape knobs at their extremes (one classification tile per
    workgroup, radix sorts from 257 candidates, every selection over many
    workgroups, the fewest hybrid and global workgroups) and the knobs the
    autotuner picks give the single runs' results."""
    alone = [qm.refine_workload(w) for w in mix]
    extreme = {"groups": 2, "classify_tiles": 1, "rank_max": 256, "select_one_wg": 0, "hybrid_wgs": 16,
               "global_wgs": 4}
    for k, g in enumerate(qm.refine_lockstep(mix, tune=extreme)):
        assert same(g, alone[k]), ("extreme", mix[k].name)
    tune, sec = qm.lockstep_autotune(mix, probe=6)
    print(f"[lockstep] autotuned knobs {tune} ({sec:.2f}s for the probe)", flush=True)
    assert 1 <= tune["groups"] <= 8 and 256 <= tune["rank_max"] <= 4096
    for k, g in enumerate(qm.refine_lockstep(mix, tune=tune)):
        assert same(g, alone[k]), ("tuned", mix[k].name)


def test_lockstep_small_instances_match_oracle(mix):
    small = [w for w in mix if len(w.xyz) <= 1300]
    got = qm.refine_lockstep(small)
    for w, g in zip(small, got):
        assert same(g, oracle.refine(w)), w.name


def test_lockstep_with_a_large_instance(mix):
    """The 50K-point workload beside small ones: its rounds take the
    per-instance paths (radix sort, device-wide scans, selection in batches
    of passes) while the small instances share the batched launches; the
    result matches the oracle's digests."""
    import json
    import os
    import hashlib
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2.json")))
    w2 = qi.config(2)
    got = qm.refine_lockstep([mix[0], w2, mix[4], mix[7]])
    g = got[1]
    t = np.sort(np.asarray(g.tets, dtype=np.int32), axis=1)
    t = t[np.lexsort(t.T[::-1])]
    dig = hashlib.sha256(np.ascontiguousarray(t).tobytes()).hexdigest()
    print(f"[lockstep] config2 in a batch: rounds={g.rounds} nv={len(g.xyz)} nt={len(g.tets)} "
          f"| oracle rounds={gold['rounds']} nv={gold['nv']} nt={gold['nt']}", flush=True)
    assert g.rounds == gold["rounds"] and len(g.xyz) == gold["nv"] and len(g.tets) == gold["nt"]
    assert dig == gold["tets_sha256"]
    assert hashlib.sha256(np.ascontiguousarray(np.asarray(g.xyz, dtype=np.float64)).tobytes()).hexdigest() == \
        gold["xyz_sha256"]
    for k in (0, 2, 3):
        assert same(got[k], qm.refine_workload([mix[0], None, mix[4], mix[7]][k])), k


def test_lockstep_per_instance_options_and_failures(mix):
    """Round limits, larger grow tiers, forced equal keys, refused options,
    a bad input and a raised error word, each on one instance of a batch:
    the others are unaffected, and each finished one equals its single run
    with the same options."""
    ws = [mix[1], mix[2], mix[3], mix[5], mix[0], mix[7], mix[4], mix[6]]
    bad = qi.Workload(mix[0].name, mix[0].xyz.copy(), mix[0].tets, mix[0].adj, mix[0].ftri, mix[0].ftri_facet,
                      mix[0].seg, mix[0].B)
    bad.xyz[9, 0] = 0.1                                    # off the 2^-53 lattice
    ws[4] = bad
    flags = [0, qm.QM_TEST_TIER1, qm.QM_TEST_TIER2, qm.QM_TEST_KEY_COLLIDE, 0, qm.QM_PROFILE,
             qm.QM_TEST_ERROR_WORD, 0]
    rounds = [25, 100000, 100000, 100000, 100000, 100000, 100000, 100000]
    got, codes = qm.refine_lockstep(ws, extra_flags=flags, max_rounds=rounds, return_codes=True)
    print(f"[lockstep] per-instance codes: {codes}", flush=True)
    assert codes == [-4, 0, 0, 0, -1, -1, -6, 0]
    assert got[4] is None and got[5] is None and got[6] is None
    for k in (0, 1, 2, 3, 7):
        s = qm.refine_workload(ws[k], extra_flags=flags[k], max_rounds=rounds[k])
        assert same(got[k], s), k
    assert got[0].status == 1 and got[0].rounds == 25


def test_lockstep_edge_cases(mix):
    """An empty batch, a batch of one, and a batch whose every instance
    fails at set-up."""
    assert qm.refine_lockstep([]) == []
    one = qm.refine_lockstep([mix[9]])[0]
    assert same(one, qm.refine_workload(mix[9]))
    got, codes = qm.refine_lockstep([mix[9], mix[0]], extra_flags=[qm.QM_EARLY_STOP, qm.QM_PROFILE_GROW],
                                    return_codes=True)
    assert codes == [-1, -1] and got == [None, None]


def test_lockstep_repeated_small_batches(mix):
    """Regression: the host staging of the instance tables must not reuse a
    pinned region whose copy to the device has not run yet (a rewind at the
    start of a round without a synchronisation let the next round's table
    replace the insertion table).  Several batches in a row, each equal to
    the single runs."""
    small = [w for w in mix if len(w.xyz) <= 1300]
    alone = [qm.refine_workload(w) for w in small]
    for rep in range(5):
        got, codes = qm.refine_lockstep(small, return_codes=True)
        print(f"[lockstep] repeat {rep}: codes {codes}", flush=True)
        assert codes == [0] * len(small)
        for w, g, s in zip(small, got, alone):
            assert same(g, s), (rep, w.name)


def test_lockstep_many_parts_and_chunked_launches():
    """300 small instances in one group: launches of more than 64 parts
    (the second ballot of the part search) and of more than 256 (split into
    several launches per phase); and the same in two groups."""
    ws = [qi.uniform_cube(12 + (7 * i) % 40, seed=1000 + i, B=2.0, spheres=((0.3,) if i % 3 == 0 else ()))
          for i in range(300)]
    alone = [qm.refine_workload(w) for w in ws]
    for groups in (1, 2):
        got = qm.refine_lockstep(ws, groups=groups)
        bad = [w.name for w, g, s in zip(ws, got, alone) if not same(g, s)]
        print(f"[lockstep] 300 instances, {groups} group(s): {len(bad)} differ", flush=True)
        assert not bad, bad[:5]
