"""Profiling modes leave the refinement unchanged: QM_PROFILE (every kernel
family, region counters) and QM_PROFILE_GROW (only the small-tile and
hybrid-tier grow launches, timed with HIP events) give the same output bits
as an unprofiled call, and the grow-only mode counts the same grow
launches."""
import numpy as np
import pytest

import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu


def canon(t):
    t = np.sort(np.asarray(t), axis=1)
    return t[np.lexsort(t.T[::-1])]


def test_profiling_modes_do_not_change_the_result():
    w = qi.uniform_cube(3000, seed=21, B=1.5, spheres=(0.3,))
    plain = qm.refine_workload(w)
    full = qm.refine_workload(w, profile=True)
    grow = qm.refine_workload(w, profile="grow")
    for r in (full, grow):
        assert r.rounds == plain.rounds and np.array_equal(r.rstats, plain.rstats)
        assert np.array_equal(r.xyz.view(np.uint64), plain.xyz.view(np.uint64))
        assert np.array_equal(canon(r.tets), canon(plain.tets))
    assert plain.profile is None
    fams = ("grow_validate", "grow_hybrid")
    for fam in fams:
        assert grow.profile["launches"][fam] == full.profile["launches"][fam]
    assert grow.profile["launches"]["grow_validate"] > 0 and grow.profile["ms"]["grow_validate"] > 0.0
    others = [k for k in qm.PROF_FAMILIES if k not in fams]
    assert all(grow.profile["ms"][k] == 0.0 and grow.profile["launches"][k] == 0 for k in others)
    assert grow.profile["tested"] == 0 and full.profile["tested"] > 0
    assert full.profile["round_ms"].shape[0] >= full.rounds
