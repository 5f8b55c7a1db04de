"""The entry point without allocation (qm_refine_noalloc) against qm_refine:
the same output bit for bit (tets as sorted vertex tuples, Steiner
coordinates bitwise, subfaces and subsegments with their ids, rounds and
insertions), on two calls in a row, the second on a smaller input, and an
undersized output refused cleanly without disturbing the next call."""
import numpy as np
import pytest

import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu


def canon(t, ids=None):
    t = np.sort(np.asarray(t), axis=1)
    if ids is not None:
        t = np.concatenate([t, np.asarray(ids).reshape(-1, 1)], axis=1)
    return t[np.lexsort(t.T[::-1])]


def buffers(cv, ct, csf, css):
    import torch
    f = lambda shape, dt: torch.full(shape, -7, dtype=dt, device="cuda")   # stale values on purpose
    return {"xyz": f((cv, 3), torch.float64), "tet": f((ct, 4), torch.int32), "sf": f((csf, 3), torch.int32),
            "sf_facet": f((csf,), torch.int32), "ss": f((css, 2), torch.int32), "ss_seg": f((css,), torch.int32)}


def run_noalloc(w, ref, slack=64):
    out = buffers(len(ref.xyz) + slack, len(ref.tets) + slack, len(ref.sf) + slack, len(ref.ss) + slack)
    sizes, st = qm.refine_noalloc(w, out)
    g = {k: out[k][:sizes[n]].cpu().numpy() for k, n in
         (("xyz", "nv"), ("tet", "nt"), ("sf", "nsf"), ("sf_facet", "nsf"), ("ss", "nss"), ("ss_seg", "nss"))}
    return g, st


def assert_same(g, st, ref, label):
    print(f"[noalloc] {label}: rounds={st['rounds']} nv={len(g['xyz'])} nt={len(g['tet'])} | "
          f"qm_refine rounds={ref.rounds} nv={len(ref.xyz)} nt={len(ref.tets)}", flush=True)
    assert st["rounds"] == ref.rounds and st["status"] == ref.status
    assert st["inserted"] == ref.inserted and st["candidates"] == ref.candidates
    assert g["xyz"].shape == ref.xyz.shape
    assert np.array_equal(g["xyz"].view(np.uint64), ref.xyz.view(np.uint64)), "Steiner coordinates differ"
    assert np.array_equal(canon(g["tet"]), canon(ref.tets)), "tet sets differ"
    assert np.array_equal(canon(g["sf"], g["sf_facet"]), canon(ref.sf, ref.sf_facet)), "subfaces differ"
    assert np.array_equal(canon(g["ss"], g["ss_seg"]), canon(ref.ss, ref.ss_seg)), "subsegments differ"


def test_noalloc_matches_refine_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    big = qi.config(1)
    small = qi.uniform_cube(300, seed=21, B=1.5, spheres=(0.3,))
    for w, label in ((big, "1K-point cube"), (small, "300 points, one sphere")):
        ref = qm.refine_workload(w)
        g, st = run_noalloc(w, ref)
        assert_same(g, st, ref, label)


def test_noalloc_refuses_small_outputs_then_runs():
    import torch
    torch.cuda.set_device(0)
    w = qi.uniform_cube(200, seed=5, B=1.6, spheres=(0.25,))
    ref = qm.refine_workload(w)
    out = buffers(len(ref.xyz) + 8, len(w.tets), len(ref.sf) + 8, len(ref.ss) + 8)   # tets: input size only
    with pytest.raises(qm.QmError, match="QM_ECAPACITY"):
        qm.refine_noalloc(w, out)
    g, st = run_noalloc(w, ref)
    assert_same(g, st, ref, "after a refused call")
