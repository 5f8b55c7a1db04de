"""Rectangle PLCs (the kind of input of the paper's experiments, Section 3
and Table 1: gamma * n rectangles among n points), each rectangle split in
advance so that the Delaunay tetrahedralisation conforms.  Large planar
facets of many triangles and chains of collinear segments go through every
class of the round loop.  Small inputs must match the oracle bit for bit;
a larger one must give a conforming CDT with its facet areas kept, the same
on a second run and in a lockstep batch."""
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
    return (a.rounds == b.rounds and a.status == b.status and np.array_equal(a.rstats, b.rstats)
            and np.array_equal(a.xyz.view(np.uint64), b.xyz.view(np.uint64))
            and np.array_equal(canon(a.tets), canon(b.tets))
            and np.array_equal(canon_tri(a.sf, a.sf_facet), canon_tri(b.sf, b.sf_facet))
            and np.array_equal(canon_tri(a.ss, a.ss_seg), canon_tri(b.ss, b.ss_seg)))


SMALL = [(200, 0.1, "uniform", 1.4), (400, 0.05, "uniform", 1.4), (120, 0.25, "uniform", 1.4)]


@pytest.mark.parametrize("n,gamma,dist,B", SMALL)
def test_rectangles_match_the_oracle(n, gamma, dist, B):
    w = qi.rectangles_plc(n, gamma, seed=11, dist=dist, B=B)
    g = qm.refine_workload(w)
    o = oracle.refine(w)
    print(f"[rect] {w.name}: {len(w.xyz)} vertices, {w.meta['rectangles']} rectangles; rounds {g.rounds} "
          f"(oracle {o.rounds}), steiner {g.steiner}", flush=True)
    assert g.status == o.status == 0
    assert same(g, o)


def test_rectangles_in_a_lockstep_batch():
    ws = [qi.rectangles_plc(n, gamma, seed=11, dist=dist, B=B) for n, gamma, dist, B in SMALL]
    got = qm.refine_lockstep(ws)
    for w, g in zip(ws, got):
        assert same(g, qm.refine_workload(w)), w.name


def test_larger_rectangle_plc_is_a_conforming_cdt():
    w = qi.rectangles_plc(20000, 0.1, seed=12, dist="gauss", B=1.4)
    g = qm.refine_workload(w)
    print(f"[rect] {w.name}: {len(w.xyz)} vertices, {w.meta['rectangles']} rectangles; rounds {g.rounds}, "
          f"steiner {g.steiner}, {g.seconds_refine:.3f}s", flush=True)
    assert g.status == 0
    c = oracle.check(g.xyz, g.tets, g.sf, g.ss, g.ss_seg, w.B)
    for k in ("neg_orient", "face_overuse", "hull_not_subface", "nonlocal_delaunay", "sf_missing", "ss_missing",
              "chain_broken"):
        assert c[k] == 0, (k, c)
    assert c["euler"] == 1 and abs(c["volume"] - 1.0) < 1e-9
    a0 = oracle.facet_areas(w.xyz, w.ftri, w.ftri_facet)
    a1 = oracle.facet_areas(g.xyz, g.sf, g.sf_facet)
    assert set(a0) == set(a1) and max(abs(a0[k] - a1[k]) / a0[k] for k in a0) < 1e-9
    g2 = qm.refine_workload(w)
    assert same(g, g2)
