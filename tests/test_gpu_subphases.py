"""Three-sub-phase rounds (QM_SUBPHASE_ROUNDS, the other reading of the class order): each
round runs a subsegment, a subface and a bad-tet sub-phase in turn, so the
insertion order differs from the paper-order refinement.  It equals, bit
for bit, the oracle refined with the same reading of the class order
(``oracle.refine(..., subphases=True)``) on inputs the oracle finishes in
seconds; at larger sizes it must be reproducible, converge, and be a CDT
conforming to the PLC (every non-subface face locally Delaunay, every
subface a face, every subsegment an edge, segment chains intact, facet areas
kept) and a valid tetrahedralisation of the cube (orientation, face use,
Euler characteristic, volume)."""
import numpy as np
import pytest

import oracle
import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu


def clustered(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ng = 9 * n // 10
    pts = np.concatenate([qi.gaussmix_interior(rng, ng), qi.uniform_interior(rng, n - ng)])
    return qi.make_workload(f"clustered_{n}", pts, 1.4, [qi.sphere_inside(r) for r in (0.15, 0.30, 0.45)])


def canon(t):
    t = np.sort(np.asarray(t), axis=1)
    return t[np.lexsort(t.T[::-1])]


@pytest.mark.parametrize("make", [lambda: qi.uniform_cube(1500, seed=6, B=2.0, spheres=(0.2, 0.35)),
                                  lambda: clustered(3000, 1579), lambda: qi.config(1), lambda: qi.config(2)])
def test_subphase_output_is_a_conforming_cdt(make):
    w = make()
    g = qm.refine_workload(w, subphases=True)
    p = qm.refine_workload(w)
    cls = np.bincount(g.rstats[:, 0], minlength=3) if g.rounds else np.zeros(3, int)
    print(f"[subphases] {w.name}: rounds {g.rounds} (SS {cls[0]}, SF {cls[1]}, TET {cls[2]}; parity {p.rounds}), "
          f"steiner {g.steiner} (parity {p.steiner}), {g.seconds_refine:.3f}s (parity {p.seconds_refine:.3f}s)",
          flush=True)
    assert g.status == 0
    c = oracle.check(g.xyz, g.tets, g.sf, g.ss, g.ss_seg, w.B)
    for k in ("neg_orient", "face_overuse", "hull_not_subface", "nonlocal_delaunay", "sf_missing", "ss_missing",
              "chain_broken"):
        assert c[k] == 0, (k, c)
    assert c["euler"] == 1 and abs(c["volume"] - 1.0) < 1e-9
    a0 = oracle.facet_areas(w.xyz, w.ftri, w.ftri_facet)
    a1 = oracle.facet_areas(g.xyz, g.sf, g.sf_facet)
    assert set(a0) == set(a1) and max(abs(a0[k] - a1[k]) / a0[k] for k in a0) < 1e-9
    assert np.array_equal(g.xyz[:len(w.xyz)].view(np.uint64), np.asarray(w.xyz).view(np.uint64))
    # reproducible: the order is fixed, only the within-round timing is free
    g2 = qm.refine_workload(w, subphases=True)
    assert g2.rounds == g.rounds and np.array_equal(g2.xyz.view(np.uint64), g.xyz.view(np.uint64))
    assert np.array_equal(canon(g2.tets), canon(g.tets))


def canon_tri(tri, fid):
    a = np.concatenate([np.sort(np.asarray(tri), axis=1), np.asarray(fid).reshape(-1, 1)], axis=1)
    return a[np.lexsort(a.T[::-1])]


@pytest.mark.parametrize("make", [lambda: qi.uniform_cube(600, seed=5, B=1.6, spheres=(0.25,)),
                                  lambda: qi.uniform_cube(900, seed=4, B=1.5, spheres=(0.3,)), lambda: qi.config(1)])
def test_subphase_mode_matches_the_oracle_reading(make):
    w = make()
    g = qm.refine_workload(w, subphases=True)
    o = oracle.refine(w, subphases=True)
    print(f"[subphases] {w.name}: rounds {g.rounds} (oracle {o.rounds}), steiner {g.steiner} "
          f"(oracle {len(o.xyz) - len(w.xyz)})", flush=True)
    assert g.status == o.status == 0
    assert g.rounds == o.rounds and np.array_equal(g.rstats, o.rstats)
    assert np.array_equal(g.xyz.view(np.uint64), o.xyz.view(np.uint64))
    assert np.array_equal(canon(g.tets), canon(o.tets))
    assert np.array_equal(canon_tri(g.sf, g.sf_facet), canon_tri(o.sf, o.sf_facet))
    assert np.array_equal(canon_tri(g.ss, g.ss_seg), canon_tri(o.ss, o.ss_seg))
