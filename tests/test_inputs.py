"""The seeded workload generator: Delaunay input, PLC structure."""
import numpy as np
import pytest

import oracle
import qm_inputs as qi


@pytest.mark.parametrize("n,seed", [(30, 1), (500, 2), (2000, 3)])
def test_delaunay_is_empty_sphere(n, seed):
    w = qi.uniform_cube(n, seed=seed)
    assert oracle.check_global(w.xyz, w.tets) == 0
    c = oracle.check(w.xyz, w.tets, w.sf, w.ss, w.ss_seg, w.B)
    assert c["neg_orient"] == 0 and c["face_overuse"] == 0 and c["euler"] == 1
    assert c["hull_not_subface"] == 0 and abs(c["volume"] - 1) < 1e-12


def test_delaunay_independent_of_point_order_within_ties():
    """The generator's symbolic perturbation makes the result a function of
    the point set and ids only: rebuilding gives the same tets."""
    w = qi.uniform_cube(400, seed=4)
    t2, _ = qi.delaunay(w.xyz)
    a = np.sort(np.sort(w.tets, axis=1), axis=0)
    b = np.sort(np.sort(t2, axis=1), axis=0)
    assert np.array_equal(a, b)


def test_workload_structure():
    w = qi.uniform_cube(200, seed=5, spheres=(0.3,))
    assert np.all(w.xyz[:8] == qi.corners())
    assert np.all((w.xyz[8:] > 0) & (w.xyz[8:] < 1))
    assert np.all(np.ldexp(w.xyz, 53) == np.rint(np.ldexp(w.xyz, 53)))     # lattice
    hull = w.ftri_facet < 6
    assert hull.sum() == 12 and np.bincount(w.ftri_facet[hull]).tolist() == [2] * 6
    assert len(w.seg) >= 12
    # each internal facet is one Delaunay face and its edges are segments
    segs = set(map(tuple, np.sort(w.seg, axis=1).tolist()))
    for tri in w.ftri[~hull]:
        a, b, c = sorted(tri.tolist())
        assert {(a, b), (a, c), (b, c)} <= segs


def test_configs_are_seeded():
    a, b = qi.config(1), qi.config(1)
    assert a.sha256() == b.sha256()
    assert len(a.xyz) == 1008


@pytest.mark.parametrize("n,gamma,dist", [(200, 0.1, "uniform"), (400, 0.25, "uniform"), (1500, 0.05, "gauss")])
def test_rectangle_plc_is_a_cdt(n, gamma, dist):
    """Rectangle PLCs (the kind of input of the paper's Table 1): gamma * n
    rectangles whose corners are PLC points, each split in advance by a
    jittered grid so that the Delaunay tetrahedralisation conforms.  A grid of
    (L+1)^2 points triangulates into exactly 2 L^2 Delaunay triangles and its
    sides into 4 L edges; the input is a Delaunay tetrahedralisation (global
    empty-sphere check), a valid CDT of its PLC (every subface a face, every
    subsegment an edge), and each rectangle's triangles tile its area."""
    w = qi.rectangles_plc(n, gamma, seed=5, dist=dist)
    L = w.meta["lattice"]
    nr = w.meta["rectangles"]
    assert nr == round(gamma * n)
    assert len(w.xyz) == 8 + (n - 4 * nr) + nr * (L + 1) ** 2
    assert len(w.ftri) == 12 + nr * 2 * L * L and len(w.seg) == 12 + nr * 4 * L
    for r in range(nr):
        assert np.count_nonzero(w.ftri_facet == 6 + r) == 2 * L * L
    assert oracle.check_global(w.xyz, w.tets) == 0
    c = oracle.check(w.xyz, w.tets, w.sf, w.ss, w.ss_seg, w.B)
    for k in ("neg_orient", "face_overuse", "hull_not_subface", "nonlocal_delaunay", "sf_missing", "ss_missing",
              "chain_broken"):
        assert c[k] == 0, (k, c)
    assert c["euler"] == 1 and abs(c["volume"] - 1.0) < 1e-12
    # every rectangle is planar (one coordinate shared by its triangles)
    for r in range(nr):
        p = w.xyz[w.ftri[w.ftri_facet == 6 + r]].reshape(-1, 3)
        assert sum(np.all(p[:, a] == p[0, a]) for a in range(3)) == 1
    assert qi.rectangles_plc(n, gamma, seed=5, dist=dist).sha256() == w.sha256()


def test_rectangle_plc_edge_cases():
    """No rectangles (gamma = 0: the cube PLC alone), every point a corner
    (gamma = 0.25), and refused parameters."""
    w = qi.rectangles_plc(100, 0.0, seed=3)
    assert w.meta["rectangles"] == 0 and len(w.xyz) == 108 and len(w.ftri) == 12 and len(w.seg) == 12
    w = qi.rectangles_plc(40, 0.25, seed=3)
    assert w.meta["rectangles"] == 10 and len(w.xyz) == 8 + 10 * 16
    assert oracle.check_global(w.xyz, w.tets) == 0
    with pytest.raises(ValueError):
        qi.rectangles_plc(10, 0.3, seed=3)             # more corners than points
    with pytest.raises(ValueError):
        qi.rectangles_plc(100, 0.1, seed=3, lattice=2)
    with pytest.raises(ValueError):
        qi.rectangles_plc(100, 0.1, seed=3, dist="ball")
