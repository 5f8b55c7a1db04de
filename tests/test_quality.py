"""Quality reports: radius-edge ratio and dihedral angles against closed
forms (regular tet, trirectangular corner tet)."""
import numpy as np

from paper_1903_03406_amd import quality as q

REG = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
CORNER = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
T = np.array([[0, 1, 2, 3]])


def test_regular_tet():
    # circumradius sqrt(3), edge 2*sqrt(2): ratio sqrt(6)/4; every dihedral arccos(1/3)
    assert np.isclose(q.radius_edge(REG, T)[0], np.sqrt(6) / 4)
    assert np.allclose(q.dihedral_angles(REG, T), np.degrees(np.arccos(1 / 3)))


def test_corner_tet():
    # circumcentre (1/2,1/2,1/2): radius sqrt(3)/2 over shortest edge 1
    assert np.isclose(q.radius_edge(CORNER, T)[0], np.sqrt(3) / 2)
    d = np.sort(q.dihedral_angles(CORNER, T)[0])
    # three right angles at the corner's edges, three of arccos(1/sqrt(3)) at the far face
    assert np.allclose(d[:3], np.degrees(np.arccos(1 / np.sqrt(3))))
    assert np.allclose(d[3:], 90.0)


def test_invariance_and_report():
    rng = np.random.default_rng(5)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    moved = 3.0 * CORNER @ R.T + 0.25
    assert np.isclose(q.radius_edge(moved, T)[0], q.radius_edge(CORNER, T)[0])
    assert np.allclose(np.sort(q.dihedral_angles(moved, T)[0]), np.sort(q.dihedral_angles(CORNER, T)[0]))
    r = q.report(np.vstack([REG, CORNER]), np.array([[0, 1, 2, 3], [4, 5, 6, 7]]), B=0.7)
    assert r["over_B"] == 1 and sum(r["dihedral_hist"]["counts"]) == 12
