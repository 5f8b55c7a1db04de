"""Pins for the oracle: its predicates, constructions and round rule checked
against independent statements of the mathematics (exact rationals,
closed forms, global Delaunay emptiness, conservation laws)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import qm_inputs as qi


# ---------------------------------------------------------------- helpers
def fr3(p):
    return [Fr(float(x)) for x in p]


def det_gauss(m):
    """Determinant by fraction Gaussian elimination (independent of any
    cofactor formula)."""
    m = [row[:] for row in m]
    n, sign, d = len(m), 1, Fr(1)
    for c in range(n):
        piv = next((r for r in range(c, n) if m[r][c] != 0), None)
        if piv is None:
            return Fr(0)
        if piv != c:
            m[c], m[piv] = m[piv], m[c]
            sign = -sign
        d *= m[c][c]
        for r in range(c + 1, n):
            f = m[r][c] / m[c][c]
            for k in range(c, n):
                m[r][k] -= f * m[c][k]
    return sign * d


def sgn(x):
    return (x > 0) - (x < 0)


def solve(A, b):
    """Solve A x = b in fractions (Cramer through det_gauss)."""
    D = det_gauss(A)
    out = []
    for i in range(len(A)):
        Ai = [row[:] for row in A]
        for r in range(len(A)):
            Ai[r][i] = b[r]
        out.append(det_gauss(Ai) / D)
    return out


def exact_orient3d(a, b, c, d):
    a, b, c, d = map(fr3, (a, b, c, d))
    return sgn(det_gauss([[b[k] - a[k] for k in range(3)], [c[k] - a[k] for k in range(3)],
                          [d[k] - a[k] for k in range(3)]]))


def exact_sphere_centre(a, b, c, d):
    a, b, c, d = map(fr3, (a, b, c, d))
    A = [[2 * (p[k] - a[k]) for k in range(3)] for p in (b, c, d)]
    rhs = [sum(p[k] * p[k] - a[k] * a[k] for k in range(3)) for p in (b, c, d)]
    return solve(A, rhs)


def exact_insphere(a, b, c, d, e):
    """+1 inside, 0 on, -1 outside: distance to the exact centre."""
    cen = exact_sphere_centre(a, b, c, d)
    A, E = fr3(a), fr3(e)
    r2 = sum((A[k] - cen[k]) ** 2 for k in range(3))
    q2 = sum((E[k] - cen[k]) ** 2 for k in range(3))
    return sgn(r2 - q2)


def exact_tri_centre(a, b, c):
    a, b, c = map(fr3, (a, b, c))
    u = [b[k] - a[k] for k in range(3)]
    w = [c[k] - a[k] for k in range(3)]
    uu = sum(x * x for x in u); ww = sum(x * x for x in w); uw = sum(x * y for x, y in zip(u, w))
    s, t = solve([[2 * uu, 2 * uw], [2 * uw, 2 * ww]], [uu, ww])
    return [a[k] + s * u[k] + t * w[k] for k in range(3)]


def exact_face_encroach(a, b, c, v):
    """-1 when v is strictly inside the equatorial ball (the sign convention
    of the oracle's facedot), +1 outside, 0 on the sphere."""
    cen = exact_tri_centre(a, b, c)
    A, V = fr3(a), fr3(v)
    return sgn(sum((V[k] - cen[k]) ** 2 for k in range(3)) - sum((A[k] - cen[k]) ** 2 for k in range(3)))


def exact_seg_encroach(a, b, v):
    A, B, V = map(fr3, (a, b, v))
    m = [(A[k] + B[k]) / 2 for k in range(3)]
    half2 = sum((B[k] - A[k]) ** 2 for k in range(3)) / 4
    return sgn(sum((V[k] - m[k]) ** 2 for k in range(3)) - half2)


def lattice_points(rng, n, mode):
    if mode == "uniform":
        return rng.random((n, 3))
    if mode == "grid":      # many exact degeneracies (coplanar, cospherical)
        return rng.integers(0, 4, size=(n, 3)) / 4.0
    if mode == "nudged":    # grid points moved by one lattice step
        g = rng.integers(0, 4, size=(n, 3)) / 4.0
        return g + rng.integers(-1, 2, size=(n, 3)) * 2.0 ** -53 * (g > 0)
    raise ValueError(mode)


MODES = ["uniform", "grid", "nudged"]


# -------------------------------------------------------------- predicates
@pytest.mark.parametrize("mode", MODES)
def test_orient3d_exact(mode):
    rng = np.random.default_rng(11)
    for _ in range(300):
        p = lattice_points(rng, 4, mode)
        assert oracle.orient3d(*p) == exact_orient3d(*p)


def test_orient3d_far_points():
    rng = np.random.default_rng(12)
    for _ in range(100):
        p = rng.random((4, 3))
        p[3] = qi.snap(p[3] * 1e12 - 5e11)
        assert oracle.orient3d(*p) == exact_orient3d(*p)


def test_orient3d_unit_tet_is_positive():
    assert oracle.orient3d([0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]) == 1
    assert oracle.orient3d([0, 0, 0], [0, 1, 0], [1, 0, 0], [0, 0, 1]) == -1


@pytest.mark.parametrize("mode", MODES)
def test_insphere_exact(mode):
    rng = np.random.default_rng(13)
    n = 0
    while n < 200:
        p = lattice_points(rng, 5, mode)
        o = exact_orient3d(*p[:4])
        if o == 0:
            continue
        if o < 0:
            p[[0, 1]] = p[[1, 0]]
        assert oracle.insphere(*p) == exact_insphere(*p)
        n += 1


def test_insphere_cube_corners_cospherical():
    c = qi.corners()
    # every corner lies on the sphere through any four non-coplanar corners
    for tet in ([0, 1, 2, 4], [1, 2, 4, 7], [0, 3, 5, 6]):
        t = c[tet]
        if oracle.orient3d(*t) < 0:
            t = t[[1, 0, 2, 3]]
        for q in range(8):
            if q not in tet:
                assert oracle.insphere(*t, c[q]) == 0


@pytest.mark.parametrize("mode", MODES)
def test_orient2d_exact(mode):
    rng = np.random.default_rng(14)
    for _ in range(300):
        p = lattice_points(rng, 3, mode)
        ax = int(rng.integers(0, 3))
        i, j = (ax + 1) % 3, (ax + 2) % 3
        a, b, c = map(fr3, p)
        want = sgn(det_gauss([[b[i] - a[i], b[j] - a[j]], [c[i] - a[i], c[j] - a[j]]]))
        assert oracle.orient2d(ax, *p) == want


@pytest.mark.parametrize("mode", MODES)
def test_seg_encroach_exact(mode):
    rng = np.random.default_rng(15)
    for _ in range(300):
        p = lattice_points(rng, 3, mode)
        assert oracle.segdot(*p) == exact_seg_encroach(*p)


@pytest.mark.parametrize("mode", MODES)
def test_face_encroach_exact(mode):
    rng = np.random.default_rng(16)
    n = 0
    while n < 200:
        p = lattice_points(rng, 4, mode)
        a, b, c = map(fr3, p[:3])
        u = [b[k] - a[k] for k in range(3)]; w = [c[k] - a[k] for k in range(3)]
        if u[1] * w[2] - u[2] * w[1] == 0 and u[2] * w[0] - u[0] * w[2] == 0 and u[0] * w[1] - u[1] * w[0] == 0:
            continue                      # collinear triangle: no circle
        assert oracle.facedot(*p) == exact_face_encroach(*p)
        n += 1


def test_encroach_closed_forms():
    a, b = [0, 0, 0], [1, 0, 0]
    assert oracle.segdot(a, b, [0.5, 0.4, 0]) < 0       # inside the diametral ball
    assert oracle.segdot(a, b, [0.5, 0.5, 0]) == 0      # on the sphere
    tri = ([0, 0, 0], [1, 0, 0], [0, 1, 0])
    assert oracle.facedot(*tri, [1, 1, 0]) == 0         # fourth square corner: cocircular
    assert oracle.facedot(*tri, [0.5, 0.5, 0.5]) < 0    # |v-c|^2 = 1/4 < R^2 = 1/2
    assert oracle.facedot(*tri, [0.5, 0.5, 1.0]) > 0    # |v-c|^2 = 1 > 1/2


# ----------------------------------------------------------- constructions
def test_tet_circumcentre_closed_form():
    p, r2 = oracle.tet_cc([0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1])
    assert list(p) == [0.5, 0.5, 0.5] and r2 == 0.75


def test_tri_circumcentre_closed_form():
    assert list(oracle.tri_cc([0, 0, 0], [1, 0, 0], [0, 1, 0])) == [0.5, 0.5, 0.0]


def test_axis_plane_constructions_stay_on_plane():
    rng = np.random.default_rng(17)
    for _ in range(200):
        p = rng.random((3, 3))
        p[:, 2] = 1.0
        assert oracle.tri_cc(*p)[2] == 1.0
        assert oracle.midpoint(p[0], p[1])[2] == 1.0


def test_radius_edge_closed_forms():
    unit = ([0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1])     # ratio sqrt(3)/2 ~ 0.866
    assert not oracle.is_bad(*unit, 0.87) and oracle.is_bad(*unit, 0.86)
    reg = ([0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1])      # regular: sqrt(6)/4 ~ 0.612
    assert not oracle.is_bad(*reg, 0.613) and oracle.is_bad(*reg, 0.612)
    needle = ([0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, qi.snap(1e-3)])
    assert oracle.is_bad(*needle, 2.0)
    sliver = ([0, 0, 0], [1, 0, 0], [1, 1, 2.0 ** -20], [0, 1, 0])  # flat square: ratio -> sqrt(2)/2
    assert not oracle.is_bad(*sliver, 0.75)


def test_circumcentres_match_exact_rationals():
    rng = np.random.default_rng(18)
    for _ in range(100):
        p = rng.random((4, 3))
        c, _ = oracle.tet_cc(*p)
        ex = exact_sphere_centre(*p)
        for k in range(3):
            assert abs(Fr(float(c[k])) - ex[k]) <= Fr(1, 10 ** 9) * (1 + abs(ex[k]))
        t = oracle.tri_cc(*p[:3])
        ex = exact_tri_centre(*p[:3])
        for k in range(3):
            assert abs(Fr(float(t[k])) - ex[k]) <= Fr(1, 10 ** 9) * (1 + abs(ex[k]))


def test_midpoint_rounding():
    rng = np.random.default_rng(19)
    for _ in range(200):
        a, b = rng.random((2, 3))
        m = oracle.midpoint(a, b)
        for k in range(3):
            assert abs(Fr(float(m[k])) - (Fr(float(a[k])) + Fr(float(b[k]))) / 2) <= Fr(1, 2 ** 54)
            assert (Fr(float(m[k])) * 2 ** 53).denominator == 1     # on the lattice


def test_priority_key_is_splitmix64():
    # first output of SplitMix64 from state 0 (published reference value)
    assert oracle.key(0, [0]) == 0xE220A8397B1DCDAF


# ------------------------------------------------------------ the round rule
def struct_ok(c):
    keys = ("neg_orient", "face_overuse", "hull_not_subface", "sf_missing", "ss_missing", "chain_broken")
    return all(c[k] == 0 for k in keys) and c["euler"] == 1 and abs(c["volume"] - 1.0) < 1e-9


def test_config1_refinement_is_delaunay_and_conforming():
    w = qi.config(1)
    r = oracle.refine(w)
    assert r.status == 0                                   # no candidates left
    c = oracle.check(r.xyz, r.tets, r.sf, r.ss, r.ss_seg, w.B)
    assert struct_ok(c) and c["nonlocal_delaunay"] == 0
    assert oracle.check_global(r.xyz, r.tets) == 0
    a0 = oracle.facet_areas(w.xyz, w.ftri, w.ftri_facet)
    a1 = oracle.facet_areas(r.xyz, r.sf, r.sf_facet)
    assert set(a0) == set(a1) and max(abs(a0[k] - a1[k]) for k in a0) < 1e-12
    # every remaining bad tet was exempted (the exemption counters bound them)
    assert c["bad_tets"] <= int(r.rstats[:, 6:15].sum())
    # Steiner points on the hull stay exactly on their cube face
    hull = r.sf[r.sf_facet < 6]
    for f, axis_side in zip(hull, r.sf_facet[r.sf_facet < 6]):
        assert np.all(r.xyz[f, axis_side // 2] == float(axis_side % 2))


@pytest.mark.parametrize("n,seed,B", [(60, 1, 1.2), (150, 2, 1.6), (300, 3, 2.0)])
def test_hull_only_delaunay_after_every_round(n, seed, B):
    w = qi.uniform_cube(n, seed=seed, B=B)
    full = oracle.refine(w)
    for m in sorted(set(np.linspace(1, full.rounds, 6).astype(int))):
        r = oracle.refine(w, max_rounds=int(m))
        c = oracle.check(r.xyz, r.tets, r.sf, r.ss, r.ss_seg, B)
        assert struct_ok(c) and c["nonlocal_delaunay"] == 0
        assert oracle.check_global(r.xyz, r.tets) == 0


def test_sequential_special_case_is_delaunay():
    """One insertion per round is textbook sequential Delaunay refinement:
    the mesh stays the Delaunay tetrahedralisation of its vertices."""
    w = qi.uniform_cube(80, seed=5, B=1.5)
    r = oracle.refine(w, max_kept=1)
    assert r.status == 0 and np.all(r.rstats[:, 5] <= 1)
    assert oracle.check_global(r.xyz, r.tets) == 0
    c = oracle.check(r.xyz, r.tets, r.sf, r.ss, r.ss_seg, w.B)
    assert struct_ok(c)


@pytest.mark.parametrize("n,seed,B,spheres", [(120, 3, 1.5, (0.3,)), (250, 8, 1.5, (0.3,)),
                                              (300, 4, 1.4, (0.2, 0.35))])
def test_surface_refinement_is_cdt_after_every_round(n, seed, B, spheres):
    """Section 2: the triangulation is a CDT at the end of every round.  With
    every subface a face of the mesh, a CDT is exactly a mesh whose
    non-subface faces are all locally Delaunay (constrained Delaunay lemma),
    which qmo_check counts independently of the refinement code.  The inputs
    have internal constraint surfaces, where a cavity can wrap around a
    constraint edge."""
    w = qi.uniform_cube(n, seed=seed, B=B, spheres=spheres)
    r = oracle.refine(w, round_checks=True)
    assert r.status == 0 and r.rounds > 50
    rc = dict(zip(oracle.CHECK_FIELDS, r.round_checks.T))
    for k in ("neg_orient", "face_overuse", "hull_not_subface", "nonlocal_delaunay", "sf_missing",
              "ss_missing", "chain_broken"):
        assert np.all(rc[k] == 0), (k, np.nonzero(rc[k])[0][:5])
    assert np.all(rc["euler"] == 1)


@pytest.mark.parametrize("n,seed", [(120, 7), (250, 8)])
def test_surface_refinement_conforms(n, seed):
    w = qi.uniform_cube(n, seed=seed, B=1.5, spheres=(0.3,))
    assert len(w.ftri) > 12
    r = oracle.refine(w)
    assert r.status == 0
    c = oracle.check(r.xyz, r.tets, r.sf, r.ss, r.ss_seg, w.B)
    assert struct_ok(c) and c["nonlocal_delaunay"] == 0
    a0 = oracle.facet_areas(w.xyz, w.ftri, w.ftri_facet)
    a1 = oracle.facet_areas(r.xyz, r.sf, r.sf_facet)
    assert set(a0) == set(a1)
    assert max(abs(a0[k] - a1[k]) / max(a0[k], 1e-300) for k in a0) < 1e-9
    # every segment is still a chain of subsegments between its endpoints
    assert c["chain_broken"] == 0 and set(r.ss_seg.tolist()) == set(range(len(w.seg)))


def canon(r):
    t = np.sort(r.tets, axis=1)
    t = t[np.lexsort(t.T[::-1])]
    return t, r.xyz


def test_canonical_under_input_permutation():
    """No decision depends on slot order: shuffling the tets and rotating
    each tet's vertices (even permutations) leaves the output unchanged."""
    w = qi.uniform_cube(150, seed=9, B=1.4, spheres=(0.3,))
    r1 = oracle.refine(w)
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(w.tets))
    even = np.array([[0, 1, 2, 3], [1, 2, 0, 3], [2, 0, 1, 3], [1, 0, 3, 2], [0, 2, 3, 1],
                     [2, 3, 0, 1], [3, 2, 1, 0], [0, 3, 1, 2]])
    rot = even[rng.integers(0, len(even), size=len(w.tets))]
    w2 = qi.Workload(w.name, w.xyz, np.take_along_axis(w.tets[perm], rot, axis=1), w.adj,
                     w.ftri, w.ftri_facet, w.seg, w.B)
    r2 = oracle.refine(w2)
    t1, x1 = canon(r1)
    t2, x2 = canon(r2)
    assert np.array_equal(t1, t2) and np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
    assert np.array_equal(r1.rstats, r2.rstats)


def test_deterministic_rerun():
    w = qi.uniform_cube(100, seed=4, B=1.5, spheres=(0.3,))
    a, b = oracle.refine(w), oracle.refine(w)
    assert np.array_equal(canon(a)[0], canon(b)[0]) and np.array_equal(a.rstats, b.rstats)


# ---------------------------------------------- brute-force region and selection
def _mesh_state(w, rounds):
    """The oracle's mesh at the start of round `rounds` (after that many)."""
    r = oracle.refine(w, max_rounds=rounds)
    tets = [tuple(int(x) for x in t) for t in r.tets]
    sfs = {tuple(sorted(int(x) for x in f)): int(F) for f, F in zip(r.sf, r.sf_facet)}
    sss = {tuple(sorted(int(x) for x in e)) for e in r.ss}
    faces = {}
    for i, t in enumerate(tets):
        for f in range(4):
            faces.setdefault(tuple(sorted(t[:f] + t[f + 1:])), []).append(i)
    return r.xyz, tets, sfs, sss, faces


def _brute_region(c, xyz, tets, sfs, sss, faces):
    """Section 2's Delaunay region of candidate c, by brute force: R_F from
    the seed subfaces (the facet region's definition), then every tet whose
    circumsphere strictly holds p and that is connected to the seeds across
    faces that are not subfaces (or are R_F subfaces)."""
    p = c["p"]
    q4 = lambda i: tuple(sorted(tets[i]))
    inside = [oracle.insphere(*(xyz[v] for v in t), p) > 0 for t in tets]
    rf = []
    if c["cls"] == 0:
        a, b = c["tup"]
        seeds = [i for i, t in enumerate(tets) if a in t and b in t]
        rf = [f for f in sfs if a in f and b in f]
    elif c["cls"] == 1:
        rf = [c["rf"][0]]                      # the located subface (its walk is pinned elsewhere)
    else:
        seeds = [i for i, t in enumerate(tets) if q4(i) == c["region"][0]]
    if c["cls"] != 2:                          # grow R_F within each subface's facet
        k = 0
        while k < len(rf):
            g = rf[k]; k += 1
            for x, y in ((g[0], g[1]), (g[0], g[2]), (g[1], g[2])):
                if (x, y) in sss:
                    continue
                for h in sfs:
                    if h != g and x in h and y in h and sfs[h] == sfs[g] and h not in rf:
                        if oracle.facedot(*(xyz[v] for v in h), p) < 0:
                            rf.append(h)
        if c["cls"] == 1:
            seeds = []
        for g in rf:
            seeds += faces[g]
    region, todo = set(), list(dict.fromkeys(seeds))
    region.update(todo)
    while todo:
        i = todo.pop()
        t = tets[i]
        for f in range(4):
            fk = tuple(sorted(t[:f] + t[f + 1:]))
            if fk in sfs and fk not in rf:
                continue
            for n in faces[fk]:
                if n != i and n not in region and inside[n]:
                    region.add(n); todo.append(n)
    claims = set(region)
    for i in region:
        t = tets[i]
        for f in range(4):
            fk = tuple(sorted(t[:f] + t[f + 1:]))
            if fk in rf:
                continue
            claims.update(n for n in faces[fk] if n not in region)
    return {q4(i) for i in region}, sorted(rf), {q4(i) for i in claims}


@pytest.mark.parametrize("n,seed,B,spheres", [(40, 3, 1.5, (0.3,)), (55, 8, 1.3, (0.25,)), (50, 11, 1.6, ())])
def test_regions_and_selection_match_brute_force(n, seed, B, spheres):
    """For the first round of each class: every candidate's region (R_F and
    R_T) and claim set equal the brute-force construction from Section 2's
    definitions, and the kept points are exactly the greedy maximal set of
    pairwise disjoint claim sets in priority order (key descending, then
    ascending tuple)."""
    w = qi.uniform_cube(n, seed=seed, B=B, spheres=spheres)
    full = oracle.refine(w)
    cls = full.rstats[:, 0]
    firsts = [int(np.argmax(cls == k)) for k in range(3) if (cls == k).any()]
    assert len(firsts) >= 2
    checked = 0
    for r in firsts:
        xyz, tets, sfs, sss, faces = _mesh_state(w, r)
        d = oracle.refine(w, max_rounds=r + 1, dump_round=r).dump
        assert d and all(c["cls"] == cls[r] for c in d)
        # priority order
        assert [(-c["key"], c["tup"]) for c in d] == sorted((-c["key"], c["tup"]) for c in d)
        for c in d:
            if not c["region"]:                # rejected or exempted by the walk, nothing grown
                continue
            reg, rf, claims = _brute_region(c, xyz, tets, sfs, sss, faces)
            assert reg == set(c["region"]), (r, c["tup"])
            assert rf == sorted(c["rf"]), (r, c["tup"])
            if c["status"] == 0:
                assert claims == set(c["claims"]), (r, c["tup"])
            checked += 1
        # the greedy maximal disjoint set
        taken, kept = set(), []
        for c in d:
            ok = c["status"] == 0 and not (set(c["claims"]) & taken)
            if ok:
                taken |= set(c["claims"])
            kept.append(int(ok))
        assert kept == [c["kept"] for c in d]
    assert checked > 20


def test_priority_key_of_longer_tuples():
    """Keys of 2-4 ids chain SplitMix64's finaliser: key(cls, ids) is the
    finaliser applied to (previous key XOR next id), starting from the
    generator's state increment times (cls + 1).  The reference generator
    below is SplitMix64's published definition; its first outputs are
    checked against the published reference values first."""
    M = (1 << 64) - 1
    G = 0x9E3779B97F4A7C15

    def mix(z):                                # SplitMix64 output function
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)
    state, outs = 0, []
    for _ in range(3):
        state = (state + G) & M
        outs.append(mix(state))
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    for cls in range(3):
        assert oracle.key(cls, [0]) == outs[cls]
        for ids in ([5, 9], [1, 2, 3], [7, 11, 13, 1 << 20], [2000000, 3, 4, 5]):
            h = (G * (cls + 1)) & M
            for i in ids:
                h = mix(h ^ i)
            assert oracle.key(cls, ids) == h
    assert oracle.key(2, [1, 2, 3, 4]) != oracle.key(2, [1, 2, 4, 3])


@pytest.mark.parametrize("n,seed,B,spheres", [(120, 4, 1.5, (0.3,)), (300, 6, 1.8, ())])
def test_equal_keys_are_ordered_by_tuple(n, seed, B, spheres):
    """With every key cut to its top 3 bits (many equal keys) the round's
    candidates still come in key-descending, tuple-ascending order, and the
    refinement still ends in a valid CDT."""
    w = qi.uniform_cube(n, seed=seed, B=B, spheres=spheres)
    mask = 0xE000000000000000
    full = oracle.refine(w, key_mask=mask)
    assert full.status == 0
    c = oracle.check(full.xyz, full.tets, full.sf, full.ss, full.ss_seg, B)
    assert struct_ok(c) and c["nonlocal_delaunay"] == 0
    big = int(np.argmax(full.rstats[:, 1]))
    d = oracle.refine(w, max_rounds=big + 1, dump_round=big, key_mask=mask).dump
    keys = [c["key"] for c in d]
    assert all(k & ~mask == 0 for k in keys) and len(set(keys)) < len(keys)
    assert [(-c["key"], c["tup"]) for c in d] == sorted((-c["key"], c["tup"]) for c in d)


def test_subphase_reading_keeps_a_cdt_after_every_round():
    """The sub-phase reading of the class order (every round takes the
    three classes in turn) on surface inputs: after every round the mesh is
    a conforming CDT and a valid tetrahedralisation (the independently
    pinned mesh checks), the refinement converges, and its first round is
    the paper-order first round (both begin with the encroached
    subsegments)."""
    for w in (qi.uniform_cube(250, seed=8, B=1.5, spheres=(0.3,)), qi.uniform_cube(400, seed=3, B=2.0,
                                                                                  spheres=(0.2, 0.35))):
        a = oracle.refine(w, subphases=True, round_checks=True)
        b = oracle.refine(w, max_rounds=1)
        assert a.status == 0 and a.rounds > 0
        rc = a.round_checks
        for k, name in enumerate(oracle.CHECK_FIELDS):
            if name == "euler":
                assert (rc[:, k] == 1).all(), name
            elif name != "bad_tets":
                assert (rc[:, k] == 0).all(), (w.name, name)
        assert np.array_equal(a.rstats[0], b.rstats[0])
        # the classes of consecutive rounds follow the cyclic order SS, SF, TET
        # (a class without candidates is passed over)
        cls = a.rstats[:, 0]
        assert cls[0] == 0 and set(np.unique(cls)) <= {0, 1, 2}


def test_rectangle_plc_refinement_keeps_a_cdt_every_round():
    """The oracle on a rectangle PLC (large planar facets of many triangles,
    collinear segment chains): after every round the mesh is a conforming
    CDT and a valid tetrahedralisation (the independently pinned mesh
    checks); the refinement converges and keeps every facet's area."""
    w = qi.rectangles_plc(200, 0.1, seed=11, B=1.4)
    o = oracle.refine(w, round_checks=True)
    assert o.status == 0 and o.rounds > 0
    rc = o.round_checks
    for k, name in enumerate(oracle.CHECK_FIELDS):
        if name == "euler":
            assert (rc[:, k] == 1).all()
        elif name != "bad_tets":
            assert (rc[:, k] == 0).all(), name
    a0 = oracle.facet_areas(w.xyz, w.ftri, w.ftri_facet)
    a1 = oracle.facet_areas(o.xyz, o.sf, o.sf_facet)
    assert set(a0) == set(a1) and max(abs(a0[k] - a1[k]) / a0[k] for k in a0) < 1e-12


def test_resume_from_the_state_equals_the_uninterrupted_run():
    """What the round rule carries beyond the mesh is exactly the queued and
    exempt flags and h_min: a run stopped by the round guard and started
    again from its output mesh and that state gives the uninterrupted run
    (round records, point bits, tets), in both readings of the class order;
    with the flags cleared it is a different refinement at some cut."""
    import types

    def canon(t):
        t = np.sort(np.asarray(t), axis=1)
        return t[np.lexsort(t.T[::-1])]

    w = qi.uniform_cube(400, seed=3, B=2.0, spheres=(0.2, 0.35))
    differ = 0
    for sub in (False, True):
        full = oracle.refine(w, subphases=sub)
        assert full.state.rounds == full.rounds
        for k in (1, 9, full.rounds // 2, full.rounds - 1):
            a = oracle.refine(w, max_rounds=k, subphases=sub)
            assert a.status == 1 and a.state.rounds == k
            m = types.SimpleNamespace(xyz=a.xyz, tets=a.tets, sf=a.sf, sf_facet=a.sf_facet, ss=a.ss,
                                      ss_seg=a.ss_seg, ftri=w.ftri, ftri_facet=w.ftri_facet, B=w.B)
            b = oracle.refine(m, state=a.state, subphases=sub)
            assert b.status == 0 and b.state.rounds == full.rounds
            assert np.array_equal(np.concatenate([a.rstats, b.rstats]), full.rstats), (sub, k)
            assert np.array_equal(b.xyz.view(np.uint64), full.xyz.view(np.uint64))
            assert np.array_equal(canon(b.tets), canon(full.tets))
            st = a.state
            clear = oracle.OracleState(st.hmin2, st.rounds, st.next_class, np.zeros_like(st.tet_flags),
                                       np.zeros_like(st.sf_flags), np.zeros_like(st.ss_flags))
            c = oracle.refine(m, state=clear, subphases=sub)
            differ += not (c.rounds == b.rounds and np.array_equal(c.xyz.view(np.uint64), b.xyz.view(np.uint64)))
    assert differ > 0


def test_oracle_behind_the_library_call_layout():
    """qm_oracle_refine takes the arguments the GPU library's refine call
    takes (qm_plc, qm_mesh, qm_options, marshalled once by the binding) and
    answers with its codes, so a test can hand one argument set to either
    engine.  Its results equal the oracle's own runs, option flags included,
    and its refusals are the library's."""
    import paper_1903_03406_amd as qm
    w = qi.uniform_cube(300, seed=2, B=1.6, spheres=(0.3,))
    keep = []
    plc, mesh = qm._marshal(w, keep)

    def run(flags=0, max_rounds=100000, B=None):
        return oracle.refine_call(plc, mesh, qm._Opts(float(w.B if B is None else B), 0.5, max_rounds, 0, flags))

    for flags, ref in ((0, oracle.refine(w)), (qm.QM_SUBPHASE_ROUNDS, oracle.refine(w, subphases=True)),
                       (qm.QM_TEST_KEY_COLLIDE, oracle.refine(w, key_mask=0xE000000000000000)),
                       (qm.QM_PROFILE | qm.QM_OUTPUT_DEVICE, oracle.refine(w))):
        rc, o = run(flags)
        assert rc == 0 and o.rounds == ref.rounds and np.array_equal(o.rstats, ref.rstats)
        assert np.array_equal(o.xyz.view(np.uint64), ref.xyz.view(np.uint64))
        assert np.array_equal(np.sort(o.tets, axis=1), np.sort(ref.tets, axis=1))
    rc, o = run(max_rounds=5)
    assert rc == -4 and o.status == 1 and o.rounds == 5            # QM_EROUNDS, result returned
    assert run(qm.QM_EARLY_STOP)[0] == -1 and run(qm.QM_INPUT_DEVICE)[0] == -1 and run(B=0.0)[0] == -1
    flipped = w.tets.copy()
    flipped[0, [0, 1]] = flipped[0, [1, 0]]
    k2 = []
    p2, m2 = qm._marshal(qi.Workload(w.name, w.xyz, flipped, w.adj, w.ftri, w.ftri_facet, w.seg, w.B), k2)
    assert oracle.refine_call(p2, m2, qm._Opts(w.B, 0.5, 100, 0, 0))[0] == -2      # QM_ENONCONFORM
    xyz = w.xyz.copy()
    xyz[9, 0] = 0.1                                                  # off the 2^-53 lattice
    k3 = []
    p3, m3 = qm._marshal(qi.Workload(w.name, xyz, w.tets, w.adj, w.ftri, w.ftri_facet, w.seg, w.B), k3)
    assert oracle.refine_call(p3, m3, qm._Opts(w.B, 0.5, 100, 0, 0))[0] == -1      # QM_EINVAL
