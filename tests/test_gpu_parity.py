"""GPU parity: the HIP path against the oracle, bit for bit.

The output is combinatorial and every predicate is exact, so the tolerance
is zero: the same tets (as sorted vertex-id tuples), the same Steiner
coordinates bitwise, the same subfaces and subsegments with their facet and
segment ids, and the same per-round record (class, candidates, verdicts by
reason, insertions, sizes)."""
import os

import numpy as np
import pytest

import oracle
import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu


def canon_tets(t):
    t = np.sort(np.asarray(t), axis=1)
    return t[np.lexsort(t.T[::-1])]


def canon_tri(tri, fid):
    t = np.sort(np.asarray(tri), axis=1)
    a = np.concatenate([t, np.asarray(fid).reshape(-1, 1)], axis=1)
    return a[np.lexsort(a.T[::-1])]


def assert_same(g, o, label=""):
    print(f"[parity] {label}: gpu rounds={g.rounds} nv={len(g.xyz)} nt={len(g.tets)} | "
          f"oracle rounds={o.rounds} nv={len(o.xyz)} nt={len(o.tets)}", flush=True)
    assert g.rounds == o.rounds and g.status == o.status
    assert np.array_equal(g.rstats, o.rstats), "per-round records differ"
    assert g.xyz.shape == o.xyz.shape
    assert np.array_equal(g.xyz.view(np.uint64), o.xyz.view(np.uint64)), "Steiner coordinates differ"
    assert np.array_equal(canon_tets(g.tets), canon_tets(o.tets)), "tet sets differ"
    assert np.array_equal(canon_tri(g.sf, g.sf_facet), canon_tri(o.sf, o.sf_facet)), "subfaces differ"
    assert np.array_equal(canon_tri(g.ss, g.ss_seg), canon_tri(o.ss, o.ss_seg)), "subsegments differ"


def run_both(w, **kw):
    g = qm.refine_workload(w, **kw)
    o = oracle.refine(w, **kw)
    return g, o


def test_config1_parity():
    w = qi.config(1)
    g, o = run_both(w)
    assert_same(g, o, "config1")
    c = oracle.check(g.xyz, g.tets, g.sf, g.ss, g.ss_seg, w.B)
    assert c["nonlocal_delaunay"] == 0 and c["euler"] == 1


@pytest.mark.parametrize("n,seed,B", [(40, 1, 2.0), (200, 2, 1.4), (700, 3, 1.8)])
def test_hull_only_parity(n, seed, B):
    g, o = run_both(qi.uniform_cube(n, seed=seed, B=B))
    assert_same(g, o, f"hull n={n}")


@pytest.mark.parametrize("n,seed,B,spheres", [(150, 4, 1.5, (0.3,)), (600, 5, 1.6, (0.25,)),
                                              (1500, 6, 2.0, (0.2, 0.35))])
def test_surface_parity(n, seed, B, spheres):
    g, o = run_both(qi.uniform_cube(n, seed=seed, B=B, spheres=spheres))
    assert_same(g, o, f"surface n={n}")


def clustered_instance(n, seed):
    """A small instance of the 1M-point workload's generator: 90% of the
    points from 8 Gaussians, 10% uniform, three nested sphere surfaces,
    B = 1.4 (many small cavities next to the clusters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ng = 9 * n // 10
    pts = np.concatenate([qi.gaussmix_interior(rng, ng), qi.uniform_interior(rng, n - ng)])
    return qi.make_workload(f"clustered_{n}", pts, 1.4, [qi.sphere_inside(r) for r in (0.15, 0.30, 0.45)])


def test_clustered_instance_parity():
    w = clustered_instance(1500, 1577)
    g, o = run_both(w)
    assert o.rounds > 100 and len(o.xyz) > len(w.xyz) + 1000
    assert_same(g, o, "clustered 1500")
    # the served form runs the same refinement
    with qm.Server(4 << 30, nworkers=2) as srv:
        assert_same(srv.result(srv.submit(w)), o, "clustered 1500 served")


@pytest.mark.parametrize("flag,label", [(qm.QM_TEST_TIER1, "hybrid tier"),
                                        (qm.QM_TEST_TIER2, "global-memory tiles")])
def test_larger_tiers_parity(flag, label):
    """Every region grown by the hybrid tier (256-lane workgroups, hash
    tables in LDS, lists in global memory) or by the global-memory tier: the
    same output as the oracle, bit for bit."""
    for w in (qi.uniform_cube(300, seed=21, B=1.5, spheres=(0.3,)), clustered_instance(600, 1578)):
        g = qm.refine_workload(w, extra_flags=flag)
        assert_same(g, oracle.refine(w), f"{w.name} {label}")


@pytest.mark.parametrize("n,seed,B,spheres", [(120, 4, 1.5, (0.3,)), (300, 6, 1.8, ()), (1500, 6, 2.0, (0.2, 0.35))])
def test_equal_keys_parity(n, seed, B, spheres):
    """Keys cut to their top 3 bits on both sides: most keys are equal, so
    the order comes from the tie rule (ascending tuple) in the one-workgroup
    ranking of small rounds and in the sort's tie fix of large ones; the
    output still matches the oracle bit for bit."""
    w = qi.uniform_cube(n, seed=seed, B=B, spheres=spheres)
    o = oracle.refine(w, key_mask=0xE000000000000000)
    assert o.rstats[:, 1].max() > 256            # a round takes the sort path
    g = qm.refine_workload(w, extra_flags=qm.QM_TEST_KEY_COLLIDE)
    assert_same(g, o, f"equal keys n={n}")


def test_device_resident_output():
    """QM_OUTPUT_DEVICE: the output mesh stays in device memory; copied out,
    it equals the host result bit for bit."""
    w = qi.uniform_cube(600, seed=5, B=1.6, spheres=(0.25,))
    d, st = qm.refine_to_device(w)
    h = qm.refine_workload(w)
    assert all(t.is_cuda for t in d.values())
    assert st["rounds"] == h.rounds and st["nt_out"] == len(h.tets)
    assert np.array_equal(d["xyz"].cpu().numpy().view(np.uint64), h.xyz.view(np.uint64))
    assert np.array_equal(canon_tets(d["tets"].cpu().numpy()), canon_tets(h.tets))
    assert np.array_equal(canon_tri(d["sf"].cpu().numpy(), d["sf_facet"].cpu().numpy()),
                          canon_tri(h.sf, h.sf_facet))
    assert np.array_equal(canon_tri(d["ss"].cpu().numpy(), d["ss_seg"].cpu().numpy()), canon_tri(h.ss, h.ss_seg))


def test_ellipsoid_instance_parity():
    # a small instance of the batched workload's generator (rotated ellipsoid)
    rng = np.random.Generator(np.random.PCG64(44))
    axes = rng.uniform(0.15, 0.40, size=3)
    rot = qi.quat_rotation(rng.standard_normal(4))
    w = qi.make_workload("ellipsoid_small", qi.uniform_interior(rng, 2000), 2.0,
                         [qi.ellipsoid_inside(axes, rot)])
    g, o = run_both(w)
    assert_same(g, o, "ellipsoid 2000")


def test_sequential_special_case_parity():
    g, o = run_both(qi.uniform_cube(100, seed=8, B=1.5, spheres=(0.3,)), max_kept=1)
    assert_same(g, o, "max_kept=1")
    assert np.all(g.rstats[:, 5] <= 1)


def test_round_guard_parity():
    w = qi.uniform_cube(400, seed=9, B=1.4, spheres=(0.3,))
    g, o = run_both(w, max_rounds=7)
    assert g.status == 1 and g.rounds == 7
    assert_same(g, o, "max_rounds=7")


def test_empty_interior_and_no_work():
    # the eight corners alone: nothing is bad or encroached at B = 2
    w = qi.uniform_cube(0, seed=1, B=2.0)
    g, o = run_both(w)
    assert_same(g, o, "corners only")
    assert g.steiner == o.xyz.shape[0] - 8
    # a huge bound: only encroachment rounds can run
    w = qi.uniform_cube(300, seed=10, B=1e9)
    g, o = run_both(w)
    assert_same(g, o, "B=1e9")
    assert np.all(g.rstats[:, 0] != 2)


def test_rerun_is_deterministic():
    w = qi.uniform_cube(500, seed=11, B=1.5, spheres=(0.3,))
    a, b = qm.refine_workload(w), qm.refine_workload(w)
    assert np.array_equal(a.xyz.view(np.uint64), b.xyz.view(np.uint64))
    assert np.array_equal(canon_tets(a.tets), canon_tets(b.tets)) and np.array_equal(a.rstats, b.rstats)


def test_shuffled_input_gives_same_output():
    w = qi.uniform_cube(300, seed=12, B=1.5, spheres=(0.3,))
    rng = np.random.default_rng(1)
    perm = rng.permutation(len(w.tets))
    w2 = qi.Workload(w.name, w.xyz, w.tets[perm][:, [1, 2, 0, 3]], w.adj, w.ftri, w.ftri_facet, w.seg, w.B)
    a, b = qm.refine_workload(w), qm.refine_workload(w2)
    assert np.array_equal(canon_tets(a.tets), canon_tets(b.tets)) and np.array_equal(a.rstats, b.rstats)


def test_device_inputs_match_host_inputs():
    torch = pytest.importorskip("torch")
    w = qi.uniform_cube(300, seed=13, B=1.5, spheres=(0.3,))
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(w, k))).cuda()
           for k in ("xyz", "tets", "sf", "sf_facet", "ss", "ss_seg", "ftri", "ftri_facet")}
    s = torch.cuda.Stream()
    a = qm.refine(dev["xyz"], dev["tets"], dev["sf"], dev["sf_facet"], dev["ss"], dev["ss_seg"],
                  dev["ftri"], dev["ftri_facet"], w.B, stream=s)
    b = qm.refine_workload(w)
    assert np.array_equal(canon_tets(a.tets), canon_tets(b.tets)) and np.array_equal(a.rstats, b.rstats)


def test_invalid_inputs_fail_cleanly():
    w = qi.uniform_cube(50, seed=14)
    bad = w.xyz.copy(); bad[10, 0] = 0.1          # 0.1 is not a multiple of 2^-53
    with pytest.raises(qm.QmError, match="EINVAL"):
        qm.refine(bad, w.tets, w.sf, w.sf_facet, w.ss, w.ss_seg, w.ftri, w.ftri_facet, 2.0)
    flipped = w.tets.copy(); flipped[0, [0, 1]] = flipped[0, [1, 0]]
    with pytest.raises(qm.QmError, match="ENONCONFORM"):
        qm.refine(w.xyz, flipped, w.sf, w.sf_facet, w.ss, w.ss_seg, w.ftri, w.ftri_facet, 2.0)
    faces = {tuple(sorted(t[i] for i in f)) for t in w.tets.tolist() for f in qi.FACE.tolist()}
    nonface = next((a, b, c) for a in range(8, 40) for b in range(a + 1, 40) for c in range(b + 1, 40)
                   if (a, b, c) not in faces)
    sf = w.sf.copy(); sf[0] = nonface             # not a face of the mesh
    with pytest.raises(qm.QmError, match="ENONCONFORM"):
        qm.refine(w.xyz, w.tets, sf, w.sf_facet, w.ss, w.ss_seg, w.ftri, w.ftri_facet, 2.0)
    with pytest.raises(qm.QmError, match="EINVAL"):
        qm.refine(w.xyz, w.tets, w.sf, w.sf_facet, w.ss, w.ss_seg, w.ftri, w.ftri_facet, -1.0)
    # the library is still usable afterwards
    g, o = run_both(w)
    assert_same(g, o, "after errors")


@pytest.mark.parametrize("flags,max_rounds", [(0, 100000), (qm.QM_SUBPHASE_ROUNDS, 100000), (0, 20)])
def test_one_argument_set_to_both_engines(flags, max_rounds):
    """The same marshalled qm_plc, qm_mesh and qm_options go to the GPU
    library (qm_refine) and to the oracle behind the same call layout
    (qm_oracle_refine): the return codes and the results are equal."""
    import ctypes
    w = qi.uniform_cube(700, seed=9, B=1.5, spheres=(0.25, 0.4))
    keep = []
    plc, mesh = qm._marshal(w, keep)
    opts = qm._Opts(float(w.B), 0.5, int(max_rounds), 0, int(flags))
    lib = qm._load()
    res = ctypes.c_void_p()
    rc_g = lib.qm_refine(ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(opts), None, ctypes.byref(res))
    g = qm._take_result(lib, res, False)
    rc_o, o = oracle.refine_call(plc, mesh, opts)
    print(f"[engines] flags={flags} max_rounds={max_rounds}: codes {rc_g}/{rc_o}, rounds {g.rounds}/{o.rounds}",
          flush=True)
    assert rc_g == rc_o and rc_g in (0, -4)
    assert g.rounds == o.rounds and g.status == o.status and np.array_equal(g.rstats, o.rstats)
    assert np.array_equal(g.xyz.view(np.uint64), o.xyz.view(np.uint64))
    t1, t2 = np.sort(g.tets, axis=1), np.sort(o.tets, axis=1)
    assert np.array_equal(t1[np.lexsort(t1.T[::-1])], t2[np.lexsort(t2.T[::-1])])
    s1, s2 = np.sort(g.sf, axis=1), np.sort(o.sf, axis=1)
    assert np.array_equal(s1[np.lexsort(s1.T[::-1])], s2[np.lexsort(s2.T[::-1])])
