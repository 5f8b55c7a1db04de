"""Full-size parity: the HIP path on the 50K-point and 1M-point workloads
against expected values that tests/golden/make_golden.py wrote with the
oracle (digests of the canonical output and of the per-round records), and
properties that hold at any size."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import paper_1903_03406_amd as qm
import qm_inputs as qi

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def canonical(r):
    t = np.sort(np.asarray(r.tets, dtype=np.int32), axis=1)
    t = t[np.lexsort(t.T[::-1])]
    sf = np.concatenate([np.sort(r.sf, axis=1), r.sf_facet.reshape(-1, 1)], axis=1).astype(np.int32)
    sf = sf[np.lexsort(sf.T[::-1])]
    ss = np.concatenate([np.sort(r.ss, axis=1), r.ss_seg.reshape(-1, 1)], axis=1).astype(np.int32)
    ss = ss[np.lexsort(ss.T[::-1])]
    return {"tets_sha256": digest(t), "xyz_sha256": digest(np.asarray(r.xyz, dtype=np.float64)),
            "sf_sha256": digest(sf), "ss_sha256": digest(ss),
            "rounds_sha256": digest(np.asarray(r.rstats, dtype=np.int32)),
            "nv": int(len(r.xyz)), "nt": int(len(r.tets)), "nsf": int(len(r.sf)), "nss": int(len(r.ss)),
            "rounds": int(r.rounds), "status": int(r.status)}


def load(name):
    p = os.path.join(GOLD, name)
    if not os.path.exists(p):
        pytest.skip(f"{name} not generated (tests/golden/make_golden.py)")
    return json.load(open(p))


def compare(g, gold, label):
    got = canonical(g)
    print(f"[fullsize] {label}: gpu rounds={got['rounds']} nv={got['nv']} nt={got['nt']} "
          f"| oracle rounds={gold['rounds']} nv={gold['nv']} nt={gold['nt']}", flush=True)
    for k in ("rounds", "status", "nv", "nt", "nsf", "nss", "rounds_sha256", "xyz_sha256", "tets_sha256",
              "sf_sha256", "ss_sha256"):
        assert got[k] == gold[k], f"{label}: {k} differs"


def assert_cdt(g, w, label):
    """The output is a valid tetrahedralisation of the cube that conforms to
    the PLC and is a CDT (every non-subface face locally Delaunay)."""
    c = oracle.check(g.xyz, g.tets, g.sf, g.ss, g.ss_seg, w.B)
    print(f"[fullsize] {label} check: {c}", flush=True)
    for k in ("neg_orient", "face_overuse", "hull_not_subface", "nonlocal_delaunay", "sf_missing", "ss_missing",
              "chain_broken"):
        assert c[k] == 0, (k, c)
    assert c["euler"] == 1 and abs(c["volume"] - 1.0) < 1e-9


def test_config2_full_parity():
    gold = load("cfg2.json")
    w = qi.config(2)
    assert w.sha256() == gold["input_sha256"]
    g = qm.refine_workload(w)
    compare(g, gold, "config2")
    assert_cdt(g, w, "config2")


@pytest.fixture(scope="module")
def cfg3():
    return qi.config(3)


@pytest.mark.parametrize("name", ["cfg3_rounds8.json", "cfg3_rounds1099.json", "cfg3_rounds1110.json"])
def test_config3_first_rounds_parity(cfg3, name):
    """The first 8 rounds, and the first 1099 and 1110 rounds (subsegment,
    subface and bad-tet rounds; the oracle takes about 4.9 hours for the
    1099-round golden)."""
    gold = load(name)
    assert cfg3.sha256() == gold["input_sha256"]
    compare(qm.refine_workload(cfg3, max_rounds=gold["max_rounds"]), gold, f"config3 {gold['max_rounds']} rounds")


def test_config3_full_properties(cfg3):
    """At full size: the refinement converges, is a CDT conforming to the PLC
    (every subface is a face, every subsegment an edge, segment chains
    intact, facet areas kept, every non-subface face locally Delaunay) and a
    valid tetrahedralisation of the cube (orientation, face use, Euler
    characteristic, volume)."""
    g = qm.refine_workload(cfg3, verbose=True)
    print(f"[fullsize] config3: rounds={g.rounds} steiner={g.steiner} tets={len(g.tets)}", flush=True)
    assert g.status == 0
    assert_cdt(g, cfg3, "config3")
    a0 = oracle.facet_areas(cfg3.xyz, cfg3.ftri, cfg3.ftri_facet)
    a1 = oracle.facet_areas(g.xyz, g.sf, g.sf_facet)
    assert set(a0) == set(a1)
    assert max(abs(a0[k] - a1[k]) / a0[k] for k in a0) < 1e-9


def test_config3_subphase_rounds_properties(cfg3):
    """The three-sub-phase mode (not a parity mode) at full size: converges
    and is a CDT conforming to the PLC and a valid tetrahedralisation."""
    g = qm.refine_workload(cfg3, subphases=True)
    print(f"[fullsize] config3 sub-phase rounds: rounds={g.rounds} steiner={g.steiner} tets={len(g.tets)} "
          f"{g.seconds_refine:.2f}s", flush=True)
    assert g.status == 0
    assert_cdt(g, cfg3, "config3 sub-phase rounds")
    a0 = oracle.facet_areas(cfg3.xyz, cfg3.ftri, cfg3.ftri_facet)
    a1 = oracle.facet_areas(g.xyz, g.sf, g.sf_facet)
    assert set(a0) == set(a1) and max(abs(a0[k] - a1[k]) / a0[k] for k in a0) < 1e-9
