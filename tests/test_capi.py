"""The C-ABI library loads and exports every entry point include/qm.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1903_03406_amd as qm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "qm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    assert {"qm_refine", "qm_result_view", "qm_result_rounds", "qm_result_free", "qm_last_error"} <= set(names)
    assert set(names) == set(qm.EXPORTS)


@pytest.mark.skipif(not os.path.exists(qm._SO), reason="libqm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(qm._SO)
    for name in declared():
        assert hasattr(lib, name), name
    lib.qm_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.qm_version()
    lib.qm_last_error.restype = ctypes.c_char_p
    assert lib.qm_last_error() == b""


def test_binding_has_no_cpu_path(monkeypatch, tmp_path):
    """Without the built library the binding fails loudly (no fallback)."""
    monkeypatch.setattr(qm, "_SO", str(tmp_path / "missing.so"))
    monkeypatch.setattr(qm, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        qm.refine([[0, 0, 0]] * 8, [[0, 1, 2, 3]], [], [], [], [], [], [], B=2.0)


@pytest.mark.skipif(not os.path.exists(qm._SO), reason="libqm.so not built")
def test_server_estimate_is_host_arithmetic():
    """qm_estimate_bytes needs no device: 8 KB per input tet at B >= 1.6,
    16 KB below, plus 320 MiB."""
    import qm_inputs as qi
    w = qi.uniform_cube(60, seed=3, B=2.0)
    nt = len(w.tets)
    assert qm.estimate_bytes(w) == nt * 8192 + (320 << 20)
    w.B = 1.4
    assert qm.estimate_bytes(w) == nt * 16384 + (320 << 20)


def test_binding_constants_match_the_header():
    text = open(os.path.join(ROOT, "include", "qm.h")).read()
    defs = {m.group(1): m.group(2) for m in re.finditer(r"#define (QM_[A-Z_0-9]+)\s+\(?(-?\w+)\)?", text)}
    assert int(defs["QM_PROFILE"].rstrip("u")) == qm.QM_PROFILE
    assert int(defs["QM_PROFILE_GROW"].rstrip("u")) == qm.QM_PROFILE_GROW
    assert int(defs["QM_ROUND_FIELDS"]) == qm.ROUND_FIELDS
    assert int(defs["QM_PROF_FAMILIES"]) == len(qm.PROF_FAMILIES)
    for flag in ("QM_INPUT_DEVICE", "QM_VERBOSE", "QM_EARLY_STOP", "QM_TEST_ERROR_WORD", "QM_TEST_TIER1",
                 "QM_TEST_TIER2", "QM_TEST_KEY_COLLIDE", "QM_OUTPUT_DEVICE", "QM_SUBPHASE_ROUNDS"):
        assert int(defs[flag].rstrip("u")) == getattr(qm, flag), flag
    codes = {int(v): k for k, v in defs.items() if k.startswith("QM_E") and v.startswith("-")}
    assert codes == qm.ERRORS


@pytest.mark.skipif(not os.path.exists(qm._SO), reason="libqm.so not built")
def test_lockstep_knobs_are_checked_before_any_device_call():
    """Out-of-range lockstep knobs are refused with QM_EINVAL (host check)."""
    for bad in ({"groups": 0}, {"classify_tiles": 65}, {"rank_max": 5000}, {"hybrid_wgs": 8},
                {"select_one_wg": -1}, {"global_wgs": 2000}):
        with pytest.raises(qm.QmError, match="EINVAL"):
            qm.refine_lockstep([], tune=bad)


@pytest.mark.skipif(not os.path.exists(qm._SO), reason="libqm.so not built")
def test_resume_state_is_checked_before_any_device_call():
    """A resume state that does not describe the mesh, or holds flag bits,
    a sub-phase, a round count or an h_min outside their ranges, is refused
    with QM_EINVAL (host check)."""
    import numpy as np
    import qm_inputs as qi
    w = qi.uniform_cube(60, seed=2, B=2.0, spheres=(0.3,))
    nt, nsf, nss = len(w.tets), len(w.sf), len(w.ss)
    good = dict(hmin2=1e-6, rounds=3, next_class=0, tet_flags=np.zeros(nt, np.uint8),
                sf_flags=np.zeros(nsf, np.uint8), ss_flags=np.zeros(nss, np.uint8))
    bads = [dict(tet_flags=np.zeros(nt - 1, np.uint8)), dict(sf_flags=np.zeros(nsf + 1, np.uint8)),
            dict(ss_flags=np.zeros(max(nss - 1, 0), np.uint8)), dict(next_class=3), dict(next_class=-1),
            dict(hmin2=-1.0), dict(hmin2=float("nan")), dict(hmin2=float("inf")), dict(rounds=-1),
            dict(tet_flags=np.full(nt, 2, np.uint8)), dict(sf_flags=np.full(nsf, 4, np.uint8)),
            dict(ss_flags=np.full(nss, 8, np.uint8))]
    assert nss > 0 and nsf > 0
    for b in bads:
        st = qm.RefineState(**{**good, **b})
        with pytest.raises(qm.QmError, match="EINVAL"):
            qm.refine(w.xyz, w.tets, w.sf, w.sf_facet, w.ss, w.ss_seg, w.ftri, w.ftri_facet, w.B, seg=w.seg,
                      state=st)
