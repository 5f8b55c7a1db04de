"""ORACLE for the constrained Delaunay refinement loop -- test infrastructure.

A plain sequential C implementation (``qmo.c``, ``qmo_exact.h``) of the
round rule the GPU library executes, with its own exact big-integer
predicates.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
path never does.  It shares no code with ``paper_1903_03406_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_qmo.so")
_lib = None

NSTAT = 17
STAT_FIELDS = ("cls", "ncand", "nok", "nrej", "nexempt", "nkept",
               "ex_nonfinite", "ex_walk", "ex_enc_exempt", "ex_hmin", "ex_rftet",
               "ex_face", "ex_edge2d", "ex_manifold", "ex_delaunay", "nv_after", "nt_after")


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _SO + ".tmp", os.path.join(_HERE, "qmo.c"), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built; run oracle.build()")
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.qmo_refine.restype = ctypes.c_int
        lib.qmo_refine.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P,
                                   ctypes.c_int, P, P, ctypes.c_int, P, P,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(P)]
        lib.qmo_result_counts.argtypes = [P, P]
        lib.qmo_result_seconds.argtypes = [P]
        lib.qmo_result_seconds.restype = ctypes.c_double
        lib.qmo_result_copy.argtypes = [P] * 8
        lib.qmo_result_free.argtypes = [P]
        for name in ("qmo_p_orient3d", "qmo_p_insphere", "qmo_p_segdot", "qmo_p_facedot"):
            getattr(lib, name).restype = ctypes.c_int
        lib.qmo_p_orient2d.restype = ctypes.c_int
        lib.qmo_p_orient2d.argtypes = [ctypes.c_int, P, P, P]
        lib.qmo_c_is_bad.restype = ctypes.c_int
        lib.qmo_c_is_bad.argtypes = [P, P, P, P, ctypes.c_double]
        lib.qmo_c_key.restype = ctypes.c_uint64
        lib.qmo_c_key.argtypes = [ctypes.c_int, P, ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data


@dataclass
class OracleResult:
    xyz: np.ndarray
    tets: np.ndarray
    sf: np.ndarray
    sf_facet: np.ndarray
    ss: np.ndarray
    ss_seg: np.ndarray
    rstats: np.ndarray        # (rounds, NSTAT)
    rounds: int
    status: int               # 0 done, 1 round guard reached
    seconds: float
    last_cands: np.ndarray = None   # last round: tuple(4), status, reason, kept, region, bfaces
    dump: list = None               # dump_round's candidates (see _take_dump)
    round_checks: np.ndarray = None  # (rounds, len(CHECK_FIELDS)): check() after every round
    state: "OracleState" = None     # the flags and h_min the rounds carry (see OracleState)


@dataclass
class OracleState:
    """What the round rule carries beyond the mesh (Section 2's filtering):
    per tet an exempt bit, per subface and subsegment queued (bit0) and
    exempt (bit1) bits, aligned with the result's arrays; h_min^2 of the
    first input; rounds run over every call; the sub-phase due next (the
    sub-phase reading)."""
    hmin2: float
    rounds: int
    next_class: int
    tet_flags: np.ndarray
    sf_flags: np.ndarray
    ss_flags: np.ndarray


def refine(w, B=None, hmin_factor=0.5, max_rounds=100000, max_kept=0,
           round_checks=False, dump_round=None, key_mask=None, subphases=False, state=None) -> OracleResult:
    """Run the oracle on a workload (qm_inputs.Workload or compatible).
    round_checks: run check() on the mesh at the end of every round.
    dump_round: record that round's candidates (result.dump, see dump()).
    key_mask: AND every priority key with this mask (forces equal keys).
    subphases: the sub-phase reading of the class order (every round takes
    the three classes in turn).
    state: resume from it (an OracleState, or any object with its fields);
    w then holds the mesh that state belongs to."""
    lib = _load()
    lib.qmo_set_subphases.argtypes = [ctypes.c_int]
    lib.qmo_set_subphases(1 if subphases else 0)
    lib.qmo_set_dump_round.argtypes = [ctypes.c_int]
    lib.qmo_set_dump_round(-1 if dump_round is None else int(dump_round))
    lib.qmo_set_key_mask.argtypes = [ctypes.c_uint64]
    lib.qmo_set_key_mask((1 << 64) - 1 if key_mask is None else int(key_mask))
    lib.qmo_set_round_check.argtypes = [ctypes.c_int]
    lib.qmo_set_round_check(1 if round_checks else 0)
    c = lambda a, t: np.ascontiguousarray(a, dtype=t)
    xyz = c(w.xyz, np.float64); tets = c(w.tets, np.int32)
    sf = c(w.sf, np.int32); sff = c(w.sf_facet, np.int32)
    ss = c(w.ss, np.int32); sss = c(w.ss_seg, np.int32)
    ft = c(w.ftri, np.int32); ftf = c(w.ftri_facet, np.int32)
    lib.qmo_clear_resume.argtypes = []
    if state is not None:
        fl = [c(state.tet_flags, np.uint8), c(state.sf_flags, np.uint8), c(state.ss_flags, np.uint8)]
        if (len(fl[0]), len(fl[1]), len(fl[2])) != (len(tets), len(sf), len(ss)):
            lib.qmo_set_key_mask((1 << 64) - 1)
            lib.qmo_set_subphases(0)
            lib.qmo_set_round_check(0)
            lib.qmo_set_dump_round(-1)
            raise ValueError("the state does not describe this mesh")
        lib.qmo_set_resume.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_int]
        lib.qmo_set_resume(_ptr(fl[0]), _ptr(fl[1]), _ptr(fl[2]), float(state.hmin2), int(state.next_class))
    res = ctypes.c_void_p()
    rc = lib.qmo_refine(len(xyz), _ptr(xyz), len(tets), _ptr(tets), len(sf), _ptr(sf), _ptr(sff),
                        len(ss), _ptr(ss), _ptr(sss), len(ft), _ptr(ft), _ptr(ftf),
                        float(w.B if B is None else B), float(hmin_factor), int(max_rounds),
                        int(max_kept), ctypes.byref(res))
    lib.qmo_clear_resume()
    if rc != 0:
        lib.qmo_set_key_mask((1 << 64) - 1)
        lib.qmo_set_subphases(0)
        raise ValueError(f"oracle rejected the input (code {rc})")
    out = _collect(lib, res, round_checks, int(state.rounds) if state is not None else 0)
    lib.qmo_set_key_mask((1 << 64) - 1)
    lib.qmo_set_subphases(0)
    if dump_round is not None:
        out.dump = _take_dump(lib)
        lib.qmo_set_dump_round(-1)
    return out


def refine_call(plc, mesh, opts):
    """qm_oracle_refine: the oracle behind the GPU library's call layout.
    plc, mesh and opts are ctypes structures laid out as qm_plc, qm_mesh
    and qm_options (host arrays).  Returns (code, OracleResult or None) with
    the library's codes: 0, -4 (round guard; result returned), -1 (invalid
    argument), -2 (not a conforming tetrahedralisation), -6."""
    lib = _load()
    lib.qm_oracle_refine.restype = ctypes.c_int
    lib.qm_oracle_refine.argtypes = [ctypes.c_void_p] * 3 + [ctypes.POINTER(ctypes.c_void_p)]
    res = ctypes.c_void_p()
    rc = lib.qm_oracle_refine(ctypes.addressof(plc), ctypes.addressof(mesh), ctypes.addressof(opts),
                              ctypes.byref(res))
    if rc not in (0, -4) and rc != -6:
        return rc, None
    return rc, _collect(lib, res, False, 0)


def _collect(lib, res, round_checks, rounds_before):
    """Copy a qmo_result into an OracleResult and free it."""
    cnt = np.zeros(6, dtype=np.int32)
    lib.qmo_result_counts(res, _ptr(cnt))
    nv, nt, nsf, nss, rounds, status = (int(x) for x in cnt)
    out = OracleResult(np.empty((nv, 3)), np.empty((nt, 4), np.int32), np.empty((nsf, 3), np.int32),
                       np.empty(nsf, np.int32), np.empty((nss, 2), np.int32), np.empty(nss, np.int32),
                       np.empty((rounds, NSTAT), np.int32), rounds, status,
                       float(lib.qmo_result_seconds(res)))
    lib.qmo_result_copy(res, _ptr(out.xyz), _ptr(out.tets), _ptr(out.sf), _ptr(out.sf_facet),
                        _ptr(out.ss), _ptr(out.ss_seg), _ptr(out.rstats))
    if round_checks:
        lib.qmo_result_round_checks.restype = ctypes.c_int
        lib.qmo_result_round_checks.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        out.round_checks = np.zeros((rounds, len(CHECK_FIELDS)), dtype=np.int32)
        if rounds:
            lib.qmo_result_round_checks(res, _ptr(out.round_checks))
        lib.qmo_set_round_check(0)
    tfl, sfl, ssl = np.zeros(nt, np.uint8), np.zeros(nsf, np.uint8), np.zeros(nss, np.uint8)
    h2 = ctypes.c_double()
    lib.qmo_result_state.restype = ctypes.c_int
    lib.qmo_result_state.argtypes = [ctypes.c_void_p] * 4 + [ctypes.POINTER(ctypes.c_double)]
    nxt = lib.qmo_result_state(res, _ptr(tfl), _ptr(sfl), _ptr(ssl), ctypes.byref(h2))
    out.state = OracleState(float(h2.value), rounds_before + rounds, int(nxt), tfl, sfl, ssl)
    lib.qmo_result_lastc.restype = ctypes.c_int
    lib.qmo_result_lastc.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    nl = lib.qmo_result_lastc(res, None)
    out.last_cands = np.zeros((nl, 9), dtype=np.int32)
    if nl:
        lib.qmo_result_lastc(res, _ptr(out.last_cands))
    lib.qmo_result_free(res)
    return out


def _take_dump(lib):
    """The recorded round's candidates in priority order, as dicts: cls,
    tup, key, status, reason, kept, p, region (set of sorted vertex
    quadruples), rf (list of sorted triples), claims (set of quadruples)."""
    lib.qmo_dump_sizes.restype = ctypes.c_int
    lib.qmo_dump_sizes.argtypes = [ctypes.c_void_p]
    lib.qmo_dump_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    sz = np.zeros(2, dtype=np.int32)
    n = lib.qmo_dump_sizes(_ptr(sz))
    ib = np.zeros(max(int(sz[0]), 1), dtype=np.int32)
    db = np.zeros(max(int(sz[1]), 1), dtype=np.float64)
    lib.qmo_dump_copy(_ptr(ib), _ptr(db))
    out, o = [], 0
    for i in range(n):
        cls, ntup = int(ib[o]), int(ib[o + 1])
        tup = tuple(int(x) for x in ib[o + 2:o + 2 + ntup])
        key = (int(np.uint32(ib[o + 6])) << 32) | int(np.uint32(ib[o + 7]))
        status, reason, kept, nrt, nrf, ncl = (int(x) for x in ib[o + 8:o + 14])
        o += 14
        quad = lambda m: [tuple(int(x) for x in ib[o + 4 * j:o + 4 * j + 4]) for j in range(m)]
        region = quad(nrt); o += 4 * nrt
        claims = quad(ncl); o += 4 * ncl
        rf = [tuple(int(x) for x in ib[o + 3 * j:o + 3 * j + 3]) for j in range(nrf)]; o += 3 * nrf
        out.append({"cls": cls, "tup": tup, "key": key, "status": status, "reason": reason, "kept": kept,
                    "p": db[3 * i:3 * i + 3].copy(), "region": region, "claims": claims, "rf": rf})
    return out


# --- the oracle's predicates and constructions, for its own pin tests -------
def _v3(p):
    return np.ascontiguousarray(p, dtype=np.float64)


def orient3d(a, b, c, d) -> int:
    L = _load(); a, b, c, d = map(_v3, (a, b, c, d))
    return L.qmo_p_orient3d(*(ctypes.c_void_p(_ptr(x)) for x in (a, b, c, d)))


def insphere(a, b, c, d, e) -> int:
    L = _load(); xs = list(map(_v3, (a, b, c, d, e)))
    return L.qmo_p_insphere(*(ctypes.c_void_p(_ptr(x)) for x in xs))


def orient2d(axis, a, b, c) -> int:
    L = _load(); xs = list(map(_v3, (a, b, c)))
    return L.qmo_p_orient2d(int(axis), *(_ptr(x) for x in xs))


def segdot(a, b, v) -> int:
    L = _load(); xs = list(map(_v3, (a, b, v)))
    return L.qmo_p_segdot(*(ctypes.c_void_p(_ptr(x)) for x in xs))


def facedot(a, b, c, v) -> int:
    L = _load(); xs = list(map(_v3, (a, b, c, v)))
    return L.qmo_p_facedot(*(ctypes.c_void_p(_ptr(x)) for x in xs))


def midpoint(a, b):
    L = _load(); a, b = _v3(a), _v3(b); p = np.empty(3)
    L.qmo_c_midpoint(ctypes.c_void_p(_ptr(a)), ctypes.c_void_p(_ptr(b)), ctypes.c_void_p(_ptr(p)))
    return p


def tri_cc(a, b, c):
    L = _load(); xs = list(map(_v3, (a, b, c))); p = np.empty(3)
    L.qmo_c_tri_cc(*(ctypes.c_void_p(_ptr(x)) for x in xs), ctypes.c_void_p(_ptr(p)))
    return p


def tet_cc(a, b, c, d):
    L = _load(); xs = list(map(_v3, (a, b, c, d))); p = np.empty(3); r2 = np.empty(1)
    L.qmo_c_tet_cc(*(ctypes.c_void_p(_ptr(x)) for x in xs), ctypes.c_void_p(_ptr(p)),
                   ctypes.c_void_p(_ptr(r2)))
    return p, float(r2[0])


def is_bad(a, b, c, d, B) -> bool:
    L = _load(); xs = list(map(_v3, (a, b, c, d)))
    return bool(L.qmo_c_is_bad(*(_ptr(x) for x in xs), float(B)))


def key(cls, ids) -> int:
    L = _load(); ids = np.ascontiguousarray(ids, dtype=np.int32)
    return int(L.qmo_c_key(int(cls), _ptr(ids), len(ids)))


CHECK_FIELDS = ("neg_orient", "face_overuse", "hull_not_subface", "nonlocal_delaunay",
                "sf_missing", "ss_missing", "euler", "bad_tets", "chain_broken")


def check(xyz, tets, sf, ss, ss_seg, B) -> dict:
    """Mesh property checks (see qmo_check in qmo.c)."""
    L = _load()
    c = lambda a, t: np.ascontiguousarray(a, dtype=t)
    xyz = c(xyz, np.float64); tets = c(tets, np.int32); sf = c(sf, np.int32)
    ss = c(ss, np.int32); ss_seg = c(ss_seg, np.int32)
    out = np.zeros(len(CHECK_FIELDS), dtype=np.int32); vol = np.zeros(1)
    L.qmo_check.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    L.qmo_check(len(xyz), _ptr(xyz), len(tets), _ptr(tets), len(sf), _ptr(sf), len(ss), _ptr(ss),
                _ptr(ss_seg), float(B), _ptr(out), _ptr(vol))
    d = dict(zip(CHECK_FIELDS, (int(x) for x in out)))
    d["volume"] = float(vol[0])
    return d


def check_global(xyz, tets) -> int:
    """Brute force: tets whose circumsphere strictly encloses a mesh vertex."""
    L = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64); tets = np.ascontiguousarray(tets, dtype=np.int32)
    L.qmo_check_global.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    L.qmo_check_global.restype = ctypes.c_int
    return int(L.qmo_check_global(len(xyz), _ptr(xyz), len(tets), _ptr(tets)))


def facet_areas(xyz, tri, tri_facet) -> dict:
    """Sum of triangle areas per facet id (FP64)."""
    a, b, c = (xyz[tri[:, k]] for k in range(3))
    ar = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    out = {}
    for f, x in zip(tri_facet.tolist(), ar.tolist()):
        out[f] = out.get(f, 0.0) + x
    return out
