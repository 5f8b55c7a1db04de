"""Round-based constrained Delaunay refinement on the AMD MI355X (gfx950).

Thin ctypes binding of ``libqm.so`` (C-ABI in ``include/qm.h``): argument
marshalling only, every step of the refinement runs in the HIP kernels.
PyTorch, when used, only supplies device memory and the HIP stream.

    import paper_1903_03406_amd as qm
    out = qm.refine(xyz, tets, sf, sf_facet, ss, ss_seg, ftri, ftri_facet, B=2.0)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_SO = os.path.join(_HERE, "libqm.so")
_SRC = os.path.join(_HERE, "csrc", "qm_lib.hip")
_lib = None

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

QM_INPUT_DEVICE = 1
QM_PROFILE = 2
QM_PROFILE_GROW = 8   # time only the small-tile grow launches (family grow_validate)
QM_VERBOSE = 4
QM_EARLY_STOP = 256       # non-parity mode: early-stop blasting (timing-dependent result)
QM_OUTPUT_DEVICE = 512    # the result's arrays stay on the device
QM_SUBPHASE_ROUNDS = 1024  # other class-order reading: three sub-phase rounds (SS, SF, TET in turn)
QM_TEST_ERROR_WORD = 16   # tests only: the call ends with QM_EINTERNAL through its own error word
QM_TEST_TIER1 = 32        # tests only: every region grown with the medium tiles (or larger)
QM_TEST_TIER2 = 64        # tests only: every region grown with the global-memory tiles
QM_TEST_KEY_COLLIDE = 128  # tests only: keys cut to their top 3 bits (equal keys, tie rule)
PROF_FAMILIES = ("classify", "split_order", "locate", "grow_validate", "flags_stats", "select",
                 "scans", "insert", "grow_hybrid", "grow_global")
TIER_FIELDS = ("evals", "overflowed", "tested", "region", "bfaces", "max_region", "max_tested", "max_bfaces",
               "ov_region", "ov_hash", "ov_facet_region", "ov_queue", "ov_bfaces", "ov_edges2d", "ov_claims",
               "ov_edge_table", "accepted", "acc_region", "acc_bfaces", "acc_claims",
               "cyc_setup_seeds", "cyc_facet_region", "cyc_tet_region", "cyc_encroach", "cyc_radius_rftets",
               "cyc_bfaces", "cyc_edges_closure", "cyc_claims_results")
ROUND_FIELDS = 17
ROUND_NAMES = ("cls", "ncand", "nok", "nrej", "nexempt", "nkept",
               "ex_nonfinite", "ex_walk", "ex_enc_exempt", "ex_hmin", "ex_rftet",
               "ex_face", "ex_edge2d", "ex_manifold", "ex_delaunay", "nv_after", "nt_after")
NOALLOC_SCRATCH_BYTES = 256 << 20   # QM_NOALLOC_SCRATCH_BYTES
ERRORS = {-1: "QM_EINVAL", -2: "QM_ENONCONFORM", -3: "QM_ENOMEM", -4: "QM_EROUNDS",
          -5: "QM_EDEVICE", -6: "QM_EINTERNAL", -7: "QM_ECAPACITY", -8: "QM_EAGAIN"}


def build() -> str:
    """Compile libqm.so for gfx950 (in-tree)."""
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(_ROOT, "include"), "-o", _SO + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class _Plc(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("nseg", ctypes.c_int32), ("seg", ctypes.c_void_p),
                ("nftri", ctypes.c_int32), ("ftri", ctypes.c_void_p), ("ftri_facet", ctypes.c_void_p)]


class _Mesh(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("nt", ctypes.c_int32),
                ("tet", ctypes.c_void_p), ("nsf", ctypes.c_int32), ("sf", ctypes.c_void_p),
                ("sf_facet", ctypes.c_void_p), ("nss", ctypes.c_int32), ("ss", ctypes.c_void_p),
                ("ss_seg", ctypes.c_void_p)]


class _State(ctypes.Structure):
    _fields_ = [("hmin2", ctypes.c_double), ("rounds", ctypes.c_int32), ("next_class", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("nsf", ctypes.c_int32), ("nss", ctypes.c_int32),
                ("tet_flags", ctypes.c_void_p), ("sf_flags", ctypes.c_void_p), ("ss_flags", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("B", ctypes.c_double), ("hmin_factor", ctypes.c_double),
                ("max_rounds", ctypes.c_int32), ("max_kept", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("status", ctypes.c_int32),
                ("inserted", ctypes.c_int64 * 3), ("candidates", ctypes.c_int64),
                ("mis_passes", ctypes.c_int64), ("deferred", ctypes.c_int64), ("device_bytes_peak", ctypes.c_int64), ("nv_out", ctypes.c_int64), ("nt_out", ctypes.c_int64),
                ("seconds_setup", ctypes.c_double), ("seconds_refine", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("prof_ms", ctypes.c_double * 10),
                ("prof_launches", ctypes.c_int64 * 10), ("prof_tested", ctypes.c_int64),
                ("prof_region", ctypes.c_int64), ("prof_bfaces", ctypes.c_int64),
                ("prof_claims", ctypes.c_int64), ("prof_scan_tets", ctypes.c_int64),
                ("prof_scan_verts", ctypes.c_int64), ("prof_overflow", ctypes.c_int64),
                ("prof_poolfull", ctypes.c_int64), ("prof_grow_cycles", ctypes.c_int64 * 8),
                ("prof_tier", (ctypes.c_int64 * 28) * 3)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built: run paper_1903_03406_amd.build() "
                               "(the refinement has no CPU fallback)")
        try:                       # share torch's HIP runtime when torch is present:
            import torch  # noqa: F401  (one runtime per process)
        except ImportError:
            pass
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.qm_refine.restype = ctypes.c_int
        lib.qm_refine.argtypes = [ctypes.POINTER(_Plc), ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts), P,
                                  ctypes.POINTER(P)]
        lib.qm_result_view.restype = ctypes.c_int
        lib.qm_result_view.argtypes = [P, ctypes.POINTER(_Mesh), ctypes.POINTER(_Stats)]
        lib.qm_result_rounds.restype = ctypes.c_int
        lib.qm_result_rounds.argtypes = [P, P, ctypes.c_int32]
        lib.qm_result_free.argtypes = [P]
        lib.qm_last_error.restype = ctypes.c_char_p
        lib.qm_version.restype = ctypes.c_char_p
        _lib = lib
    return _lib


EXPORTS = ("qm_refine", "qm_refine_resume", "qm_result_state", "qm_refine_noalloc", "qm_test_geometry", "qm_refine_batch", "qm_refine_lockstep", "qm_lockstep_autotune", "qm_result_view", "qm_result_rounds", "qm_result_last_round",
           "qm_result_round_profile", "qm_result_free", "qm_last_error", "qm_version",
           "qm_estimate_bytes", "qm_server_create", "qm_server_submit", "qm_server_step", "qm_server_poll",
           "qm_server_info", "qm_server_evict", "qm_server_readmit",
           "qm_server_destroy")


class QmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


@dataclass
class RefineResult:
    xyz: np.ndarray
    tets: np.ndarray
    sf: np.ndarray
    sf_facet: np.ndarray
    ss: np.ndarray
    ss_seg: np.ndarray
    rstats: np.ndarray          # (rounds, 16), same fields as ROUND_NAMES
    rounds: int
    status: int                 # 0 converged, 1 round guard reached
    inserted: tuple
    candidates: int
    mis_passes: int
    seconds_setup: float
    seconds_refine: float
    seconds_total: float
    profile: dict = None        # QM_PROFILE: per-family ms/launches and region counters
    last_cands: np.ndarray = None   # last round: tuple(4), status, reason, kept, region, bfaces
    deferred: int = 0               # QM_EARLY_STOP: evaluations stopped early
    device_bytes_peak: int = 0      # most device memory the call held at once
    state: "RefineState" = None     # checkpoint: flags and h_min to resume from (qm_result_state)

    @property
    def steiner(self) -> int:
        return int(sum(self.inserted))


@dataclass
class RefineState:
    """The refinement state beyond the mesh (qm_state): per output tet an
    exempt bit, per subface and subsegment queued (bit0) and exempt (bit1)
    bits, aligned with the result's arrays; h_min^2 of the first call; rounds
    run over every call; the next sub-phase (three-sub-phase mode)."""
    hmin2: float
    rounds: int
    next_class: int
    tet_flags: np.ndarray
    sf_flags: np.ndarray
    ss_flags: np.ndarray


def _prof_flag(profile):
    """profile=True: every kernel family and the region counters (QM_PROFILE);
    profile="grow": only the small-tile grow launches (QM_PROFILE_GROW)."""
    if profile == "grow":
        return QM_PROFILE_GROW
    return QM_PROFILE if profile else 0


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def refine(xyz, tets, sf, sf_facet, ss, ss_seg, ftri, ftri_facet, B, *, seg=None, hmin_factor=0.5,
           max_rounds=100000, max_kept=0, stream=None, profile=False, verbose=False,
           extra_flags=0, early_stop=False, subphases=False, state=None) -> RefineResult:
    """Refine a CDT.  Arrays are numpy (host) or torch CUDA tensors (device);
    ``stream`` is a torch.cuda.Stream or a raw hipStream_t handle.
    ``state``: a RefineState to resume from (qm_refine_resume); the mesh is
    then the output the state belongs to."""
    lib = _load()
    dev = False
    keep = []

    def ptr(a, dtype):
        nonlocal dev
        if a is None:
            return None, 0
        if hasattr(a, "is_cuda") and a.is_cuda:
            dev = True
            import torch
            t = a.contiguous().to(dtype={np.float64: torch.float64, np.int32: torch.int32}[dtype])
            keep.append(t)
            return t.data_ptr(), t.shape[0]
        h = _arr(a, dtype)
        keep.append(h)
        return h.ctypes.data, h.shape[0]

    pxyz, nv = ptr(xyz, np.float64)
    ptet, nt = ptr(tets, np.int32)
    psf, nsf = ptr(sf, np.int32)
    psff, _ = ptr(sf_facet, np.int32)
    pss, nss = ptr(ss, np.int32)
    pssg, _ = ptr(ss_seg, np.int32)
    pft, nft = ptr(ftri, np.int32)
    pftf, _ = ptr(ftri_facet, np.int32)
    pseg, nseg = ptr(seg if seg is not None else np.zeros((0, 2), np.int32), np.int32)
    plc = _Plc(nv, nseg, pseg, nft, pft, pftf)
    mesh = _Mesh(nv, pxyz, nt, ptet, nsf, psf, psff, nss, pss, pssg)
    opts = _Opts(float(B), float(hmin_factor), int(max_rounds), int(max_kept),
                 (QM_INPUT_DEVICE if dev else 0) | (_prof_flag(profile))
                 | (QM_VERBOSE if verbose else 0) | (QM_EARLY_STOP if early_stop else 0)
                 | (QM_SUBPHASE_ROUNDS if subphases else 0) | int(extra_flags))
    if stream is None:
        hs = None
    elif hasattr(stream, "cuda_stream"):
        hs = stream.cuda_stream
    else:
        hs = int(stream)
    res = ctypes.c_void_p()
    if state is None:
        rc = lib.qm_refine(ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(opts), hs, ctypes.byref(res))
    else:
        fl = [_arr(a, np.uint8) for a in (state.tet_flags, state.sf_flags, state.ss_flags)]
        keep.extend(fl)
        cst = _State(float(state.hmin2), int(state.rounds), int(state.next_class), len(fl[0]), len(fl[1]),
                     len(fl[2]), fl[0].ctypes.data, fl[1].ctypes.data, fl[2].ctypes.data)
        lib.qm_refine_resume.restype = ctypes.c_int
        lib.qm_refine_resume.argtypes = [ctypes.POINTER(_Plc), ctypes.POINTER(_Mesh), ctypes.POINTER(_State),
                                         ctypes.POINTER(_Opts), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        rc = lib.qm_refine_resume(ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(cst), ctypes.byref(opts),
                                  hs, ctypes.byref(res))
    if rc not in (0, -4):
        raise QmError(rc, lib.qm_last_error().decode())
    return _take_result(lib, res, profile)


def _take_result(lib, res, profile) -> RefineResult:
    """Copy a qm_result into numpy arrays and free it."""
    P_ = ctypes.c_void_p
    try:
        view, st = _Mesh(), _Stats()
        lib.qm_result_view(res, ctypes.byref(view), ctypes.byref(st))

        def grab(p, n, cols, dtype):
            if n == 0:
                return np.zeros((0, cols) if cols > 1 else (0,), dtype=dtype)
            ctype = ctypes.c_double if dtype == np.float64 else ctypes.c_int32
            buf = ctypes.cast(p, ctypes.POINTER(ctype * (n * cols))).contents
            a = np.frombuffer(buf, dtype=dtype).copy()
            return a.reshape(n, cols) if cols > 1 else a

        lib.qm_result_last_round.restype = ctypes.c_int
        lib.qm_result_last_round.argtypes = [P_, P_, ctypes.c_int32]
        nl = lib.qm_result_last_round(res, None, 0)
        last = np.zeros((max(nl, 0), 9), dtype=np.int32)
        if nl:
            lib.qm_result_last_round(res, last.ctypes.data, nl)
        round_ms = None
        if profile:
            lib.qm_result_round_profile.restype = ctypes.c_int
            lib.qm_result_round_profile.argtypes = [P_, P_, ctypes.c_int32]
            npr = lib.qm_result_round_profile(res, None, 0)
            round_ms = np.zeros((max(npr, 0), len(PROF_FAMILIES)), dtype=np.float64)
            if npr:
                lib.qm_result_round_profile(res, round_ms.ctypes.data, npr)
        cs = _State()
        lib.qm_result_state.restype = ctypes.c_int
        lib.qm_result_state.argtypes = [P_, ctypes.POINTER(_State)]
        lib.qm_result_state(res, ctypes.byref(cs))

        def flags(p, n):
            return (np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_uint8)), shape=(n,)).copy()
                    if n else np.zeros(0, np.uint8))
        state = RefineState(float(cs.hmin2), int(cs.rounds), int(cs.next_class), flags(cs.tet_flags, cs.nt),
                            flags(cs.sf_flags, cs.nsf), flags(cs.ss_flags, cs.nss))
        nr = lib.qm_result_rounds(res, None, 0)
        rs = np.zeros((max(nr, 0), ROUND_FIELDS), dtype=np.int32)
        if nr:
            lib.qm_result_rounds(res, rs.ctypes.data, nr)
        return RefineResult(grab(view.xyz, view.nv, 3, np.float64), grab(view.tet, view.nt, 4, np.int32),
                            grab(view.sf, view.nsf, 3, np.int32), grab(view.sf_facet, view.nsf, 1, np.int32),
                            grab(view.ss, view.nss, 2, np.int32), grab(view.ss_seg, view.nss, 1, np.int32),
                            rs, int(st.rounds), int(st.status), tuple(int(x) for x in st.inserted),
                            int(st.candidates), int(st.mis_passes), float(st.seconds_setup),
                            float(st.seconds_refine), float(st.seconds_total),
                            ({"ms": dict(zip(PROF_FAMILIES, list(st.prof_ms))),
                              "launches": dict(zip(PROF_FAMILIES, [int(x) for x in st.prof_launches])),
                              "tested": int(st.prof_tested), "region": int(st.prof_region),
                              "bfaces": int(st.prof_bfaces), "claims": int(st.prof_claims),
                              "scan_tets": int(st.prof_scan_tets), "scan_verts": int(st.prof_scan_verts),
                              "overflow": int(st.prof_overflow), "poolfull": int(st.prof_poolfull),
                              "grow_cycles": [int(x) for x in st.prof_grow_cycles],
                              "tiers": [dict(zip(TIER_FIELDS, [int(x) for x in st.prof_tier[k]]))
                                        for k in range(3)],
                              "round_ms": round_ms}
                             if profile else None), last, int(st.deferred), int(st.device_bytes_peak), state)
    finally:
        lib.qm_result_free(res)


class _MeshBuf(ctypes.Structure):
    _fields_ = [("cap_v", ctypes.c_int32), ("cap_t", ctypes.c_int32), ("cap_sf", ctypes.c_int32),
                ("cap_ss", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("tet", ctypes.c_void_p),
                ("sf", ctypes.c_void_p), ("sf_facet", ctypes.c_void_p), ("ss", ctypes.c_void_p),
                ("ss_seg", ctypes.c_void_p), ("nv", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("nsf", ctypes.c_int32), ("nss", ctypes.c_int32)]


def refine_noalloc(w, out, *, hmin_factor=0.5, max_rounds=100000, max_kept=0, stream=None):
    """qm_refine_noalloc: refine workload ``w`` (its arrays are copied to the
    device here, by torch) into the caller's device tensors ``out`` (a dict:
    xyz float64 [cap_v,3], tet int32 [cap_t,4], sf int32 [cap_sf,3], sf_facet
    int32 [cap_sf], ss int32 [cap_ss,2], ss_seg int32 [cap_ss]).  The library
    allocates nothing.  Returns (sizes dict nv/nt/nsf/nss, stats dict);
    raises QmError on failure (sizes still in the error's ``sizes``)."""
    import torch
    lib = _load()
    lib.qm_refine_noalloc.restype = ctypes.c_int
    lib.qm_refine_noalloc.argtypes = [ctypes.POINTER(_Plc), ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts),
                                      ctypes.c_void_p, ctypes.POINTER(_MeshBuf), ctypes.POINTER(_Stats)]
    keep = []

    def d(a, dtype, cols):
        t = torch.as_tensor(_arr(a, dtype).reshape(-1, cols) if cols > 1 else _arr(a, dtype).reshape(-1),
                            device="cuda").contiguous()
        keep.append(t)
        return t.data_ptr(), t.shape[0]
    pxyz, nv = d(w.xyz, np.float64, 3)
    ptet, nt = d(w.tets, np.int32, 4)
    psf, nsf = d(w.sf, np.int32, 3)
    psff, _ = d(w.sf_facet, np.int32, 1)
    pss, nss = d(w.ss, np.int32, 2)
    pssg, _ = d(w.ss_seg, np.int32, 1)
    pft, nft = d(w.ftri, np.int32, 3)
    pftf, _ = d(w.ftri_facet, np.int32, 1)
    pseg, nseg = d(w.seg if w.seg is not None else np.zeros((0, 2), np.int32), np.int32, 2)
    plc = _Plc(nv, nseg, pseg, nft, pft, pftf)
    mesh = _Mesh(nv, pxyz, nt, ptet, nsf, psf, psff, nss, pss, pssg)
    opts = _Opts(float(w.B), float(hmin_factor), int(max_rounds), int(max_kept), QM_INPUT_DEVICE)
    buf = _MeshBuf(out["xyz"].shape[0], out["tet"].shape[0], out["sf"].shape[0], out["ss"].shape[0],
                   out["xyz"].data_ptr(), out["tet"].data_ptr(), out["sf"].data_ptr(),
                   out["sf_facet"].data_ptr(), out["ss"].data_ptr(), out["ss_seg"].data_ptr(), -1, -1, -1, -1)
    st = _Stats()
    if stream is None:
        hs = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        hs = stream.cuda_stream
    else:
        hs = int(stream)
    torch.cuda.current_stream().synchronize()        # the input copies are complete
    rc = lib.qm_refine_noalloc(ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(opts), hs,
                               ctypes.byref(buf), ctypes.byref(st))
    sizes = {"nv": buf.nv, "nt": buf.nt, "nsf": buf.nsf, "nss": buf.nss}
    if rc not in (0, -4):
        e = QmError(rc, lib.qm_last_error().decode())
        e.sizes = sizes
        raise e
    stats = {"rounds": int(st.rounds), "status": int(st.status), "inserted": tuple(int(x) for x in st.inserted),
             "candidates": int(st.candidates), "mis_passes": int(st.mis_passes), "nv_out": int(st.nv_out),
             "nt_out": int(st.nt_out), "seconds_refine": float(st.seconds_refine)}
    return sizes, stats


def _marshal(w, keep):
    """qm_plc and qm_mesh views of a workload's host arrays (the arrays are
    appended to `keep`, which must outlive the views)."""
    def h(a, dtype):
        a = _arr(a, dtype)
        keep.append(a)
        return a.ctypes.data, a.shape[0]
    pxyz, nv = h(w.xyz, np.float64)
    ptet, nt = h(w.tets, np.int32)
    psf, nsf = h(w.sf, np.int32)
    psff, _ = h(w.sf_facet, np.int32)
    pss, nss = h(w.ss, np.int32)
    pssg, _ = h(w.ss_seg, np.int32)
    pft, nft = h(w.ftri, np.int32)
    pftf, _ = h(w.ftri_facet, np.int32)
    pseg, nseg = h(w.seg if w.seg is not None else np.zeros((0, 2), np.int32), np.int32)
    return (_Plc(nv, nseg, pseg, nft, pft, pftf),
            _Mesh(nv, pxyz, nt, ptet, nsf, psf, psff, nss, pss, pssg))


def refine_batch(workloads, *, nstreams=8, hmin_factor=0.5, max_rounds=100000, max_kept=0,
                 profile=False, extra_flags=None, return_codes=False) -> list:
    """Refine independent instances concurrently (qm_refine_batch): each
    workload exposes the PLC and CDT arrays and B (host arrays).  With
    return_codes, returns (results, per-instance return codes) and raises
    nothing for failed instances (their result is None)."""
    lib = _load()
    n = len(workloads)
    plcs, meshes, opts, keep = (_Plc * n)(), (_Mesh * n)(), (_Opts * n)(), []
    for i, w in enumerate(workloads):
        plcs[i], meshes[i] = _marshal(w, keep)
        opts[i] = _Opts(float(w.B), float(hmin_factor), int(max_rounds), int(max_kept),
                        _prof_flag(profile) | (int(extra_flags[i]) if extra_flags else 0))
    outs = (ctypes.c_void_p * max(n, 1))()
    codes = (ctypes.c_int32 * max(n, 1))()
    lib.qm_refine_batch.restype = ctypes.c_int
    lib.qm_refine_batch.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    rc = lib.qm_refine_batch(n, ctypes.addressof(plcs), ctypes.addressof(meshes), ctypes.addressof(opts),
                             int(nstreams), ctypes.addressof(outs), ctypes.addressof(codes))
    results = []
    for i in range(n):
        if outs[i]:
            results.append(_take_result(lib, ctypes.c_void_p(outs[i]), profile))
        else:
            results.append(None)
    if return_codes:
        return results, [int(codes[i]) for i in range(n)]
    if rc not in (0, -4):
        raise QmError(rc, lib.qm_last_error().decode())
    return results


class _Tune(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32), ("classify_tiles", ctypes.c_int32), ("rank_max", ctypes.c_int32),
                ("select_one_wg", ctypes.c_int32), ("hybrid_wgs", ctypes.c_int32), ("global_wgs", ctypes.c_int32)]


LOCKSTEP_DEFAULTS = {"groups": 1, "classify_tiles": 8, "rank_max": 4096, "select_one_wg": 65536,
                     "hybrid_wgs": 1024, "global_wgs": 256}


def _batch_arrays(workloads, hmin_factor, max_rounds, max_kept, extra_flags):
    n = len(workloads)
    plcs, meshes, opts, keep = (_Plc * max(n, 1))(), (_Mesh * max(n, 1))(), (_Opts * max(n, 1))(), []
    for i, w in enumerate(workloads):
        plcs[i], meshes[i] = _marshal(w, keep)
        mr = max_rounds[i] if isinstance(max_rounds, (list, tuple)) else max_rounds
        opts[i] = _Opts(float(w.B), float(hmin_factor), int(mr), int(max_kept),
                        int(extra_flags[i]) if extra_flags else 0)
    return plcs, meshes, opts, keep


def refine_lockstep(workloads, *, groups=None, tune=None, hmin_factor=0.5, max_rounds=100000, extra_flags=None,
                    return_codes=False, max_kept=0) -> list:
    """Refine independent instances in lockstep (qm_refine_lockstep): one
    launch per phase per round over all instances of a group.  `tune` is a
    dict of qm_lockstep_tune knobs (missing ones take the defaults), or None
    for one group on the default stream; `groups` overrides tune["groups"].
    max_rounds may be one value or one per instance.  Results and
    return_codes as refine_batch."""
    lib = _load()
    n = len(workloads)
    plcs, meshes, opts, keep = _batch_arrays(workloads, hmin_factor, max_rounds, max_kept, extra_flags)
    knobs = None
    if tune is not None or groups is not None:
        k = dict(LOCKSTEP_DEFAULTS, **(tune or {}))
        if groups is not None:
            k["groups"] = int(groups)
        knobs = _Tune(*[int(k[f]) for f, _ in _Tune._fields_])
    outs = (ctypes.c_void_p * max(n, 1))()
    codes = (ctypes.c_int32 * max(n, 1))()
    lib.qm_refine_lockstep.restype = ctypes.c_int
    lib.qm_refine_lockstep.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rc = lib.qm_refine_lockstep(n, ctypes.addressof(plcs), ctypes.addressof(meshes), ctypes.addressof(opts),
                                None, ctypes.addressof(knobs) if knobs is not None else None,
                                ctypes.addressof(outs), ctypes.addressof(codes))
    results = [_take_result(lib, ctypes.c_void_p(outs[i]), False) if outs[i] else None for i in range(n)]
    if return_codes:
        return results, [int(codes[i]) for i in range(n)]
    if rc not in (0, -4):
        raise QmError(rc, lib.qm_last_error().decode())
    return results


def lockstep_autotune(workloads, *, probe=16, hmin_factor=0.5, max_rounds=100000):
    """Knobs for refine_lockstep chosen by qm_lockstep_autotune on a probe
    batch of `probe` of the workloads; returns (dict of knobs, probe
    seconds)."""
    lib = _load()
    plcs, meshes, opts, keep = _batch_arrays(workloads, hmin_factor, max_rounds, 0, None)
    best = _Tune()
    sec = ctypes.c_double()
    lib.qm_lockstep_autotune.restype = ctypes.c_int
    lib.qm_lockstep_autotune.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    rc = lib.qm_lockstep_autotune(len(workloads), ctypes.addressof(plcs), ctypes.addressof(meshes),
                                  ctypes.addressof(opts), int(probe), ctypes.addressof(best), ctypes.byref(sec))
    if rc:
        raise QmError(rc, lib.qm_last_error().decode())
    return {f: int(getattr(best, f)) for f, _ in _Tune._fields_}, float(sec.value)


def refine_workload(w, **kw) -> RefineResult:
    """Refine a workload object exposing the PLC and CDT arrays
    (xyz, tets, sf, sf_facet, ss, ss_seg, ftri, ftri_facet, seg, B)."""
    return refine(w.xyz, w.tets, w.sf, w.sf_facet, w.ss, w.ss_seg, w.ftri, w.ftri_facet,
                  kw.pop("B", w.B), seg=w.seg, **kw)


def resume(w, r, **kw) -> RefineResult:
    """Continue the refinement of workload ``w`` from result ``r`` (a run cut
    by max_rounds): its output mesh and state, ``w``'s PLC and bound.  In the
    deterministic modes the rounds of ``r`` and of this call together equal
    one uninterrupted refinement."""
    if r.state is None:
        raise ValueError("the result carries no refinement state")
    return refine(r.xyz, r.tets, r.sf, r.sf_facet, r.ss, r.ss_seg, w.ftri, w.ftri_facet,
                  kw.pop("B", w.B), seg=w.seg, state=r.state, **kw)


def test_geometry(op, tuples, param=0.0):
    """Tests only (qm_test_geometry): the device predicates (ops 0-5, signs)
    or constructions (10-13) on an (n, k, 3) array of point tuples; returns
    an (n, 4) array."""
    lib = _load()
    lib.qm_test_geometry.restype = ctypes.c_int
    lib.qm_test_geometry.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_void_p]
    a = np.ascontiguousarray(tuples, dtype=np.float64)
    out = np.zeros((len(a), 4))
    rc = lib.qm_test_geometry(int(op), len(a), a.ctypes.data, float(param), out.ctypes.data)
    if rc != 0:
        raise QmError(rc, lib.qm_last_error().decode())
    return out


def refine_to_device(w, *, hmin_factor=0.5, max_rounds=100000):
    """Refine workload w with QM_OUTPUT_DEVICE: the output mesh stays in
    device memory.  Returns (dict of torch CUDA tensors copied device to
    device from the result's arrays: xyz, tets, sf, sf_facet, ss, ss_seg;
    the result's statistics)."""
    import torch
    lib = _load()
    keep = []
    plc, mesh = _marshal(w, keep)
    opts = _Opts(float(w.B), float(hmin_factor), int(max_rounds), 0, QM_OUTPUT_DEVICE)
    res = ctypes.c_void_p()
    rc = lib.qm_refine(ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(opts), None, ctypes.byref(res))
    if rc not in (0, -4):
        raise QmError(rc, lib.qm_last_error().decode())
    try:
        view, st = _Mesh(), _Stats()
        lib.qm_result_view(res, ctypes.byref(view), ctypes.byref(st))
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        out = {}
        for name, p, n, cols, dt in (("xyz", view.xyz, view.nv, 3, torch.float64), ("tets", view.tet, view.nt, 4, torch.int32),
                                     ("sf", view.sf, view.nsf, 3, torch.int32), ("sf_facet", view.sf_facet, view.nsf, 1, torch.int32),
                                     ("ss", view.ss, view.nss, 2, torch.int32), ("ss_seg", view.ss_seg, view.nss, 1, torch.int32)):
            t = torch.empty((n, cols) if cols > 1 else (n,), dtype=dt, device="cuda")
            if n:
                e = hip.hipMemcpy(t.data_ptr(), p, t.numel() * t.element_size(), 3)   # device to device
                if e != 0:
                    raise QmError(-5, f"hipMemcpy failed ({e})")
            out[name] = t
        return out, {"rounds": int(st.rounds), "nv_out": int(st.nv_out), "nt_out": int(st.nt_out)}
    finally:
        lib.qm_result_free(res)


def version() -> str:
    return _load().qm_version().decode()


def estimate_bytes(w, *, hmin_factor=0.5) -> int:
    """Device bytes the server budgets for refining workload w
    (qm_estimate_bytes; host arithmetic only)."""
    lib = _load()
    lib.qm_estimate_bytes.restype = ctypes.c_size_t
    lib.qm_estimate_bytes.argtypes = [ctypes.POINTER(_Plc), ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts)]
    keep = []
    plc, mesh = _marshal(w, keep)
    opt = _Opts(float(w.B), float(hmin_factor), 1, 0, 0)
    return int(lib.qm_estimate_bytes(ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(opt)))


class _SrvStats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_size_t), ("resident", ctypes.c_size_t), ("queued", ctypes.c_int32),
                ("running", ctypes.c_int32), ("admitted", ctypes.c_int64), ("refused", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("evictions", ctypes.c_int64), ("parked", ctypes.c_int32)]


class Server:
    """Served refinement (qm_server_*): jobs are admitted against a
    device-memory budget and refined by `nworkers` worker threads, each with
    its own HIP stream, on the current device."""

    def __init__(self, hbm_budget_bytes: int, nworkers: int = 8):
        lib = self._lib = _load()
        P = ctypes.c_void_p
        lib.qm_server_create.restype = ctypes.c_int
        lib.qm_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(P)]
        lib.qm_server_submit.restype = ctypes.c_int
        lib.qm_server_submit.argtypes = [P, ctypes.POINTER(_Plc), ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts),
                                         ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64)]
        lib.qm_server_poll.restype = ctypes.c_int
        lib.qm_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(P),
                                       ctypes.POINTER(ctypes.c_int32), P]
        lib.qm_server_info.restype = ctypes.c_int
        lib.qm_server_info.argtypes = [P, ctypes.POINTER(_SrvStats)]
        lib.qm_server_destroy.argtypes = [P]
        lib.qm_estimate_bytes.restype = ctypes.c_size_t
        lib.qm_estimate_bytes.argtypes = [ctypes.POINTER(_Plc), ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts)]
        h = P()
        rc = lib.qm_server_create(int(hbm_budget_bytes), int(nworkers), ctypes.byref(h))
        if rc:
            raise QmError(rc, lib.qm_last_error().decode())
        self._h = h
        self._profile = {}

    @staticmethod
    def _opts(w, hmin_factor, max_rounds, max_kept, profile):
        return _Opts(float(w.B), float(hmin_factor), int(max_rounds), int(max_kept),
                     _prof_flag(profile))

    def estimate_bytes(self, w, *, hmin_factor=0.5) -> int:
        return estimate_bytes(w, hmin_factor=hmin_factor)

    def step(self) -> int:
        """Stepped server (nworkers=0): one round for every resident job
        (qm_server_step); returns the number still resident."""
        self._lib.qm_server_step.restype = ctypes.c_int
        self._lib.qm_server_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
        n = ctypes.c_int32()
        rc = self._lib.qm_server_step(self._h, ctypes.byref(n))
        if rc:
            raise QmError(rc, self._lib.qm_last_error().decode())
        return int(n.value)

    def submit(self, w, *, est_bytes=0, hmin_factor=0.5, max_rounds=100000, max_kept=0, profile=False):
        """Ticket of the admitted job, or None when the budget has no room
        now (QM_EAGAIN)."""
        keep = []
        plc, mesh = _marshal(w, keep)
        opt = self._opts(w, hmin_factor, max_rounds, max_kept, profile)
        t = ctypes.c_uint64()
        rc = self._lib.qm_server_submit(self._h, ctypes.byref(plc), ctypes.byref(mesh), ctypes.byref(opt),
                                        int(est_bytes), ctypes.byref(t))
        if rc == -8:
            return None
        if rc:
            raise QmError(rc, self._lib.qm_last_error().decode())
        self._profile[t.value] = profile
        return t.value

    def poll(self, ticket, wait_ms=0):
        """None while the job runs; else (result or None, code, message,
        seconds queued, seconds from submission to completion)."""
        res, code = ctypes.c_void_p(), ctypes.c_int32()
        sec = (ctypes.c_double * 2)()
        rc = self._lib.qm_server_poll(self._h, int(ticket), int(wait_ms), ctypes.byref(res), ctypes.byref(code),
                                      ctypes.addressof(sec))
        if rc == -8:
            return None
        if rc:
            raise QmError(rc, self._lib.qm_last_error().decode())
        msg = self._lib.qm_last_error().decode()
        prof = self._profile.pop(int(ticket), False)
        out = _take_result(self._lib, res, prof) if res.value else None
        return out, int(code.value), msg, float(sec[0]), float(sec[1])

    def result(self, ticket):
        """Wait for a job and return its RefineResult (QmError if it failed
        or is evicted)."""
        got = self.poll(ticket, wait_ms=-1)
        if got is None:
            raise QmError(-8, self._lib.qm_last_error().decode())
        out, code, msg, _, _ = got
        if code not in (0, -4):
            raise QmError(code, msg)
        return out

    def evict(self, ticket) -> bool:
        """Take a job off the device at a round boundary, its mesh and state
        kept on the host (qm_server_evict).  True when evicted, False when it
        finished first."""
        self._lib.qm_server_evict.restype = ctypes.c_int
        self._lib.qm_server_evict.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        rc = self._lib.qm_server_evict(self._h, int(ticket))
        if rc == -8:
            return False
        if rc:
            raise QmError(rc, self._lib.qm_last_error().decode())
        return True

    def readmit(self, ticket) -> bool:
        """Admit an evicted job again (qm_server_readmit): True when admitted,
        False while the budget has no room."""
        self._lib.qm_server_readmit.restype = ctypes.c_int
        self._lib.qm_server_readmit.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        rc = self._lib.qm_server_readmit(self._h, int(ticket))
        if rc == -8:
            return False
        if rc:
            raise QmError(rc, self._lib.qm_last_error().decode())
        return True

    def info(self) -> dict:
        st = _SrvStats()
        self._lib.qm_server_info(self._h, ctypes.byref(st))
        return {k: int(getattr(st, k)) for k, _ in _SrvStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.qm_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()


class PipelinedServer:
    """Served refinement with the input preparation pipelined, as the
    paper's gQM3D+ splits the work (Section 3): the host builds each job's
    initial Delaunay tetrahedralisation and CDT while the device refines
    other jobs.  submit(prep, *args) runs prep(*args) (which returns a
    workload) on a pool of `prep_threads` host threads; a dispatcher thread
    hands each prepared workload to an underlying Server (`nworkers` device
    workers, `budget` bytes) in the order the preparations finish, waiting
    while the budget has no room.  poll/result give the result with the
    preparation, queueing and total seconds of the job."""

    def __init__(self, budget, nworkers=8, prep_threads=8):
        import collections
        import threading
        from concurrent.futures import ThreadPoolExecutor
        self._srv = Server(budget, nworkers=nworkers)
        self._pool = ThreadPoolExecutor(max_workers=prep_threads)
        self._mu = threading.Condition()
        self._ready = collections.deque()       # (handle, workload or exception, t_prepared)
        self._jobs = {}                         # handle -> dict(t0, t_prep, ticket, error)
        self._next = 1
        self._stop = False
        self._thread = threading.Thread(target=self._dispatch, daemon=True)
        self._thread.start()

    def submit(self, prep, *args) -> int:
        import time
        with self._mu:
            h = self._next
            self._next += 1
            self._jobs[h] = {"t0": time.perf_counter(), "t_prep": None, "ticket": None, "error": None}
        fut = self._pool.submit(prep, *args)

        def done(f, h=h):
            import time
            try:
                item = f.result()
            except Exception as e:          # the preparation failed: the job ends with it
                item = e
            with self._mu:
                self._ready.append((h, item, time.perf_counter()))
                self._mu.notify_all()
        fut.add_done_callback(done)
        return h

    def _dispatch(self):
        import time
        while True:
            with self._mu:
                while not self._ready and not self._stop:
                    self._mu.wait()
                if self._stop:
                    return
                h, item, t_prep = self._ready[0]
            job = self._jobs[h]
            if isinstance(item, Exception):
                tk, err = None, item
            else:
                try:
                    tk, err = self._srv.submit(item), None
                except QmError as e:
                    tk, err = None, e
                if tk is None and err is None:    # no room yet: wait for completions
                    time.sleep(0.0005)
                    continue
            with self._mu:
                self._ready.popleft()
                job["t_prep"] = t_prep - job["t0"]
                job["ticket"], job["error"] = tk, err
                self._mu.notify_all()

    def poll(self, handle, wait_ms=0):
        """None while the job is being prepared, queued or refined; else
        (result or None, code, message, preparation s, total s)."""
        import time
        deadline = None if wait_ms < 0 else time.perf_counter() + wait_ms / 1000.0
        while True:
            with self._mu:
                job = self._jobs[handle]
                if job["error"] is not None:
                    del self._jobs[handle]
                    e = job["error"]
                    return None, getattr(e, "code", -1), str(e), job["t_prep"] or 0.0, \
                        time.perf_counter() - job["t0"]
                tk = job["ticket"]
            if tk is not None:
                got = self._srv.poll(tk, wait_ms=0)
                if got is not None:
                    res, code, msg, _, _ = got
                    with self._mu:
                        del self._jobs[handle]
                    return res, code, msg, job["t_prep"], time.perf_counter() - job["t0"]
            if deadline is not None and time.perf_counter() >= deadline:
                return None
            time.sleep(0.0005)

    def result(self, handle):
        out, code, msg, _, _ = self.poll(handle, wait_ms=-1)
        if code not in (0, -4):
            raise QmError(code, msg)
        return out

    def close(self):
        with self._mu:
            self._stop = True
            self._mu.notify_all()
        self._thread.join()
        self._pool.shutdown(wait=True)
        self._srv.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
