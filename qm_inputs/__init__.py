"""Seeded synthetic workloads for the constrained Delaunay refinement loop.

This module holds the input generators only: point sets, the initial
Delaunay tetrahedralisation (built by ``qmi_dt.c``) and the piecewise linear
complex (PLC) read off it.  It contains none of the refinement arithmetic;
both the oracle and the GPU library receive its arrays.

Conventions shared by every workload (the reading of the paper's Section 1
data model used throughout):

* coordinates are FP64 multiples of 2^-53 inside the closed unit cube;
* vertices 0..7 are the cube corners, corner ``i = (i&1, (i>>1)&1, (i>>2)&1)``;
  the remaining vertices lie strictly inside and are numbered in Morton
  order of their coordinates (spatially coherent ids);
* the PLC always contains the six cube faces as facets 0..5 (facet
  ``2*axis + side``), each given by its two hull triangles, and the twelve
  cube edges as segments 0..11; internal constraint surfaces add one facet
  per Delaunay face and one segment per distinct edge of those faces, and
  rectangle PLCs (``rectangles_plc``) one facet per rectangle and one segment
  per Delaunay edge along its sides;
* the initial CDT is the Delaunay tetrahedralisation itself: its subfaces are
  the PLC triangles and its subsegments the PLC segments.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qmi_dt.c")
_SO = os.path.join(_HERE, "_qmi_dt.so")
_lib = None

LATTICE_BITS = 53


def build() -> str:
    """Compile the Delaunay builder into an in-tree shared object."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is not built; run qm_inputs.build()")
        lib = ctypes.CDLL(_SO)
        lib.qmi_delaunay.restype = ctypes.c_int
        lib.qmi_delaunay.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                     ctypes.c_void_p]
        _lib = lib
    return _lib


def snap(x: np.ndarray) -> np.ndarray:
    """Round to the nearest multiple of 2^-53 (exact in FP64)."""
    return np.ldexp(np.rint(np.ldexp(np.asarray(x, dtype=np.float64), LATTICE_BITS)),
                    -LATTICE_BITS)


def corners() -> np.ndarray:
    i = np.arange(8)
    return np.stack([(i & 1), (i >> 1) & 1, (i >> 2) & 1], axis=1).astype(np.float64)


def _morton(pts: np.ndarray, bits: int = 10) -> np.ndarray:
    q = np.minimum((pts * (1 << bits)).astype(np.int64), (1 << bits) - 1)
    code = np.zeros(len(pts), dtype=np.int64)
    for b in range(bits):
        for k in range(3):
            code |= ((q[:, k] >> b) & 1) << (3 * b + k)
    return code


def finalize_points(interior: np.ndarray) -> np.ndarray:
    """Snap, keep strictly-interior distinct points, Morton-order, add corners."""
    p = snap(interior)
    ok = np.all((p > 0.0) & (p < 1.0), axis=1)
    p = p[ok]
    p = np.unique(p, axis=0)            # exact duplicates removed (sorted)
    order = np.argsort(_morton(p), kind="stable")
    return np.concatenate([corners(), p[order]], axis=0)


def uniform_interior(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform points of the open unit cube (exact zeros are redrawn)."""
    p = rng.random((n, 3))
    bad = np.any(p == 0.0, axis=1)
    while bad.any():
        p[bad] = rng.random((int(bad.sum()), 3))
        bad = np.any(p == 0.0, axis=1)
    return p


def gaussmix_interior(rng: np.random.Generator, n: int, ncomp: int = 8,
                      sigma: float = 0.05) -> np.ndarray:
    """n points from ncomp equal-weight isotropic Gaussians with centres in
    [0.2,0.8]^3, redrawn until strictly inside the unit cube."""
    centres = rng.uniform(0.2, 0.8, size=(ncomp, 3))
    comp = rng.integers(0, ncomp, size=n)
    p = centres[comp] + sigma * rng.standard_normal((n, 3))
    bad = np.any((p <= 0.0) | (p >= 1.0), axis=1)
    while bad.any():
        k = int(bad.sum())
        p[bad] = centres[comp[bad]] + sigma * rng.standard_normal((k, 3))
        bad = np.any((p <= 0.0) | (p >= 1.0), axis=1)
    return p


def delaunay(xyz: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Delaunay tetrahedralisation (tets positively oriented, adjacency t<<2|f)."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    n = len(xyz)
    cap = 8 * n + 64
    tets = np.empty((cap, 4), dtype=np.int32)
    adj = np.empty((cap, 4), dtype=np.int32)
    nt = ctypes.c_int(0)
    rc = lib.qmi_delaunay(n, xyz.ctypes.data, cap, ctypes.byref(nt),
                          tets.ctypes.data, adj.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"qmi_delaunay failed with code {rc}")
    return tets[:nt.value].copy(), adj[:nt.value].copy()


# inward face triples of a positively oriented tet (face i is opposite v_i)
FACE = np.array([[1, 3, 2], [0, 2, 3], [0, 3, 1], [0, 1, 2]], dtype=np.int64)


def centroids(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    a, b, c, d = (xyz[tets[:, k]] for k in range(4))
    return ((a + b) + (c + d)) * 0.25


@dataclass
class Workload:
    """One refinement instance: PLC + initial CDT + quality bound."""
    name: str
    xyz: np.ndarray            # (nv,3) f64
    tets: np.ndarray           # (nt,4) i32, positively oriented
    adj: np.ndarray            # (nt,4) i32, t<<2|f or -1
    ftri: np.ndarray           # (nftri,3) i32  PLC polygons as triangles
    ftri_facet: np.ndarray     # (nftri,) i32   polygon (facet) id
    seg: np.ndarray            # (nseg,2) i32   PLC segments
    B: float
    meta: dict = field(default_factory=dict)

    @property
    def sf(self):
        return self.ftri

    @property
    def sf_facet(self):
        return self.ftri_facet

    @property
    def ss(self):
        return self.seg

    @property
    def ss_seg(self):
        return np.arange(len(self.seg), dtype=np.int32)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.xyz, self.tets, self.ftri, self.ftri_facet, self.seg):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(repr(self.B).encode())
        return h.hexdigest()


def _faces_of(tets: np.ndarray, adj: np.ndarray):
    """Yield (tet index, face index) arrays of faces, and their neighbours."""
    t = np.repeat(np.arange(len(tets)), 4)
    f = np.tile(np.arange(4), len(tets))
    return t, f, adj.reshape(-1)


def build_plc(xyz: np.ndarray, tets: np.ndarray, adj: np.ndarray, inside_fns=()):
    """Hull facets + cube-edge segments, plus one facet per Delaunay face that
    separates a tet whose centroid satisfies ``fn`` from one that does not,
    for each ``fn`` in inside_fns; every edge of such a face is a segment."""
    t, f, nb = _faces_of(tets, adj)
    fv = np.sort(tets[t[:, None], FACE[f]], axis=1)        # sorted face triples
    # hull triangles, grouped by cube face
    hull = nb < 0
    hv = fv[hull]
    hx = xyz[hv]                                           # (h,3,3)
    facet_of = np.full(len(hv), -1, dtype=np.int64)
    for axis in range(3):
        for side in (0, 1):
            on = np.all(hx[:, :, axis] == float(side), axis=1)
            facet_of[on] = 2 * axis + side
    if np.any(facet_of < 0):
        raise RuntimeError("hull face not on a cube face")
    order = np.lexsort((hv[:, 2], hv[:, 1], hv[:, 0], facet_of))
    tri = [hv[order]]
    tri_facet = [facet_of[order]]
    # cube edges: corners differing in one coordinate
    segs = [(i, j) for i in range(8) for j in range(i + 1, 8) if bin(i ^ j).count("1") == 1]
    seg = [np.array(segs, dtype=np.int64)]
    if inside_fns:
        cen = centroids(xyz, tets)
        inner = (~hull) & (t < (nb >> 2))                  # each interior face once
        ti, ni = t[inner], nb[inner] >> 2
        sep = np.zeros(len(ti), dtype=bool)
        for fn in inside_fns:
            ins = fn(cen)
            sep |= ins[ti] != ins[ni]
        sv = fv[inner][sep]
        sv = sv[np.lexsort((sv[:, 2], sv[:, 1], sv[:, 0]))]
        tri.append(sv)
        tri_facet.append(6 + np.arange(len(sv)))
        e = np.concatenate([sv[:, [0, 1]], sv[:, [0, 2]], sv[:, [1, 2]]], axis=0)
        e = np.unique(e, axis=0)
        seg.append(e)
    return (np.concatenate(tri).astype(np.int32), np.concatenate(tri_facet).astype(np.int32),
            np.concatenate(seg).astype(np.int32))


def sphere_inside(r: float, c=(0.5, 0.5, 0.5)):
    c = np.asarray(c, dtype=np.float64)
    rr = r * r

    def fn(x):
        d = x - c
        return ((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]) < rr
    return fn


def ellipsoid_inside(axes, rot, c=(0.5, 0.5, 0.5)):
    c = np.asarray(c, dtype=np.float64)
    axes = np.asarray(axes, dtype=np.float64)

    def fn(x):
        y = (x - c) @ rot            # R^T (x - c) for row vectors
        y = y / axes
        return ((y[:, 0] * y[:, 0] + y[:, 1] * y[:, 1]) + y[:, 2] * y[:, 2]) < 1.0
    return fn


def quat_rotation(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def make_workload(name: str, interior: np.ndarray, B: float, inside_fns=(), meta=None) -> Workload:
    xyz = finalize_points(interior)
    tets, adj = delaunay(xyz)
    ftri, ftri_facet, seg = build_plc(xyz, tets, adj, inside_fns)
    return Workload(name, xyz, tets, adj, ftri, ftri_facet, seg, float(B), dict(meta or {}))


def uniform_cube(n: int, seed: int, B: float = 2.0, spheres=(), name=None) -> Workload:
    """Corners + n uniform points; optional spherical constraint surfaces."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = uniform_interior(rng, n)
    fns = [sphere_inside(r) for r in spheres]
    return make_workload(name or f"uniform{n}_s{seed}", pts, B, fns,
                         {"n": n, "seed": seed, "spheres": list(spheres)})


def config(k: int, instance: int = 0) -> Workload:
    """The five synthetic workloads (k = 1..4; k = 4 takes an instance index).

    1: corners + 1 000 uniform points, hull PLC, B = 2.0.
    2: corners + 50 000 uniform points, hull + sphere r = 0.3 surface, B = 1.5.
    3: corners + 900 000 points from 8 Gaussians (sigma 0.05) + 100 000
       uniform, hull + spheres r = 0.15/0.30/0.45, B = 1.4.
    4: instance i of 256: log-uniform n in [2 000, 200 000] uniform points,
       hull + one randomly rotated ellipsoid surface, B = 2.0.
    """
    if k == 1:
        return uniform_cube(1000, seed=1, B=2.0, name="cfg1_uniform1k")
    if k == 2:
        return uniform_cube(50000, seed=2, B=1.5, spheres=(0.3,), name="cfg2_uniform50k_sphere")
    if k == 3:
        rng = np.random.Generator(np.random.PCG64(3))
        g = gaussmix_interior(rng, 900000)
        u = uniform_interior(rng, 100000)
        fns = [sphere_inside(r) for r in (0.15, 0.30, 0.45)]
        return make_workload("cfg3_gauss1m_3spheres", np.concatenate([g, u]), 1.4, fns,
                             {"n": 1000000, "seed": 3})
    if k == 4:
        ss = np.random.SeedSequence(4).spawn(256)[instance]
        rng = np.random.Generator(np.random.PCG64(ss))
        n = int(np.floor(np.exp(rng.uniform(np.log(2000.0), np.log(200000.0)))))
        axes = rng.uniform(0.15, 0.40, size=3)
        rot = quat_rotation(rng.standard_normal(4))
        pts = uniform_interior(rng, n)
        return make_workload(f"cfg4_inst{instance}", pts, 2.0, [ellipsoid_inside(axes, rot)],
                             {"n": n, "instance": instance})
    raise ValueError(f"unknown workload {k}")


def serve_job(i: int, max_points: int = 500000, seed: int = 5) -> Workload:
    """Job i of the served workload: n log-uniform in [1 000, max_points];
    half the jobs use the clustered generator of workload 3 (90% from 8
    Gaussians, 10% uniform, three nested spheres), half the one of workload 4
    (uniform, one rotated ellipsoid); B drawn from {1.4, 2.0}."""
    ss = np.random.SeedSequence(seed).spawn(i + 1)[i]
    rng = np.random.Generator(np.random.PCG64(ss))
    n = int(np.floor(np.exp(rng.uniform(np.log(1000.0), np.log(float(max_points))))))
    B = 1.4 if rng.uniform() < 0.5 else 2.0
    if rng.uniform() < 0.5:
        ng = (9 * n) // 10
        pts = np.concatenate([gaussmix_interior(rng, ng), uniform_interior(rng, n - ng)])
        fns = [sphere_inside(r) for r in (0.15, 0.30, 0.45)]
        kind = "clustered"
    else:
        axes = rng.uniform(0.15, 0.40, size=3)
        rot = quat_rotation(rng.standard_normal(4))
        pts = uniform_interior(rng, n)
        fns = [ellipsoid_inside(axes, rot)]
        kind = "ellipsoid"
    return make_workload(f"serve_job{i}_{kind}{n}", pts, B, fns, {"n": n, "job": i, "kind": kind})


def rectangles_plc(n: int, gamma: float, seed: int, B: float = 1.4, dist: str = "uniform",
                   lattice: int = 3, name=None) -> Workload:
    """A PLC of the kind the paper's experiments use (Section 3, Table 1):
    n points, of which round(gamma * n) polygons are axis-aligned rectangles
    whose four corners are PLC points; the other points are uniform
    (``dist="uniform"``) or from the Gaussian mixture of workload 3
    (``dist="gauss"``).

    The paper's inputs are made a CDT by TetGen's constraint recovery, which
    is not built here.  Instead each rectangle is split in advance so that
    the Delaunay tetrahedralisation of all points conforms to it:

    * the cube is cut into k^3 cells (k^3 >= the number of rectangles); each
      rectangle lies in a cell of its own, chosen at random, in a plane
      normal to a random axis, with a random size and position inside the
      cell;
    * every rectangle carries a (lattice+1) x (lattice+1) grid of points,
      exactly in its plane and on its sides (coordinates on the 2^-53 grid).
      The grid points inside the rectangle are moved by up to 15% of the
      spacing within the plane, and those on a side are moved along it, so
      that no four are cocircular;
    * no other point lies within twice the grid spacing of the rectangle's
      plane over the rectangle grown by that margin.  A Delaunay triangle of
      the grid then has an empty equatorial ball in 3D, so the rectangle is
      a union of Delaunay faces and its sides unions of Delaunay edges.

    Both facts are checked on the result: the Delaunay faces with all three
    vertices on one rectangle cover its area, and every pair of consecutive
    points of a side is a Delaunay edge.  Each rectangle is one facet (id 6 +
    its index); each edge between consecutive side points is a segment.
    The grid points are Steiner points of the recovery, so gamma counts the
    rectangles against the PLC's own points (corners and others)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nrect = int(round(gamma * n))
    nother = n - 4 * nrect
    if nrect < 0 or nother < 0 or lattice < 3:
        raise ValueError("need 4 * round(gamma * n) <= n and lattice >= 3")
    k = max(1, int(np.ceil(nrect ** (1.0 / 3.0) - 1e-9)))
    while k ** 3 < nrect:
        k += 1
    cell = 1.0 / k
    cells = rng.choice(k ** 3, size=nrect, replace=False)
    boxes = np.zeros((nrect, 2, 3))
    rect = []                                          # (axis, plane, lo(2), hi(2)) per rectangle
    pts = []
    sides = []                                         # per rectangle: 4 lists of point indices along its sides
    base = 0
    for r, c in enumerate(cells):
        ci = np.array([c % k, (c // k) % k, c // (k * k)], dtype=np.float64)
        lo_cell, hi_cell = ci * cell, (ci + 1) * cell
        axis = int(rng.integers(0, 3))
        u, v = [a for a in range(3) if a != axis]
        size = rng.uniform(0.2, 0.35, size=2) * cell     # size (1 + 4 / lattice) <= cell for lattice >= 3
        h = float(np.max(size)) / lattice
        m = 2.0 * h                                    # slab margin
        # rectangle and its slab inside the cell (away from the cube faces)
        lo = np.empty(2)
        for j, a in enumerate((u, v)):
            lo[j] = rng.uniform(lo_cell[a] + m, hi_cell[a] - m - size[j])
        plane = snap(rng.uniform(lo_cell[axis] + m, hi_cell[axis] - m))
        lo = snap(lo)
        hi = snap(lo + size)
        # grid with in-plane jitter (sides move along themselves, corners stay)
        gi = np.arange(lattice + 1)
        I, J = np.meshgrid(gi, gi, indexing="ij")
        I, J = I.reshape(-1), J.reshape(-1)
        su, sv = (hi[0] - lo[0]) / lattice, (hi[1] - lo[1]) / lattice
        pu = lo[0] + I * su + rng.uniform(-0.15, 0.15, size=len(I)) * su
        pv = lo[1] + J * sv + rng.uniform(-0.15, 0.15, size=len(J)) * sv
        on_u = (I == 0) | (I == lattice)
        on_v = (J == 0) | (J == lattice)
        pu = np.where(I == 0, lo[0], np.where(I == lattice, hi[0], pu))
        pv = np.where(J == 0, lo[1], np.where(J == lattice, hi[1], pv))
        # a point on a side keeps that side's coordinate; pu/pv already hold it
        p = np.empty((len(I), 3))
        p[:, axis] = plane
        p[:, u] = snap(pu)
        p[:, v] = snap(pv)
        p[:, u] = np.where(on_u, np.where(I == 0, lo[0], hi[0]), p[:, u])
        p[:, v] = np.where(on_v, np.where(J == 0, lo[1], hi[1]), p[:, v])
        pts.append(p)
        idx = base + np.arange(len(I))
        sides.append([idx[(I == 0)][np.argsort(J[I == 0])], idx[(I == lattice)][np.argsort(J[I == lattice])],
                      idx[(J == 0)][np.argsort(I[J == 0])], idx[(J == lattice)][np.argsort(I[J == lattice])]])
        rect.append((axis, plane, lo.copy(), hi.copy(), base, len(I)))
        base += len(I)
        box_lo = np.empty(3); box_hi = np.empty(3)
        box_lo[axis], box_hi[axis] = plane - m, plane + m
        box_lo[u], box_hi[u] = lo[0] - m, hi[0] + m
        box_lo[v], box_hi[v] = lo[1] - m, hi[1] + m
        boxes[r] = (box_lo, box_hi)
    rect_pts = np.concatenate(pts) if pts else np.zeros((0, 3))
    # the other points, outside every slab
    other = np.zeros((0, 3))
    while len(other) < nother:
        want = nother - len(other)
        if dist == "uniform":
            q = uniform_interior(rng, want)
        elif dist == "gauss":
            q = gaussmix_interior(rng, want)
        else:
            raise ValueError("dist is 'uniform' or 'gauss'")
        q = snap(q)
        cidx = np.minimum((q / cell).astype(np.int64), k - 1)
        cid = cidx[:, 0] + k * cidx[:, 1] + k * k * cidx[:, 2]
        slot = np.full(k ** 3, -1, dtype=np.int64)
        slot[cells] = np.arange(nrect)
        rr = slot[cid]
        inside = np.zeros(len(q), dtype=bool)
        has = rr >= 0
        if has.any():
            bl, bh = boxes[rr[has], 0], boxes[rr[has], 1]
            inside[has] = np.all((q[has] >= bl) & (q[has] <= bh), axis=1)
        ok = ~inside & np.all((q > 0.0) & (q < 1.0), axis=1)
        other = np.concatenate([other, q[ok]])
    allp = np.concatenate([rect_pts, other[:nother]])
    if len(np.unique(allp, axis=0)) != len(allp):
        raise RuntimeError("coincident points")
    order = np.argsort(_morton(allp), kind="stable")
    xyz = np.concatenate([corners(), allp[order]], axis=0)
    vid = np.empty(len(allp), dtype=np.int64)
    vid[order] = 8 + np.arange(len(allp))
    tets, adj = delaunay(xyz)
    ftri, ftri_facet, seg = build_plc(xyz, tets, adj)
    # Delaunay faces (each once) and edges
    t, f, nb = _faces_of(tets, adj)
    once = (nb < 0) | (t < (nb >> 2))
    fv = np.sort(tets[t[once][:, None], FACE[f[once]]], axis=1)
    owner = np.full(len(xyz), -1, dtype=np.int64)
    for r, (_, _, _, _, b0, cnt) in enumerate(rect):
        owner[vid[b0:b0 + cnt]] = r
    o = owner[fv]
    same = (o[:, 0] >= 0) & (o[:, 0] == o[:, 1]) & (o[:, 0] == o[:, 2])
    tri, tri_rect = fv[same], o[same, 0]
    # coverage: the faces on each rectangle tile its area
    a, b_, c_ = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b_ - a, c_ - a), axis=1)
    cover = np.bincount(tri_rect, weights=area, minlength=nrect)
    want = np.array([(hi[0] - lo[0]) * (hi[1] - lo[1]) for (_, _, lo, hi, _, _) in rect])
    if nrect and np.max(np.abs(cover - want) / want) > 1e-9:
        raise RuntimeError("a rectangle is not a union of Delaunay faces")
    e6 = np.concatenate([tets[:, [0, 1]], tets[:, [0, 2]], tets[:, [0, 3]], tets[:, [1, 2]], tets[:, [1, 3]],
                         tets[:, [2, 3]]]).astype(np.int64)
    e6.sort(axis=1)
    ekeys = np.unique(e6[:, 0] * (1 << 32) + e6[:, 1])
    sseg = []
    for r in range(nrect):
        for side in sides[r]:
            ids = vid[side]
            sseg.append(np.stack([ids[:-1], ids[1:]], axis=1))
    sseg = np.sort(np.concatenate(sseg), axis=1) if sseg else np.zeros((0, 2), dtype=np.int64)
    if len(sseg) and not np.all(np.isin(sseg[:, 0] * (1 << 32) + sseg[:, 1], ekeys)):
        raise RuntimeError("a rectangle side is not a union of Delaunay edges")
    order_t = np.lexsort((tri[:, 2], tri[:, 1], tri[:, 0], tri_rect))
    ftri = np.concatenate([ftri, tri[order_t]]).astype(np.int32)
    ftri_facet = np.concatenate([ftri_facet, 6 + tri_rect[order_t]]).astype(np.int32)
    seg = np.concatenate([seg, sseg]).astype(np.int32)
    return Workload(name or f"rect{n}_g{gamma}_{dist}_s{seed}", xyz, tets, adj, ftri, ftri_facet, seg, float(B),
                    {"n": n, "gamma": gamma, "rectangles": nrect, "dist": dist, "seed": seed,
                     "grid_points": int(len(rect_pts)), "lattice": lattice})
