"""Mesh quality reports of a refinement's output (host-side numpy analysis,
not part of the refinement): radius-edge ratios, the quality measure the
bound B applies to (paper, Section 1), and dihedral angles, whose
distribution the paper compares between meshers (Section 4, Fig. 2)."""
import numpy as np

_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def radius_edge(xyz, tets, chunk=1 << 20):
    """Circumradius over shortest edge of each tet (float64)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets)
    out = np.empty(len(tets))
    for lo in range(0, len(tets), chunk):
        t = tets[lo:lo + chunk]
        a = xyz[t[:, 0]]
        u, v, w = xyz[t[:, 1]] - a, xyz[t[:, 2]] - a, xyz[t[:, 3]] - a
        # circumcentre offset from a: solves [u;v;w] c = (|u|^2, |v|^2, |w|^2) / 2
        uv, vw, wu = np.cross(u, v), np.cross(v, w), np.cross(w, u)
        det = np.einsum("ij,ij->i", u, vw)
        c = (np.einsum("ij,ij->i", u, u)[:, None] * vw + np.einsum("ij,ij->i", v, v)[:, None] * wu
             + np.einsum("ij,ij->i", w, w)[:, None] * uv) / (2.0 * det)[:, None]
        r = np.sqrt(np.einsum("ij,ij->i", c, c))
        p = xyz[t]
        lmin = np.min([np.linalg.norm(p[:, i] - p[:, j], axis=1) for i, j in _EDGES], axis=0)
        out[lo:lo + chunk] = r / lmin
    return out


def dihedral_angles(xyz, tets, chunk=1 << 20):
    """The six interior dihedral angles of each tet in degrees, shape (nt, 6):
    the angle at edge (i, j) between the two faces that share it."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets)
    out = np.empty((len(tets), 6))
    for lo in range(0, len(tets), chunk):
        p = xyz[tets[lo:lo + chunk]]
        for e, (i, j) in enumerate(_EDGES):
            k, l = [m for m in range(4) if m not in (i, j)]
            d = p[:, j] - p[:, i]
            d /= np.linalg.norm(d, axis=1)[:, None]
            # components of the two other vertices orthogonal to the edge
            a, b = p[:, k] - p[:, i], p[:, l] - p[:, i]
            a -= np.einsum("ij,ij->i", a, d)[:, None] * d
            b -= np.einsum("ij,ij->i", b, d)[:, None] * d
            cosang = np.einsum("ij,ij->i", a, b) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
            out[lo:lo + chunk, e] = np.degrees(np.arccos(np.clip(cosang, -1.0, 1.0)))
    return out


def report(xyz, tets, B, bin_deg=10):
    """Summary: tets over the bound, ratio extremes, dihedral extremes and a
    histogram of all dihedral angles in `bin_deg` bins over [0, 180]."""
    rho = radius_edge(xyz, tets)
    dih = dihedral_angles(xyz, tets)
    hist, _ = np.histogram(dih, bins=np.arange(0, 180 + bin_deg, bin_deg))
    return {"tets": int(len(tets)), "over_B": int(np.count_nonzero(rho > B)),
            "over_B_frac": float(np.count_nonzero(rho > B) / max(len(tets), 1)),
            "ratio_max": float(rho.max()) if len(rho) else 0.0,
            "ratio_median": float(np.median(rho)) if len(rho) else 0.0,
            "dihedral_min_deg": float(dih.min()) if len(dih) else 0.0,
            "dihedral_max_deg": float(dih.max()) if len(dih) else 0.0,
            "dihedral_hist": {"bin_deg": bin_deg, "counts": hist.tolist()}}
