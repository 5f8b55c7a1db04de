"""Write the stored expected values for the full-size parity tests.

Calls only the seeded input generator and the oracle; the GPU path is never
involved.  Each record holds SHA-256 digests of the canonical output (tets
as sorted vertex-id tuples in lexicographic order, coordinates as raw FP64
bytes, subfaces and subsegments with their facet / segment ids) and of the
per-round records, plus the sizes.

    python tests/golden/make_golden.py cfg2            # full refinement
    python tests/golden/make_golden.py cfg3 --rounds 8
    python tests/golden/make_golden.py cfg3 --rounds 1099   # about 3.4 h of oracle time
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import qm_inputs as qi  # noqa: E402


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["cfg1", "cfg2", "cfg3"])
    ap.add_argument("--rounds", type=int, default=100000)
    args = ap.parse_args()
    w = qi.config(int(args.config[-1]))
    t0 = time.time()
    r = oracle.refine(w, max_rounds=args.rounds)
    rec = {"workload": w.name, "input_sha256": w.sha256(), "max_rounds": args.rounds,
           "oracle_seconds": round(time.time() - t0, 1), **canonical(r)}
    name = f"{args.config}_rounds{args.rounds}" if args.rounds < 100000 else args.config
    out = os.path.join(HERE, f"{name}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out, rec)


if __name__ == "__main__":
    main()
