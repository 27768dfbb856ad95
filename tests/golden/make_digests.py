"""Write tests/golden/digests.json: oracle results for the larger seeded
workloads, so GPU parity tests at those sizes need not re-run the oracle.

Every value is computed by ``oracle/`` alone from inputs drawn by
``graphgen`` (never from the GPU library).  Per workload it stores m, the
triangle count, the SHA-256 of the canonical-order support array (int32
little-endian), and, where the decomposition is affordable, kmax, the
SHA-256 of the truss numbers and, for each requested k, |F_k| and the SHA-256
of the k-truss mask (uint8).

Usage:  python tests/golden/make_digests.py [name ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "digests.json")

# name -> (generator call, decomposition route or None, ks)
WORKLOADS = {
    "rmat_s16_ef16_seed1": (lambda: gg.rmat(16, 16, seed=1), "peel", [3, 4, 5, 6]),
    "rmat_s18_ef16_seed1": (lambda: gg.rmat(18, 16, seed=1), "peel", [3, 4, 5, 6]),
    "rmat_s20_ef16_seed1": (lambda: gg.rmat(20, 16, seed=1), "peel", [3, 4, 5, 6]),
    "er_n20_m16n_seed2": (lambda: gg.er(1 << 20, 16 << 20, seed=2), "peel", [3, 4]),
    "rmat_s22_ef16_seed1": (lambda: gg.rmat(22, 16, seed=1), "search", [3, 4, 5, 6]),
    "rmat_s24_ef16_seed1": (lambda: gg.rmat(24, 16, seed=1), "search", [3, 4, 5, 6]),
    "er_n24_m16n_seed2": (lambda: gg.er(1 << 24, 16 << 24, seed=2), "search", [3, 4]),
}


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def digest(name: str, stored: dict | None = None) -> dict:
    """The record of one workload.  With ``stored``, only the decomposition
    is computed and added to a copy of it."""
    gen, decomp, ks = WORKLOADS[name]
    t0 = time.time()
    src, dst, n = gen()
    u, v = oracle.normalise(src, dst, n)
    del src, dst
    rec = {"n": int(n), "m": int(len(u)), "edges_sha256": sha(np.stack([u, v], 1))}
    print(name, "normalised", len(u), "%.1fs" % (time.time() - t0), flush=True)
    if stored is not None:
        for key in ("n", "m", "edges_sha256"):
            assert stored[key] == rec[key], (name, key)
        rec = dict(stored)
        t0 -= stored.get("oracle_seconds", 0.0)
    else:
        rec["triangles"] = oracle.triangle_count(n, u, v)
        print(name, "T", rec["triangles"], "%.1fs" % (time.time() - t0), flush=True)
        sup = oracle.support(n, u, v, "listing")
        assert int(sup.astype(np.int64).sum()) == 3 * rec["triangles"]
        rec["support_sha256"] = sha(sup.astype("<i4"))
        rec["support_max"] = int(sup.max()) if len(sup) else 0
        print(name, "support", "%.1fs" % (time.time() - t0), flush=True)
        del sup
    if decomp:
        tau, kmax = oracle.truss_decomposition(n, u, v, decomp)
        rec["kmax"] = kmax
        rec["truss_sha256"] = sha(tau.astype("<i4"))
        rec["ktruss"] = {}
        for k in ks:
            mask = (tau >= k).astype(np.uint8)
            rec["ktruss"][str(k)] = {"m_k": int(mask.sum()), "mask_sha256": sha(mask)}
        print(name, "decomposition kmax", kmax, "%.1fs" % (time.time() - t0), flush=True)
    rec["oracle_seconds"] = round(time.time() - t0, 1)
    return rec


def main(args):
    add_truss = "--add-truss" in args
    names = [a for a in args if a != "--add-truss"]
    for name in names or list(WORKLOADS):
        rec = None
        if add_truss:
            with open(OUT) as f:
                rec = json.load(f)[name]
        rec = digest(name, rec)
        # re-read before writing: several workloads may run side by side
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as f:
                data = json.load(f)
        data[name] = rec
        tmp = "%s.%d.tmp" % (OUT, os.getpid())
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
