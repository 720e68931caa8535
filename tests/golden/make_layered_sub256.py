"""Writes layered_sub256.json: the oracle's hierarchy fingerprint and FP64 PCG
solution for the 256^3 system sampled from the 512^3 layered field
(problems.layered_subsampled(512, seed=2)).  Calls only the oracle; run from
the repository root:  python tests/golden/make_layered_sub256.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1209_0960_amd import problems as P  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    t = time.time()
    s = P.layered_subsampled(512, seed=2)
    print(f"system {s.n} rows {s.nnz} nnz ({time.time() - t:.1f} s)", flush=True)
    t = time.time()
    H = O.Hierarchy(s.rowptr, s.colind, s.vals, vcycle_fp32=0)
    print(f"oracle setup {time.time() - t:.1f} s, {H.levels} levels", flush=True)
    levels = []
    for l in range(H.levels):
        L = H.level(l)
        levels.append({"n": int(L.n), "nnz": int(L.nnz), "ncolours": int(L.ncol),
                       "agg_sha256": sha(L.agg.astype(np.int32)) if L.agg is not None else None,
                       "colour_sha256": sha(L.colour.astype(np.int32)),
                       "rowptr_sha256": sha(L.rowptr.astype(np.int32)),
                       "colind_sha256": sha(L.colind.astype(np.int32)),
                       "vals_sha256": sha(L.vals.astype(np.float64))})
    t = time.time()
    out = H.pcg(s.b, rtol=1e-8)
    print(f"oracle PCG {time.time() - t:.1f} s, {out['iterations']} iterations", flush=True)
    x = np.asarray(out["x"])
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(s.n, size=4096, replace=False))
    res = {
        "source": "oracle (oracle/amg_oracle.cpp), FP64 V-cycle PCG, default parameters, rtol 1e-8",
        "system": "problems.layered_subsampled(512, seed=2): layered K sampled at even cells of the 512^3 field",
        "n": s.n, "nnz": s.nnz, "levels": levels, "iterations": int(out["iterations"]),
        "res_hist": [float(v) for v in out["res_hist"]],
        "x_norm": float(np.linalg.norm(x)), "sample_rows": idx.tolist(), "x_sample": x[idx].tolist(),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "layered_sub256.json"), "w") as f:
        json.dump(res, f)
    H.close()


if __name__ == "__main__":
    main()
