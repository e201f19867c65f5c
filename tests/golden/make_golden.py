"""Writes oracle_8x8.json: the FP64 oracle's output on a tiny seeded input.
Calls only oracle/ and the seeded generator; rerun only when the oracle's
arithmetic changes for a reason stated in the commit."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle.ils import ils  # noqa: E402
from synth import voronoi_image  # noqa: E402

f = voronoi_image(8, 8, 1, 4, 0.05, seed=123)[0].astype("float64")
lam, p, eps, N = 1.0, 0.8, 1e-4, 4
u = ils(f, lam, p, eps, N)
out = {"lam": lam, "p": p, "eps": eps, "N": N, "f": f.tolist(), "u": u.tolist()}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_8x8.json"), "w") as fh:
    json.dump(out, fh, indent=1)
