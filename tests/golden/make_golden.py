"""Writes oracle_uniform2d.json: the oracle's selections, means and scales on
the first 8 locations of the 2-d uniform workload (N = 4000, n = 50, 500
candidates), exhaustive and ray (2 rays) search.  Calls only the oracle;
floats are stored as hex so the fixture pins every bit.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1409_0074_amd import workloads as W  # noqa: E402


def main():
    w = W.tiny_2d(M=8)
    out = {}
    for tag, prm in (("exhaustive", w.params), ("ray2", w.params.replace(search=W.SEARCH_RAY, numrays=2))):
        r = oracle.predict(w.X, w.y, w.XX, prm, nthreads=1)
        out[tag] = dict(sel=r["sel"].tolist(), mean=[float(v).hex() for v in r["mean"]],
                        s2=[float(v).hex() for v in r["s2"]])
    with open(os.path.join(HERE, "oracle_uniform2d.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
