"""Write pair_counts.json: the oracle's exact count of connected ordered
determinant pairs (singles, doubles) of the benchmarked spaces.

CPU only; calls the oracle (every pair of each space is visited) and the
seeded input generator, nothing of the GPU library.  Run from the
repository root:  python tests/golden/make_pair_counts.py  (about 10 minutes
on 8 cores for the 2,000,000-determinant space).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import sc  # noqa: E402
from paper_2501_18185_amd import synth  # noqa: E402

CASES = [("sci-n64-10a10b-2e6", 1, 0), ("spinor-40kp-20e-1e6", 2, 0)] + \
        [(f"batch16-problem{i}", 3, i) for i in range(16)]


def main():
    out = {}
    for name, k, i in CASES:
        t0 = time.time()
        p = synth.workload(k, i)
        s, d = sc.pair_counts(p)
        out[name] = {"workload": k, "problem": i, "ndet": int(p.ndet), "single_pairs": s, "double_pairs": d}
        print(f"{name}: ndet={p.ndet} singles={s} doubles={d} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "pair_counts.json"), "w") as f:
        json.dump({"source": "oracle.sc.pair_counts over every ordered pair of each space "
                             "(tests/golden/make_pair_counts.py)", "cases": out}, f, indent=1)


if __name__ == "__main__":
    main()
