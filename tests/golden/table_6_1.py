"""Network diagnostics of Sec. 6.1 (Table 6.1) and Sec. 6.2.1 (Table 6.3) on
the oracle: homogeneity sigma and connectivity mu (oracle/diagnostics.py) of

  grid     the Example 3.7 grid with (2^9 + 1)^2 nodes, boxes of side H for
           H^-1 = 4, 8, 16, 32 (Table 6.3, pinned by the tests), and
  uniform  the Sec. 6.1 uniform fiber network (fibers of length 0.05, midpoints
           in [-0.025, 1.025]^2, clipped, placed until the clipped length
           reaches 1000), boxes B_R of side 2R for R^-1 = 4 ... 64, joining
           paths within R0 = 1/64 (Table 6.1; the instance is not the paper's,
           so its row is a statistic).

In both tables the box side s (H, or 2R) is the length in mu_box =
1 / (s sqrt(lambda_2)), the reading under which the grid row of Table 6.3 is
reproduced.

Calls only the oracle and the seeded input generators. Usage:
    python tests/golden/table_6_1.py [--rows grid,uniform]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.join(ROOT, "oracle"), HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import diagnostics as D  # noqa: E402  (oracle/diagnostics.py)
from paper_2207_07488_amd import workloads as W  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", default="grid,uniform")
    a = ap.parse_args()
    for row in a.rows.split(","):
        if row == "grid":
            x, e = W.grid_network(512)
            sizes, r0 = (4, 8, 16, 32), None
        else:
            import oracle as O
            import table_6_2 as T
            net = O.Network.from_segments(2, T.fiber_segments_sec61(), merge_tol=W.merge_tol(T.FIBER_LENGTH),
                                          dir_lo=3, dir_hi=3)
            x, e, _ = net.arrays()
            sizes, r0 = (2, 4, 8, 16, 32), 1.0 / 64
        print(f"# {row}: {len(x)} nodes, {len(e)} edges", flush=True)
        for nb in sizes:
            t = time.time()
            _, sigma, _ = D.homogeneity(x, e, nb)
            _, mu = D.connectivity(x, e, nb, r0)
            label = f"H^-1 = {nb}" if row == "grid" else f"R^-1 = {2 * nb}"
            print(f"{label}: sigma {sigma:.3f} mu {mu:.3f} ({time.time() - t:.1f} s)", flush=True)


if __name__ == "__main__":
    main()
