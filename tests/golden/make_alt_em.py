"""Writes the oracle's whole-lattice (E, M) of the alternative dynamics on
the HBM-resident 262144^2 lattice.

Calls only the oracle (never the HIP path).  Each case is summed over bands
of rows with light-cone margins of 2n + 1 rows (``oracle.lcg_band_em``,
``oracle.pool_band_em``).  Output, in this directory, one line per case and
sweep:

  alt_em.txt  - "L T seed stream_id init dynamics sweep E M"

with dynamics "lcg" (the per-thread LCG of section 5.3, thread seeds of
Eq. (7) from the seed) or "pool22" / "pool22-linear" (a pool of 2^22
Boltzmann patterns, random addresses or linear reads).  Cases: 262144^2,
T = 2.0, hot start from seed 7, stream id 0, sweeps 1..3, each dynamics.
A case already present in the file is skipped, so the script resumes.

Run:  python tests/golden/make_alt_em.py [threads]
(about 15 min for the LCG and 20 min per pool case on 8 cores).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402

OUT = os.path.join(HERE, "alt_em.txt")
HOT = 2
L, T, SEED, SID, N, BAND = 262144, 2.0, 7, 0, 3, 2048
CASES = ["lcg", "pool22", "pool22-linear"]


def _done():
    have = set()
    if os.path.exists(OUT):
        for line in open(OUT):
            if line.startswith("#") or not line.strip():
                continue
            have.add(line.split()[5])
    return have


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    if not os.path.exists(OUT):
        with open(OUT, "w") as f:
            f.write("# written by tests/golden/make_alt_em.py from the oracle alone\n")
            f.write("# whole-lattice oracle E and M after each sweep of the alternative "
                    "dynamics, summed over bands of rows\n")
            f.write("# L T seed stream_id init dynamics sweep E M\n")
    have = _done()
    beta = 1.0 / T
    for dyn in CASES:
        if dyn in have:
            print("%s: already written" % dyn, flush=True)
            continue
        t0 = time.time()
        pool = None
        if dyn.startswith("pool"):
            pool = oracle.pool_fill(beta, SEED, SID, 22)
        total = np.zeros((N, 2), dtype=np.int64)
        for y0 in range(0, L, BAND):
            if dyn == "lcg":
                total += oracle.lcg_band_em(L, beta, SEED, SID, HOT, N, y0, BAND)
            else:
                total += oracle.pool_band_em(L, beta, SEED, SID, HOT, 0, N, 22,
                                             dyn.endswith("linear"), y0, BAND, pool=pool)
            if (y0 // BAND) % 16 == 15:
                print("%s: %d of %d rows, %.0f s" % (dyn, y0 + BAND, L, time.time() - t0),
                      flush=True)
        with open(OUT, "a") as f:
            for k in range(N):
                f.write("%d %r %d %d %d %s %d %d %d\n" % (L, T, SEED, SID, HOT, dyn, k + 1,
                                                          int(total[k, 0]), int(total[k, 1])))
        print("%s done in %.0f s" % (dyn, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
