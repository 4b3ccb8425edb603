"""Writes the oracle's whole-lattice (E, M) for lattices too large to hold.

Calls only the oracle (never the HIP path).  Each case is summed over bands
of rows with ``oracle.lattice_em_by_bands`` (light-cone margins of 2n + 1
rows), so memory stays near (band + 4n + 2) L bytes.  Output, in this
directory, one line per case and sweep:

  huge_em.txt   - "L T seed stream_id init sweep E M"

Cases (hot start unless noted):
  262144^2, T = 2.0 and 3.0, seed 7, sweeps 1..10 (the HBM-resident
      benchmark lattice: more than 2^32 sites, so every E/M sum passes 32 bits)
  185368^2, T = 2.269185, seed 11, sweeps 1..4 (L not a power of two; more
      than 2^32 Philox blocks per colour)
  1048576^2, T = 2.0, seed 7, sweep 1 (2^33 words per colour plane)
  65536^2, T = 2.0, seed 3, stream id 1, cold +1 start, sweeps 1..2 (2^32
      up spins at the start: the batched path's 64-bit lattice totals)
A case already present in the file is skipped, so the script resumes.

Run:  python tests/golden/make_huge_em.py [threads] [max_L]
(the 262144^2 cases take about 1.5 h each on 8 cores; the oracle is plain).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

OUT = os.path.join(HERE, "huge_em.txt")
HOT, COLD_UP = 2, 0
# (L, T, seed, stream_id, init, sweeps, band rows)
CASES = [
    (262144, 2.0, 7, 0, HOT, 10, 2048),
    (262144, 3.0, 7, 0, HOT, 10, 2048),
    (185368, 2.269185, 11, 0, HOT, 4, 2048),
    (1048576, 2.0, 7, 0, HOT, 1, 1024),
    (65536, 2.0, 3, 1, COLD_UP, 2, 4096),
]


def _done():
    have = set()
    if os.path.exists(OUT):
        for line in open(OUT):
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            have.add((int(f[0]), float(f[1]), int(f[2]), int(f[3]), int(f[4])))
    return have


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    max_L = int(sys.argv[2]) if len(sys.argv) > 2 else None
    if not os.path.exists(OUT):
        with open(OUT, "w") as f:
            f.write("# written by tests/golden/make_huge_em.py from the oracle alone\n")
            f.write("# whole-lattice oracle E and M after each sweep, summed over bands of rows\n")
            f.write("# L T seed stream_id init sweep E M\n")
    have = _done()
    for (L, T, seed, sid, init, n, band) in CASES:
        if max_L is not None and L > max_L:
            continue
        if (L, T, seed, sid, init) in have:
            print("L=%d T=%r: already written" % (L, T), flush=True)
            continue
        t0 = time.time()

        def progress(y, L=L, t0=t0):
            if y % (16 * band) == 0 or y == L:
                print("L=%d: %d of %d rows, %.0f s" % (L, y, L, time.time() - t0), flush=True)

        EM = oracle.lattice_em_by_bands(L, 1.0 / T, seed, sid, init, n, band, progress)
        with open(OUT, "a") as f:
            for k in range(n):
                f.write("%d %r %d %d %d %d %d %d\n"
                        % (L, T, seed, sid, init, k + 1, int(EM[k, 0]), int(EM[k, 1])))
        print("L=%d T=%r done in %.0f s" % (L, T, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
