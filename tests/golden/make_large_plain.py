"""Writes the oracle's reference for the 16384 x 16384 plain workload.

Calls only the oracle (never the HIP path).  Outputs, in this directory:
  large_plain_em.txt      - per-sweep "E M" (int64) for all 2000 sweeps
  large_plain_sha256.txt  - "sweep sha256" of the int8 L x L spin array
                            (row-major [y][x], +1/-1) after sweeps 1, 10, 2000
Run:  python tests/golden/make_large_plain.py [threads]
(about 1-2 hours on 8 cores; the oracle is deliberately plain).
"""
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    w = workloads.LARGE
    beta = 1.0 / w.T
    s = oracle.init(w.L, w.seed, w.stream_id, w.init)
    checkpoints = {1, 10, w.sweeps}
    em = []
    digests = []
    t = 0
    t0 = time.time()
    while t < w.sweeps:
        nxt = min(c for c in sorted(checkpoints | {w.sweeps}) if c > t)
        EM = oracle.sweeps(s, beta, w.seed, w.stream_id, t, nxt - t)
        em.extend((int(a), int(b)) for a, b in EM)
        t = nxt
        if t in checkpoints:
            digests.append((t, hashlib.sha256(np.ascontiguousarray(s).tobytes()).hexdigest()))
        print("sweep %d done, %.0f s" % (t, time.time() - t0), flush=True)
    origin = "# written by tests/golden/make_large_plain.py from the oracle alone\n"
    with open(os.path.join(HERE, "large_plain_em.txt"), "w") as f:
        f.write(origin)
        f.write("# oracle E M after each sweep: L=%d T=%r init=%d seed=%d stream_id=%d\n"
                % (w.L, w.T, w.init, w.seed, w.stream_id))
        for a, b in em:
            f.write("%d %d\n" % (a, b))
    with open(os.path.join(HERE, "large_plain_sha256.txt"), "w") as f:
        f.write(origin)
        f.write("# sha256 of the int8 spin array (row-major, +1/-1) after the given sweep\n")
        for t, d in digests:
            f.write("%d %s\n" % (t, d))


if __name__ == "__main__":
    main()
