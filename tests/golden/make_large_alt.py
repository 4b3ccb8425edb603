"""Writes the oracle's reference for the 16384 x 16384 workload under the
alternative dynamics the benchmark times there.

Calls only the oracle (never the HIP path).  For each dynamics ("lcg": the
per-thread LCG of section 5.3 with the thread seeds of Eq. (7); "pool22":
a pool of 2^22 Boltzmann patterns at random addresses, section 5.1), the
workload's cold +1 start at T = 2.269185 (seed 1, stream id 0), all 2000
sweeps.  Outputs, in this directory, appended per dynamics:
  large_alt_em.txt      - "dynamics sweep E M" for every sweep
  large_alt_sha256.txt  - "dynamics sweep sha256" of the int8 L x L spin
                          array (row-major [y][x], +1/-1) after sweeps 1,
                          10 and 2000
A dynamics already present is skipped, so the script resumes.
Run:  python tests/golden/make_large_alt.py [threads] [dynamics ...]
(about 1 hour per dynamics on 8 cores).
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

EM_OUT = os.path.join(HERE, "large_alt_em.txt")
SHA_OUT = os.path.join(HERE, "large_alt_sha256.txt")
ORIGIN = "# written by tests/golden/make_large_alt.py from the oracle alone\n"


def _done():
    have = set()
    if os.path.exists(SHA_OUT):
        for line in open(SHA_OUT):
            if not line.startswith("#") and line.strip():
                have.add(line.split()[0])
    return have


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    todo = sys.argv[2:] or ["lcg", "pool22"]
    w = workloads.LARGE
    beta = 1.0 / w.T
    for path, what in ((EM_OUT, "E M after each sweep"),
                       (SHA_OUT, "sha256 of the int8 spin array (row-major, +1/-1)")):
        if not os.path.exists(path):
            with open(path, "w") as f:
                f.write(ORIGIN)
                f.write("# oracle %s: L=%d T=%r init=%d seed=%d stream_id=%d\n"
                        % (what, w.L, w.T, w.init, w.seed, w.stream_id))
                f.write("# dynamics sweep %s\n" % ("E M" if path == EM_OUT else "sha256"))
    have = _done()
    for dyn in todo:
        if dyn in have:
            print("%s: already written" % dyn, flush=True)
            continue
        s = oracle.init(w.L, w.seed, w.stream_id, w.init)
        st = oracle.lcg_seed(w.L, w.seed) if dyn == "lcg" else None
        em, digests, t, t0 = [], [], 0, time.time()
        for nxt in (1, 10, 500, 1000, 1500, w.sweeps):
            if dyn == "lcg":
                EM = oracle.lcg_sweeps(s, beta, st, nxt - t)
            else:
                EM = oracle.pool_sweeps(s, beta, w.seed, w.stream_id, t, nxt - t, 22, False)
            em.extend((int(a), int(b)) for a, b in EM)
            t = nxt
            if t in (1, 10, w.sweeps):
                digests.append((t, hashlib.sha256(np.ascontiguousarray(s).tobytes()).hexdigest()))
            print("%s: sweep %d done, %.0f s" % (dyn, t, time.time() - t0), flush=True)
        with open(EM_OUT, "a") as f:
            for k, (a, b) in enumerate(em):
                f.write("%s %d %d %d\n" % (dyn, k + 1, a, b))
        with open(SHA_OUT, "a") as f:
            for t, d in digests:
                f.write("%s %d %s\n" % (dyn, t, d))


if __name__ == "__main__":
    main()
