"""Writes the oracle's per-sweep (E, M) for the larger lattices of the
finite-size-scaling grid (L >= 512: 128 lattices), 40 sweeps from the hot
start, as the batched parity test runs them.

Calls only the oracle (never the HIP path).  Output, in this directory:
  fss_grid_em.txt  - one line per lattice: "L stream_id E_1 M_1 ... E_40 M_40"
Run:  python tests/golden/make_fss_grid_em.py [threads]   (a few minutes on 8 cores)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

SWEEPS = 40


def main():
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    lines = []
    for g in workloads.fss_grid():
        if g.L < 512:
            continue
        _, EM = oracle.run(g.L, 1.0 / g.T, g.seed, g.stream_id, g.init, SWEEPS)
        lines.append("%d %d %s\n" % (g.L, g.stream_id, " ".join(str(int(v)) for v in EM.ravel())))
        print("L=%d stream %d done" % (g.L, g.stream_id), flush=True)
    with open(os.path.join(HERE, "fss_grid_em.txt"), "w") as f:
        f.write("# written by tests/golden/make_fss_grid_em.py from the oracle alone\n")
        f.write("# fss grid (seed 1, hot start, T = linspace(2.20, 2.34, 32)[stream_id %% 32]), "
                "%d sweeps: L stream_id E_1 M_1 ... E_n M_n\n" % SWEEPS)
        f.writelines(lines)


if __name__ == "__main__":
    main()
