"""Multi-process check of the row-strip exchange protocol on the CPU (gloo,
CPU tensors only).

Each rank owns a band of rows of an L x L lattice plus one halo row above
and below, and updates its own rows site by site with the oracle's
per-site uniform and acceptance rule (keyed by global coordinates).  After
every colour step the ranks exchange their boundary rows: each sends its
first row to the rank above (that rank's halo below) and its last row to
the rank below (its halo above), which is the order the GPU strips follow
(ising_strip_exchange after each colour); tags keep the two directions
apart when both neighbours are the same rank.  Per sweep, each rank counts
anti-aligned bonds at their colour-1 ends and up spins over its own rows,
and an all-reduce sums them.  The gathered lattice and the (E, M) series
must equal the oracle's whole-lattice run exactly."""
import os
import socket
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _free_port():
    with socket.socket() as s:
        s.bind(("127.0.0.1", 0))
        return s.getsockname()[1]


def _rank_main(rank, world, port, L, n, beta, seed, sid, out_dir):
    sys.path.insert(0, ROOT)
    import torch
    import torch.distributed as dist
    import oracle
    import workloads
    dist.init_process_group("gloo", init_method="tcp://127.0.0.1:%d" % port, rank=rank,
                            world_size=world)
    rows = L // world
    y0 = rank * rows
    full = oracle.init(L, seed, sid, workloads.INIT_HOT)
    band = np.zeros((rows + 2, L), dtype=np.int8)  # rows 0 and rows + 1 are halos
    band[1:rows + 1] = full[y0:y0 + rows]
    t4, t8 = oracle.thresholds(beta)
    up, down = (rank - 1) % world, (rank + 1) % world

    def exchange():
        first = torch.from_numpy(band[1].copy())
        last = torch.from_numpy(band[rows].copy())
        halo_above = torch.empty(L, dtype=torch.int8)
        halo_below = torch.empty(L, dtype=torch.int8)
        # tags tell the two directions apart when up and down are the same
        # rank (two strips): rows travelling up become the receiver's halo
        # below (tag 1), rows travelling down its halo above (tag 0)
        ops = [dist.P2POp(dist.isend, first, up, tag=1), dist.P2POp(dist.isend, last, down, tag=0),
               dist.P2POp(dist.irecv, halo_above, up, tag=0),
               dist.P2POp(dist.irecv, halo_below, down, tag=1)]
        for req in dist.batch_isend_irecv(ops):
            req.wait()
        band[0] = halo_above.numpy()
        band[rows + 1] = halo_below.numpy()

    exchange()
    EM = np.zeros((n, 2), dtype=np.int64)
    for k in range(n):
        for c in (0, 1):
            for r in range(1, rows + 1):
                y = y0 + r - 1
                for x in range((y + c) & 1, L, 2):
                    v = int(band[r, x])
                    u = oracle.uniform(seed, sid, c, k, L, x, y)
                    if oracle.accept(v, int(band[r, (x - 1) % L]), int(band[r, (x + 1) % L]),
                                     int(band[r - 1, x]), int(band[r + 1, x]), u, t4, t8):
                        band[r, x] = -v
            exchange()
        anti = up_spins = 0
        for r in range(1, rows + 1):
            y = y0 + r - 1
            up_spins += int(np.sum(band[r] > 0))
            for x in range((y + 1) & 1, L, 2):  # colour-1 sites own their four bonds
                v = band[r, x]
                anti += int(band[r, (x - 1) % L] != v) + int(band[r, (x + 1) % L] != v)
                anti += int(band[r - 1, x] != v) + int(band[r + 1, x] != v)
        counts = torch.tensor([anti, up_spins], dtype=torch.int64)
        dist.all_reduce(counts)
        EM[k] = (2 * int(counts[0]) - 2 * L * L, 2 * int(counts[1]) - L * L)
    bands = [torch.zeros((rows, L), dtype=torch.int8) for _ in range(world)]
    dist.all_gather(bands, torch.from_numpy(band[1:rows + 1].copy()))
    if rank == 0:
        np.save(os.path.join(out_dir, "spins.npy"), torch.cat(bands).numpy())
        np.save(os.path.join(out_dir, "em.npy"), EM)
    dist.destroy_process_group()


@pytest.mark.parametrize("world,L", [(2, 16), (4, 16)])
def test_gloo_strips_reproduce_the_lattice(tmp_path, world, L):
    import torch.multiprocessing as mp
    import oracle
    import workloads
    n, beta, seed, sid = 4, 1 / 2.269185, 13, 2
    mp.spawn(_rank_main, args=(world, _free_port(), L, n, beta, seed, sid, str(tmp_path)),
             nprocs=world, join=True)
    spins = np.load(tmp_path / "spins.npy")
    em = np.load(tmp_path / "em.npy")
    s, oem = oracle.run(L, beta, seed, sid, workloads.INIT_HOT, n)
    assert np.array_equal(spins, s)
    assert np.array_equal(em, oem)
