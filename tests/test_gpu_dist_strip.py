"""The distributed row-strip driver (DistStrip) in one to three processes
that share the one GPU: gloo ranks (the halo rows staged through host
memory; RCCL cannot put two ranks on one device), one strip per rank; a
single rank exchanges with itself in place.  The gathered
lattice and the per-sweep (E, M) must equal the oracle's whole-lattice run
bit for bit."""
import os
import socket
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def _free_port():
    with socket.socket() as s:
        s.bind(("127.0.0.1", 0))
        return s.getsockname()[1]


def _rank_main(rank, world, port, L, n, beta, seed, sid, out_dir):
    sys.path.insert(0, ROOT)
    import torch
    import torch.distributed as dist
    from paper_1007_3726_amd import ising
    import workloads
    dist.init_process_group("gloo", init_method="tcp://127.0.0.1:%d" % port, rank=rank,
                            world_size=world)
    print("rank %d/%d: L=%d" % (rank, world, L), flush=True)
    st = ising.DistStrip(L, seed=seed, stream_id=sid, init=workloads.INIT_HOT, beta=beta)
    em = st.sweep_em(n).cpu()
    rows = torch.from_numpy(st.get_rows())
    sizes = [torch.zeros(1, dtype=torch.int64) for _ in range(world)]
    dist.all_gather(sizes, torch.tensor([rows.shape[0]], dtype=torch.int64))
    # all_gather needs equal shapes: gather padded bands
    pad = int(max(int(sz) for sz in sizes))
    padded = torch.zeros((pad, L), dtype=torch.int8)
    padded[:rows.shape[0]] = rows
    gathered = [torch.zeros((pad, L), dtype=torch.int8) for _ in range(world)]
    dist.all_gather(gathered, padded)
    if rank == 0:
        full = torch.cat([g[:int(sz)] for g, sz in zip(gathered, sizes)])
        np.save(os.path.join(out_dir, "spins.npy"), full.numpy())
        np.save(os.path.join(out_dir, "em.npy"), em.numpy())
    st.close()
    dist.destroy_process_group()


@pytest.mark.parametrize("world,L", [(1, 128), (2, 256), (3, 384)])
def test_distributed_strips_on_one_gpu(tmp_path, world, L):
    import torch
    import torch.multiprocessing as mp
    import oracle
    import workloads
    if torch.cuda.device_count() < 1:  # counts devices without initialising them
        pytest.skip("no GPU")
    n, beta, seed, sid = 5, 1 / 2.269185, 17, 4
    print("case world=%d L=%d" % (world, L), flush=True)
    mp.spawn(_rank_main, args=(world, _free_port(), L, n, beta, seed, sid, str(tmp_path)),
             nprocs=world, join=True)
    spins = np.load(tmp_path / "spins.npy")
    em = np.load(tmp_path / "em.npy")
    s, oem = oracle.run(L, beta, seed, sid, workloads.INIT_HOT, n)
    assert np.array_equal(em, oem)
    assert np.array_equal(spins, s)
