"""The allocation-free cluster entry point, ising_batch_cluster_static, against
ising_batch_cluster with a caller-owned workspace: two calls in a row (the
second on a smaller batch, so the library's workspace still holds the first
call's labels), traces and lattices bit for bit, both algorithms; and the
size limit, rejected on the host before any work is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _descs(shapes, seed0):
    return [dict(Lx=Lx, Ly=Ly, J=1.0, beta=1.0 / T, seed=seed0 + r, replica=r, init=0)
            for r, (Lx, Ly, T) in enumerate(shapes)]


LARGER = [(256, 128, 2.27), (512, 64, 2.0), (128, 130, 3.1), (1024, 256, 2.4)]
SMALLER = [(64, 16, 2.5), (128, 6, 1.8)]


@pytest.mark.parametrize("algorithm", ["sw", "wolff"])
def test_static_workspace_equals_caller_workspace(algorithm):
    import torch
    import paper_2404_16990_amd as P
    for k, shapes in enumerate((LARGER, SMALLER)):
        descs = _descs(shapes, 7000 + 100 * k)
        a, s = P.Batch(descs), P.Batch(descs)
        need = P.ising_cluster_ws_bytes(s.h)
        assert need <= P.ISING_CLUSTER_STATIC_WS_BYTES
        a.run(3)
        s.run(3)
        n, every = 21, 3   # a captured 16-step chunk plus a direct remainder on the caller-workspace path
        ta = a.cluster(n, algorithm, every)
        bond = torch.empty((len(descs), n // every), dtype=torch.int64, device="cuda")
        mag = torch.empty_like(bond)
        s.cluster_static(n, algorithm, bond, mag, every)
        torch.cuda.synchronize()
        assert torch.equal(ta[0], bond) and torch.equal(ta[1], mag), (k, algorithm)
        for r in range(len(descs)):
            assert np.array_equal(a.get_spins(r), s.get_spins(r)), (k, algorithm, r)
        # without traces, then Metropolis sweeps on the shared counter
        a.cluster(5, algorithm)
        s.cluster_static(5, algorithm)
        ga, gs = a.run(4, 2), s.run(4, 2)
        torch.cuda.synchronize()
        assert torch.equal(ga[0], gs[0]) and torch.equal(ga[1], gs[1])
        assert [a.get_sweep(r) for r in range(len(descs))] == [s.get_sweep(r) for r in range(len(descs))]
        a.close()
        s.close()


def test_static_workspace_rejects_batches_beyond_its_size():
    import paper_2404_16990_amd as P
    b = P.Batch(_descs([(8192, 2048, 2.3)], 9))   # 2^24 labels of 4 bytes > 64 MiB
    assert P.ising_cluster_ws_bytes(b.h) > P.ISING_CLUSTER_STATIC_WS_BYTES
    with pytest.raises(P.IsingError) as e:
        b.cluster_static(1, "sw")
    assert e.value.code == P.ISING_E_NOMEM and "67" in str(e.value)
    assert b.get_sweep(0) == 0
    b.close()
