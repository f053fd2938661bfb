"""The decomposition entry point that allocates nothing (its workspace is the
library's static scratch array) against the one that takes a workspace:
two calls in a row, the second smaller, identical bits; plus the size
limit, rejected before any device work."""
import numpy as np
import pytest

from _parity import assert_c64
from oracle import statevector as sv
from paper_1912_03243_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_03243_amd import juqcs
    return juqcs


def cases():
    # (rows, cols, depth, seed, crossings kept, bitstrings, group size)
    return [(4, 5, 6, 41, 6, 3000, 0), (2, 6, 4, 42, 3, 700, 2)]


def test_noalloc_matches_workspace_entry_point(J):
    import torch
    for rows, cols, depth, seed, cross, count, group in cases():
        print("CASE noalloc", rows, cols, depth, seed, cross, count, group, flush=True)
        circ, side = W.grid_circuit(rows, cols, depth, seed, max_cross=cross)
        n = rows * cols
        z = np.random.default_rng(seed).integers(0, 1 << n, count, dtype=np.uint64)
        dz = torch.from_numpy(z.view(np.int64).reshape(-1, 1)).cuda()
        ref = torch.empty(2 * count, dtype=torch.float64, device="cuda")
        got = torch.full((2 * count,), float("nan"), dtype=torch.float64, device="cuda")
        J.juqcs_branch_amplitudes_device(n, circ, side, dz, ref, group_size=group)
        J.juqcs_branch_amplitudes_noalloc(n, circ, side, dz, got, group_size=group)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(a, b)
        full = sv.run_circuit(n, circ)
        assert_c64(b.view(np.complex128), full[z.astype(np.int64)])


def test_noalloc_rejects_decompositions_beyond_the_scratch(J):
    import torch
    # 2 x 24-qubit halves: one part state alone is 128 MiB
    circ, side = W.grid_circuit(6, 8, 2, 5, max_cross=2)
    dz = torch.zeros((4, 1), dtype=torch.int64, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_branch_amplitudes_noalloc(48, circ, side, dz, out)
    assert e.value.status == J.ERR_SIZE
    assert torch.count_nonzero(out).item() == 0
