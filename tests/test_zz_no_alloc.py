"""erpp_bin_static (the allocation-free binning) against erpp_bin through the
C ABI: bit-exact keys and bin starts, the same particles in every cell; two
calls in a row, the second on a smaller box, so that the static scratch keeps
nothing of the first call.  (The size limits are checked on the CPU in
test_abi.py: they are rejected before any launch.)"""
import numpy as np
import pytest

import oracle
import workloads
from helpers import upload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
erpp = pytest.importorskip("paper_1405_6969_amd")


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _box(shape, np_, seed):
    spec = workloads.BoxSpec(n=shape, L=tuple(0.05 * s for s in shape), np_=np_,
                             placement="clustered", n_blobs=20, carrier="zero", seed=seed)
    box = workloads.make_box(spec)
    # positions on the box faces and at the last cell's upper edge
    box.x[:, :3] = np.array([[0.0, spec.L[0] * (1 - 1e-17), spec.L[0] - 1e-12],
                             [0.0, 1e-300, spec.L[1] - 1e-12],
                             [spec.L[2] * (1 - 1e-17), 0.0, 0.0]])
    return box


def _per_cell_sets(perm, start):
    return [np.sort(perm[start[c]:start[c + 1]]) for c in range(start.size - 1)
            if start[c + 1] > start[c]]


def _compare(box):
    db = upload(box, 2, erpp.F32_FAST)
    with erpp.Plan([db], 2, 1e-3) as plan:
        k1, p1, s1 = plan.bin(0, db.x)
        torch.cuda.synchronize()
        k1, p1, s1 = k1.cpu().numpy(), p1.cpu().numpy(), s1.cpu().numpy()
    k2, p2, s2 = erpp.bin_static(box.n, box.L, db.x)
    torch.cuda.synchronize()
    k2, p2, s2 = k2.cpu().numpy(), p2.cpu().numpy(), s2.cpu().numpy()
    assert np.array_equal(k1, k2)
    assert np.array_equal(s1, s2)
    for a, b in zip(_per_cell_sets(p1, s1), _per_cell_sets(p2, s2)):
        assert np.array_equal(a, b)
    # and both agree with the oracle's cell keys
    P = oracle.params_for_box(box, 2, 1e-3)
    ko, so, _ = oracle.bin_cells(P, box.x)
    assert np.array_equal(k2, ko) and np.array_equal(s2, so)
    return k2, s2


def test_bin_static_matches_bin_on_two_calls():
    _cuda()
    big = _box((72, 64, 48), 60000, 901)        # 221,184 cells
    small = _box((20, 16, 12), 3000, 902)       # 3,840 cells, fewer particles
    _compare(big)
    k, s = _compare(small)
    assert s[-1] == 3000 and k.max() < 20 * 16 * 12
