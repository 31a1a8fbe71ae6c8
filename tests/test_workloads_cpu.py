"""CPU checks of the seeded input generators: the device-side feature
generator (torch, here on the CPU) reproduces the numpy generator bit for
bit, on whole batches and on image subsets written into a slice."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")


def test_splitmix64_torch_matches_numpy():
    x = np.array([0, 1, 2, 12345, 2**40 + 7, 2**63 - 1, 2**63, 2**64 - 1], dtype=np.uint64)
    ref = workloads.splitmix64(x)
    got = workloads._splitmix64_torch(torch.from_numpy(x.view(np.int64))).numpy().view(np.uint64)
    assert np.array_equal(ref, got)
    for v in x.tolist():
        assert workloads.splitmix64_scalar(v) == int(ref[x.tolist().index(v)])


@pytest.mark.parametrize("make", [workloads.config1, workloads.config2, workloads.uneven_batch])
def test_device_features_equal_host_features(make):
    wl = make()
    ref = wl.features()
    got = workloads.features_device(wl, "cpu").numpy()
    assert ref.shape == got.shape
    assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))


def test_device_features_image_subset():
    wl = workloads.uneven_batch()
    ref = wl.features()
    lo = wl.pyramids[1].levels[0].cell_offset
    sub = workloads.features_device(wl, "cpu", images=range(1, 3)).numpy()
    assert np.array_equal(sub.view(np.uint32), ref[lo:].view(np.uint32))
    # written into a caller's buffer at a cell base
    out = torch.zeros((ref.shape[0] - lo, 32), dtype=torch.float32)
    workloads.features_device(wl, "cpu", out=out, cell_base=lo, images=range(1, 3))
    assert np.array_equal(out.numpy().view(np.uint32), ref[lo:].view(np.uint32))
