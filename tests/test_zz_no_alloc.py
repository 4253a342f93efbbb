"""The allocation-free query entry point (mknn_knn_static) through the C ABI: its rows equal
mknn_knn's bit for bit, on consecutive calls that reuse the fixed scratch with a smaller
batch the second time, and batches above its fixed capacity are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_02224_amd import _lib
    from paper_2605_02224_amd import api as A
    from paper_2605_02224_amd import workloads as W
    return torch, _lib, A, W


def _call(torch, L, fn, cl, qd, k, m):
    nq = qd.shape[0]
    idx = torch.full((nq, k), -9, dtype=torch.int32, device="cuda")
    dist = torch.full((nq, k), -9.0, dtype=torch.float32, device="cuda")
    st = getattr(L, fn)(cl._h, qd.data_ptr(), nq, k, m, idx.data_ptr(), dist.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    assert st == 0, L.mknn_last_error()
    return idx, dist


def test_static_scratch_matches_allocating_entry_point(env):
    torch, _lib, A, W = env
    L = _lib.lib()
    c = W.random_cloud(60000, seed=41, shape="torus")
    P = c.by_rank
    cl = A.Cloud.build(P).upload()
    lo, hi = W.bbox_expanded(P, 1.1)
    rng = np.random.default_rng(17)
    # first a large sorted batch, then a smaller sorted one and an unsorted one: the fixed
    # scratch keeps the previous call's contents, which must not leak into the next answer
    for nq, k, m in ((200000, 16, 60000), (9001, 7, 41234), (5000, 33, 60000),
                     (1 << 20, 1, 60000)):
        Q = W.uniform_in_box(rng, nq, lo, hi)
        qd = torch.from_numpy(Q).cuda()
        a = _call(torch, L, "mknn_knn_static", cl, qd, k, m)
        b = _call(torch, L, "mknn_knn", cl, qd, k, m)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), (nq, k, m)
        assert (a[0][:, 0] >= 0).all()


def test_static_scratch_rejects_batches_above_capacity(env):
    torch, _lib, A, W = env
    L = _lib.lib()
    c = W.random_cloud(3000, seed=42, shape="sphere")
    cl = A.Cloud.build(c.by_rank).upload()
    nq = (1 << 20) + 1
    q = torch.zeros((nq, 3), dtype=torch.float32, device="cuda")
    idx = torch.empty((nq, 4), dtype=torch.int32, device="cuda")
    dist = torch.empty((nq, 4), dtype=torch.float32, device="cuda")
    st = L.mknn_knn_static(cl._h, q.data_ptr(), nq, 4, 3000, idx.data_ptr(), dist.data_ptr(),
                           None)
    assert st == _lib.EINVAL and b"fixed scratch" in L.mknn_last_error()
