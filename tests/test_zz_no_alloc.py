"""petar_clusters_noalloc (the clusters pass on the library's fixed scratch)
against petar_clusters, through the C ABI: two calls in a row on one
context, the first at the largest N the fixed scratch takes and the second
smaller, bit for bit (labels, cluster offsets, members are integers); the
second also against the oracle. The context that makes the calls holds no
workspace afterwards, and an N beyond the maximum is rejected before any
launch."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_MAX = 1 << 20


@pytest.fixture(scope="module")
def pt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_16560_amd as pt
    return pt


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def random_graph(n, seed):
    """Symmetric neighbour CSR (rows ascending, no self) of about 0.6 n
    pairs, mostly between nearby indices, so that components of every size
    from 1 up to several hundred occur."""
    rng = np.random.default_rng(seed)
    m = int(0.6 * n)
    i = rng.integers(0, n, m)
    j = np.where(rng.random(m) < 0.9, i + rng.integers(1, 12, m), rng.integers(0, n, m))
    keep = (j < n) & (j != i)
    i, j = i[keep], j[keep]
    a = np.concatenate([i, j])
    b = np.concatenate([j, i])
    key = np.unique(a.astype(np.int64) * n + b)
    a, b = key // n, key % n
    offs = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offs, a + 1, 1)
    return np.cumsum(offs), b.astype(np.int32)


def test_clusters_noalloc_matches_clusters(pt, orc):
    ref_ctx = pt.petar_create(0)
    ctx = pt.petar_create(0)
    try:
        for k, n in enumerate((N_MAX, 30011)):
            offs, idx = random_graph(n, 700 + k)
            o_d, i_d = T(offs), T(idx)
            out = (torch.full((n,), -7, dtype=torch.int32, device="cuda:0"),
                   torch.full((n + 1,), -7, dtype=torch.int64, device="cuda:0"),
                   torch.full((n,), -7, dtype=torch.int32, device="cuda:0"))
            label, cl, members = pt.petar_clusters_noalloc(ctx, o_d, i_d, out=out)
            r_label, r_cl, r_members = pt.petar_clusters(ref_ctx, o_d, i_d)
            torch.cuda.synchronize()
            print("noalloc call %d: N = %d, %d clusters" % (k, n, cl.shape[0] - 1), flush=True)
            assert label.data_ptr() == out[0].data_ptr()
            assert torch.equal(label, r_label)
            assert torch.equal(cl, r_cl)
            assert torch.equal(out[1][cl.shape[0]:], torch.full_like(out[1][cl.shape[0]:], n))
            assert torch.equal(members, r_members)
            assert 1 < cl.shape[0] - 1 < n
            if n < N_MAX:
                l_ref, cl_ref, m_ref = orc.clusters(n, offs, idx)
                assert np.array_equal(label.cpu().numpy(), l_ref)
                assert np.array_equal(cl.cpu().numpy(), cl_ref)
                assert np.array_equal(members.cpu().numpy(), m_ref)
        assert pt.petar_get_stats(ctx)["workspace_bytes"] == 0
        assert pt.petar_get_stats(ref_ctx)["workspace_bytes"] > 0
    finally:
        pt.petar_destroy(ctx)
        pt.petar_destroy(ref_ctx)


def test_clusters_noalloc_rejects_large_n(pt):
    ctx = pt.petar_create(0)
    try:
        n = N_MAX + 1
        offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda:0")
        idx = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        with pytest.raises(pt.PetarError) as ei:
            pt.petar_clusters_noalloc(ctx, offs, idx)
        assert ei.value.status == pt.PETAR_E_INVALID
        assert "fixed scratch" in str(ei.value)
        # the context still works after the rejection
        label, cl, members = pt.petar_clusters_noalloc(ctx, offs[:1001], idx)
        assert torch.equal(label.cpu(), torch.arange(1000, dtype=torch.int32))
        assert pt.petar_get_stats(ctx)["workspace_bytes"] == 0
    finally:
        pt.petar_destroy(ctx)
