"""hk_kdist_noalloc, the k-distribution call that allocates nothing, through
the C ABI: the same results as hk_kdist, bit for bit, on two calls in a row
(the second smaller, so the fixed array still holds the first call's
values), for bins above one LDS sort (which go through the fixed array) and
for bins within one (which need no scratch); and the size limit."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hk = pytest.importorskip("paper_1503_03806_amd")


@pytest.fixture(scope="module")
def ctx():
    c = hk.Context(0)
    yield c
    c.close()


def both(ctx, kap, ppb, g, precision):
    n = kap.numel()
    nb = -(-n // ppb)
    a = torch.empty((nb, len(g)), dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    sa = torch.empty_like(kap)
    sb = torch.empty_like(kap)
    hk.hk_kdist(ctx.h, kap, precision, n, ppb, g, a, sa)
    hk.hk_kdist_noalloc(ctx.h, kap, precision, n, ppb, g, b, sb)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), sa.cpu().numpy(), sb.cpu().numpy()


@pytest.mark.parametrize("precision", [hk.HK_F64, hk.HK_F32_KAHAN])
def test_noalloc_equals_kdist_on_two_calls(ctx, precision):
    g, _ = oracle.g_nodes(20)
    rng = np.random.default_rng(41)
    dt = torch.float64 if precision == hk.HK_F64 else torch.float32
    for n, ppb in ((400_000, 100_000), (150_001, 100_000), (60_000, 10_000), (20_017, 10_000)):
        kap = torch.from_numpy(10.0 ** rng.uniform(-30, -18, n)).to(dt).cuda()
        a, b, sa, sb = both(ctx, kap, ppb, g, precision)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (n, ppb)
        assert np.array_equal(sa, sb), (n, ppb)
        ref = oracle.kdist(kap.double().cpu().numpy(), ppb, g)
        assert np.array_equal(b, ref), (n, ppb)


def test_noalloc_rejects_inputs_beyond_its_array(ctx):
    g, _ = oracle.g_nodes(20)
    n = hk.HK_KDIST_NOALLOC_SCRATCH_BYTES // 16 + 1  # binary64 keys, two halves
    kap = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty((2, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(hk.HKError) as ex:
        hk.hk_kdist_noalloc(ctx.h, kap, hk.HK_F64, n, n // 2 + 1, g, out)
    assert ex.value.code == hk.HK_EINVAL and "fixed" in str(ex.value)
    # bins within one LDS sort need no scratch, whatever the grid size
    hk.hk_kdist_noalloc(ctx.h, kap, hk.HK_F64, n, 1000, g, torch.empty((-(-n // 1000), 20), dtype=torch.float64,
                                                                       device="cuda"))
    torch.cuda.synchronize()
