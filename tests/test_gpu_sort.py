"""The radix sort of the neighbour structure (Morton keys, work-item order)
against numpy's stable argsort, through the C ABI: random and heavily tied
keys, ragged sizes around the 4096-key tile, and the full-size species."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2603_24688_amd as dmb
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dmb.Context(0)
    yield c
    c.close()


def _check(ctx, keys, lo_bit, passes):
    import torch
    n = keys.size
    vals = np.arange(n, dtype=np.int64)[::-1].astype(np.int32).copy()   # payload = reversed index
    kt = torch.from_numpy(keys.view(np.int64)).cuda()
    vt = torch.from_numpy(vals).cuda()
    ko, vo = ctx.sort_pairs(kt, vt, lo_bit, passes)
    ko = ko.cpu().numpy().view(np.uint64)
    vo = vo.cpu().numpy()
    nbits = 8 * passes
    mask = np.uint64((1 << nbits) - 1) if nbits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    digit = (keys >> np.uint64(lo_bit)) & mask
    order = np.argsort(digit, kind="stable")
    assert np.array_equal(vo, vals[order])
    assert np.array_equal(ko, keys[order])


@pytest.mark.parametrize("n", [1, 63, 4095, 4096, 4097, 12289, 100_003])
def test_sort_random_and_tied(ctx, n):
    r = np.random.default_rng(n)
    keys = r.integers(0, 2 ** 63, n, dtype=np.uint64)
    _check(ctx, keys, 31, 4)
    tied = r.integers(0, 7, n, dtype=np.uint64) << np.uint64(40)     # few distinct digits: stability
    _check(ctx, tied, 33, 3)
    _check(ctx, r.integers(0, 256, n, dtype=np.uint64), 0, 1)        # the work-item order (one pass)


@pytest.mark.parametrize("n,passes", [(4_000_000, 4), (32_000_000, 4), (1_000_000, 8)])
def test_sort_full_size(ctx, n, passes):
    r = np.random.default_rng(7)
    keys = r.integers(0, 2 ** 63, n, dtype=np.uint64)
    keys[: n // 3] = keys[: n // 3] & np.uint64(~((1 << 52) - 1) & 0xFFFFFFFFFFFFFFFF)   # long runs of equal digits
    _check(ctx, keys, 64 - 8 * passes, passes)


def test_sort_rejects_bad_bits(ctx):
    import torch
    import paper_2603_24688_amd as dmb
    k = torch.zeros(10, dtype=torch.int64, device="cuda")
    v = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(dmb.DmbError, match="EINVAL"):
        ctx.sort_pairs(k, v, 60, 1)
    with pytest.raises(dmb.DmbError, match="EINVAL"):
        ctx.sort_pairs(k, v, 0, 9)
