"""cs_sort_pairs_noalloc (the sort entry point that allocates nothing)
against cs_sort_pairs on the same seeded keys, through the C ABI: two calls
in a row on one context, the second smaller, bit-exact (integer sort), plus
numpy's stable argsort; sizes beyond the fixed scratch are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pairs(n, bits, seed):
    rng = np.random.default_rng(seed)
    if bits > 31:
        tiles = rng.integers(0, min(1 << (bits - 31), 300), size=n).astype(np.uint64)
        depth = rng.uniform(0.2, 90.0, size=n).astype(np.float32)
        depth[rng.uniform(size=n) < 0.2] = 7.5  # exact ties
        keys = (tiles << np.uint64(31)) | depth.view(np.uint32).astype(np.uint64)
    else:
        keys = rng.integers(0, 1 << bits, size=n).astype(np.uint64)
    return keys, rng.permutation(n).astype(np.uint32)


def test_noalloc_sort_matches_the_allocating_sort():
    import torch

    from paper_2501_17792_amd import crowdsplat as cs

    r = cs.Renderer(0)
    # first the largest size the scratch takes (4 passes of 11 bits), then a
    # smaller ragged one with an odd pass count (the result is copied back
    # from the scratch), then a 2-pass one
    for n, bits, seed in [(cs.CS_NOALLOC_MAX_PAIRS, 44, 1), (123_457, 46, 2), (70_001, 13, 3)]:
        print(f"noalloc sort: n={n} bits={bits} seed={seed}", flush=True)
        keys, vals = _pairs(n, bits, seed)
        ka = torch.from_numpy(keys.view(np.int64).copy()).cuda()
        va = torch.from_numpy(vals.view(np.int32).copy()).cuda()
        kb, vb = ka.clone(), va.clone()
        r.sort_pairs(ka, va, bits)
        r.sort_pairs_noalloc(kb, vb, bits)
        torch.cuda.synchronize()
        got_k, got_v = kb.cpu().numpy().view(np.uint64), vb.cpu().numpy().view(np.uint32)
        assert np.array_equal(got_k, ka.cpu().numpy().view(np.uint64))
        assert np.array_equal(got_v, va.cpu().numpy().view(np.uint32))
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(got_k, keys[order])
        assert np.array_equal(got_v, vals[order])
    # beyond the scratch: refused with a capacity error, nothing enqueued
    n = cs.CS_NOALLOC_MAX_PAIRS + 1
    kd = torch.zeros(n, dtype=torch.int64, device="cuda")
    vd = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(cs.CrowdSplatError) as e:
        r.sort_pairs_noalloc(kd, vd, 44)
    assert e.value.code == cs.CS_ERR_CAPACITY
    assert "scratch" in str(e.value)
    r.sort_pairs_noalloc(kd, vd, 44, n=0)  # empty: a no-op
    r.close()
