"""The merge microbenchmark kernels (five algorithms of the paper's merge
evaluation) through the C ABI, against the oracle's stable merge."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

ALGS = ("ranking", "merge_path", "odd_even", "bitonic", "bitonic_advanced")
STABLE = ("ranking", "merge_path")


def _pairs(rng, l, pairs, distinct=True):
    """Pairs of ascending length-l runs (uint32 keys), 2l entries per pair."""
    if distinct:
        k = np.argsort(rng.random((pairs, 2 * l)), axis=1).astype(np.uint64) * 2654435 + 17
        k = (k % (1 << 32)).astype(np.uint32)
    else:
        k = rng.integers(0, 5, (pairs, 2 * l), dtype=np.uint32)
    k[:, :l].sort(axis=1)
    k[:, l:].sort(axis=1)
    return k.reshape(-1)


def _run(alg, keys, vals, l, threads):
    import torch
    from paper_1504_05022_amd import lib as L
    dk = torch.from_numpy(keys.view(np.int32)).cuda()
    dv = None if vals is None else torch.from_numpy(vals).cuda()
    print("case: %s l %d threads %d entries %d values %s" %
          (alg, l, threads, keys.size, None if vals is None else vals.dtype), flush=True)
    ko, vo = L.merge_pairs(dk, dv, l, alg, threads)
    torch.cuda.synchronize()
    return ko.cpu().numpy().view(np.uint32), None if vo is None else vo.cpu().numpy()


def _tile_pairs(l, threads):
    return max(2 * l, 2 * threads) // (2 * l)


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("vb", [0, 4, 8])
@pytest.mark.parametrize("l", [1, 16, 256, 4096])
@pytest.mark.parametrize("threads", [64, 1024])
def test_merge_matches_oracle(alg, vb, l, threads):
    if alg == "merge_path" and max(2 * l, 2 * threads) // threads > 32:
        pytest.skip("merge path holds at most 32 outputs per thread")
    if max(2 * l, 2 * threads) * (4 + vb) * (2 if alg == "ranking" else 1) > 160 * 1024:
        pytest.skip("tile larger than LDS")
    rng = np.random.default_rng(ALGS.index(alg) * 100000 + vb * 10000 + l + threads)
    pairs = 3 * _tile_pairs(l, threads) + 1  # a ragged last tile
    keys = _pairs(rng, l, pairs)
    vals = None if vb == 0 else (np.arange(keys.size, dtype=np.int32 if vb == 4 else np.int64)
                                 + (0 if vb == 4 else (1 << 40)))
    ko, vo = _run(alg, keys, vals, l, threads)
    rk, rv = oracle.merge_pairs(keys, vals, l)
    assert np.array_equal(ko, rk)
    if vals is not None:
        assert np.array_equal(vo, rv)


@pytest.mark.parametrize("alg", ALGS)
def test_merge_equal_keys(alg):
    """Many equal keys: keys match exactly; values match for the stable
    algorithms and are a permutation within every run of equal keys (per
    pair) for the networks."""
    l, threads = 64, 128
    rng = np.random.default_rng(7)
    keys = _pairs(rng, l, 40, distinct=False)
    vals = np.arange(keys.size, dtype=np.int64)
    ko, vo = _run(alg, keys, vals, l, threads)
    rk, rv = oracle.merge_pairs(keys, vals, l)
    assert np.array_equal(ko, rk)
    if alg in STABLE:
        assert np.array_equal(vo, rv)
    else:
        grp = np.repeat(np.arange(keys.size // (2 * l)), 2 * l)
        a = np.lexsort((vo, ko, grp))
        b = np.lexsort((rv, rk, grp))
        assert np.array_equal(vo[a], rv[b])
        # every value still sits with its own key
        assert np.array_equal(keys[vo], ko)


def test_merge_rejects_bad_arguments():
    import torch
    from paper_1504_05022_amd import lib as L
    from paper_1504_05022_amd import SpgemmError
    k = torch.zeros(2 * 4096, dtype=torch.int32, device="cuda")
    v = torch.zeros(2 * 4096, dtype=torch.int64, device="cuda")
    with pytest.raises(SpgemmError):
        L.merge_pairs(k, None, 4096, "merge_path", 64)  # 128 outputs per thread
    with pytest.raises(SpgemmError):
        L.merge_pairs(torch.zeros(6, dtype=torch.int32, device="cuda"), None, 3, "ranking", 64)
    big = torch.zeros(2 * 8192, dtype=torch.int32, device="cuda")
    with pytest.raises(SpgemmError):
        L.merge_pairs(big, torch.zeros(2 * 8192, dtype=torch.int64, device="cuda"), 8192,
                      "ranking", 256)  # 384 KB of LDS
    L.merge_pairs(k, v, 4096, "odd_even", 256)
    torch.cuda.synchronize()
