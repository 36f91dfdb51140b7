"""GPU parity of the learned-splitter sort and its model fit.

The learned sort must equal the oracle's stable sort byte for byte whatever the
model: fitted on the same data, on an earlier (drifted) window, a constant
model that puts every key in one bucket (forced overflow), and invalid models
(decreasing or NaN knots), which must be detected and counted."""
import numpy as np
import pytest
import torch

import datagen
from datagen.rows import mix64_int
from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def zipf_mix_keys(n, s, k, seed):
    """Zipf ranks mapped to pseudo-random 64-bit keys (heavy hitters)."""
    u = datagen.splitmix64(seed, 1, torch.arange(n, dtype=torch.int64))
    r = datagen.zipf_ranks(u, s, k)
    table = datagen.key_table(k, seed ^ 77)
    return table[r - 1].numpy().view(np.uint64).copy()


def rank_zipf_keys(n, s, seed, offset=0):
    """Rank-ordered Zipf keys: o + (r-1)*2^12 (steep CDF at the low end)."""
    u = datagen.splitmix64(seed, 1, torch.arange(n, dtype=torch.int64))
    r = datagen.zipf_ranks(u, s, 1 << 20).numpy().astype(np.uint64)
    return np.uint64(offset) + (r - np.uint64(1)) * np.uint64(4096)


def gen_keys(dist, n, seed):
    rng = np.random.default_rng(seed)
    if dist == "uniform64":
        return rng.integers(0, 1 << 63, size=n, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=n, dtype=np.uint64)
    if dist == "zipf_mix":
        return zipf_mix_keys(n, 1.1, 1 << 16, seed)
    if dist == "zipf_rank":
        return rank_zipf_keys(n, 1.2, seed, offset=(5 << 40))
    if dist == "few":
        pool = rng.integers(0, 1 << 63, size=5, dtype=np.uint64)
        return pool[rng.integers(0, 5, size=n)]
    if dist == "narrow":
        return np.uint64(1 << 50) + rng.integers(0, 3000, size=n, dtype=np.uint64)
    raise ValueError(dist)


def seg_offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)


def fit_models(K, keys, off):
    """Sort with the radix path, then fit per-segment models on the GPU."""
    sk, _ = K.kpa_sort_segmented(dev_u64(keys), dev_u32(np.arange(len(keys), dtype=np.uint32)),
                                 dev_u64(off))
    return K.kpa_pwl_fit(sk, dev_u64(off), 1024), sk


def check_learned(K, orc, keys, rids, off, models):
    stats = K.new_sort_stats("cuda")
    ok, orr = K.kpa_sort_segmented(dev_u64(keys), dev_u32(rids), dev_u64(off),
                                   algo=K.KPA_SORT_LEARNED, models=models, stats=stats)
    torch.cuda.synchronize()
    ek, er = orc.sort_segmented(keys, rids, off)
    assert np.array_equal(u64(ok), ek), "keys differ from the oracle"
    assert np.array_equal(u32(orr), er), "rids (tie order) differ from the oracle"
    st = stats.cpu().numpy()
    # every entry is accounted for once: on chip, single-key chunk, or fallback
    assert int(st[1] + st[2] + st[3]) == len(keys), st
    return st


def test_pwl_fit_matches_oracle(K, orc):
    rng = np.random.default_rng(1)
    sizes = [0, 1, 2, 1000, 4097, 100000, 7]
    off = seg_offsets(sizes)
    keys = np.concatenate([np.sort(gen_keys(d, s, i)) for i, (d, s) in enumerate(
        zip(["uniform64", "few", "narrow", "zipf_mix", "zipf_rank", "uniform64", "narrow"],
            sizes))])
    for S in (1, 7, 1024):
        say(f"pwl_fit S={S}")
        models = K.kpa_pwl_fit(dev_u64(keys), dev_u64(off), S)
        torch.cuda.synchronize()
        got = K.model_fields(models)
        for s, (a, b) in enumerate(zip(off[:-1], off[1:])):
            a, b = int(a), int(b)
            kmin, kmax, ns, knots = got[s]
            if b == a:
                assert ns == 0
                continue
            ekmin, ekmax, eknots = orc.pwl_fit(keys[a:b], S)
            assert (kmin, kmax, ns) == (ekmin, ekmax, S)
            assert np.array_equal(knots, eknots)   # bit-exact floats


@pytest.mark.parametrize("dist", ["uniform64", "zipf_mix", "zipf_rank", "few", "narrow"])
@pytest.mark.parametrize("n", [3000, 70001, 1 << 20])
def test_learned_sort_with_fitted_model(K, orc, dist, n):
    keys = gen_keys(dist, n, 11)
    rids = np.arange(n, dtype=np.uint32)
    off = seg_offsets([n])
    say(f"learned {dist} n={n} (model from the same data)")
    models, _ = fit_models(K, keys, off)
    st = check_learned(K, orc, keys, rids, off, models)
    if dist in ("uniform64", "narrow") and n >= 70001:
        assert st[1] > 0.9 * n   # a good model finishes nearly everything on chip
    # drifted: the model comes from another draw of the distribution
    keys2 = gen_keys(dist, n, 12)
    if dist == "zipf_rank":
        keys2 = keys2 + np.uint64(1 << 26)      # key offset drift between windows
    say(f"learned {dist} n={n} (model from an earlier window)")
    check_learned(K, orc, keys2, rids, off, models)


def test_learned_sort_segmented_ragged(K, orc):
    rng = np.random.default_rng(3)
    sizes = [0, 5, 4096, 4097, 0, 150000, 1, 33333, 8192, 0, 600001]
    dists = ["uniform64", "few", "zipf_mix", "narrow", "uniform64", "zipf_rank", "few",
             "uniform64", "zipf_mix", "narrow", "zipf_rank"]
    keys = np.concatenate([gen_keys(d, s, 20 + i) for i, (d, s) in enumerate(zip(dists, sizes))])
    rids = rng.permutation(len(keys)).astype(np.uint32)
    off = seg_offsets(sizes)
    models, _ = fit_models(K, keys, off)
    keys2 = np.concatenate([gen_keys(d, s, 40 + i) for i, (d, s) in enumerate(zip(dists, sizes))])
    say("learned segmented ragged")
    check_learned(K, orc, keys2, rids, off, models)


def test_learned_chunk_with_few_inversions(K, orc):
    """One window of the drifting-skew batch's control variant (Zipf ranks
    hashed over 2^32; window 107 of 300, model fitted on the previous epoch):
    it has a finishing chunk whose only out-of-order keys lie in its first
    bucket while a long in-order run of one key holds its largest refined ids,
    so both byte passes over the refined ids must run."""
    n = 101515
    gen = lambda e: datagen.gen_c4_window(107, e, n, n_windows=300, control=True,
                                          device="cuda")[:, 0].cpu().numpy().view(np.uint64)
    off = seg_offsets([n])
    models, _ = fit_models(K, gen(0), off)
    say("learned, chunk with few inversions")
    check_learned(K, orc, gen(1), np.arange(n, dtype=np.uint32), off, models)


def test_forced_overflow_constant_model(K, orc):
    """All knots 0: every key lands in bucket 0 -> the whole segment overflows."""
    n = 200003
    keys = gen_keys("uniform64", n, 5)
    off = seg_offsets([n])
    models, _ = fit_models(K, keys, off)
    raw = models.view(torch.uint8)
    knots = raw[24:24 + 4 * 1025].view(torch.float32)
    knots.zero_()
    say("forced overflow")
    st = check_learned(K, orc, keys, np.arange(n, dtype=np.uint32), off, models)
    # all but the one maximal key overflow; the pivot split settles one more
    assert st[3] >= n - 2 and st[4] >= 1


def test_pivot_split_heavy_key_with_light_neighbours(K, orc):
    """One oversize chunk over many tiles (all knots 0: every key in bucket 0)
    holding a heavy key and repeated light keys on both sides of it: the
    three-way split around the heavy key must keep each class in input order
    (the light parts are then sorted on chip)."""
    rng = np.random.default_rng(9)
    n = 300001
    H = 1 << 40
    keys = np.full(n, H, dtype=np.int64)
    light = rng.choice(n, 3000, replace=False)
    keys[light] = H + rng.integers(-2000, 2000, size=3000)
    keys = keys.astype(np.uint64)
    off = seg_offsets([n])
    models, _ = fit_models(K, keys, off)
    models.view(torch.uint8)[24:24 + 4 * 1025].view(torch.float32).zero_()
    say("pivot split, heavy key with light neighbours")
    rids = rng.permutation(n).astype(np.uint32)
    st = check_learned(K, orc, keys, rids, off, models)
    assert st[4] >= 1 and st[2] >= n - 3000   # split around the heavy key


def heavy_with_close_neighbours(seed, n=300001):
    """Half the keys one heavy key H = 2^39; 6000 light keys within 2^18 of
    it (with a model fitted on such data they share H's bucket but spread
    over its refined ids); the rest uniform over [0, 2^40)."""
    rng = np.random.default_rng(seed)
    H = 1 << 39
    keys = rng.integers(0, 1 << 40, size=n, dtype=np.int64)
    idx = rng.permutation(n)
    keys[idx[: n // 2]] = H
    keys[idx[n // 2: n // 2 + 6000]] = H + rng.integers(-(1 << 18), 1 << 18, size=6000)
    return keys.astype(np.uint64)


def test_pivot_split_parts_sorted_by_model(K, orc):
    """An oversize bucket holding a heavy key and a few thousand light keys
    close to it, with a model fitted on an earlier draw: the split leaves
    parts of 512 to FCAP entries, which are sorted on chip by their window's
    refined bucket ids."""
    off = seg_offsets([300001])
    models, _ = fit_models(K, heavy_with_close_neighbours(21), off)
    keys = heavy_with_close_neighbours(22)
    say("pivot split, parts sorted by the model")
    rids = np.random.default_rng(23).permutation(len(keys)).astype(np.uint32)
    st = check_learned(K, orc, keys, rids, off, models)
    assert st[4] >= 1   # an oversize bucket was split around its heavy key


@pytest.mark.parametrize("bad", ["decreasing", "nan", "above_one"])
def test_invalid_model_detected(K, orc, bad):
    n = 100001
    keys = gen_keys("uniform64", n, 6)
    off = seg_offsets([n])
    models, _ = fit_models(K, keys, off)
    knots = models.view(torch.uint8)[24:24 + 4 * 1025].view(torch.float32)
    if bad == "decreasing":
        knots[500] = 0.9
        knots[501] = 0.1
    elif bad == "nan":
        knots[10] = float("nan")
    else:
        knots[1024] = 1.5
    say(f"invalid model {bad}")
    st = check_learned(K, orc, keys, np.arange(n, dtype=np.uint32), off, models)
    assert st[5] == 1   # order violation counted


def test_learned_equals_radix_bytes(K, orc):
    """Cross-algorithm equality on a C2-shaped window set."""
    rows = datagen.gen_c2(1 << 21, seed=8, n_keys=1 << 16, span_ns=10 ** 6)
    from datagen.rows import LAYOUT32
    d = rows.cuda()
    keys, rids, woff, _ = K.kpa_partition_windows(d, LAYOUT32, 10 ** 5, 10)
    rk, rr = K.kpa_sort_segmented(keys, rids, woff, algo=K.KPA_SORT_RADIX)
    models = K.kpa_pwl_fit(rk, woff, 1024)
    rows2 = datagen.gen_c2(1 << 21, seed=9, n_keys=1 << 16, span_ns=10 ** 6)
    d2 = rows2.cuda()
    keys2, rids2, woff2, _ = K.kpa_partition_windows(d2, LAYOUT32, 10 ** 5, 10)
    say("learned vs radix bytes")
    lk, lr = K.kpa_sort_segmented(keys2, rids2, woff2, algo=K.KPA_SORT_LEARNED, models=models)
    rk2, rr2 = K.kpa_sort_segmented(keys2, rids2, woff2, algo=K.KPA_SORT_RADIX)
    torch.cuda.synchronize()
    assert torch.equal(lk, rk2) and torch.equal(lr, rr2)


def test_segments_beyond_2_31_entries(K, orc):
    """Segments placed across and above entry 2^31 of a buffer of 2^31 + 2^20
    + 4096 entries (only they are filled): tile bases at or above 2^31 must
    stay unsigned 64-bit offsets in every pass (radix, then learned with
    models fitted on the radix output)."""
    n_cap = (1 << 31) + (1 << 20) + 4096
    a0 = (1 << 31) - 3 * 4096 - 5
    a1 = (1 << 31) + (1 << 19) + 11
    a2 = (1 << 31) + (1 << 20) + 1000
    m = a2 - a0
    keys = np.concatenate([gen_keys("zipf_mix", a1 - a0, 51), gen_keys("zipf_rank", a2 - a1, 52)])
    rids = np.random.default_rng(53).permutation(m).astype(np.uint32) + np.uint32(7)
    ek, er = orc.sort_segmented(keys, rids, np.array([0, a1 - a0, m], dtype=np.uint64))
    say(f"segments [{a0}, {a1}, {a2}) in a buffer of {n_cap} entries")
    kin = torch.empty(n_cap, dtype=torch.int64, device="cuda")
    rin = torch.empty(n_cap, dtype=torch.int32, device="cuda")
    kin[a0:a2] = dev_u64(keys)
    rin[a0:a2] = dev_u32(rids)
    off = dev_u64(np.array([a0, a1, a2], dtype=np.uint64))
    kout = torch.empty_like(kin)
    rout = torch.empty_like(rin)
    try:
        K.kpa_sort_segmented(kin, rin, off, n_cap=n_cap, keys_out=kout, rids_out=rout)
        torch.cuda.synchronize()
        assert np.array_equal(u64(kout[a0:a2]), ek) and np.array_equal(u32(rout[a0:a2]), er)
        models = K.kpa_pwl_fit(kout, off, 1024)
        kout.zero_()
        rout.zero_()
        say("learned, same segments")
        stats = K.new_sort_stats("cuda")
        K.kpa_sort_segmented(kin, rin, off, n_cap=n_cap, algo=K.KPA_SORT_LEARNED, models=models,
                             stats=stats, keys_out=kout, rids_out=rout)
        torch.cuda.synchronize()
        assert np.array_equal(u64(kout[a0:a2]), ek) and np.array_equal(u32(rout[a0:a2]), er)
        st = stats.cpu().numpy()
        assert int(st[1] + st[2] + st[3]) == m, st
    finally:
        del kin, rin, kout, rout
        torch.cuda.empty_cache()
