"""The allocation-free keyed reduction (kpa_reduce_by_key_noalloc, scratch in
the library's static device array) gives the same groups as the workspace
form, on two calls in a row, the second with a smaller input (so stale
contents of the shared array from the first call would show)."""
import numpy as np
import pytest
import torch

from datagen.rows import LAYOUT32
from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u64

pytestmark = pytest.mark.gpu


def make(rng, n, n_seg, n_keys):
    keys = rng.integers(0, n_keys, size=n, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    vals = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    rows = np.zeros((n, 4), np.uint64)
    rows[:, 0], rows[:, 1] = keys, vals
    cuts = np.sort(rng.integers(0, n + 1, size=n_seg - 1))
    off = np.concatenate([[0], cuts, [n]]).astype(np.uint64)
    rids = np.arange(n, dtype=np.uint32)
    order = np.lexsort((rids, keys))  # any sort inside segments works for both forms
    sk, sr = np.empty_like(keys), np.empty_like(rids)
    for s in range(n_seg):
        a, b = int(off[s]), int(off[s + 1])
        o = a + np.lexsort((rids[a:b], keys[a:b]))
        sk[a:b], sr[a:b] = keys[o], rids[o]
    del order
    return sk, sr, off, rows


def test_noalloc_matches_workspace_form_twice():
    need_gpu()
    K = kpa_mod()
    rng = np.random.default_rng(7)
    for call, (n, n_seg, n_keys) in enumerate([(1_000_003, 9, 30_000), (54_321, 3, 500)]):
        say(f"no-alloc reduce call {call}: n={n} segments={n_seg}")
        sk, sr, off, rows = make(rng, n, n_seg, n_keys)
        dk, dr, doff = dev_u64(sk), dev_u32(sr), dev_u64(off)
        drows = torch.from_numpy(rows.view(np.int64)).cuda()
        ref_k, ref, ref_seg = K.kpa_reduce_by_key(dk, dr, doff, drows, LAYOUT32,
                                                  want=("cnt", "sum", "max", "gstart"))
        outs = {name: torch.full((n,), -1, dtype=torch.int64, device="cuda")
                for name in ("gkey", "cnt", "sum", "max", "gstart")}
        outs["gseg_off"] = torch.full((n_seg + 1,), -1, dtype=torch.int64, device="cuda")
        K.kpa_reduce_by_key_noalloc(dk, dr, doff, drows, LAYOUT32, outs,
                                    want=("cnt", "sum", "max"))
        torch.cuda.synchronize()
        gs = u64(ref_seg)
        assert np.array_equal(u64(outs["gseg_off"]), gs)
        g = int(gs[-1])
        assert np.array_equal(u64(outs["gkey"])[:g], u64(ref_k)[:g])
        for name in ("cnt", "sum", "max", "gstart"):
            assert np.array_equal(u64(outs[name])[:g], u64(ref[name])[:g]), name


def test_noalloc_rejects_oversize_before_enqueueing():
    need_gpu()
    K = kpa_mod()
    z = torch.zeros(4, dtype=torch.int64, device="cuda")
    outs = {"gkey": z, "gseg_off": torch.zeros(2, dtype=torch.int64, device="cuda")}
    with pytest.raises(K.KpaError) as e:
        K.kpa_reduce_by_key_noalloc(z, torch.zeros(4, dtype=torch.int32, device="cuda"),
                                    torch.zeros(2, dtype=torch.int64, device="cuda"), None,
                                    LAYOUT32, outs, n_cap=(1 << 32) - 1, want=())
    assert e.value.code == K.KPA_EUNSUPPORTED
