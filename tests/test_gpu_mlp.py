"""GPU parity of the monotone CDF network: forward pass, loss and gradients
(float32 on the GPU against the float64 oracle), the Adam step, training,
distillation to PWL knots, and the gain of the trained network over the
untrained one in the learned-splitter sort (identical output either way).

Tolerances: every gradient entry must lie within its own bound, derived in
tests/mlp_bound.py from the kernel's float32 operation and summation order
(first-order error propagation through the forward and backward pass, sums of
256 samples per workgroup then the workgroups in order, so gamma_256 +
gamma_nblk times the sum of the term magnitudes, plus whole terms of samples
that sit on a ramp kink within their error); the forward pass to 1e-5
absolute (values in [0, ~1])."""
import numpy as np
import pytest
import torch

from gpu_util import dev_u32, dev_u64, kpa_mod, need_gpu, say, u32, u64
from mlp_bound import grad_bound
from oracle import mlp as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    need_gpu()
    return kpa_mod()


def skewed_keys(n, seed, offset=1 << 40):
    rng = np.random.default_rng(seed)
    # rank-ordered Zipf-like keys: steep CDF at the low end
    r = np.floor(np.exp(rng.random(n) * np.log(1 << 20))).astype(np.uint64)
    return np.uint64(offset) + r * np.uint64(4096)


def params0(seed=0):
    u = np.random.default_rng(seed).random(M.N_PARAMS)   # the method's random draws, as input
    return M.init_params(u)


def test_training_set_definition(K):
    keys = np.sort(skewed_keys(10007, 1))
    S = 1000
    model = K.new_models(1, "cuda")
    x, y = K.kpa_mlp_training_set(dev_u64(keys), S, model)
    torch.cuda.synchronize()
    kmin, kmax = int(keys[0]), int(keys[-1])
    idx = (np.arange(S, dtype=np.uint64) * np.uint64(len(keys))) // np.uint64(S)
    ex = ((keys[idx] - np.uint64(kmin)).astype(np.float64) / float(kmax - kmin)).astype(np.float32)
    ey = (idx.astype(np.float64) / len(keys)).astype(np.float32)
    assert np.array_equal(x.cpu().numpy(), ex) and np.array_equal(y.cpu().numpy(), ey)
    kmin_g, kmax_g, ns, _ = K.model_fields(model)[0]
    assert (kmin_g, kmax_g) == (kmin, kmax)


def test_forward_matches_oracle(K):
    p = params0(1)
    x = np.linspace(0, 1, 5001)
    f = K.kpa_mlp_forward(torch.tensor(p, dtype=torch.float32, device="cuda"),
                          torch.tensor(x, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    ef, _ = M.forward(p.astype(np.float32).astype(np.float64), x.astype(np.float32))
    assert np.allclose(f.cpu().numpy(), ef, rtol=0, atol=1e-5)


@pytest.mark.parametrize("m", [1, 255, 256, 1000, 1 << 16])
def test_loss_grad_matches_oracle(K, m):
    keys = np.sort(skewed_keys(max(m, 2) * 3, 2))
    model = K.new_models(1, "cuda")
    x, y = K.kpa_mlp_training_set(dev_u64(keys), m, model)
    p = params0(2)
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    say(f"loss_grad m={m}")
    loss, g = K.kpa_mlp_loss_grad(pt, x, y)
    torch.cuda.synchronize()
    el, eg = M.loss_grad(p.astype(np.float32).astype(np.float64), x.cpu().numpy().astype(np.float64),
                         y.cpu().numpy().astype(np.float64))
    gg = g.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(eg))
    assert abs(float(loss.item()) - el) <= 1e-5 + 1e-3 * el
    bound, amb = grad_bound(p.astype(np.float32).astype(np.float64),
                            x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64))
    err = np.abs(gg - eg)
    say(f"m={m}: max |err|/bound {np.max(err / np.maximum(bound, 1e-300)):.3g}, "
        f"max |err|/max|g| {np.max(err) / scale:.3g}, bound/max|g| {np.max(bound) / scale:.3g}, "
        f"samples on a kink {amb}")
    assert np.all(err <= bound), np.argmax(err / np.maximum(bound, 1e-300))
    # deterministic: the same call gives the same bits
    loss2, g2 = K.kpa_mlp_loss_grad(pt, x, y)
    torch.cuda.synchronize()
    assert torch.equal(g, g2) and torch.equal(loss, loss2)


def test_adam_step_matches_oracle(K):
    rng = np.random.default_rng(3)
    p = params0(3)
    g = rng.normal(size=M.N_PARAMS) * 0.01
    m0 = rng.normal(size=M.N_PARAMS) * 0.001
    v0 = np.abs(rng.normal(size=M.N_PARAMS)) * 1e-4
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    mt = torch.tensor(m0, dtype=torch.float32, device="cuda")
    vt = torch.tensor(v0, dtype=torch.float32, device="cuda")
    K.kpa_mlp_adam_step(pt, torch.tensor(g, dtype=torch.float32, device="cuda"), mt, vt, 5,
                        lr=1e-2)
    torch.cuda.synchronize()
    ep, em, ev = M.adam_step(p, g, m0, v0, 5, lr=1e-2)
    assert np.allclose(pt.cpu().numpy(), ep, rtol=1e-5, atol=1e-6)
    assert np.allclose(mt.cpu().numpy(), em, rtol=1e-5, atol=1e-9)
    assert np.all(pt.cpu().numpy()[M.weight_mask() > 0] >= 0)


def train(K, keys_sorted, steps, seed=4, S=1 << 14, lr=1e-2):
    model = K.new_models(1, "cuda")
    x, y = K.kpa_mlp_training_set(dev_u64(keys_sorted), S, model)
    p = torch.tensor(params0(seed), dtype=torch.float32, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    l0, _ = K.kpa_mlp_loss_grad(p, x, y)
    loss = K.kpa_mlp_train(p, m, v, x, y, 1, steps, lr=lr) if steps else l0
    return p, model, float(l0.item()), float(loss.item()), x, y


def test_training_lowers_loss_and_stays_monotone(K):
    keys = np.sort(skewed_keys(200000, 5))
    p, model, l0, l1, x, y = train(K, keys, 300)
    torch.cuda.synchronize()
    assert l1 < 0.2 * l0, (l0, l1)
    pn = p.cpu().numpy()
    assert np.all(pn[M.weight_mask() > 0] >= 0)
    K.kpa_mlp_to_pwl(p, model, 1024)
    torch.cuda.synchronize()
    _, _, ns, knots = K.model_fields(model)[0]
    assert ns == 1024 and np.all(np.diff(knots) >= 0) and knots.min() >= 0 and knots.max() <= 1
    ek = M.to_pwl(pn.astype(np.float64))
    assert np.allclose(knots, ek, rtol=0, atol=1e-4)


def test_trained_network_gains_over_untrained(K, orc):
    """Gain: the trained network's buckets overflow less than the untrained
    network's on a skewed, drifting key distribution; both sort identically."""
    n = 1 << 21
    prev = np.sort(skewed_keys(n, 6))
    cur = skewed_keys(n, 7) + np.uint64(1 << 24)      # the next window, drifted
    rids = np.arange(n, dtype=np.uint32)
    off = dev_u64([0, n])
    stats = {}
    outs = {}
    for name, steps in (("untrained", 0), ("trained", 400)):
        p, model, l0, l1, _, _ = train(K, prev, steps)
        K.kpa_mlp_to_pwl(p, model, 1024)
        st = K.new_sort_stats("cuda")
        ok, orr = K.kpa_sort_segmented(dev_u64(cur), dev_u32(rids), off, algo=K.KPA_SORT_LEARNED,
                                       models=model, stats=st)
        torch.cuda.synchronize()
        stats[name] = st.cpu().numpy()
        outs[name] = (u64(ok), u32(orr))
        say(f"{name}: loss {l0:.4g} -> {l1:.4g}, stats {stats[name].tolist()}")
    ek, er = orc.sort(cur, rids)
    for name in outs:
        assert np.array_equal(outs[name][0], ek) and np.array_equal(outs[name][1], er)
    # entries needing more than the model's buckets: pivot splits and fallbacks
    assert stats["trained"][3] < stats["untrained"][3]
    assert stats["trained"][1] > stats["untrained"][1]


def test_init_matches_oracle(K):
    """The network's starting parameters from the same uniforms, on the GPU
    (float32) and in the oracle (float64)."""
    u = np.random.default_rng(11).random(M.N_PARAMS)
    p = K.kpa_mlp_init(torch.tensor(u, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    e = M.init_params(u.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(p.cpu().numpy().astype(np.float64), e, rtol=2e-6, atol=1e-7)
