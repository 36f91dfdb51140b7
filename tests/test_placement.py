"""The demand balance knob of hybrid placement (Sec. 5) and the serving
loop's creation-time checks, on the host (no GPU).

The knob rule as the paper states it: {k_low, k_high} start at 1 and move in
steps of 0.05; k_low moves first; only when k_low already sits at the end it
would move toward does k_high move, and only while the output delay keeps 10%
headroom below the target.  Here capacity pressure (HBM use above host-link
use by more than 0.1) moves allocations toward the host, bandwidth pressure
toward HBM."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def K():
    import paper_1901_01328_amd as P
    return P.load()


CASES = [
    # (k_low, k_high, hbm_util, bw_util, delay_ms, target_ms) -> (k_low, k_high)
    ((1.0, 1.0, 0.9, 0.1, 100, 1000), (0.95, 1.0)),     # capacity-short: k_low first
    ((0.0, 1.0, 0.9, 0.1, 100, 1000), (0.0, 0.95)),     # k_low at 0: k_high, headroom ok
    ((0.0, 1.0, 0.9, 0.1, 950, 1000), (0.0, 1.0)),      # no 10% headroom: nothing moves
    ((0.0, 1.0, 0.9, 0.1, 900, 1000), (0.0, 0.95)),     # exactly 10% headroom counts
    ((0.5, 0.7, 0.50, 0.45, 100, 1000), (0.5, 0.7)),    # balanced (within 0.1): no change
    ((0.5, 0.3, 0.1, 0.9, 100, 1000), (0.55, 0.3)),     # bandwidth-short: toward HBM
    ((1.0, 0.3, 0.1, 0.9, 100, 1000), (1.0, 0.35)),     # k_low at 1: k_high moves up
    ((0.02, 1.0, 0.9, 0.1, 100, 1000), (0.0, 1.0)),     # clamped at 0
    ((1.0, 1.0, 0.1, 0.9, 100, 1000), (1.0, 1.0)),      # both at 1 already
]


@pytest.mark.parametrize("args,exp", CASES)
def test_knob_rule(K, args, exp):
    lo, hi = K.kpa_balance_knob_update(*args)
    assert lo == pytest.approx(exp[0], abs=1e-12) and hi == pytest.approx(exp[1], abs=1e-12)


def test_sustained_capacity_pressure_walks_low_then_high(K):
    lo, hi, steps = 1.0, 1.0, 0
    while lo > 0:
        lo, hi = K.kpa_balance_knob_update(lo, hi, 1.0, 0.0, 0, 1000)
        steps += 1
    assert steps == 20 and hi == 1.0      # 1 / 0.05 steps of k_low, k_high untouched
    lo, hi = K.kpa_balance_knob_update(lo, hi, 1.0, 0.0, 0, 1000)
    assert lo == 0.0 and hi == pytest.approx(0.95)


def _create(K, **fields):
    cfg = K.kpa_server_config()
    assert K._lib.kpa_server_config_default(ctypes.byref(cfg)) == 0
    for k, v in fields.items():
        setattr(cfg, k, v)
    h = ctypes.c_void_p(None)
    rc = K._lib.kpa_server_create(ctypes.byref(cfg), ctypes.byref(h))
    return rc, h, K._lib.kpa_last_error_string()


def test_defaults(K):
    cfg = K.kpa_server_config()
    assert K._lib.kpa_server_config_default(ctypes.byref(cfg)) == 0
    assert cfg.placement == K.KPA_PLACE_DEVICE and cfg.host_pool_bytes == 0
    assert cfg.monitor_ms == 10 and cfg.target_delay_ms == 1000.0 and cfg.keep_groups == 0


def test_unadmissible_bundle_is_refused_at_creation(K):
    # the slots' scratch fits, but a largest bundle (rows + KPA) never could
    rc, h, msg = _create(K, budget_bytes=300 << 20, slots=1, max_bundle_rows=1 << 22)
    assert rc == K.KPA_EBUDGET and b"bundle" in msg and not h.value


def test_host_placement_needs_a_host_pool(K):
    rc, h, msg = _create(K, placement=K.KPA_PLACE_BALANCED)
    assert rc == K.KPA_EINVAL and b"host pool" in msg and not h.value
    rc, h, msg = _create(K, placement=7)
    assert rc == K.KPA_EINVAL
