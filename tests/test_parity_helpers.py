"""CPU checks of the test-side storage rounding (it prepares oracle inputs)."""
import numpy as np

from parity_helpers import iou, round_storage


def test_round_bf16_known_values():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.3, -2.5], np.float32)
    r = round_storage(x, "bf16")
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2.0 ** -6
    # every result is a bf16 value (low 16 bits zero) within half an ulp
    u = r.astype(np.float32).view(np.uint32)
    assert np.all(u & 0xFFFF == 0)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_round_f16_matches_numpy_half():
    x = np.random.default_rng(0).random(1000).astype(np.float32)
    np.testing.assert_array_equal(round_storage(x, "f16"), x.astype(np.float16).astype(np.float64))
    np.testing.assert_array_equal(round_storage(x, "f32"), x.astype(np.float64))


def test_iou():
    a = np.zeros((4, 4), bool)
    b = np.zeros((4, 4), bool)
    assert iou(a, b) == 1.0
    a[0, :2] = True
    b[0, 1:3] = True
    assert iou(a, b) == 1.0 / 3.0
