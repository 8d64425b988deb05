"""Storage-form emulation used to weigh 16-bit forms against the 1e-3
acoustic-pressure bar (tests/storage_forms_study.py)."""
import numpy as np

from tests.storage_forms_study import round_float, run


def test_round_float_reproduces_binary16_and_binary32():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 0.05, 20000), rng.normal(0, 1e-6, 5000),
                        np.ldexp(rng.uniform(0.5, 1.0, 3000), rng.integers(-30, 10, 3000)),
                        [0.0, 2.0 ** -24, 3 * 2.0 ** -25, 1.0 + 2.0 ** -11, -6e-8]])
    h16 = round_float(x, 10, -14, 15)
    np.testing.assert_array_equal(h16, x.astype(np.float16).astype(np.float64))
    h32 = round_float(x, 23, -126, 127)
    np.testing.assert_array_equal(h32, x.astype(np.float32).astype(np.float64))


def test_custom_format_grid():
    # 4 exponent bits, 11 mantissa bits: one more bit than binary16 at every
    # normal magnitude, subnormal step 2^-25, largest value 2 - 2^-11
    x = np.array([1.0 + 2.0 ** -12, 1.0 + 3 * 2.0 ** -12, 2.0 ** -14 * (1 + 2.0 ** -11),
                  2.0 ** -26, 3 * 2.0 ** -26, 5.0, 0.3])
    y = round_float(x, 11, -14, 0)
    assert y[0] == 1.0                              # half an ulp, ties to even
    assert y[1] == 1.0 + 2 * 2.0 ** -11             # ties to even upwards
    assert y[2] == x[2]                             # representable
    assert y[3] == 0.0 and y[4] == 2.0 ** -24       # subnormal ties to even
    assert y[5] == 2.0 - 2.0 ** -11                 # saturates
    assert abs(y[6] - 0.3) <= 2.0 ** -2 * 2.0 ** -12


def test_custom_format_beats_binary16_on_a_short_run():
    res = run(n=20, horizons=(60,), forms=("f16s", "f16c", "f32s"))
    row = res[60]
    assert row["f32s"] < 1e-4
    assert row["f16c"] < row["f16s"]
