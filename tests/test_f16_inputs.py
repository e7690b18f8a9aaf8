"""Half-precision array-of-structures hit coordinates (the paper's storage
optimisation, Section 4 optimisation table): host-side conversion and the
method's physics on the rounded coordinates (CPU).  GPU parity of the
half-precision entry point is in test_gpu_parity.py."""

import numpy as np

import oracle
from paper_2207_03936_amd import indicators, sbt, synth
from _util import rounded_to_f16


def test_conversion_rounds_to_nearest_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -10)          # binary16 spacing at 1
    cases = [
        (one + ulp / 2, one),             # tie -> even (1.0)
        (one + 3 * ulp / 2, one + 2 * ulp),   # tie -> even (mantissa ...10)
        (one + ulp * 0.49, one),
        (one + ulp * 0.51, one + ulp),
        (np.float32(725.0), np.float32(725.0)),   # plane positions are exact
        (np.float32(-275.0), np.float32(-275.0)),
        (np.float32(41.99), np.float32(42.0)),    # spacing 2^-5 on [32, 64)
    ]
    for v, want in cases:
        got = np.float32(np.float16(v))
        assert got == want, (v, got, want)


def test_aos_layout():
    x = np.array([1.0, -2.5, 3.25], np.float32)
    y = np.array([0.5, 7.0, -0.125], np.float32)
    z = np.array([725.0, 685.0, -275.0], np.float32)
    a = sbt.to_f16_aos(x, y, z)
    assert a.shape == (3, 4) and a.dtype == np.uint16
    h = a.view(np.float16)
    assert np.array_equal(h[:, 0].astype(np.float32), x)
    assert np.array_equal(h[:, 1].astype(np.float32), y)
    assert np.array_equal(h[:, 2].astype(np.float32), z)
    assert not a[:, 3].any()


def test_rounding_error_within_half_spacing():
    b = synth.make_batch("mu7.6", 5)
    r = rounded_to_f16(b)
    for a, q in ((b.x, r.x), (b.y, r.y)):
        mag = np.maximum(np.abs(a), np.float32(2.0 ** -14))       # subnormal spacing below 2^-14
        spacing = np.float32(2.0) ** (np.floor(np.log2(mag)) - 10)
        assert np.all(np.abs(q - a) <= spacing / 2)
    assert np.array_equal(r.z, b.z)


def test_physics_holds_on_half_precision_coordinates():
    """Binary16 spacing is at most 31 um inside the 42 mm annulus, beside
    12 um of hit smear, so the default tolerances keep the indicators."""
    b = rounded_to_f16(synth.make_batch("tiny", 100))
    res = indicators.evaluate(b, *oracle.reconstruct(b))
    assert res["efficiency"] >= 0.98
    assert res["fake_fraction"] <= 0.01
    assert res["hit_purity"] >= 0.99


def test_server_conversion_matches_numpy():
    """The server's host conversion (F16C where the CPU has it, eight hits at
    a time, then one by one) gives numpy's binary16 rounding bit for bit:
    ties to even, subnormals, signed zeros, values near the binary16 limit,
    and lengths that are not a multiple of eight."""
    import os
    if not os.path.exists(sbt.LIB_PATH):
        import pytest
        pytest.skip("libsbt.so is not built")
    rng = np.random.default_rng(16)
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -10)
    special = np.array([0.0, -0.0, one + ulp / 2, one + 3 * ulp / 2, -(one + ulp / 2), 6.0e-8, -3.0e-6, 2.0 ** -24,
                        65504.0, -65504.0, 65519.0, 725.0, -275.0, 41.99, 1e-3, 123.456], np.float32)
    for n in (0, 1, 7, 8, 9, 16, 23, 1000, 4097):
        x = np.concatenate([special, rng.normal(0, 40, n).astype(np.float32)])[:n]
        y = rng.uniform(-60, 60, n).astype(np.float32)
        z = rng.choice(np.float32(synth.PLANE_Z), n).astype(np.float32) + rng.normal(0, 2, n).astype(np.float32)
        got = sbt.half_records(x, y, z)
        assert np.array_equal(got, sbt.to_f16_aos(x, y, z)), n
