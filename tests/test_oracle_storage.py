"""Pins of the oracle's storage rounding (oracle/storage.py): values fixed by
the formats' definitions, and the conversions of an independent library
(torch's CPU casts) on random inputs."""
import numpy as np
import pytest

from oracle import storage


def test_bf16_definition_values():
    # bfloat16 keeps 8 significant bits: the spacing just above 1 is 2^-7
    cases = {1.0: 1.0, 1 + 2 ** -7: 1 + 2 ** -7,
             1 + 2 ** -8: 1.0,                          # tie, to even
             1 + 3 * 2 ** -8: 1 + 2 ** -6,              # tie, to even (up)
             1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7,       # just above the tie
             -3.0: -3.0, 0.0: 0.0,
             3.140625: 3.140625,                        # 11.001001b: 8 significant bits
             1 / 3: 0.333984375}                        # 0.0101010101b rounds up
    for x, want in cases.items():
        assert storage.to_bf16(np.array([x]))[0] == want, x


def test_f16_definition_values():
    cases = {1.0: 1.0, 1 / 3: 0.333251953125, 65504.0: 65504.0, 2.0 ** -24: 2.0 ** -24,
             1 + 2 ** -11: 1.0, 1 + 3 * 2 ** -11: 1 + 2 ** -9}
    for x, want in cases.items():
        assert storage.to_f16(np.array([x]))[0] == want, x


def test_f32_is_binary32():
    x = np.array([1 / 3, np.pi, 1e-40, 1 + 2 ** -24, 1 + 3 * 2 ** -24])
    got = storage.to_f32(x)
    assert got[0] == 0.3333333432674408 and got[1] == 3.1415927410125732
    assert got[3] == 1.0 and got[4] == 1 + 2 ** -22
    assert got[2] != 0.0 and abs(got[2] - 1e-40) < 2 ** -149     # binary32 subnormal


def test_against_torch_casts():
    """Same results as torch's float32 -> bfloat16 / float16 casts (an
    independent implementation) on values spread over many binades."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(200000) * np.exp2(rng.integers(-20, 20, 200000))
    x32 = torch.from_numpy(x.astype(np.float32))
    np.testing.assert_array_equal(storage.to_bf16(x), x32.to(torch.bfloat16).to(torch.float64).numpy())
    xs = x[np.abs(x) < 6e4]
    x32 = torch.from_numpy(xs.astype(np.float32))
    np.testing.assert_array_equal(storage.to_f16(xs), x32.to(torch.float16).to(torch.float64).numpy())


def test_scaled_storage():
    # a value below binary16's normal range survives storage with a 2^10 scale
    x = np.array([3.0e-6])
    assert abs(storage.stored(x, "f16")[0] - 3.0e-6) > 1e-9
    assert abs(storage.stored(x, "f16", 2.0 ** 10)[0] - 3.0e-6) < 3.0e-6 * 2 ** -10
    with pytest.raises(AssertionError):
        storage.stored(x, "f16", 3.0)
