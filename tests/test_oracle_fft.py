"""Pins for the oracle's own FFT (no GPU).

The oracle's radix-2 FFT is checked against the textbook O(N^2) DFT sum, a
library FFT, the inverse round trip, Parseval's identity and two closed
forms (impulse and shift theorem)."""

import numpy as np
import pytest

from oracle import fft


def _rand(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("shape,axes", [((1,), (0,)), ((2,), (0,)), ((8,), (0,)),
                                        ((16,), (0,)), ((8, 16), (0, 1)),
                                        ((4, 8, 2), (0, 1, 2)), ((3, 8, 4), (1, 2))])
@pytest.mark.parametrize("inverse", [False, True])
def test_fft_matches_brute_force_dft(shape, axes, inverse):
    x = _rand(shape, 1)
    ref = fft.dft_brute(x, axes, inverse=inverse)
    got = fft.ifftn(x, axes) if inverse else fft.fftn(x, axes)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [32, 64, 256])
def test_fft_matches_library(n):
    x = _rand((3, n), 2)
    assert np.max(np.abs(fft.fftn(x, (1,)) - np.fft.fft(x, axis=1))) <= 1e-13 * n
    assert np.max(np.abs(fft.ifftn(x, (1,)) - np.fft.ifft(x, axis=1))) <= 1e-13


def test_round_trip_and_parseval():
    x = _rand((2, 32, 64), 3)
    X = fft.fftn(x, (1, 2))
    assert np.max(np.abs(fft.ifftn(X, (1, 2)) - x)) <= 1e-14 * 10
    P = 32 * 64
    lhs = np.sum(np.abs(x) ** 2)
    rhs = np.sum(np.abs(X) ** 2) / P
    assert abs(lhs - rhs) <= 1e-14 * lhs * 10


def test_impulse_and_shift_theorem():
    n = 16
    d = np.zeros(n, dtype=complex)
    d[0] = 1.0
    assert np.max(np.abs(fft.fftn(d, (0,)) - 1.0)) == 0.0
    x = _rand((n,), 4)
    s = 3
    k = np.arange(n)
    shifted = fft.fftn(np.roll(x, s), (0,))
    expect = fft.fftn(x, (0,)) * np.exp(-2j * np.pi * k * s / n)
    assert np.max(np.abs(shifted - expect)) <= 1e-13


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        fft.fft_axis(np.ones(12), 0)


def test_threaded_field_transforms_are_bit_identical():
    # the per-field threads of fftn / ifftn / fs_run change no arithmetic
    from oracle import fs
    from paper_2306_04322_amd import inputs as I
    rng = np.random.default_rng(11)
    a = rng.random((5, 16, 32)) + 1j * rng.random((5, 16, 32))
    assert np.array_equal(fft.fftn(a, (1, 2), workers=4), fft.fftn(a, (1, 2)))
    assert np.array_equal(fft.ifftn(a, (1, 2), workers=3), fft.ifftn(a, (1, 2)))
    for cfg in (I.make_config(2, (32, 16), 1.0, 4, I.PAPER_FE),
                I.make_config(3, (8, 16, 8), 1.0, 2, I.PAPER_FE)):
        u0 = I.random_ic(cfg, 3)
        assert np.array_equal(fs.fs_run(u0, cfg, 0.1, 3, workers=5), fs.fs_run(u0, cfg, 0.1, 3))
