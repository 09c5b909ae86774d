"""Pins of the oracle's own DFT/FFT (oracle/fft.py)."""
import numpy as np
import pytest

from oracle import fft as offt

LENGTHS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 15, 16, 18, 24, 25, 27, 30, 32, 33, 48, 60, 64, 96, 128]


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_definition(n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=(3, n)) + 1j * rng.normal(size=(3, n))
    ref = offt.dft(x)
    got = offt.fft(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    refi = offt.dft(x, inverse=True)
    goti = offt.fft(x, inverse=True)
    assert np.max(np.abs(goti - refi)) <= 1e-13 * max(1.0, np.max(np.abs(refi)))


@pytest.mark.parametrize("n", [8, 12, 64, 96, 384])
def test_fft_matches_numpy(n):
    # numpy.fft (pocketfft) is an independent third-party implementation.
    rng = np.random.default_rng(100 + n)
    x = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    assert np.allclose(offt.fft2(x), np.fft.fft2(x), rtol=0, atol=1e-12 * n)
    assert np.allclose(offt.fft2(x, inverse=True), np.fft.ifft2(x) * n * n, rtol=0, atol=1e-12 * n)


def test_dft_single_frequency():
    # A pure exponential exp(2 pi i 3 j / n) transforms to n at bin 3 only.
    n = 16
    j = np.arange(n)
    x = np.exp(2j * np.pi * 3 * j / n)
    X = offt.dft(x)
    expect = np.zeros(n, complex)
    expect[3] = n
    assert np.max(np.abs(X - expect)) < 1e-12


def test_parseval_and_roundtrip():
    rng = np.random.default_rng(7)
    x = rng.normal(size=48) + 1j * rng.normal(size=48)
    X = offt.fft(x)
    assert abs(np.sum(abs(X) ** 2) / 48 - np.sum(abs(x) ** 2)) < 1e-10
    assert np.max(np.abs(offt.fft(X, inverse=True) / 48 - x)) < 1e-14


def test_axis_argument():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(6, 10))
    a = offt.fft(x, axis=0)
    b = offt.dft(x.T).T
    assert np.max(np.abs(a - b)) < 1e-12
