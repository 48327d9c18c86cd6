"""Pins of the Fourier ring correlation used to compare ICD with full
Dykstra (the paper compares reconstructions by FRC, Sec. 2.5).  Known answers:
an image against itself or a positive multiple gives 1 on every ring, against
its negative -1; a single spatial frequency lands on its own ring with the
cosine of the phase difference (the other rings are empty); and two images built in the Fourier domain as
S + N and S - N with |S| = s, |N| = n and N in quadrature with S give
(s^2 - n^2) / (s^2 + n^2) on every ring (the signal-to-noise form of FRC)."""
import numpy as np
import pytest

import bench
import smre_inputs as gi


def test_self_and_scaled_copies():
    a = gi.emitters(64, 80, n_e=12, seed=1) + 0.1 * gi.gaussian(64, 80, seed=2)
    np.testing.assert_allclose(bench.frc_rings(a, a), 1.0, atol=1e-12)
    np.testing.assert_allclose(bench.frc_rings(a, 3.5 * a), 1.0, atol=1e-12)
    np.testing.assert_allclose(bench.frc_rings(a, -a), -1.0, atol=1e-12)
    s = bench.frc_summary(a, a)
    assert s["mean"] == pytest.approx(1.0) and s["first_ring_below_1_7"] is None
    assert s["rings"] == 32


@pytest.mark.parametrize("f,theta", [(5, 0.7), (11, 2.0)])
def test_single_frequency_lands_on_its_ring(f, theta):
    H = W = 64
    xx = np.arange(W)[None, :].repeat(H, 0)
    a = np.cos(2 * np.pi * f * xx / W)
    b = np.cos(2 * np.pi * f * xx / W + theta)
    r = bench.frc_rings(a, b)
    # (the other rings hold only rounding noise, whose ratio is meaningless)
    assert r[f - 1] == pytest.approx(np.cos(theta), abs=1e-12)


@pytest.mark.parametrize("s,n", [(2.0, 1.0), (1.0, 3.0)])
def test_signal_plus_quadrature_noise(s, n):
    H, W = 64, 96
    rng = np.random.default_rng(3)
    phi = rng.uniform(0, 2 * np.pi, size=(H, W))
    A = (s + 1j * n) * np.exp(1j * phi)
    B = (s - 1j * n) * np.exp(1j * phi)
    # real images: keep one of each pair of mirrored bins, drop the bins that
    # are their own mirror image (DC and Nyquist rows / columns)
    ky, kx = np.meshgrid(np.fft.fftfreq(H) * H, np.fft.fftfreq(W) * W, indexing="ij")
    keep = (ky > 0) | ((ky == 0) & (kx > 0))
    keep &= (np.abs(ky) != H // 2) & (np.abs(kx) != W // 2)
    A, B = np.where(keep, A, 0), np.where(keep, B, 0)
    a = np.fft.ifft2(A).real * 2
    b = np.fft.ifft2(B).real * 2
    want = (s * s - n * n) / (s * s + n * n)
    r = bench.frc_rings(a, b)
    np.testing.assert_allclose(r, want, atol=1e-10)
    assert bench.frc_summary(a, b)["mean"] == pytest.approx(want, abs=1e-10)
