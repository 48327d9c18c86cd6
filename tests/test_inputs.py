"""The seeded input generators: shapes, determinism and the recipe of the
fluctuation movie (checked against a direct per-frame construction)."""
import numpy as np
from scipy.ndimage import gaussian_filter

import smre_inputs as gi


def test_movie_is_deterministic_and_normalised():
    a = gi.blinking_movie(40, 30, 50, seed=2, dtype=np.float64)
    b = gi.blinking_movie(40, 30, 50, seed=2, dtype=np.float64)
    assert a.shape == (40, 30, 50) and np.array_equal(a, b)
    assert abs(np.sqrt(np.mean(a * a)) - 1.0) < 1e-12
    # fluctuations about each emitter's time average: every pixel averages to 0
    assert np.max(np.abs(a.mean(axis=0))) < 1e-12
    assert not np.array_equal(a, gi.blinking_movie(40, 30, 50, seed=3, dtype=np.float64))


def test_movie_frames_are_blurred_fluctuation_images():
    # every frame is a combination of the emitters' PSFs (the constant-mode
    # Gaussian filter of a unit impulse at each emitter pixel): least squares
    # on that basis leaves no residual
    n, H, W = 30, 24, 33
    m = gi.blinking_movie(n, H, W, n_e=6, seed=4, dtype=np.float64)
    rng = gi.rng_for(4)
    rows = rng.integers(0, H, size=6)
    cols = rng.integers(0, W, size=6)
    basis = []
    for r, c in zip(rows, cols):
        D = np.zeros((H, W))
        D[r, c] = 1.0
        basis.append(gaussian_filter(D, 1.5, mode="constant", truncate=4.0).ravel())
    B = np.stack(basis, axis=1)
    for t in (0, 17):
        coef, *_ = np.linalg.lstsq(B, m[t].ravel(), rcond=None)
        assert np.max(np.abs(B @ coef - m[t].ravel())) < 1e-10


def test_movie_blinks():
    m = gi.blinking_movie(200, 16, 16, n_e=1, seed=7, dtype=np.float64)
    peak = np.unravel_index(np.argmax(np.abs(m).sum(axis=0)), (16, 16))
    trace = m[:, peak[0], peak[1]]
    # on and off frames both occur: two clusters of values
    assert trace.max() - trace.min() > 1.0
    assert len(np.unique(np.round(trace, 9))) > 2
