"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module draws random numbers and shapes images; it holds none of the
projection's arithmetic.  Every generator takes an explicit seed and uses
numpy's PCG64 behind SeedSequence, so the oracle and the GPU path see the same
bytes.

Workload shapes (the paper's test data -- a blurred, noisy test image and a
quantum-dot fluorescence movie, Sec. 4.1 -- are not available; these stand in):

* noise_blob: i.i.d. N(0,1) residual plus one Gaussian blob (amplitude 4,
  sigma 3 px) at the image centre ((H-1)/2, (W-1)/2).
* emitters: residual of a fluorescence frame following the fluctuation model of
  Sec. 2.4: n_e point emitters at uniform pixel positions with Poisson(50)
  photon counts, blurred by a Gaussian PSF (sigma 1.5 px, truncated at 4 sigma,
  zero outside the image), minus the blurred mean (50 per emitter), divided by
  its population standard deviation.  Pixels far from every emitter stay 0.
"""
import numpy as np
from scipy.ndimage import gaussian_filter


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def noise_blob(H=64, W=64, seed=0, amp=4.0, sigma=3.0):
    rng = rng_for(seed)
    x = rng.standard_normal((H, W))
    r = np.arange(H)[:, None] - (H - 1) / 2.0
    c = np.arange(W)[None, :] - (W - 1) / 2.0
    x = x + amp * np.exp(-(r * r + c * c) / (2.0 * sigma * sigma))
    return x.astype(np.float64)


def emitters(H, W, n_e=None, seed=0, rng=None, mean_count=50.0, psf_sigma=1.5):
    if rng is None:
        rng = rng_for(seed)
    if n_e is None:
        n_e = int(round(H * W / 1300.0))
    rows = rng.integers(0, H, size=n_e)
    cols = rng.integers(0, W, size=n_e)
    counts = rng.poisson(mean_count, size=n_e).astype(np.float64)
    E = np.zeros((H, W))
    np.add.at(E, (rows, cols), counts)
    M = np.zeros((H, W))
    np.add.at(M, (rows, cols), mean_count)
    R = gaussian_filter(E - M, psf_sigma, mode="constant", truncate=4.0)
    sd = R.std()
    if sd == 0.0:
        return R
    return (R / sd).astype(np.float64)


def gaussian(H, W, seed=0, scale=1.0):
    return scale * rng_for(seed).standard_normal((H, W))


BATCH_SIDES = (128, 256, 384, 512, 768)


def batch_images(n=64, seed=0, sides=BATCH_SIDES):
    """n emitter images with sides drawn uniformly from `sides`, 1 emitter per
    1300 px^2, each from its own spawned seed sequence."""
    ss = np.random.SeedSequence(seed)
    pick = np.random.Generator(np.random.PCG64(ss))
    chosen = pick.choice(np.asarray(sides), size=n)
    children = ss.spawn(n)
    out = []
    for s, child in zip(chosen, children):
        rng = np.random.Generator(np.random.PCG64(child))
        out.append(emitters(int(s), int(s), rng=rng))
    return out


def serve_trace(n, rate=200.0, seed=0, lo=256, hi=1024):
    """Poisson arrivals: (arrival_times_s, sides, images_rng_children).

    Inter-arrival gaps ~ Exp(1/rate); side = round(exp(U(ln lo, ln hi)))."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps)
    sides = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))).astype(int)
    return t, sides, ss.spawn(n)


def serve_image(side, child):
    rng = np.random.Generator(np.random.PCG64(child))
    return emitters(int(side), int(side), rng=rng)


def serve_sides(side):
    """Window sides 1..max(8, side // 64)."""
    return list(range(1, max(8, int(side) // 64) + 1))


def blinking_movie(n_frames, H, W, n_e=None, seed=0, mean_count=50.0, psf_sigma=1.5,
                   exponent=1.5, dtype=np.float32, chunk=256):
    """Fluorescence fluctuation movie (n_frames, H, W) of blinking emitters.

    Emitters sit at fixed random pixels (n_e = round(H W / 1300) by default).
    Each one blinks: on- and off-times in frames are drawn from a power law
    P(tau) ~ tau^-exponent (tau >= 1), its first state at random; an emitter
    that is on in a frame emits Poisson(mean_count) counts, otherwise none.
    Frame t is the PSF-blurred fluctuation sum_k (K_kt - <K_k>) G(r - r_k)
    about each emitter's time-averaged count (Gaussian PSF of psf_sigma px,
    the same kernel as `emitters`), divided by the movie-wide standard
    deviation.
    """
    rng = rng_for(seed)
    if n_e is None:
        n_e = int(round(H * W / 1300.0))
    rows = rng.integers(0, H, size=n_e)
    cols = rng.integers(0, W, size=n_e)
    on = np.zeros((n_e, n_frames), dtype=bool)
    for k in range(n_e):
        t, state = 0, bool(rng.integers(0, 2))
        while t < n_frames:
            tau = int(np.ceil(rng.random() ** (-1.0 / (exponent - 1.0))))
            on[k, t:t + tau] = state
            t += tau
            state = not state
    counts = np.where(on, rng.poisson(mean_count, size=on.shape), 0).astype(np.float64)
    fluct = counts - counts.mean(axis=1, keepdims=True)          # (n_e, n_frames)
    # PSF stamp: the constant-mode Gaussian filter of a unit impulse
    rad = int(4.0 * psf_sigma + 0.5)
    imp = np.zeros((2 * rad + 1, 2 * rad + 1))
    imp[rad, rad] = 1.0
    stamp = gaussian_filter(imp, psf_sigma, mode="constant", truncate=4.0)
    dy, dx = np.meshgrid(np.arange(-rad, rad + 1), np.arange(-rad, rad + 1), indexing="ij")
    rr = rows[:, None] + dy.ravel()[None, :]
    cc = cols[:, None] + dx.ravel()[None, :]
    keep = (rr >= 0) & (rr < H) & (cc >= 0) & (cc < W)
    kk = np.broadcast_to(np.arange(n_e)[:, None], rr.shape)
    from scipy.sparse import csr_matrix
    S = csr_matrix((np.broadcast_to(stamp.ravel(), rr.shape)[keep],
                    (kk[keep], (rr * W + cc)[keep])), shape=(n_e, H * W))
    out = np.empty((n_frames, H, W), dtype=dtype)
    ss = 0.0
    for f0 in range(0, n_frames, chunk):
        blk = np.asarray((S.T @ fluct[:, f0:f0 + chunk]).T)     # (frames, H W)
        ss += float(np.sum(blk * blk))
        out[f0:f0 + chunk] = blk.reshape(-1, H, W)
    sd = np.sqrt(ss / (n_frames * H * W))
    if sd > 0:
        out /= dtype(sd) if dtype != np.float64 else sd
    return out


def test_scene(H, W, seed=0, n_shapes=40):
    """Piecewise-smooth gray-level scene (0..255): a smooth background
    gradient plus random filled ellipses and rectangles of random gray levels,
    standing in for a natural test image."""
    rng = rng_for(seed)
    yy, xx = np.meshgrid(np.arange(H) / max(H - 1, 1), np.arange(W) / max(W - 1, 1),
                         indexing="ij")
    img = 60.0 + 60.0 * yy + 40.0 * xx
    for _ in range(n_shapes):
        cy, cx = rng.uniform(0, 1, size=2)
        ry, rx = rng.uniform(0.03, 0.25, size=2)
        level = rng.uniform(0, 255)
        if rng.random() < 0.5:
            mask = ((yy - cy) / ry) ** 2 + ((xx - cx) / rx) ** 2 <= 1.0
        else:
            mask = (np.abs(yy - cy) <= ry) & (np.abs(xx - cx) <= rx)
        img[mask] = level
    return np.clip(img, 0.0, 255.0)


def deblur_problem(H, W, seed=0, psf_sigma=4.0, noise_sigma=1.0):
    """(I, x_true): the scene blurred by a Gaussian PSF (zero outside the
    image) plus N(0, noise_sigma^2) noise, both divided by noise_sigma so the
    noise has unit variance."""
    x = test_scene(H, W, seed=seed)
    blurred = gaussian_filter(x, psf_sigma, mode="constant", truncate=4.0)
    noise = rng_for(seed + 1).standard_normal((H, W)) * noise_sigma
    return (blurred + noise) / noise_sigma, x / noise_sigma
