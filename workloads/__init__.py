"""Seeded synthetic inputs shared by the HIP library's tests/benchmark and the oracle.

This module holds none of the method's arithmetic: it draws images, blur
matrices and raw noise only.  Each side forms the observation
C = M(X_true) + nu * ||M(X_true)||_F / ||N0||_F * N0 with its own operator.

Everything is FP64 numpy, laid out (n3, rows, cols) = (p, n, s).

The paper's test images are not available, so every image here is a
synthetic stand-in with the paper's shapes, value range [0, 1] and kind of
structure (smooth regions plus edges), blurred by the banded Gaussian
Toeplitz matrix of Sec. 4 and contaminated by Gaussian noise at a relative
level nu (Sec. 4).

Seeds: workload c (1-based), instance i uses numpy.random.default_rng(1000 c + i).
"""
import math

import numpy as np

# Mixing tubes (A(:,:,k) = a_k T, the recipe of eq. tensor_form in Sec. 4).
COLOUR_TUBE = (0.7, 0.15, 0.15)
PAPER_COLOUR_TUBE = (0.8, 0.0, 0.1)     # th(0.8, 0, 0.1) is the printed A_color


def gaussian_toeplitz(n, sigma, r):
    """Banded Gaussian blur of Sec. 4: a_kl = exp(-(k-l)^2/(2 sigma^2))/(sigma sqrt(2 pi)), |k-l| <= r."""
    T = np.zeros((n, n))
    c = 1.0 / (sigma * math.sqrt(2.0 * math.pi))
    for d in range(-r, r + 1):
        val = c * math.exp(-(d * d) / (2.0 * sigma * sigma))
        idx = np.arange(max(0, -d), min(n, n - d))
        T[idx, idx + d] = val
    return T


def _minmax(X):
    lo, hi = X.min(), X.max()
    return (X - lo) / (hi - lo) if hi > lo else np.zeros_like(X)


def smooth_field(rng, p, n, s, count=8):
    """Sum of ``count`` random 2-D Gaussians per channel, globally scaled to [0, 1]."""
    X = np.zeros((p, n, s))
    ii = np.arange(n)[:, None]
    jj = np.arange(s)[None, :]
    for k in range(p):
        for _ in range(count):
            ci = rng.uniform(0, n)
            cj = rng.uniform(0, s)
            w = rng.uniform(n / 16.0, n / 4.0)
            amp = rng.uniform(0.2, 1.0)
            X[k] += amp * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * w * w))
    return _minmax(X)


def edges_field(rng, p, n, s, count=20):
    """Smooth field plus ``count`` axis-aligned rectangles per channel, scaled to [0, 1]."""
    X = smooth_field(rng, p, n, s)
    for k in range(p):
        for _ in range(count):
            h = int(rng.uniform(n / 32.0, n / 4.0))
            w = int(rng.uniform(s / 32.0, s / 4.0))
            i0 = int(rng.integers(0, max(1, n - h)))
            j0 = int(rng.integers(0, max(1, s - w)))
            X[k, i0:i0 + h, j0:j0 + w] += rng.uniform(0.1, 0.6)
    return _minmax(X)


def moving_blobs(rng, p, n, s, count=8, speed=2.0):
    """Video: ``count`` Gaussian blobs (width U[8, 32] px) drifting ``speed`` px/frame,
    reflected at the borders; frame k is slice k."""
    X = np.zeros((p, n, s))
    ii = np.arange(n)[:, None]
    jj = np.arange(s)[None, :]
    blobs = []
    for _ in range(count):
        ang = rng.uniform(0.0, 2.0 * math.pi)
        blobs.append([rng.uniform(0, n), rng.uniform(0, s), speed * math.cos(ang),
                      speed * math.sin(ang), rng.uniform(8.0, 32.0), rng.uniform(0.3, 1.0)])
    for k in range(p):
        for b in blobs:
            X[k] += b[5] * np.exp(-((ii - b[0]) ** 2 + (jj - b[1]) ** 2) / (2.0 * b[4] ** 2))
            b[0] += b[2]
            b[1] += b[3]
            if b[0] < 0 or b[0] >= n:
                b[2] = -b[2]
                b[0] = min(max(b[0], 0.0), n - 1.0)
            if b[1] < 0 or b[1] >= s:
                b[3] = -b[3]
                b[1] = min(max(b[1], 0.0), s - 1.0)
    return _minmax(X)


def mixed_blur(tube, T):
    """A with frontal slices A(:,:,k) = tube_k * T."""
    return np.ascontiguousarray(np.stack([c * T for c in tube], axis=0))


def tube_for(p):
    """Mixing tube used for a given n3: the colour tube for p = 3, the
    half-kernel (0.5, 0.25, 0, ...) of [0.25, 0.5, 0.25] otherwise."""
    if p == 3:
        return COLOUR_TUBE
    t = np.zeros(p)
    t[0] = 0.5
    if p > 1:
        t[1] = 0.25
    return tuple(t)


def colour_small():
    """n1 = n2 = s = 32, n3 = 3, sigma = 2, r = 4, smooth field, nu = 1e-3, 20 iterations, FP64."""
    rng = np.random.default_rng(1000 * 1 + 0)
    n, p = 32, 3
    A = mixed_blur(COLOUR_TUBE, gaussian_toeplitz(n, 2.0, 4))
    X = smooth_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    return {"name": "colour_32x32x3", "A": A, "B": None, "X_true": X, "N0": N0,
            "nu": 1e-3, "iters": 20}


def colour_256(instance=0):
    """n1 = n2 = s = 256, n3 = 3, sigma = 3, r = 8, smooth + edges field, nu = 1e-2, 40 iterations."""
    rng = np.random.default_rng(1000 * 2 + instance)
    n, p = 256, 3
    A = mixed_blur(COLOUR_TUBE, gaussian_toeplitz(n, 3.0, 8))
    X = edges_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    return {"name": "colour_256x256x3", "A": A, "B": None, "X_true": X, "N0": N0,
            "nu": 1e-2, "iters": 40}


def video_256(instance=0, frames=32):
    """Two-sided A *c X *c B, n = s = 256, n3 = 32 frames: A = e_1 (x) T_{2.5,7}
    (per-frame blur), B(:,:,k) = t_k T_{1.5,4}^T with t = (0.5, 0.25, 0, ...),
    moving blobs, nu = 5e-3, 40 Arnoldi steps."""
    rng = np.random.default_rng(1000 * 3 + instance)
    n, p = 256, frames
    A = np.zeros((p, n, n))
    A[0] = gaussian_toeplitz(n, 2.5, 7)
    Tb = gaussian_toeplitz(n, 1.5, 4).T
    B = mixed_blur(tube_for(p), Tb)
    X = moving_blobs(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    return {"name": "video_256x256x32", "A": A, "B": B, "X_true": X, "N0": N0,
            "nu": 5e-3, "iters": 40}


def paper_shaped(n, nu, instance=0):
    """Stand-in for the paper's colour experiments (Sec. 4: two-sided
    A *c X *c B, n3 = 3, Gaussian Toeplitz blur sigma = 4, r = 6, noise level
    nu): A(:,:,k) = t_k T with the printed A_color tube t = (0.8, 0, 0.1), B =
    e_1 (x) T^T (the same blur along the other image direction, no channel
    mixing), a smooth-plus-edges field in place of the images (papav256,
    cat1024), which are not available."""
    rng = np.random.default_rng(1000 * 7 + 10 * instance + (n // 256))
    p = 3
    T = gaussian_toeplitz(n, 4.0, 6)
    A = mixed_blur(PAPER_COLOUR_TUBE, T)
    B = mixed_blur((1.0, 0.0, 0.0), np.ascontiguousarray(T.T))
    X = edges_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    return {"name": "paper_%dx%dx3" % (n, n), "A": A, "B": B, "X_true": X, "N0": N0, "nu": nu}


def batch_instance(i):
    """Instance i (0..63) of the uneven batched set: n = s in {64, ..., 512},
    n3 in {3, 8, 31}, sigma ~ U[1, 4], r = ceil(2.5 sigma), nu ~ logU[1e-3, 1e-2]."""
    rng = np.random.default_rng(1000 * 4 + i)
    n = int(rng.choice([64, 128, 192, 256, 384, 512]))
    p = int(rng.choice([3, 8, 31]))
    sigma = float(rng.uniform(1.0, 4.0))
    r = int(math.ceil(2.5 * sigma))
    nu = float(10.0 ** rng.uniform(-3.0, -2.0))
    A = mixed_blur(tube_for(p), gaussian_toeplitz(n, sigma, r))
    X = edges_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    return {"name": "batch_%02d" % i, "A": A, "B": None, "X_true": X, "N0": N0,
            "nu": nu, "iters": 40}


def tiny_random(seed, p, n1, n2, s, two_sided=False):
    """Dense random operator and tensors for the small parity cases."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((p, n1, n2))
    B = rng.standard_normal((p, s, s)) if two_sided else None
    X = rng.standard_normal((p, n2, s))
    Y = rng.standard_normal((p, n1, s))
    return {"A": A, "B": B, "X": X, "Y": Y}


def band_blur(p, n, sig_lo=1.5, sig_hi=4.0, last_weight=None):
    """Hyperspectral-like operator: frontal slice k is w_k T_{sigma_k, ceil(2.5 sigma_k)}
    with sigma_k spanning [sig_lo, sig_hi] linearly over the p bands.

    last_weight=None: w_k = 2^-(k+1) (the first few bands carry the operator).
    last_weight=c: w_k = c^(k/(p-1)), a geometric decay from 1 at the first band
    to c at the last (c = 0.005 at p = 64 is a factor 0.919 per band), so every
    band's sigma enters every transform-domain slice.  With all blurs equal the
    tube transform of such a decay stays positive while (1-r)/(1+r) > r^p for the
    ratio r, which holds for c = 0.005 at every p >= 2."""
    A = np.zeros((p, n, n))
    for k in range(p):
        sk = sig_lo + (sig_hi - sig_lo) * (k / max(1, p - 1))
        if last_weight is None:
            wk = 2.0 ** -(k + 1)
        else:
            wk = float(last_weight) ** (k / max(1, p - 1))
        A[k] = wk * gaussian_toeplitz(n, sk, int(math.ceil(2.5 * sk)))
    return A


HYPER_LAST_WEIGHT = 0.005


def spectral_field(rng, p, n, s, count=8):
    """8 spatial Gaussians, each with a smooth spectral profile across the p bands, in [0, 1]."""
    ii = np.arange(n)[:, None]
    jj = np.arange(s)[None, :]
    t = np.arange(p) / max(1, p - 1)
    X = np.zeros((p, n, s))
    for _ in range(count):
        ci, cj = rng.uniform(0, n), rng.uniform(0, s)
        w = rng.uniform(n / 16.0, n / 4.0)
        spat = np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * w * w))
        mu, sd, amp = rng.uniform(0.0, 1.0), rng.uniform(0.15, 0.6), rng.uniform(0.2, 1.0)
        prof = amp * np.exp(-((t - mu) ** 2) / (2.0 * sd * sd))
        X += prof[:, None, None] * spat[None, :, :]
    return _minmax(X)


def hyperspectral(instance=0, n=512, p=64, seed_base=5000):
    """The hyperspectral-like workload: n1 = n2 = s = n, n3 = p, band-dependent blur
    sigma from 1.5 to 4 with slice weights decaying geometrically to 0.005 at the
    last band, spectral Gaussian field, noise nu ~ logU[1e-3, 2e-2]."""
    rng = np.random.default_rng(seed_base + instance)
    A = band_blur(p, n, last_weight=HYPER_LAST_WEIGHT)
    X = spectral_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    nu = float(10.0 ** rng.uniform(-3.0, math.log10(2e-2)))
    return {"name": "hyperspectral_%dx%dx%d" % (n, n, p), "A": A, "B": None, "X_true": X, "N0": N0,
            "nu": nu, "iters": 40}


def learned_stop_instance(i, n=64, p_choices=(8, 16)):
    """Training / evaluation instance for the learned stopping rule: a hyperspectral-like
    problem with random blur range, band count and noise level (seed 6000 + i)."""
    rng = np.random.default_rng(6000 + i)
    p = int(rng.choice(p_choices))
    lo = float(rng.uniform(1.0, 2.5))
    hi = float(rng.uniform(lo + 0.5, 5.0))
    A = band_blur(p, n, lo, hi)
    X = spectral_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    nu = float(10.0 ** rng.uniform(-3.0, math.log10(3e-2)))
    return {"name": "learned_%d" % i, "A": A, "B": None, "X_true": X, "N0": N0, "nu": nu, "iters": 40}


def batch_train_instance(i):
    """Training problem for the learned stop on the uneven batch: the batch's
    distributions with smaller slices, n = s in {64, 96, 128} (seed 7000 + i)."""
    rng = np.random.default_rng(7000 + i)
    n = int(rng.choice([64, 96, 128]))
    p = int(rng.choice([3, 8, 31]))
    sigma = float(rng.uniform(1.0, 4.0))
    r = int(math.ceil(2.5 * sigma))
    nu = float(10.0 ** rng.uniform(-3.0, -2.0))
    A = mixed_blur(tube_for(p), gaussian_toeplitz(n, sigma, r))
    X = edges_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    return {"name": "batch_train_%d" % i, "A": A, "B": None, "X_true": X, "N0": N0, "nu": nu, "iters": 40}


def colour_video(instance=0, n=128, frames=16):
    """Order-4 colour video deblurring (the higher-order extension of Sec. 1):
    A in R^{n x n x 3 x frames}, stored (frames, 3, n, n), A[f, c] = t_f a_c T
    with the colour tube a = (0.7, 0.15, 0.15) along mode 3, the temporal
    half-kernel t = (0.5, 0.25, 0, ...) of [0.25, 0.5, 0.25] along mode 4 and
    the sigma = 2, r = 5 Gaussian blur T; X_true moving blobs (2 px/frame),
    each with its own colour weights; nu = 5e-3, 40 GKB steps (seed 8000 + i)."""
    rng = np.random.default_rng(1000 * 8 + instance)
    T = gaussian_toeplitz(n, 2.0, 5)
    t = tube_for(frames)
    A = np.zeros((frames, 3, n, n))
    for f in range(frames):
        for c in range(3):
            A[f, c] = t[f] * COLOUR_TUBE[c] * T
    V = np.zeros((frames, 3, n, n))
    for _ in range(3):          # three layers of blobs, each with a random colour mix
        w = rng.uniform(0.2, 1.0, 3)
        layer = moving_blobs(rng, frames, n, n, count=4)
        for c in range(3):
            V[:, c] += w[c] * layer
    X = _minmax(V)
    N0 = rng.standard_normal((frames, 3, n, n))
    return {"name": "colour_video_%dx%dx3x%d" % (n, n, frames), "A": A, "B": None, "X_true": X, "N0": N0,
            "nu": 5e-3, "iters": 40}


_HYPER_OPS = {}


def hyper_family_operator(n=128, p=64):
    """The band-dependent blur of the hyperspectral workload at size n (cached:
    every instance of the family shares it)."""
    key = (n, p)
    if key not in _HYPER_OPS:
        _HYPER_OPS[key] = band_blur(p, n, last_weight=HYPER_LAST_WEIGHT)
    return _HYPER_OPS[key]


def hyper_family_instance(i, n=128, p=64):
    """Training / evaluation problem of the learned stop for the hyperspectral
    workload: its operator (sigma 1.5 to 4, slice weights to 0.005) at size n,
    its own spectral field and noise, nu ~ logU[1e-3, 2e-2] (seed 9000 + i;
    A is shared by all instances of one n)."""
    rng = np.random.default_rng(9000 + i)
    X = spectral_field(rng, p, n, n)
    N0 = rng.standard_normal((p, n, n))
    nu = float(10.0 ** rng.uniform(-3.0, math.log10(2e-2)))
    return {"name": "hyper_family_%d_%d" % (n, i), "A": hyper_family_operator(n, p), "B": None, "X_true": X,
            "N0": N0, "nu": nu, "iters": 40}
