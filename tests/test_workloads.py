"""The seeded input generators: shapes, ranges, determinism, and the blur of Sec. 4."""
import math

import numpy as np

import workloads as W


def test_gaussian_toeplitz_entries():
    """a_kl = exp(-(k-l)^2/(2 sigma^2)) / (sigma sqrt(2 pi)) inside the band, 0 outside."""
    T = W.gaussian_toeplitz(20, 4.0, 6)
    for k in range(20):
        for l in range(20):
            d = k - l
            ref = math.exp(-d * d / 32.0) / (4.0 * math.sqrt(2 * math.pi)) if abs(d) <= 6 else 0.0
            assert abs(T[k, l] - ref) < 1e-15
    assert np.allclose(T, T.T)


def test_generators_deterministic_and_in_range():
    a = W.colour_small()
    b = W.colour_small()
    assert np.array_equal(a["X_true"], b["X_true"]) and np.array_equal(a["N0"], b["N0"])
    assert a["X_true"].shape == (3, 32, 32) and a["A"].shape == (3, 32, 32)
    assert a["X_true"].min() == 0.0 and a["X_true"].max() == 1.0
    c = W.colour_256()
    assert c["X_true"].shape == (3, 256, 256) and c["nu"] == 1e-2


def test_batch_instances_span_sizes():
    sizes = {W.batch_instance(i)["A"].shape for i in range(6)}
    for p, n, n2 in sizes:
        assert n == n2 and p in (3, 8, 31) and n in (64, 128, 192, 256, 384, 512)


def test_paper_shaped_structure():
    """The paper-shaped workload: A(:,:,k) = t_k T with t = (0.8, 0, 0.1), B =
    e_1 (x) T^T, T the sigma = 4, r = 6 Gaussian Toeplitz blur; the field in
    [0, 1]; seeded (two calls agree)."""
    w = W.paper_shaped(64, 1e-3)
    T = W.gaussian_toeplitz(64, 4.0, 6)
    for k, t in enumerate((0.8, 0.0, 0.1)):
        assert np.array_equal(w["A"][k], t * T)
    assert np.array_equal(w["B"][0], T.T)
    assert not w["B"][1].any() and not w["B"][2].any()
    assert w["X_true"].min() >= 0.0 and w["X_true"].max() <= 1.0
    w2 = W.paper_shaped(64, 1e-3)
    assert np.array_equal(w["X_true"], w2["X_true"]) and np.array_equal(w["N0"], w2["N0"])



def test_hyperspectral_band_weights():
    """The hyperspectral-like operator: slice k is w_k T_{sigma_k} with sigma_k
    linear from 1.5 to 4 and w_k decaying geometrically from 1 to 0.005, so the
    last band still carries 0.5 % of the first band's weight."""
    p, n = 64, 40
    A = W.band_blur(p, n, last_weight=W.HYPER_LAST_WEIGHT)
    for k in (0, 1, 31, 63):
        sk = 1.5 + 2.5 * k / 63.0
        T = W.gaussian_toeplitz(n, sk, int(math.ceil(2.5 * sk)))
        assert np.allclose(A[k], 0.005 ** (k / 63.0) * T, rtol=1e-14, atol=0.0)
    ratios = [np.abs(A[k + 1]).max() / np.abs(A[k]).max() for k in range(p - 1)]
    assert 0.85 < min(ratios) and max(ratios) < 0.95


def test_colour_video_structure():
    """Order-4 colour video: A[f, c] = t_f a_c T (mode-3 colour tube, mode-4
    temporal half-kernel), X_true in [0, 1], seeded."""
    w = W.colour_video(0, n=32, frames=4)
    assert w["A"].shape == (4, 3, 32, 32) and w["X_true"].shape == (4, 3, 32, 32)
    T = W.gaussian_toeplitz(32, 2.0, 5)
    for f, tf in enumerate((0.5, 0.25, 0.0, 0.0)):
        for c, ac in enumerate((0.7, 0.15, 0.15)):
            assert np.array_equal(w["A"][f, c], tf * ac * T)
    assert w["X_true"].min() == 0.0 and w["X_true"].max() == 1.0
    w2 = W.colour_video(0, n=32, frames=4)
    assert np.array_equal(w["X_true"], w2["X_true"])
