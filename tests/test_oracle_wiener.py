"""Pins of the oracle's nonstationary Wiener deblurring (appendix D of the
paper: regularised per-block inverse eigenvalues, eq. sol, overlap-add with
valences).

The paper prints no values; the pins are algebraic identities of the filter:

* the tapers of the two windows over every node add up to one;
* unregularised, filtering the blurred image itself returns the reference
  image exactly (this fails if the complex conjugate is dropped or misplaced);
* identical reference and blurred images give the identity filter, a blur
  that is a scalar multiple gives the inverse scale;
* the filter is invariant to a common scale of its inputs (relative eps) and
  vanishes as eps grows.
"""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O


@pytest.mark.parametrize("n,block", [(37, 16), (64, 64), (5, 8), (100, 32)])
def test_tapers_partition_unity(n, block):
    t = O.wiener_taper(block)
    acc = np.zeros(n)
    for o in O.wiener_starts(n, block):
        for u in range(block):
            if 0 <= o + u < n:
                acc[o + u] += t[u]
    assert np.max(np.abs(acc - 1.0)) <= 1e-14


@pytest.mark.parametrize("shape,block", [((37, 45), 16), ((12, 14, 10), 8)])
def test_filtering_the_blurred_image_returns_the_reference(shape, block):
    rng = np.random.default_rng(1)
    ref = rng.standard_normal(shape)
    blur = rng.standard_normal(shape)
    out = O.wiener_deblur(ref, blur, blur, block, 0.0)
    assert np.max(np.abs(out - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape,block", [((37, 45), 16), ((12, 14, 10), 8)])
def test_identity_and_scalar_blur(shape, block):
    rng = np.random.default_rng(2)
    m = rng.standard_normal(shape)
    x = rng.standard_normal(shape)
    assert np.max(np.abs(O.wiener_deblur(m, m, x, block, 0.0) - x)) <= 1e-10 * np.max(np.abs(x))
    assert np.max(np.abs(O.wiener_deblur(m, 2.5 * m, x, block, 0.0) - x / 2.5)) <= 1e-10 * np.max(np.abs(x))


def test_scale_invariance_and_regularisation():
    rng = np.random.default_rng(3)
    ref, blur, x = (rng.standard_normal((30, 41)) for _ in range(3))
    a = O.wiener_deblur(ref, blur, x, 16, 1e-2)
    b = O.wiener_deblur(3.0 * ref, 3.0 * blur, 3.0 * x, 16, 1e-2)
    assert np.max(np.abs(b - 3.0 * a)) <= 1e-12 * np.max(np.abs(b))
    big = O.wiener_deblur(ref, blur, x, 16, 1e8)
    assert np.linalg.norm(big) <= 1e-6 * np.linalg.norm(a)
