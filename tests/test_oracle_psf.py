"""Pins of the oracle's point-spread-function Hessian (appendix C of the
paper: PSF images of a scatterer lattice, windowed and interpolated with
multilinear weights, eq. trilinear).

The paper prints no values; the pins are mathematical:

* the column of a lattice node is exactly the window of the PSF image
  around that node (weight 1 on one corner);
* PSF images made of one fixed kernel at every scatterer give a Hessian that
  applies that kernel as a convolution (translation invariance reproduced
  exactly, every block, asymmetric kernels so a flipped shift fails);
* kernels whose amplitude varies linearly across the lattice are
  interpolated exactly (bilinear / trilinear weights);
* PSF images are columns of the symmetric L^T L: <P_q, S_q'> = <S_q, P_q'>;
* the monoparameter Hessian is the lnIp block of the multiparameter one.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth


def _window(arr, c, W):
    """arr[c + o] for |o| <= W as a dict offset -> value (inside only)."""
    out = {}
    nd = arr.ndim
    for o in np.ndindex(*([2 * W + 1] * nd)):
        oo = tuple(x - W for x in o)
        idx = tuple(c[k] + oo[k] for k in range(nd))
        if all(0 <= idx[k] < arr.shape[k] for k in range(nd)):
            out[oo] = arr[idx]
    return out


@pytest.mark.parametrize("shape,spacing", [((13, 11), 5), ((9, 10, 8), 4)])
def test_column_of_a_scatterer_is_its_window(shape, spacing):
    rng = np.random.default_rng(1)
    P = rng.standard_normal((2, 2) + shape)
    H = O.psf_hessian(P, spacing).toarray()
    N = int(np.prod(shape))
    W = O.psf_halfwidth(spacing)
    nd = len(shape)
    lat = [O.psf_lattice(shape[k], spacing) for k in range(nd)]   # numpy-axis order here
    for c in [tuple(l[0] for l in lat), tuple(l[-1] for l in lat)]:
        j = np.ravel_multi_index(c, shape)
        for p in range(2):
            for q in range(2):
                col = H[p * N:(p + 1) * N, q * N + j].reshape(shape)
                ref = np.zeros(shape)
                for oo, v in _window(P[q][p], c, W).items():
                    ref[tuple(c[k] + oo[k] for k in range(nd))] = v
                assert np.array_equal(col, ref), (c, p, q)


def _stationary(shape, spacing, kernels):
    """PSF images with kernel K_pq placed at every scatterer."""
    W = O.psf_halfwidth(spacing)
    nd = len(shape)
    P = np.zeros((2, 2) + shape)
    spikes = O.psf_scatterers(shape, spacing, 0)[0]
    for p in range(2):
        for q in range(2):
            P[q][p] = signal.convolve(spikes, kernels[p][q], mode="same")
    return P, W


def test_stationary_kernel_is_convolution():
    spacing = 5
    W = O.psf_halfwidth(spacing)
    # sizes with the last scatterer at least W from the far edge
    shape = (W + 3 * spacing + W + 1, W + 4 * spacing + W + 1)
    rng = np.random.default_rng(2)
    K = [[rng.standard_normal((2 * W + 1, 2 * W + 1)) for _ in range(2)] for _ in range(2)]
    P, _ = _stationary(shape, spacing, K)
    H = O.psf_hessian(P, spacing)
    x = rng.standard_normal((2,) + shape)
    y = (H @ x.reshape(-1)).reshape((2,) + shape)
    for p in range(2):
        ref = sum(signal.convolve2d(x[q], K[p][q], mode="same") for q in range(2))
        assert np.max(np.abs(y[p] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_linear_amplitude_is_interpolated_exactly():
    """P = alpha(c) K with alpha affine in the scatterer position: the column
    of any point inside the lattice hull is alpha(j) K (bilinear weights)."""
    spacing = 6
    W = O.psf_halfwidth(spacing)
    shape = (W + 2 * spacing + W + 1, W + 3 * spacing + W + 1)
    rng = np.random.default_rng(3)
    K = rng.standard_normal((2 * W + 1, 2 * W + 1))
    alpha = lambda i0, i1: 1.0 + 0.3 * i0 - 0.2 * i1
    P = np.zeros((2, 2) + shape)
    lat0 = O.psf_lattice(shape[0], spacing)
    lat1 = O.psf_lattice(shape[1], spacing)
    for c0 in lat0:
        for c1 in lat1:
            for o0 in range(-W, W + 1):
                for o1 in range(-W, W + 1):
                    P[0][0][c0 + o0, c1 + o1] = alpha(c0, c1) * K[o0 + W, o1 + W]
    H = O.psf_hessian(P, spacing).toarray()
    N = int(np.prod(shape))
    for j0, j1 in [(lat0[0] + 2, lat1[1] + 1), (lat0[1] + 5, lat1[2] + 3), (lat0[0] + 1, lat1[0] + 4)]:
        col = H[:N, np.ravel_multi_index((j0, j1), shape)].reshape(shape)
        ref = np.zeros(shape)
        ref[j0 - W:j0 + W + 1, j1 - W:j1 + W + 1] = alpha(j0, j1) * K
        assert np.max(np.abs(col - ref)) <= 1e-12


def test_mono_is_the_lnip_block():
    rng = np.random.default_rng(4)
    P = rng.standard_normal((2, 2, 12, 14))
    H = O.psf_hessian(P, 4).toarray()
    Hm = O.psf_hessian(P, 4, mono=True).toarray()
    N = 12 * 14
    # the same entries (duplicate corner contributions may be summed in another order)
    assert np.max(np.abs(Hm - H[N:, N:])) <= 1e-14 * np.max(np.abs(Hm))


def test_psf_images_are_columns_of_a_symmetric_operator():
    w = synth.small((18, 22), nt=60, npml=3, seed=5, nshot=2, uneven=True)
    prob = O.Problem(w.h, w.dt, w.nt, w.npml, w.pml_R, w.pml_freq, w.win, w.src, w.rec,
                     w.wavelet.astype(np.float64))
    lnvp, lnip = w.lnvp.astype(np.float64), w.lnip.astype(np.float64)
    P = O.psf_images(prob, lnvp, lnip, 5)
    S = [O.psf_scatterers(lnvp.shape, 5, q) for q in range(2)]
    a = np.vdot(P[0], S[1])
    b = np.vdot(S[0], P[1])
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    assert np.vdot(P[0], S[0]) > 0 and np.vdot(P[1], S[1]) > 0
