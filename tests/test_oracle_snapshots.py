"""Pins of the oracle's compressed snapshots (appendix A: the background
history may be kept by checkpointing or compression; the storage format is
a reading: per-snapshot max-abs scale, round to nearest with ties to even,
FP16 or BF16).

* rounding to 8 significant bits equals torch's float32 -> bfloat16
  conversion on float32 inputs (a library routine), ties go to even, the
  relative error stays within 2^-8 and representable values are unchanged;
* the FP16 path keeps the largest magnitude exactly (it maps to 2^14) and
  every value within 2^-11 relative in the normal range;
* a history replayed from compressed snapshots gives an image whose error
  against the exact history is between u / 8 and 4 u (u = 2^-11 FP16,
  2^-8 BF16), and FP64 snapshots give the exact image bit for bit.
"""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth


def test_round_significand_ties_and_bound():
    one = 1.0
    assert O.round_significand(np.array([one + 2.0 ** -8]), 8)[0] == 1.0            # tie -> even
    assert O.round_significand(np.array([one + 3 * 2.0 ** -8]), 8)[0] == 1.0 + 2.0 ** -6
    assert O.round_significand(np.array([-(one + 2.0 ** -8)]), 8)[0] == -1.0
    assert O.round_significand(np.array([0.0]), 8)[0] == 0.0
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000) * np.exp(rng.uniform(-20, 20, 10000))
    r = O.round_significand(x, 8)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    assert np.array_equal(O.round_significand(r, 8), r)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_significand(x.astype(np.float64), 8), ref)


@pytest.mark.parametrize("dtype,bits", [("f16", 11), ("bf16", 8)])
def test_compress_field_bounds(dtype, bits):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((40, 30)) * 3e-7
    c = O.compress_field(x, dtype)
    i = np.unravel_index(np.argmax(np.abs(x)), x.shape)
    assert c[i] == x[i]                                  # the scale's own value is exact
    big = np.abs(x) >= 2.0 ** -14 * np.max(np.abs(x))    # normal range of both formats
    assert np.all(np.abs(c - x)[big] <= 2.0 ** -bits * np.abs(x)[big])
    assert np.array_equal(O.compress_field(np.zeros(5), dtype), np.zeros(5))
    assert np.array_equal(O.compress_field(x, "f64"), x)


def test_compressed_history_image_error():
    w = synth.small((40, 56), nt=160, npml=6, seed=81, nshot=2, uneven=True)
    prob = O.Problem(w.h, w.dt, w.nt, w.npml, w.pml_R, w.pml_freq, w.win, w.src, w.rec,
                     w.wavelet.astype(np.float64))
    lnvp, lnip = w.lnvp.astype(np.float64), w.lnip.astype(np.float64)
    rng = np.random.default_rng(3)
    ys = [rng.standard_normal((w.nt, len(r))) for r in w.rec]
    exact = O.adjoint(prob, lnvp, lnip, ys)
    assert np.array_equal(O.adjoint(prob, lnvp, lnip, ys, ckpt_every=20, ckpt_dtype="f64"), exact)
    for dtype, u in (("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        img = O.adjoint(prob, lnvp, lnip, ys, ckpt_every=20, ckpt_dtype=dtype)
        e = max(np.linalg.norm(img[k] - exact[k]) / np.linalg.norm(exact[k]) for k in range(2))
        print(dtype, e, e / u)
        assert u / 8 <= e <= 4 * u
