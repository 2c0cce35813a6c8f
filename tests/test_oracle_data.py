"""Pins of the oracle's data preparation (section 4.1: nonlinear residual
with a top mute) and of the monoparameter inversion (section 4.2's
impedance-only mode) expressed through the preconditioned CGNR.

* mute: what the paper uses it for (section 4.1: keep the near-offset
  reflections, remove the direct wave) checked on the oracle's own
  wavefields: in a homogeneous medium the muted record of every receiver
  keeps under 1e-5 of the direct wave's energy, and the reflection from a
  layer below keeps over 0.999 of its energy at the near offsets; the same
  checks fail for a cut time computed in grid units, with the axes' spacings
  swapped, with the delay's sign flipped or with the weights inverted;
* mute: zero before the cut time, one after cut + taper, the cosine ramp
  between (checked sample by sample against its closed form at the receiver
  where the cut falls mid-record), linear, and idempotent without a taper;
* a 0/1 mask as the CGNR preconditioner is CGNR on the restricted operator
  (the masked parameter stays exactly zero).
"""
import numpy as np

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth


def _problem(w):
    return O.Problem(w.h, w.dt, w.nt, w.npml, w.pml_R, w.pml_freq, w.win, w.src, w.rec,
                     w.wavelet.astype(np.float64))


def test_mute_removes_direct_wave_keeps_reflection():
    nz, nx, h, npml, nt, dt, f0 = 60, 120, (10.0, 12.5), 10, 900, 1e-3, 15.0
    vp = np.full((nx, nz), 2000.0)
    rho = np.full((nx, nz), 2000.0)
    vp2, rho2 = vp.copy(), rho.copy()
    vp2[:, 40:], rho2[:, 40:] = 3000.0, 2300.0          # a layer 400 m down
    src = (2, 10)
    rx = np.arange(10, 111, 5)                          # offsets 0 .. 1250 m
    rec = np.stack([np.full_like(rx, 2), rx], 1)
    wav = synth.ricker(f0, nt, dt)[None].astype(np.float64)

    def prob_with(hh):
        return O.Problem(hh, dt, nt, npml, 1e-4, f0, [((0, nz), (0, nx))], [src], [rec], wav)

    prob = prob_with(h)
    direct = O.forward(prob, np.log(vp), np.log(vp * rho))[0]
    refl = O.forward(prob, np.log(vp2), np.log(vp2 * rho2))[0] - direct
    near = rx - src[1] <= 55                             # offsets up to 687.5 m
    # cut at the direct arrival plus the wavelet's length (delay 1.5 / f0 to
    # its peak, the same again to its end)
    v, t0, ntap = 2000.0, 3.0 / f0, 20

    def kept(W, d):
        return np.sum((W * d) ** 2, 0) / np.sum(d ** 2, 0)

    W = O.mute_weights(prob, 0, v, t0, ntap)
    assert np.all(kept(W, direct) < 1e-5)
    assert np.all(kept(W, refl)[near] > 0.999)
    bad = {"grid units": O.mute_weights(prob_with((1.0, 1.0)), 0, v, t0, ntap),
           "spacings swapped": O.mute_weights(prob_with(h[::-1]), 0, v, t0, ntap),
           "delay sign": O.mute_weights(prob, 0, v, -t0, ntap),
           "inverted": 1.0 - W}
    for name, Wb in bad.items():
        assert np.any(kept(Wb, direct) > 1e-3) or np.any(kept(Wb, refl)[near] < 0.9), name


def test_mute_weights_closed_form():
    w = synth.small((30, 40), nt=200, npml=4, seed=71, nshot=2, uneven=True)
    prob = _problem(w)
    v, t0, L = 1500.0, 0.02, 10
    for s in range(2):
        W = O.mute_weights(prob, s, v, t0, L)
        rec = np.asarray(prob.rec[s], float).reshape(-1, 2)
        src = np.asarray(prob.src[s], float)
        for r in range(W.shape[1]):
            D = np.hypot((rec[r, 0] - src[0]) * prob.h[0], (rec[r, 1] - src[1]) * prob.h[1])
            tc = t0 + D / v
            for n in range(prob.nt):
                t = (n + 1) * prob.dt
                if t < tc:
                    assert W[n, r] == 0.0
                elif t >= tc + L * prob.dt:
                    assert W[n, r] == 1.0
                else:
                    assert abs(W[n, r] - 0.5 * (1 - np.cos(np.pi * (t - tc) / (L * prob.dt)))) <= 1e-15
    assert np.any((W > 0) & (W < 1))


def test_mute_linear_and_idempotent():
    w = synth.small((30, 40), nt=120, npml=4, seed=72, nshot=2, uneven=True)
    prob = _problem(w)
    rng = np.random.default_rng(0)
    ds = [rng.standard_normal((prob.nt, len(r))) for r in prob.rec]
    a = O.mute(prob, [2.0 * d for d in ds], 2000.0, 0.01, 5)
    b = O.mute(prob, ds, 2000.0, 0.01, 5)
    assert all(np.array_equal(x, 2.0 * y) for x, y in zip(a, b))
    c = O.mute(prob, ds, 2000.0, 0.01, 0)
    cc = O.mute(prob, c, 2000.0, 0.01, 0)
    assert all(np.array_equal(x, y) for x, y in zip(c, cc))


def test_mask_preconditioner_is_restricted_cgnr():
    rng = np.random.default_rng(5)
    m, n = 40, 10
    A = rng.standard_normal((m, 2 * n))
    d = rng.standard_normal(m)
    mask = np.concatenate([np.zeros(n), np.ones(n)])
    for k in (1, 4, 8):
        x, h = O.pcgnr(lambda p: A @ p, lambda r: A.T @ r, d, k, mask)
        A2 = A[:, n:]
        y, h2 = O.cgnr(lambda p: A2 @ p, lambda r: A2.T @ r, d, k)
        assert np.all(x[:n] == 0.0)
        assert np.linalg.norm(x[n:] - y) <= 1e-10 * np.linalg.norm(y)
        assert np.allclose(h, h2, rtol=1e-10, atol=0)
