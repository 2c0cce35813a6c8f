"""Nonstationary Wiener deblurring (appendix D) on the GPU (hipFFT), through
the C ABI, against the FP64 oracle (numpy FFT).

Bar: FP32 transforms of tapered blocks followed by a regularised division;
relative L2 error 1e-4 against the FP64 oracle, as for the operators.
"""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth
from gpu_common import f64, oracle_problem, rel, require_gpu, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


CASES = [((37, 45), 16, 1e-3), ((64, 75), 32, 1e-2), ((240, 100), 64, 1e-3), ((12, 14, 10), 8, 1e-3),
         # blocks larger than the image along every axis
         ((20, 24), 64, 1e-3), ((5, 6, 4), 8, 1e-3)]


@pytest.mark.parametrize("n,block,eps", CASES)
def test_wiener_vs_oracle_random(torch, n, block, eps):
    from paper_2508_10405_amd import lsrtm
    print(f"[case] wiener {n} block {block} eps {eps}", flush=True)
    shape = tuple(reversed(n))
    ctx = lsrtm.Context(n, (10.0,) * len(n), 10, 1e-3)
    rng = np.random.default_rng(sum(n) + block)
    ref, blur, x = (rng.standard_normal(shape) for _ in range(3))
    out = ctx.wiener(to_dev(torch, ref), to_dev(torch, blur), to_dev(torch, x), block=block, eps_rel=eps)
    expect = O.wiener_deblur(ref, blur, x, block, eps)
    e = rel(out.cpu().numpy(), expect)
    print("wiener rel", e, flush=True)
    assert e <= TOL
    ctx.close()


def test_wiener_identity(torch):
    """Unregularised filter of an image by itself is the identity."""
    from paper_2508_10405_amd import lsrtm
    n = (50, 61)
    ctx = lsrtm.Context(n, (10.0, 10.0), 10, 1e-3)
    rng = np.random.default_rng(7)
    m = to_dev(torch, rng.standard_normal((61, 50)))
    x = to_dev(torch, rng.standard_normal((61, 50)))
    out = ctx.wiener(m, m, x, block=16, eps_rel=0.0)
    e = rel(out.cpu().numpy(), x.cpu().numpy())
    print("identity rel", e, flush=True)
    assert e <= 1e-5
    ctx.close()


def test_wiener_on_migrated_images(torch):
    """The paper's use: m_ref = m_in = RTM image, m_blur = its remigration
    L^T L m_rtm, both parameters in one call (each filtered on its own)."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((48, 64), nt=140, npml=8, seed=61, nshot=3, uneven=True)
    ctx = lsrtm.context_for(w)
    m_rtm = ctx.adjoint(ctx.born(to_dev(torch, w.dm)))
    m_rem = ctx.adjoint(ctx.born(m_rtm))
    out = ctx.wiener(m_rtm, m_rem, block=16, eps_rel=1e-3)
    for k in range(2):
        expect = O.wiener_deblur(m_rtm[k].cpu().numpy().astype(np.float64),
                                 m_rem[k].cpu().numpy().astype(np.float64),
                                 m_rtm[k].cpu().numpy().astype(np.float64), 16, 1e-3)
        e = rel(out[k].cpu().numpy(), expect)
        print("migrated wiener", k, e, flush=True)
        assert e <= TOL
    single = ctx.wiener(m_rtm[1].contiguous(), m_rem[1].contiguous(), block=16, eps_rel=1e-3)
    assert torch.equal(single, out[1])
    ctx.close()
    # oracle-only chain: the oracle's RTM image and remigration, then its filter
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    LtL = lambda m: O.adjoint(prob, lnvp, lnip, O.born(prob, lnvp, lnip, m))
    r_rtm = LtL(f64(w.dm))
    r_rem = LtL(r_rtm)
    for k in range(2):
        expect = O.wiener_deblur(r_rtm[k], r_rem[k], r_rtm[k], 16, 1e-3)
        e = rel(out[k].cpu().numpy(), expect)
        print("migrated wiener, oracle-only chain", k, e, flush=True)
        assert e <= TOL


def test_wiener_errors(torch):
    from paper_2508_10405_amd import lsrtm
    ctx = lsrtm.Context((20, 24), (10.0, 10.0), 10, 1e-3)
    m = torch.zeros((24, 20), device="cuda")
    for block, eps in ((15, 1e-3), (0, 1e-3), (16, -1.0)):
        with pytest.raises(lsrtm.LsrtmError):
            ctx.wiener(m, m, block=block, eps_rel=eps)
    ctx.close()
