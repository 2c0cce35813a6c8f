"""The allocation-free mute (lsrtm_mute_noalloc) against lsrtm_mute, through
the C ABI, on two calls in a row, the second on a smaller acquisition (fewer
shots and receivers: the shared scratch array keeps the first call's longer
tables, which the second must not read)."""
import numpy as np
import pytest

from paper_2508_10405_amd import synth
from gpu_common import require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _muted(torch, w, noalloc, v_mute=1800.0, t0=0.012, ntaper=7):
    from paper_2508_10405_amd import lsrtm
    ctx = lsrtm.context_for(w)
    rng = np.random.default_rng(3)
    d = to_dev(torch, rng.standard_normal(ctx.data_len))
    if noalloc:
        ctx.mute_noalloc(d, v_mute, t0, ntaper)
    else:
        ctx.mute(d, v_mute, t0, ntaper)
    out = d.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_mute_noalloc_matches_mute(torch, ndim):
    if ndim == 2:
        big = synth.small((40, 64), nt=90, npml=5, seed=101, nshot=4, uneven=True)
        small = synth.small((30, 40), nt=70, npml=4, seed=102, nshot=2, uneven=True)
    else:
        big = synth.small((14, 17, 11), nt=50, npml=3, seed=103, nshot=3, uneven=True, h=12.5)
        small = synth.small((12, 13, 9), nt=40, npml=3, seed=104, nshot=1, h=12.5)
    print(f"[case] mute_noalloc {ndim}D: {sum(len(r) for r in big.rec)} then "
          f"{sum(len(r) for r in small.rec)} receivers", flush=True)
    for w in (big, small):
        a = _muted(torch, w, noalloc=True)
        b = _muted(torch, w, noalloc=False)
        assert np.any(a == 0.0) and np.any((a != 0.0))
        assert np.array_equal(a, b)


def test_mute_noalloc_rejects_too_many_receivers(torch):
    from paper_2508_10405_amd import lsrtm
    n = (8, 600)
    rx = np.arange(600)
    rec = np.stack([np.full(600, 1), rx], axis=1)
    nshot = 450                                   # 270000 receivers > 2^18
    ctx = lsrtm.Context(n, (10.0, 10.0), 4, 1e-3, npml=2)
    lnvp = torch.full((600, 8), np.log(2000.0), device="cuda")
    lnip = torch.full((600, 8), np.log(2000.0 * 2000.0), device="cuda")
    ctx.set_model(lnvp, lnip)
    ctx.set_acquisition([((0, 8), (0, 600))] * nshot, [(1, 300)] * nshot, [rec] * nshot,
                        torch.zeros((nshot, 4), device="cuda"))
    d = torch.zeros(ctx.data_len, device="cuda")
    with pytest.raises(lsrtm.LsrtmError) as ei:
        ctx.mute_noalloc(d, 1500.0)
    assert ei.value.status == lsrtm.EINVAL
    ctx.mute(d, 1500.0)                           # the allocating entry point has no such limit
    ctx.close()
