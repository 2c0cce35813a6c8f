"""Failure detection and recovery on the GPU, forced from the host.

* A non-finite wavelet sample makes the background non-finite; the max-abs
  reduction of the next stored snapshot flags it and the pass returns
  LSRTM_ENONFINITE (forward, Born, migration, and the per-group checkpoint
  layout, whose migration re-runs the background); a finite wavelet set
  afterwards gives the results of a fresh context bit for bit.
* A CG run saved to a file after two iterations and resumed in a new
  context continues with the same iterates, bit for bit (plain and
  preconditioned).
"""
import os

import numpy as np
import pytest

from paper_2508_10405_amd import synth
from gpu_common import require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _with_wavelet(w, wav):
    return synth.Workload(w.name, w.h, w.dt, w.nt, w.npml, w.f0, w.lnvp, w.lnip, w.dm, w.win, w.src, w.rec,
                          np.ascontiguousarray(wav, dtype=np.float32), pml_R=w.pml_R, pml_f0=w.pml_f0)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("ckpt_per_group", [False, True])
def test_nonfinite_wavelet_flagged_by_snapshots(torch, bad, ckpt_per_group):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((30, 44), nt=60, npml=4, seed=91, nshot=3, uneven=True)
    print(f"[case] wavelet sample {bad}, per-group checkpoints {ckpt_per_group}", flush=True)
    wav = w.wavelet.copy()
    wav[1, 3] = bad
    wb = _with_wavelet(w, wav)
    opts = dict(ckpt_every=10, shots_per_launch=2, ckpt_per_group=ckpt_per_group)
    dm = to_dev(torch, w.dm)
    y = to_dev(torch, np.random.default_rng(0).standard_normal(sum(w.nt * len(r) for r in w.rec)))
    calls = [lambda c: c.adjoint(y)] if ckpt_per_group else \
        [lambda c: c.forward(), lambda c: c.born(dm), lambda c: c.adjoint(y)]
    for call in calls:
        ctx = lsrtm.context_for(wb, **opts)
        with pytest.raises(lsrtm.LsrtmError) as ei:
            call(ctx)
            torch.cuda.synchronize()
        assert ei.value.status == lsrtm.ENONFINITE
        # recovery: a finite wavelet on the same context
        ctx.set_acquisition(w.win, w.src, w.rec, to_dev(torch, w.wavelet))
        ref = lsrtm.context_for(w, **opts)
        assert torch.equal(ctx.born(dm), ref.born(dm))
        assert torch.equal(ctx.adjoint(y), ref.adjoint(y))
        ctx.close()
        ref.close()


@pytest.mark.parametrize("precond", [False, True])
def test_cg_state_file_resume(torch, tmp_path, precond):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((36, 50), nt=90, npml=5, seed=92, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    if precond:
        _, minv = ctx.pseudo_hessian()
        ctx.set_preconditioner(minv)
    dobs = ctx.born(to_dev(torch, w.dm)).clone()
    x = ctx.cgnr_begin(dobs)
    m = [ctx.cgnr_iterate(x) for _ in range(4)]
    x_ref = x.cpu().numpy()
    x = ctx.cgnr_begin(dobs)
    ctx.cgnr_iterate(x)
    ctx.cgnr_iterate(x)
    path = os.path.join(str(tmp_path), "cg.npz")
    ctx.cgnr_save(path, x)
    ctx.close()
    # a new context (a restarted job) resumes from the file
    ctx = lsrtm.context_for(w, tile=1)
    x = ctx.cgnr_load(path)
    m34 = [ctx.cgnr_iterate(x) for _ in range(2)]
    assert np.array_equal(x.cpu().numpy(), x_ref)
    assert m34 == m[2:]
    with pytest.raises(ValueError):
        lsrtm.context_for(synth.small((30, 50), nt=90, npml=5, seed=92, nshot=2, uneven=True)).cgnr_load(path)
    ctx.close()
