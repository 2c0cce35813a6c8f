"""Failure detection and recovery on the GPU, forced from the host.

* A non-finite wavelet sample makes the background non-finite; the max-abs
  reduction of the next stored snapshot flags it and the pass returns
  LSRTM_ENONFINITE (forward, Born, migration, and the per-group checkpoint
  layout, whose migration re-runs the background); a finite wavelet set
  afterwards gives the results of a fresh context bit for bit.
* A CG run saved to a file after two iterations and resumed in a new
  context continues with the same iterates, bit for bit (plain and
  preconditioned).
* Tensors of the wrong size, device or dtype are refused by the binding
  before any launch.
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


def test_binding_refuses_wrong_sizes(torch):
    """Every binding method that hands a caller's tensor to the library checks
    its device, dtype, contiguity and size first (the library trusts the sizes
    it is given), so a wrong tensor raises before any launch and leaves the
    context usable: a Born call afterwards equals one on a fresh context."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((30, 40), nt=60, npml=5, seed=93, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    shape, nd = ctx.shape, ctx.data_len
    dm = to_dev(torch, w.dm)
    good_d = torch.zeros(nd, device="cuda")
    short_d = torch.zeros(nd - 1, device="cuda")
    bad_img = torch.zeros((1,) + shape, device="cuda")
    x = ctx.cgnr_begin(good_d.clone() + 1.0)
    st = ctx.cgnr_get_state()
    refused = {
        "born dm": lambda: ctx.born(bad_img),
        "born d": lambda: ctx.born(dm, short_d),
        "adjoint d": lambda: ctx.adjoint(short_d),
        "adjoint img": lambda: ctx.adjoint(good_d, bad_img),
        "cgnr d_obs": lambda: ctx.cgnr(short_d, 1),
        "cgnr niter": lambda: ctx.cgnr(good_d, -1),
        "cgnr x": lambda: ctx.cgnr(good_d, 1, bad_img),
        "cgnr_begin d_obs": lambda: ctx.cgnr_begin(short_d),
        "cgnr_begin x": lambda: ctx.cgnr_begin(good_d, bad_img),
        "cgnr_iterate x": lambda: ctx.cgnr_iterate(x[:1]),
        "cgnr_set_state r": lambda: ctx.cgnr_set_state({**st, "r": st["r"][:-1]}),
        "cgnr_set_state z": lambda: ctx.cgnr_set_state({**st, "z": st["z"][:1]}),
        "cgnr_set_state p": lambda: ctx.cgnr_set_state({**st, "p": st["p"][:1]}),
        "cgnr_set_state scalars": lambda: ctx.cgnr_set_state({**st, "scalars": st["scalars"][:3]}),
        "set_preconditioner": lambda: ctx.set_preconditioner(bad_img),
        "psf_apply psf": lambda: ctx.psf_apply(torch.zeros((2, 1) + shape, device="cuda"), 8, dm),
        "psf_apply x": lambda: ctx.psf_apply(torch.zeros((2, 2) + shape, device="cuda"), 8, bad_img),
        "psf_cgnr psf": lambda: ctx.psf_cgnr(torch.zeros((1, 2) + shape, device="cuda"), 8, dm, 1),
        "psf_cgnr niter": lambda: ctx.psf_cgnr(torch.zeros((2, 2) + shape, device="cuda"), 8, dm, -1),
        "mute": lambda: ctx.mute(short_d, 1500.0),
        "mute_noalloc": lambda: ctx.mute_noalloc(short_d, 1500.0),
        "dot": lambda: ctx.dot(good_d, short_d),
        "axpy": lambda: ctx.axpy(1.0, good_d, short_d),
    }
    for name, call in refused.items():
        print("[case]", name, flush=True)
        with pytest.raises(ValueError):
            call()
    with pytest.raises(TypeError):
        ctx.adjoint(good_d.cpu())
    with pytest.raises(TypeError):
        ctx.adjoint(good_d.double())
    torch.cuda.synchronize()
    d = ctx.born(dm).cpu().numpy()
    ctx.close()
    fresh = lsrtm.context_for(w, tile=1)
    assert np.array_equal(d, fresh.born(dm).cpu().numpy())
    fresh.close()
