"""Pseudo-Hessian preconditioner (appendix B) and preconditioned CGNR
(section 3) on the GPU, through the C ABI, against the FP64 oracle.

Bar: the pseudo-Hessian is a time sum of squares accumulated in FP32 over
nt steps, so its relative L2 error against the oracle is held to 1e-4 like
the seismograms; PCGNR iterates and misfits are held to 1e-4 relative, both
for the oracle-only chain (oracle pseudo-Hessian -> oracle PCGNR) and with
the GPU's preconditioner vector on both sides, and every iteration from the
GPU's state is checked against one oracle iteration.
"""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth
from gpu_common import cg_step_parity, concat, f64, oracle_problem, rel, require_gpu, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


CASES = [
    # n, nt, npml, nshot, uneven
    ((37, 45), 160, 4, 1, False),
    ((70, 83), 200, 20, 3, True),
    ((33, 40), 120, 0, 2, True),
    ((14, 17, 11), 70, 4, 2, True),
]


@pytest.mark.parametrize("n,nt,npml,nshot,uneven", CASES)
def test_pseudo_hessian_vs_oracle(torch, n, nt, npml, nshot, uneven):
    from paper_2508_10405_amd import lsrtm
    w = synth.small(n, nt=nt, npml=npml, seed=sum(n) + 40, nshot=nshot, uneven=uneven)
    print(f"[case] pseudo-Hessian {n} nt={nt} npml={npml} nshot={nshot}", flush=True)
    prob = oracle_problem(w)
    ref = O.pseudo_hessian(prob, f64(w.lnvp), f64(w.lnip))
    ctx = lsrtm.context_for(w)
    h, minv = ctx.pseudo_hessian(eps_rel=1e-3)
    e = rel(h.cpu().numpy(), ref)
    print("pseudo-Hessian rel", e, flush=True)
    assert e <= TOL
    mref = O.preconditioner(ref, 1e-3)
    e = rel(minv.cpu().numpy(), mref)
    print("preconditioner rel", e, flush=True)
    assert e <= TOL
    ctx.close()


def test_pseudo_hessian_invariant_to_launch_layout(torch):
    """Batched or per-shot launches, any tile, either 2D schedule: the same
    bits (pointwise accumulation, fixed shot-order reduction)."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((61, 77), nt=90, npml=10, seed=44, nshot=3, uneven=True)
    ref = None
    for spl, tile, fused in ((0, 1, False), (1, 0, False), (2, 4, True), (0, 8, True)):
        ctx = lsrtm.context_for(w, shots_per_launch=spl, tile=tile, fused=fused)
        h, _ = ctx.pseudo_hessian(preconditioner=False)
        h = h.cpu().numpy()
        ctx.close()
        if ref is None:
            ref = h
        assert np.array_equal(h, ref), (spl, tile, fused)


def test_pseudo_hessian_3d_invariant_to_tiles(torch):
    """3D: the accumulation inside the velocity and pressure kernels gives
    the same bits on every kind of tile (64-row tiles in blocks of 256 and
    512 threads, tall tiles spanning the whole z extent in blocks of 1024)."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((20, 18, 30), nt=40, npml=4, seed=46, nshot=2, uneven=True, h=12.5)
    ref = None
    for spl, tile in ((0, 0), (1, 6), (0, 7), (2, 9), (0, 10)):
        ctx = lsrtm.context_for(w, shots_per_launch=spl, tile=tile)
        h, _ = ctx.pseudo_hessian(preconditioner=False)
        h = h.cpu().numpy()
        ctx.close()
        if ref is None:
            ref = h
        assert np.array_equal(h, ref), (spl, tile)


def test_pseudo_hessian_leaves_checkpoints_valid(torch):
    """The pseudo-Hessian pass runs through the field buffers; Born data and
    images computed afterwards are unchanged."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((40, 52), nt=100, npml=6, seed=45, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    dm = to_dev(torch, w.dm)
    d0 = ctx.born(dm).clone()
    i0 = ctx.adjoint(d0).clone()
    ctx.pseudo_hessian()
    assert torch.equal(ctx.born(dm), d0)
    assert torch.equal(ctx.adjoint(d0), i0)
    ctx.close()


def test_pcgnr_vs_oracle(torch):
    """Three preconditioned CGNR iterations.

    * Oracle only: the oracle's pseudo-Hessian, its preconditioner and its
      PCGNR against the GPU's pseudo-Hessian, preconditioner and PCGNR
      (iterate and misfit within 1e-4).
    * The same GPU run against the oracle's PCGNR with the GPU's
      preconditioner vector (isolates the solver from the preconditioner).
    * Every iteration from the GPU's own state against one FP64 oracle
      iteration with the GPU's preconditioner (1e-4 on x, r, z and p)."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((36, 52), nt=110, npml=6, seed=14, nshot=2, uneven=True)
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    L = lambda m: O.born(prob, lnvp, lnip, m)
    Lt = lambda d: O.adjoint(prob, lnvp, lnip, d)
    dobs = L(f64(w.dm))
    minv_ref = O.preconditioner(O.pseudo_hessian(prob, lnvp, lnip), 1e-3)
    x_ref, hist_ref = O.pcgnr(L, Lt, dobs, 3, minv_ref)
    ctx = lsrtm.context_for(w)
    _, minv = ctx.pseudo_hessian(eps_rel=1e-3)
    ctx.set_preconditioner(minv)
    x, hist = ctx.cgnr(to_dev(torch, concat(dobs)), 3)
    e = rel(x.cpu().numpy(), x_ref)
    print("pcgnr x rel (oracle-only chain)", e, hist, hist_ref, flush=True)
    assert e <= TOL
    assert np.allclose(hist, hist_ref, rtol=TOL, atol=0)
    assert all(hist[i + 1] <= hist[i] for i in range(3))
    mg = minv.cpu().numpy().astype(np.float64)
    x_mix, hist_mix = O.pcgnr(L, Lt, dobs, 3, mg)
    e = rel(x.cpu().numpy(), x_mix)
    print("pcgnr x rel (GPU preconditioner on both sides)", e, flush=True)
    assert e <= TOL
    assert np.allclose(hist, hist_mix, rtol=TOL, atol=0)
    cg_step_parity(torch, ctx, L, Lt, to_dev(torch, concat(dobs)), 3, minv=mg)
    ctx.close()


def test_pcgnr_identity_preconditioner_is_cgnr(torch):
    """minv = 1 gives the unpreconditioned iterates bit for bit; removing the
    preconditioner restores plain CGNR."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((36, 50), nt=90, npml=5, seed=17, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    dobs = ctx.born(to_dev(torch, w.dm)).clone()
    x0, h0 = ctx.cgnr(dobs, 3)
    x0 = x0.clone()
    ctx.set_preconditioner(torch.ones((2,) + ctx.shape, device="cuda"))
    x1, h1 = ctx.cgnr(dobs, 3)
    assert torch.equal(x0, x1) and h0 == h1
    ctx.set_preconditioner(None)
    x2, h2 = ctx.cgnr(dobs, 3)
    assert torch.equal(x0, x2) and h0 == h2
    ctx.close()


def test_pcgnr_resume_from_saved_state(torch):
    """A preconditioned run stopped after two iterations and resumed from its
    saved state reproduces the uninterrupted iterates."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((36, 50), nt=90, npml=5, seed=18, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    _, minv = ctx.pseudo_hessian()
    ctx.set_preconditioner(minv)
    dobs = ctx.born(to_dev(torch, w.dm)).clone()
    x = ctx.cgnr_begin(dobs)
    m = [ctx.cgnr_iterate(x) for _ in range(3)]
    x_ref = x.cpu().numpy()
    x = ctx.cgnr_begin(dobs)
    ctx.cgnr_iterate(x)
    ctx.cgnr_iterate(x)
    saved = {k: (v.clone() if hasattr(v, "clone") else list(v)) for k, v in ctx.cgnr_get_state().items()}
    x_saved = x.clone()
    ctx.cgnr_iterate(x)
    ctx.cgnr_set_state(saved)
    x = x_saved
    m3 = ctx.cgnr_iterate(x)
    assert np.array_equal(x.cpu().numpy(), x_ref)
    assert m3 == m[2]
    ctx.close()


def test_pseudo_hessian_errors(torch):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((20, 24), nt=40, npml=4, seed=46, nshot=1)
    ctx = lsrtm.context_for(w)
    with pytest.raises(lsrtm.LsrtmError):
        ctx.pseudo_hessian(eps_rel=-1.0)
    with pytest.raises(lsrtm.LsrtmError):
        ctx.pseudo_hessian(eps_rel=0.0)          # no stabilisation: undefined preconditioner
    h, m = ctx.pseudo_hessian(eps_rel=0.0, preconditioner=False)
    assert m is None and float(h.max()) > 0
    ctx.close()
