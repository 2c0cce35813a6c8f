"""Replay cache (LSRTM_OPT_REPLAY_CACHE_MB): the background replays of the
last checkpoint segments of every launch group are kept across migration
passes, and 2D Born passes read the background of those segments from them
instead of advancing it.  They depend on the background model and the acquisition only
(appendix A: the history the adjoint reads is the background's), so every
result must be bitwise that of a plan without the cache: on the pass that
fills the cache, on the passes that read it, with and without graphs, with
one or several launch groups, with a partial last segment, in CGNR, after
the model changes (the cache is refilled), in 3D and with a single segment.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2508_10405_amd import synth
from gpu_common import require_gpu, to_dev

pytestmark = pytest.mark.gpu
K = 10


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _w(seed=33, nt=95):
    # nt = 95 with checkpoints every 10 steps: 10 segments, the last one of 5 steps
    return synth.small((48, 64), nt=nt, npml=8, seed=seed, nshot=3, uneven=True)


def _mb_for(ctx, m):
    """Cache size (MB) of about m segments of every launch group (the padded
    arrays' rows are rounded up, so the plan may hold fewer)."""
    sz = ctx.sizes()
    per_seg = sz["ckpt_every"] * 3 * sz["padded_points"] * 4
    return math.ceil(m * per_seg / 2 ** 20)


def _ref(torch, w, y, spl=0):
    from paper_2508_10405_amd import lsrtm
    ctx = lsrtm.context_for(w, ckpt_every=K, shots_per_launch=spl)
    d = ctx.born(to_dev(torch, w.dm)).cpu().numpy()
    img = ctx.adjoint(y).cpu().numpy()
    ctx.close()
    return d, img


@pytest.mark.parametrize("spl", [0, 1])
@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("m", [3, "all"])
def test_replay_cache_bitwise(torch, spl, graph, m):
    from paper_2508_10405_amd import lsrtm
    w = _w()
    print(f"[case] replay cache spl={spl} graph={graph} m={m}", flush=True)
    ctx = lsrtm.context_for(w, ckpt_every=K, shots_per_launch=spl, graph=graph)
    y = to_dev(torch, np.random.default_rng(4).standard_normal(ctx.data_len))
    ref_d, ref_i = _ref(torch, w, y, spl)
    nseg = math.ceil(w.nt / K)
    ctx.set_option(lsrtm.OPT_REPLAY_CACHE_MB, 1 << 20 if m == "all" else _mb_for(ctx, m))
    held = ctx.sizes()["replay_cache_segments"]
    if m == "all":
        assert held == nseg
    else:
        assert 1 <= held < nseg, held
    dm = to_dev(torch, w.dm)
    for rep in range(3):   # fill, then read twice
        img = ctx.adjoint(y).cpu().numpy()
        assert np.array_equal(img, ref_i), rep
    assert np.array_equal(ctx.born(dm).cpu().numpy(), ref_d)
    assert np.array_equal(ctx.adjoint(y).cpu().numpy(), ref_i)
    ctx.close()


def test_replay_cache_refilled_after_model_change(torch):
    """A new background model invalidates the cached replays: the next
    migration is that of a fresh plan with the new model."""
    from paper_2508_10405_amd import lsrtm
    w, w2 = _w(seed=33), _w(seed=34)
    ctx = lsrtm.context_for(w, ckpt_every=K, replay_cache_mb=1 << 20)
    assert ctx.sizes()["replay_cache_segments"] == math.ceil(w.nt / K)
    y = to_dev(torch, np.random.default_rng(5).standard_normal(ctx.data_len))
    ctx.adjoint(y)
    ctx.adjoint(y)
    ctx.born(to_dev(torch, w.dm))
    ctx.set_model(to_dev(torch, w2.lnvp), to_dev(torch, w2.lnip))
    d = ctx.born(to_dev(torch, w.dm)).cpu().numpy()
    img = ctx.adjoint(y).cpu().numpy()
    d2 = ctx.born(to_dev(torch, w.dm)).cpu().numpy()
    ctx.close()
    w3 = dataclasses.replace(w, lnvp=w2.lnvp, lnip=w2.lnip)
    ref_d, ref = _ref(torch, w3, y)
    assert np.array_equal(img, ref)
    assert np.array_equal(d, ref_d) and np.array_equal(d2, ref_d)


def test_replay_cache_cgnr_bitwise(torch):
    from paper_2508_10405_amd import lsrtm
    w = _w()
    out = []
    for mb in (0, 1 << 20):
        ctx = lsrtm.context_for(w, ckpt_every=K, replay_cache_mb=mb)
        d_obs = ctx.born(to_dev(torch, w.dm))
        x, mis = ctx.cgnr(d_obs, 3)
        out.append((x.cpu().numpy(), mis))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_replay_cache_off_where_not_planned(torch):
    """No cache for the fused 2D schedule or with per-group checkpoints."""
    from paper_2508_10405_amd import lsrtm
    w = _w()
    for opts in (dict(fused=True), dict(ckpt_per_group=True)):
        ctx = lsrtm.context_for(w, ckpt_every=K, replay_cache_mb=1 << 20, **opts)
        assert ctx.sizes()["replay_cache_segments"] == 0, opts
        ctx.close()
    with pytest.raises(lsrtm.LsrtmError):
        ctx = lsrtm.context_for(w, ckpt_every=K)
        try:
            ctx.set_option(lsrtm.OPT_REPLAY_CACHE_MB, -1)
        finally:
            ctx.close()


@pytest.mark.parametrize("case", ["3d", "one_segment"])
def test_replay_cache_3d_and_single_segment(torch, case):
    """A 3D plan (injection kernels of their own) and a plan whose only
    segment starts from rest (no checkpoint to restore)."""
    from paper_2508_10405_amd import lsrtm
    if case == "3d":
        w, k = synth.small((14, 18, 12), nt=40, npml=3, seed=36, nshot=2, uneven=True), 7
    else:
        w, k = _w(nt=60), 100
    print(f"[case] replay cache {case}", flush=True)
    dm = to_dev(torch, w.dm)
    ref = lsrtm.context_for(w, ckpt_every=k)
    y = to_dev(torch, np.random.default_rng(6).standard_normal(ref.data_len))
    ref_i = ref.adjoint(y).cpu().numpy()
    ref_d = ref.born(dm).cpu().numpy()
    ref.close()
    ctx = lsrtm.context_for(w, ckpt_every=k, replay_cache_mb=1 << 20)
    assert ctx.sizes()["replay_cache_segments"] == math.ceil(w.nt / k)
    for rep in range(3):
        assert np.array_equal(ctx.adjoint(y).cpu().numpy(), ref_i), rep
        assert np.array_equal(ctx.born(dm).cpu().numpy(), ref_d), rep
    ctx.close()


def test_replay_cache_with_planner_interval(torch):
    """Checkpoint interval left to the planner, which may shorten it so that
    a cache of part of the history holds more steps: bitwise the results of
    the planner's plan without the cache."""
    from paper_2508_10405_amd import lsrtm
    w = _w(nt=200)
    dm = to_dev(torch, w.dm)
    ref = lsrtm.context_for(w)
    y = to_dev(torch, np.random.default_rng(7).standard_normal(ref.data_len))
    ref_i = ref.adjoint(y).cpu().numpy()
    ref_d = ref.born(dm).cpu().numpy()
    mb = math.ceil(0.4 * w.nt * 3 * ref.sizes()["padded_points"] * 4 / 2 ** 20)
    ref.close()
    ctx = lsrtm.context_for(w, replay_cache_mb=mb)
    sz = ctx.sizes()
    print(f"[case] planner interval {sz['ckpt_every']}, cached segments {sz['replay_cache_segments']}", flush=True)
    assert 1 <= sz["replay_cache_segments"] < math.ceil(w.nt / sz["ckpt_every"])
    for rep in range(2):
        assert np.array_equal(ctx.adjoint(y).cpu().numpy(), ref_i), rep
        assert np.array_equal(ctx.born(dm).cpu().numpy(), ref_d), rep
    ctx.close()
