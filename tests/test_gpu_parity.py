"""GPU (FP32, HIP) against the FP64 oracle, through the C ABI.

Bar: relative L2 error <= 1e-4 on seismograms and images, the tolerance the
benchmark target states for FP32 propagation against the FP64 oracle.  Sizes
are chosen so that grids span several tiles with ragged tails, shots use
uneven windows, and the oracle finishes in seconds.
"""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth
from gpu_common import BF16_BOUND, FP16_BOUND, cg_step_parity, concat, f64, oracle_problem, rel, require_gpu, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _ctx(torch, w, **opts):
    from paper_2508_10405_amd import lsrtm
    print(f"[case] {w.name} nshot={w.nshot} nt={w.nt} npml={w.npml} opts={opts}", flush=True)
    return lsrtm.context_for(w, **opts)


CASES = [
    # n (nz, nx), nt, npml, nshot, uneven
    ((37, 45), 160, 4, 1, False),
    ((70, 83), 220, 20, 3, True),
    ((129, 17), 150, 6, 2, True),
    # no absorbing strips (zero outside the grid), and strips one node wide
    ((33, 40), 120, 0, 2, True),
    ((20, 26), 100, 1, 1, False),
]


@pytest.mark.parametrize("n,nt,npml,nshot,uneven", CASES)
def test_forward_born_adjoint_vs_oracle(torch, n, nt, npml, nshot, uneven):
    w = synth.small(n, nt=nt, npml=npml, seed=sum(n), nshot=nshot, uneven=uneven)
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    ctx = _ctx(torch, w)
    # background data
    d0 = ctx.forward().cpu().numpy()
    ref0 = concat(O.forward(prob, lnvp, lnip))
    e = rel(d0, ref0)
    print("forward rel", e)
    assert e <= TOL
    # Born data
    dm = to_dev(torch, w.dm)
    dd = ctx.born(dm).cpu().numpy()
    refd = O.born(prob, lnvp, lnip, f64(w.dm))
    e = rel(dd, concat(refd))
    print("born rel", e)
    assert e <= TOL
    # adjoint image of seeded data
    rng = np.random.default_rng(7)
    ys = [rng.standard_normal((nt, len(r))) for r in w.rec]
    img = ctx.adjoint(to_dev(torch, concat(ys))).cpu().numpy()
    refi = O.adjoint(prob, lnvp, lnip, ys)
    for k in range(2):
        e = rel(img[k], refi[k])
        print("adjoint rel", k, e)
        assert e <= TOL


def test_dot_product_gpu(torch):
    w = synth.small((61, 77), nt=200, npml=10, seed=3, nshot=2, uneven=True)
    ctx = _ctx(torch, w)
    rng = np.random.default_rng(2)
    x = to_dev(torch, rng.standard_normal((2,) + w.shape))
    y = to_dev(torch, rng.standard_normal(ctx.data_len))
    Lx = ctx.born(x)
    Lty = ctx.adjoint(y)
    a = ctx.dot(Lx, y)
    b = ctx.dot(x.view(-1), Lty.view(-1))
    print("dot", a, b, abs(a - b) / abs(a))
    assert abs(a - b) <= TOL * abs(a)


def test_replay_is_bitwise(torch):
    """FP32 checkpoint replay reproduces the stored-everything history bit for
    bit: images for every checkpoint interval are identical."""
    w = synth.small((45, 66), nt=97, npml=8, seed=5, nshot=2, uneven=True)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(sum(w.nt * len(r) for r in w.rec))
    imgs = []
    for k, fused in ((1, True), (7, True), (32, True), (97, True), (7, False), (97, False)):
        from paper_2508_10405_amd import lsrtm
        ctx = lsrtm.context_for(w, ckpt_every=k, fused=fused)
        imgs.append(ctx.adjoint(to_dev(torch, y)).cpu().numpy())
        ctx.close()
    for im in imgs[1:]:
        assert np.array_equal(im, imgs[0])


def test_batched_equals_per_shot_and_tiles(torch):
    """Batching shots into one launch, every tile shape, and the fused
    one-kernel-per-step schedule against the two-phase one, all give bitwise
    the same data and images as plain per-shot launches."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((50, 90), nt=120, npml=6, seed=9, nshot=4, uneven=True)
    dm = to_dev(torch, w.dm)
    rng = np.random.default_rng(4)
    y = to_dev(torch, rng.standard_normal(sum(w.nt * len(r) for r in w.rec)))
    ref = None
    for spl, fused in ((1, True), (0, True), (3, True), (2, False)):
        for tile in range(9):
            ctx = lsrtm.context_for(w, shots_per_launch=spl, tile=tile, fused=fused)
            d = ctx.born(dm).cpu().numpy()
            im = ctx.adjoint(y).cpu().numpy()
            ctx.close()
            if ref is None:
                ref = (d, im)
            else:
                assert np.array_equal(d, ref[0]), (spl, tile, fused)
                assert np.array_equal(im, ref[1]), (spl, tile, fused)


def test_per_phase_tiles_bitwise(torch):
    """The velocity phases and the adjoint A phase may walk tables of their
    own tile shapes (they record and inject nothing): Born data and images are
    bitwise those of one tile shape for every phase."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((50, 90), nt=120, npml=6, seed=9, nshot=4, uneven=True)
    dm = to_dev(torch, w.dm)
    y = to_dev(torch, np.random.default_rng(4).standard_normal(sum(w.nt * len(r) for r in w.rec)))
    ctx = lsrtm.context_for(w, shots_per_launch=2, tile=1)
    ref = (ctx.born(dm).cpu().numpy(), ctx.adjoint(y).cpu().numpy())
    ctx.close()
    for tile, tv, ta in ((1, 4, 2), (0, 8, 6), (1, -1, 2), (3, 1, -1)):
        print(f"[case] tile {tile} tile_v {tv} tile_adj_a {ta}", flush=True)
        ctx = lsrtm.context_for(w, shots_per_launch=2, tile=tile, tile_v=tv, tile_adj_a=ta)
        assert np.array_equal(ctx.born(dm).cpu().numpy(), ref[0])
        assert np.array_equal(ctx.adjoint(y).cpu().numpy(), ref[1])
        ctx.close()
    with pytest.raises(lsrtm.LsrtmError):
        lsrtm.context_for(w, tile_v=9)


def test_run_twice_deterministic(torch):
    w = synth.small((40, 60), nt=90, npml=5, seed=12, nshot=3, uneven=True)
    ctx = _ctx(torch, w)
    dm = to_dev(torch, w.dm)
    a = ctx.born(dm).cpu().numpy()
    b = ctx.born(dm).cpu().numpy()
    assert np.array_equal(a, b)
    y = to_dev(torch, np.random.default_rng(0).standard_normal(ctx.data_len))
    assert np.array_equal(ctx.adjoint(y).cpu().numpy(), ctx.adjoint(y).cpu().numpy())


def test_adjoint_accumulate(torch):
    w = synth.small((30, 40), nt=60, npml=4, seed=2, nshot=1)
    ctx = _ctx(torch, w)
    y = to_dev(torch, np.random.default_rng(0).standard_normal(ctx.data_len))
    a = ctx.adjoint(y)
    b = a.clone()
    ctx.adjoint(y, img=b, accumulate=True)
    np.testing.assert_allclose(b.cpu().numpy(), 2 * a.cpu().numpy(), rtol=1e-6, atol=0)


def test_cgnr_vs_oracle(torch):
    """Three CGNR iterations: iterate and normalised misfit history against
    the FP64 oracle's CGNR on the same operators (1e-4), and every single
    iteration from the GPU's own state against one FP64 oracle iteration
    (1e-4 on x, r, z and p)."""
    w = synth.small((36, 52), nt=110, npml=6, seed=14, nshot=2, uneven=True)
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    L = lambda m: O.born(prob, lnvp, lnip, m)
    Lt = lambda d: O.adjoint(prob, lnvp, lnip, d)
    dobs = L(f64(w.dm))
    x_ref, hist_ref = O.cgnr(L, Lt, dobs, 3)
    ctx = _ctx(torch, w)
    x, hist = ctx.cgnr(to_dev(torch, concat(dobs)), 3)
    e = rel(x.cpu().numpy(), x_ref)
    print("cgnr x rel", e, hist, hist_ref)
    assert e <= TOL
    assert np.allclose(hist, hist_ref, rtol=TOL, atol=0)
    assert all(hist[i + 1] <= hist[i] for i in range(3))
    cg_step_parity(torch, ctx, L, Lt, to_dev(torch, concat(dobs)), 3)


def test_config1_full(torch):
    """Config 1 at full size (100 x 200, nt = 1000, 200 receivers)."""
    w = synth.config1()
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    ctx = _ctx(torch, w)
    dd = ctx.born(to_dev(torch, w.dm)).cpu().numpy()
    refd = O.born(prob, lnvp, lnip, f64(w.dm))
    e = rel(dd, concat(refd))
    print("config1 born rel", e)
    assert e <= TOL
    img = ctx.adjoint(to_dev(torch, concat(refd))).cpu().numpy()
    refi = O.adjoint(prob, lnvp, lnip, refd, ckpt_every=50)
    for k in range(2):
        e = rel(img[k], refi[k])
        print("config1 adjoint rel", k, e)
        assert e <= TOL


@pytest.mark.parametrize("dtype,bound,u", [("f16", FP16_BOUND, 2.0 ** -11), ("bf16", BF16_BOUND, 2.0 ** -8)])
def test_compressed_checkpoints_error(torch, dtype, bound, u):
    """FP16/BF16 snapshots with per-snapshot max-abs scaling.

    Against the oracle with exact history the image error is held to the
    stated bound (4 u).  Against the oracle replaying from snapshots
    compressed the same way (scale, round to nearest even) the two sides
    differ only where the FP32 state and the FP64 state fall on different
    sides of a rounding boundary: with a relative state difference delta a
    value flips with probability about delta / u and then moves by u, so the
    expected error is about sqrt(2 delta u), times the small gain of the
    imaging derivatives.  With delta <= 1e-5 and a gain of at most 4 the
    bound is 4 sqrt(2e-5 u): 4.0e-4 (FP16) and 1.1e-3 (BF16), 5 to 14 times
    tighter than the bound against the exact history, so that a wrong scale
    or rounding mode fails."""
    flip_bound = 4.0 * np.sqrt(2e-5 * u)
    from paper_2508_10405_amd import lsrtm
    w = synth.small((60, 80), nt=300, npml=10, seed=21, nshot=2, uneven=True)
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    rng = np.random.default_rng(5)
    ys = [rng.standard_normal((w.nt, len(r))) for r in w.rec]
    refi = O.adjoint(prob, lnvp, lnip, ys)
    for k in (10, 50):
        refc = O.adjoint(prob, lnvp, lnip, ys, ckpt_every=k, ckpt_dtype=dtype)
        ctx = lsrtm.context_for(w, ckpt_every=k, ckpt_dtype=dtype)
        img = ctx.adjoint(to_dev(torch, concat(ys))).cpu().numpy()
        ctx.close()
        e = max(rel(img[i], refi[i]) for i in range(2))
        ec = max(rel(img[i], refc[i]) for i in range(2))
        eo = max(rel(refc[i], refi[i]) for i in range(2))
        print(f"[compressed] {dtype} k={k} image rel err {e:.3e} (oracle with the same snapshots: {eo:.3e}); "
              f"against that oracle {ec:.3e}", flush=True)
        assert e <= bound
        assert ec <= flip_bound


def test_error_paths(torch):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((20, 30), nt=20, npml=4, seed=1)
    # CFL violation
    ctx = lsrtm.Context(w.n, w.h, w.nt, 0.05, npml=4)
    with pytest.raises(lsrtm.LsrtmError) as ei:
        ctx.set_model(to_dev(torch, w.lnvp), to_dev(torch, w.lnip))
    assert ei.value.status == lsrtm.EUNSTABLE
    # NaN model
    ctx = lsrtm.Context(w.n, w.h, w.nt, w.dt, npml=4)
    bad = w.lnvp.copy()
    bad[3, 4] = np.nan
    with pytest.raises(lsrtm.LsrtmError) as ei:
        ctx.set_model(to_dev(torch, bad), to_dev(torch, w.lnip))
    assert ei.value.status == lsrtm.ENONFINITE
    # call order
    ctx = lsrtm.Context(w.n, w.h, w.nt, w.dt, npml=4)
    with pytest.raises(lsrtm.LsrtmError) as ei:
        ctx.born(to_dev(torch, w.dm))
    assert ei.value.status == lsrtm.ESTATE
    ctx.set_model(to_dev(torch, w.lnvp), to_dev(torch, w.lnip))
    # receiver outside its window
    with pytest.raises(lsrtm.LsrtmError) as ei:
        ctx.set_acquisition([((0, 20), (0, 10))], [(1, 2)], [np.array([[1, 15]])],
                            to_dev(torch, w.wavelet[:1]))
    assert ei.value.status == lsrtm.EINVAL


def test_graph_replay_matches_direct_launches(torch):
    """Passes replayed from captured HIP graphs give bitwise the results of
    direct launches, on every replay, with eager work in between."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((44, 70), nt=80, npml=6, seed=15, nshot=3, uneven=True)
    dm = to_dev(torch, w.dm)
    y = to_dev(torch, np.random.default_rng(8).standard_normal(sum(w.nt * len(r) for r in w.rec)))
    ref = lsrtm.context_for(w, graph=False, tile=1)
    d_ref = ref.born(dm).cpu().numpy()
    i_ref = ref.adjoint(y).cpu().numpy()
    ctx = lsrtm.context_for(w, graph=True, tile=1)
    d = torch.empty(ctx.data_len, device="cuda")
    img = torch.empty((2,) + w.shape, device="cuda")
    for rep in range(3):
        ctx.born(dm, d)
        assert np.array_equal(d.cpu().numpy(), d_ref), rep
        torch.cuda.synchronize()
        _ = (dm * 2).sum().item()          # eager work between replays
        ctx.adjoint(y, img)
        assert np.array_equal(img.cpu().numpy(), i_ref), rep


def test_graph_cache_bounded(torch):
    """A caller handing in fresh data buffers on every call (a training loop
    through the autograd operator): the cache keeps at most the set number of
    pass graphs, replacing the least recently used, and every call gives the
    direct launches' results bit for bit."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((40, 60), nt=50, npml=5, seed=19, nshot=3, uneven=True)
    dm = to_dev(torch, w.dm)
    ref = lsrtm.context_for(w, graph=False, tile=1, shots_per_launch=2)
    d_ref = ref.born(dm).cpu().numpy()
    y = to_dev(torch, np.random.default_rng(9).standard_normal(ref.data_len))
    i_ref = ref.adjoint(y).cpu().numpy()
    ctx = lsrtm.context_for(w, graph=True, tile=1, shots_per_launch=2)
    assert ctx.sizes()["groups"] == 2
    ctx.set_option(lsrtm.OPT_GRAPH_CACHE, 3)
    for rep in range(6):
        d = torch.empty(ctx.data_len, device="cuda")        # a new pointer every call
        ctx.born(dm, d)
        img = ctx.adjoint(d if rep % 2 else y)
        assert np.array_equal(d.cpu().numpy(), d_ref), rep
        if rep % 2 == 0:
            assert np.array_equal(img.cpu().numpy(), i_ref), rep
        assert ctx.sizes()["graphs"] <= 3
    ctx.set_option(lsrtm.OPT_GRAPH_CACHE, 0)
    with pytest.raises(lsrtm.LsrtmError):
        ctx.set_option(lsrtm.OPT_GRAPH_CACHE, -1)
    ctx.close()
    ref.close()


def test_autotune_keeps_results_and_caches(torch, tmp_path, monkeypatch):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((40, 64), nt=60, npml=5, seed=16, nshot=5, uneven=True)
    dm = to_dev(torch, w.dm)
    ref = lsrtm.context_for(w, tile=0, shots_per_launch=1).born(dm).cpu().numpy()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LSRTM_TUNE_CACHE", str(cache))
    ctx = lsrtm.context_for(w)
    res = ctx.autotune(nsteps=2, groups=True)
    print("autotune", res, ctx.sizes())
    assert np.array_equal(ctx.born(dm).cpu().numpy(), ref)
    assert cache.exists() and cache.read_text().count("|") == 1
    ctx2 = lsrtm.context_for(w)
    res2 = ctx2.autotune(nsteps=2, groups=True)
    assert res2["tile"] == res["tile"] and ctx2.sizes()["shots_per_launch"] == ctx.sizes()["shots_per_launch"]
    assert (res2["tile_v"], res2["tile_adj_a"]) == (res["tile_v"], res["tile_adj_a"])
    assert cache.read_text().count("|") == 1   # served from the cache
    assert np.array_equal(ctx2.born(dm).cpu().numpy(), ref)
    y = to_dev(torch, np.random.default_rng(5).standard_normal(ctx2.data_len))
    plain = lsrtm.context_for(w, tile=0, shots_per_launch=1)
    assert np.array_equal(ctx2.adjoint(y).cpu().numpy(), plain.adjoint(y).cpu().numpy())


def test_cgnr_resume_from_saved_state(torch):
    """A CGNR run stopped after two iterations and resumed from its saved
    state (x, r, z, p, scalars) reproduces the uninterrupted iterates."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((36, 50), nt=90, npml=5, seed=17, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    dobs = ctx.born(to_dev(torch, w.dm)).clone()
    x = ctx.cgnr_begin(dobs)
    m = [ctx.cgnr_iterate(x) for _ in range(3)]
    x_ref = x.cpu().numpy()
    x = ctx.cgnr_begin(dobs)
    ctx.cgnr_iterate(x)
    ctx.cgnr_iterate(x)
    saved = {k: (v.clone() if hasattr(v, "clone") else list(v)) for k, v in ctx.cgnr_get_state().items()}
    x_saved = x.clone()
    ctx.cgnr_iterate(x)                      # disturb the solver state
    ctx.born(to_dev(torch, 0 * w.dm))
    ctx.cgnr_set_state(saved)
    x = x_saved
    m3 = ctx.cgnr_iterate(x)
    assert np.array_equal(x.cpu().numpy(), x_ref)
    assert m3 == m[2]


def test_cgnr_step_log(torch, tmp_path):
    """The CG log: one JSON line per iteration with the solver's own alpha,
    beta, ||L p||^2 and misfit.  alpha is <z, s> / ||L p||^2 of the state
    before the iteration (recomputed here with the library's Born pass and
    FP64 dot, bit for bit), beta the ratio of the new and old <z, s>, and the
    misfits equal those of the plain solver call."""
    import json
    from paper_2508_10405_amd import lsrtm
    w = synth.small((36, 50), nt=90, npml=5, seed=18, nshot=2, uneven=True)
    ctx = lsrtm.context_for(w, tile=1)
    dobs = ctx.born(to_dev(torch, w.dm)).clone()
    _, m_plain = ctx.cgnr(dobs, 3)
    log = tmp_path / "cg.jsonl"
    x, m_log = ctx.cgnr(dobs, 3, log=str(log))
    assert m_log == m_plain
    lines = [json.loads(s) for s in log.read_text().splitlines()]
    assert [e["iter"] for e in lines] == [1, 2, 3]
    assert [e["misfit"] for e in lines] == m_plain[1:]
    assert all(e["seconds"] > 0 and e["gpts"] > 0 for e in lines)
    # alpha and beta of one more iteration against the exported state
    st = ctx.cgnr_get_state()
    zs = st["scalars"][0]
    wp = ctx.born(st["p"])
    ww = ctx.dot(wp, wp)
    ctx.cgnr_iterate(x)
    step = ctx.cgnr_step()
    assert step["iter"] == 4 and step["ww"] == ww and step["alpha"] == zs / ww
    assert step["beta"] == ctx.cgnr_get_state()["scalars"][0] / zs
    ctx.close()
