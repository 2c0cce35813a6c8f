"""3D propagator (GPU, FP32) against the FP64 oracle and its properties."""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth
from gpu_common import BF16_BOUND, concat, f64, oracle_problem, rel, require_gpu, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


CASES3 = [
    # n (nz, nx, ny), nt, npml, nshot, uneven
    ((14, 17, 11), 70, 4, 2, True),
    ((70, 9, 38), 60, 5, 1, False),
    ((17, 19, 21), 60, 0, 1, False),   # no absorbing strips
]


@pytest.mark.parametrize("n,nt,npml,nshot,uneven", CASES3)
def test_3d_vs_oracle(torch, n, nt, npml, nshot, uneven):
    from paper_2508_10405_amd import lsrtm
    w = synth.small(n, nt=nt, npml=npml, seed=sum(n) + 3, nshot=nshot, uneven=uneven, h=12.5)
    print(f"[case] 3D {n} nt={nt} npml={npml} nshot={nshot}", flush=True)
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    ctx = lsrtm.context_for(w)
    d0 = ctx.forward().cpu().numpy()
    e = rel(d0, concat(O.forward(prob, lnvp, lnip)))
    print("3d forward rel", e)
    assert e <= TOL
    dd = ctx.born(to_dev(torch, w.dm)).cpu().numpy()
    e = rel(dd, concat(O.born(prob, lnvp, lnip, f64(w.dm))))
    print("3d born rel", e)
    assert e <= TOL
    rng = np.random.default_rng(1)
    ys = [rng.standard_normal((nt, len(r))) for r in w.rec]
    img = ctx.adjoint(to_dev(torch, concat(ys))).cpu().numpy()
    refi = O.adjoint(prob, lnvp, lnip, ys)
    for k in range(2):
        e = rel(img[k], refi[k])
        print("3d adjoint rel", k, e)
        assert e <= TOL


def test_3d_invariances(torch):
    """Tiles (also per phase), batching, replay interval and per-group
    checkpoints do not change a single bit of the 3D results."""
    from paper_2508_10405_amd import lsrtm
    w = synth.small((20, 18, 70), nt=50, npml=4, seed=5, nshot=3, uneven=True, h=12.5)
    dm = to_dev(torch, w.dm)
    y = to_dev(torch, np.random.default_rng(2).standard_normal(sum(w.nt * len(r) for r in w.rec)))
    ref = None
    for opts in ({"tile": 0}, {"tile": 1, "shots_per_launch": 1}, {"tile": 2, "ckpt_every": 7},
                 {"tile": 3, "ckpt_every": 50}, {"tile": 4, "ckpt_per_group": True, "shots_per_launch": 2},
                 {"tile": 5, "graph": False}, {"tile": 0, "tile_v": 1, "tile_adj_a": 2},
                 {"tile": 3, "tile_v": 5, "tile_adj_a": 0, "ckpt_per_group": True},
                 {"tile": 6}, {"tile": 7, "shots_per_launch": 1, "ckpt_every": 7},
                 {"tile": 8, "tile_v": 6, "tile_adj_a": 7, "graph": False}):
        ctx = lsrtm.context_for(w, **opts)
        out = (ctx.born(dm).cpu().numpy(), ctx.adjoint(y).cpu().numpy())
        ctx.close()
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]), opts
            assert np.array_equal(out[1], ref[1]), opts


def test_3d_tall_tiles(torch):
    """The tall tiles in blocks of 1024 threads (256 x 4, 256 x 8 and 128 x 8
    columns) and the tiles in blocks of 512 (64 x 8, 128 x 4) give the 64 x 4
    tile's results bit for bit, on a grid whose padded z extent (162 nodes)
    is spanned by one 256-row tile (no z-halo) and needs two 128-row tiles
    (a z-halo between them); and on a grid 270 nodes deep (282 padded), where
    the 256-row tiles too stage a z-halo between two tiles of a column."""
    from paper_2508_10405_amd import lsrtm
    for n, npml, nt in (((150, 21, 40), 6, 40), ((270, 9, 14), 6, 30)):
        print(f"[case] tall tiles on {n}, npml {npml}, nt {nt}", flush=True)
        w = synth.small(n, nt=nt, npml=npml, seed=5, nshot=2, uneven=True, h=12.5)
        dm = to_dev(torch, w.dm)
        y = to_dev(torch, np.random.default_rng(2).standard_normal(sum(w.nt * len(r) for r in w.rec)))
        ref = None
        for opts in ({"tile": 0}, {"tile": 6}, {"tile": 7}, {"tile": 8},
                     {"tile": 0, "tile_v": 7, "tile_adj_a": 6}, {"tile": 8, "tile_v": 6, "tile_adj_a": 7},
                     {"tile": 9}, {"tile": 10, "tile_v": 9, "tile_adj_a": 10}):
            ctx = lsrtm.context_for(w, **opts)
            out = (ctx.forward().cpu().numpy(), ctx.born(dm).cpu().numpy(), ctx.adjoint(y).cpu().numpy())
            ctx.close()
            if ref is None:
                ref = out
            else:
                for a, b in zip(out, ref):
                    assert np.array_equal(a, b), (n, opts)


def test_3d_dot_product(torch):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((24, 30, 26), nt=80, npml=6, seed=8, nshot=2, uneven=True, h=12.5)
    ctx = lsrtm.context_for(w)
    rng = np.random.default_rng(3)
    x = to_dev(torch, rng.standard_normal((2,) + w.shape))
    y = to_dev(torch, rng.standard_normal(ctx.data_len))
    a = ctx.dot(ctx.born(x), y)
    b = ctx.dot(x.view(-1), ctx.adjoint(y).view(-1))
    print("3d dot", a, b)
    assert abs(a - b) <= TOL * abs(a)


def test_config5_launch_configuration_window(torch):
    """The 3D workload's launch configuration (one shot per launch, 64 x 4 x 32
    tiles with the velocity phases on 64 x 8 x 32, BF16 checkpoints) on a
    window of the config-5 model (salt flank, 110 x 36 x 34 physical nodes,
    150 x 76 x 74 padded: 3 tiles along z and y, 19 along x, every axis
    ragged) against the FP64 oracle: Born data and the migration with FP32
    checkpoints within 1e-4, the migration with the BF16 checkpoints within
    the stated BF16 bound."""
    import oracle_jobs as J
    from paper_2508_10405_amd import lsrtm
    nt = 150
    full = synth.config5(nt=nt)
    y0, x0, nz, nx, ny = 183, 180, 110, 36, 34
    sl = (slice(y0, y0 + ny), slice(x0, x0 + nx), slice(0, nz))
    rx, ry = np.meshgrid(np.arange(0, nx, 5), np.arange(0, ny, 5), indexing="xy")
    rec = np.stack([np.full(rx.size, 2), rx.ravel(), ry.ravel()], axis=1)
    w = synth.Workload("config5 window", full.h, full.dt, nt, full.npml, full.f0,
                       np.ascontiguousarray(full.lnvp[sl]), np.ascontiguousarray(full.lnip[sl]),
                       np.ascontiguousarray(full.dm[(slice(None),) + sl]),
                       [((0, nz), (0, nx), (0, ny))], [(2, 18, 17)], [rec],
                       np.ascontiguousarray(full.wavelet[:1, :nt]), pml_R=full.pml_R, pml_f0=full.pml_f0)
    del full
    print(f"[case] config5 window {w.n} nt={nt}, launch configuration of the 3D benchmark", flush=True)
    rng = np.random.default_rng(12)
    ys = [rng.standard_normal((nt, len(rec)))]
    running = J.Running([J.born_job(w, [0], nt, w.dm), J.adjoint_job(w, [0], nt, ys, ckpt_every=30)])
    cfg = dict(shots_per_launch=1, tile=0, tile_v=1)
    assert lsrtm.tile_shape(3, 0) == (64, 4) and lsrtm.tile_shape(3, 1) == (64, 8)
    out = {}
    for dtype in ("f32", "bf16"):
        ctx = lsrtm.context_for(w, ckpt_dtype=dtype, **cfg)
        print("plan", dtype, ctx.sizes(), flush=True)
        out[dtype] = (ctx.born(to_dev(torch, w.dm)).cpu().numpy(),
                      ctx.adjoint(to_dev(torch, concat(ys))).cpu().numpy())
        ctx.close()
    # the tall 256 x 4 tiles (blocks of 1024 threads, no z-halo) give the
    # same results bit for bit
    ctx = lsrtm.context_for(w, ckpt_dtype="f32", shots_per_launch=1, tile=6, tile_v=7)
    tall = (ctx.born(to_dev(torch, w.dm)).cpu().numpy(), ctx.adjoint(to_dev(torch, concat(ys))).cpu().numpy())
    ctx.close()
    assert np.array_equal(tall[0], out["f32"][0]) and np.array_equal(tall[1], out["f32"][1])
    ref_d, ref_i = running.results()
    assert np.array_equal(out["f32"][0], out["bf16"][0])
    e = rel(out["f32"][0], concat(ref_d))
    print("config5 window born rel", e, flush=True)
    assert e <= TOL
    for dtype, bound in (("f32", TOL), ("bf16", BF16_BOUND)):
        for k in range(2):
            e = rel(out[dtype][1][k], ref_i[k])
            print(f"config5 window image {k} ({dtype} checkpoints) rel {e:.2e}", flush=True)
            assert e <= bound
