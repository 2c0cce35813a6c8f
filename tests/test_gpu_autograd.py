"""The differentiable Born operator: its backward is the library's adjoint
(migration with checkpoint replay).  Checked by central finite differences
of the misfit, by the dot-product test through autograd, and against the
FP64 oracle's gradient."""
import numpy as np
import pytest

from oracle import lsrtm_oracle as O
from paper_2508_10405_amd import synth
from gpu_common import SNAPSHOT_BOUND, concat, f64, oracle_problem, rel, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _setup(torch, k=25, dtype="f32"):
    from paper_2508_10405_amd import lsrtm
    w = synth.small((48, 96), nt=240, npml=10, seed=31, nshot=3, uneven=True)
    print(f"[case] autograd small nshot={w.nshot} nt={w.nt} k={k} {dtype}", flush=True)
    ctx = lsrtm.context_for(w, ckpt_every=k, ckpt_dtype=dtype)
    return w, ctx


def test_gradient_matches_oracle(torch):
    from paper_2508_10405_amd import autograd
    w, ctx = _setup(torch)
    rng = np.random.default_rng(1)
    d_obs = rng.standard_normal(ctx.data_len).astype(np.float32)
    m = to_dev(torch, 0.5 * w.dm).requires_grad_(True)
    J = autograd.misfit(m, ctx, to_dev(torch, d_obs))
    J.backward()
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    Lm = O.born(prob, lnvp, lnip, 0.5 * f64(w.dm))
    res, o = [], 0
    for d in Lm:
        res.append(d - d_obs[o:o + d.size].reshape(d.shape))
        o += d.size
    g_ref = O.adjoint(prob, lnvp, lnip, res)
    e = rel(m.grad.cpu().numpy(), g_ref)
    print("grad rel", e)
    assert e <= 1e-4


def test_gradient_central_differences(torch):
    """J is quadratic in dm, so the central difference along v equals <g, v>
    up to rounding; eps = 1e-3 as in the benchmark recipe."""
    from paper_2508_10405_amd import autograd
    w, ctx = _setup(torch)
    rng = np.random.default_rng(2)
    # observed data on the scale of L dm, so that J is not dominated by a
    # constant that would swamp the FP32 differences
    d_obs = ctx.born(to_dev(torch, 0.6 * w.dm + 0.02 * rng.standard_normal((2,) + w.shape))).clone()
    m = to_dev(torch, w.dm).requires_grad_(True)
    J = autograd.misfit(m, ctx, d_obs)
    J.backward()
    g = m.grad.detach()
    for trial in range(3):
        v = to_dev(torch, rng.standard_normal((2,) + w.shape))
        eps = 1e-3
        with torch.no_grad():
            rp = ctx.born((m + eps * v).detach().contiguous()) - d_obs
            rm = ctx.born((m - eps * v).detach().contiguous()) - d_obs
            fd = (0.5 * ctx.dot(rp, rp) - 0.5 * ctx.dot(rm, rm)) / (2 * eps)
        an = ctx.dot(g.view(-1).contiguous(), v.view(-1))
        print("fd", fd, "analytic", an)
        assert abs(fd - an) <= 1e-3 * abs(an)


def test_dot_product_through_autograd(torch):
    from paper_2508_10405_amd import autograd
    w, ctx = _setup(torch)
    rng = np.random.default_rng(3)
    x = to_dev(torch, rng.standard_normal((2,) + w.shape)).requires_grad_(True)
    y = to_dev(torch, rng.standard_normal(ctx.data_len))
    Lx = autograd.born(x, ctx)
    (Lx * y).sum().backward()
    a = ctx.dot(Lx.detach(), y)
    b = ctx.dot(x.detach().view(-1), x.grad.view(-1).contiguous())
    print("dot", a, b)
    assert abs(a - b) <= 1e-4 * abs(a)


@pytest.mark.parametrize("k", [10, 50, 200])
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_checkpoint_interval_and_dtype(torch, k, dtype):
    """Gradient through the autograd op for every checkpoint interval and
    snapshot precision, against the FP64 oracle: FP32 snapshots meet the
    1e-4 bar; compressed ones report their error under the bounds stated for
    compressed snapshots (4 u: 1.95e-3 FP16, 1.56e-2 BF16)."""
    from paper_2508_10405_amd import autograd
    w, ctx = _setup(torch, k=k, dtype=dtype)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(ctx.data_len).astype(np.float32)
    x = to_dev(torch, np.zeros((2,) + w.shape)).requires_grad_(True)
    (autograd.born(x, ctx) * to_dev(torch, y)).sum().backward()
    prob = oracle_problem(w)
    ys, o = [], 0
    for r in w.rec:
        ys.append(f64(y[o:o + w.nt * len(r)]).reshape(w.nt, len(r)))
        o += w.nt * len(r)
    g_ref = O.adjoint(prob, f64(w.lnvp), f64(w.lnip), ys)
    e = rel(x.grad.cpu().numpy(), g_ref)
    print(f"[ckpt] k={k} {dtype} gradient rel err {e:.3e}")
    bound = SNAPSHOT_BOUND[dtype]
    assert e <= bound


def test_config4_checkpoint_table(torch):
    """Config-4 geometry (480 x 160 at 12.5 m, 15 Hz), one shot, the first 400
    steps: gradient of the misfit through the autograd op for every checkpoint
    interval and snapshot precision against the FP64 oracle (the table the
    design notes quote)."""
    from paper_2508_10405_amd import autograd, lsrtm
    full = synth.config4(nt=400)
    s = 15
    w = synth.Workload(full.name, full.h, full.dt, full.nt, full.npml, full.f0, full.lnvp, full.lnip,
                       full.dm, full.win[s:s + 1], full.src[s:s + 1], full.rec[s:s + 1],
                       full.wavelet[s:s + 1])
    prob = oracle_problem(w)
    lnvp, lnip = f64(w.lnvp), f64(w.lnip)
    d_obs = O.born(prob, lnvp, lnip, f64(w.dm))
    m0 = 0.5 * f64(w.dm)
    Lm = O.born(prob, lnvp, lnip, m0)
    g_ref = O.adjoint(prob, lnvp, lnip, [Lm[0] - d_obs[0]], ckpt_every=50)
    rows = []
    for dtype in ("f32", "f16", "bf16"):
        for k in (10, 50, 200):
            ctx = lsrtm.context_for(w, ckpt_every=k, ckpt_dtype=dtype)
            m = to_dev(torch, m0).requires_grad_(True)
            J = autograd.misfit(m, ctx, to_dev(torch, concat(d_obs)))
            J.backward()
            e = rel(m.grad.cpu().numpy(), g_ref)
            rows.append((dtype, k, e))
            print(f"[config4 table] {dtype} k={k} gradient rel err {e:.3e}", flush=True)
            ctx.close()
            assert e <= SNAPSHOT_BOUND[dtype]


def test_config4_full_size_fd_and_dot(torch):
    """Config 4 at full size (480 x 160 at 12.5 m, 32 shots, nt = 3000) through
    the autograd operator for every checkpoint interval {10, 50, 200} and
    snapshot precision {FP32, FP16, BF16}: central differences of the misfit
    (eps = 1e-3) against <grad, v>, and the dot-product test
    <L x, y> = <x, L^T y> through autograd.  The Born data the differences use
    do not depend on the snapshots; the gradient does, so the agreement is
    held to 1e-3 (the FP32 differences' own rounding) plus the stated
    snapshot bound.  The dot test with FP32 snapshots is held to 1e-4; with
    compressed snapshots L^T is approximate, and its error
    |<x, L~^T y> - <L x, y>| is bounded by ||x|| ||L~^T y - L^T y||, so the
    difference is normalised by ||x|| ||L^T y|| and held to the snapshot
    bound, as is the relative difference of the two gradients L~^T y and
    L^T y (the FP32 run of the same interval serving as L^T y)."""
    from paper_2508_10405_amd import autograd, lsrtm
    w = synth.config4()
    print(f"[case] config4 full size, {w.nshot} shots, nt {w.nt}", flush=True)
    rng = np.random.default_rng(41)
    dm = to_dev(torch, w.dm)
    noise = to_dev(torch, 0.02 * rng.standard_normal((2,) + w.shape))
    v = to_dev(torch, rng.standard_normal((2,) + w.shape))
    x = to_dev(torch, rng.standard_normal((2,) + w.shape))
    d_obs = None
    g32 = {}
    for dtype in ("f32", "f16", "bf16"):
        for k in (10, 50, 200):
            ctx = lsrtm.context_for(w, ckpt_every=k, ckpt_dtype=dtype)
            if d_obs is None:
                d_obs = ctx.born((0.6 * dm + noise).contiguous()).clone()
                y = to_dev(torch, rng.standard_normal(ctx.data_len))
            m = dm.clone().requires_grad_(True)
            J = autograd.misfit(m, ctx, d_obs)
            J.backward()
            g = m.grad.detach()
            eps = 1e-3
            with torch.no_grad():
                rp = ctx.born((dm + eps * v).contiguous()) - d_obs
                rm = ctx.born((dm - eps * v).contiguous()) - d_obs
                fd = (0.5 * ctx.dot(rp, rp) - 0.5 * ctx.dot(rm, rm)) / (2 * eps)
            an = ctx.dot(g.reshape(-1).contiguous(), v.reshape(-1))
            e_fd = abs(fd - an) / abs(an)
            xg = x.clone().requires_grad_(True)
            Lx = autograd.born(xg, ctx)
            (Lx * y).sum().backward()
            a = ctx.dot(Lx.detach(), y)
            gy = xg.grad.reshape(-1).contiguous()
            b = ctx.dot(x.reshape(-1), gy)
            if dtype == "f32":
                g32[k] = gy.clone()
                e_dot = abs(a - b) / abs(a)
                e_g = 0.0
            else:
                nx = ctx.dot(x.reshape(-1), x.reshape(-1)) ** 0.5
                ng = ctx.dot(g32[k], g32[k]) ** 0.5
                e_dot = abs(a - b) / (nx * ng)
                dg = gy - g32[k]
                e_g = ctx.dot(dg, dg) ** 0.5 / ng
            print(f"[config4 full] {dtype} k={k}: central difference {e_fd:.2e}, dot test {e_dot:.2e}, "
                  f"migration against FP32 snapshots {e_g:.2e}", flush=True)
            ctx.close()
            assert e_fd <= 1e-3 + SNAPSHOT_BOUND[dtype]
            assert e_dot <= SNAPSHOT_BOUND[dtype]
            assert e_g <= SNAPSHOT_BOUND[dtype]
