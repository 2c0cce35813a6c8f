"""Helpers shared by the GPU tests: device setup and oracle runs."""
import numpy as np

from oracle import lsrtm_oracle as O


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    from paper_2508_10405_amd import lsrtm
    lsrtm.lib()   # fails loudly if the library is missing
    return torch


def oracle_problem(w, nt=None):
    return O.Problem(w.h, w.dt, w.nt if nt is None else nt, w.npml, w.pml_R, w.pml_freq, w.win,
                     w.src, w.rec, w.wavelet.astype(np.float64))


def f64(a):
    return np.asarray(a, dtype=np.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def concat(ds):
    return np.concatenate([np.asarray(d).ravel() for d in ds])


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# Bounds of the image error caused by FP16 / BF16 snapshots (per-snapshot
# max-abs scaling, round to nearest even).  Error model: a restored snapshot
# is the exact state plus rounding of relative size at most u (unit roundoff:
# 2^-11 for FP16, 2^-8 for BF16; the scale keeps every value of interest in
# the normal range).  A replay is a linear map of its initial state that does
# not amplify it, so the replayed background carries a relative error of
# order u; the imaging condition correlates derivatives of that background
# with the adjoint field, and the rounding error is white, so the O(2,8)
# difference amplifies it against the band-limited field by a small factor.
# Measured image errors lie between 1.6 u and 2.1 u (every checkpoint interval
# from 10 to 200 steps, 2D and 3D); the stated bound is 4 u.
FP16_BOUND = 4 * 2.0 ** -11
BF16_BOUND = 4 * 2.0 ** -8
SNAPSHOT_BOUND = {"f32": 1e-4, "f16": FP16_BOUND, "bf16": BF16_BOUND}


def cg_step_parity(torch, ctx, L, Lt, d_obs, niter, minv=None, tol=1e-4):
    """Per-iteration parity of the library's (preconditioned) CGNR: before
    every iteration the GPU's state (x, r, z, p, <z, s>) is exported and one
    FP64 iteration of the oracle's algebra (the step of O.pcgnr: w = L p,
    alpha = <z, s> / <w, w>, x += alpha p, r -= alpha w, s = L^T r,
    z = minv s, beta = <z, s>_new / <z, s>_old, p = z + beta p) is applied to
    it; the GPU's next state must agree within tol (relative L2, each of x, r,
    z, p).  L and Lt are oracle operators on numpy arrays (image of shape
    (2, *grid) <-> list of per-shot (nt, nrec) records).  Returns the largest
    error seen and the GPU iterate."""
    def data_list(v):
        return [p.cpu().numpy().astype(np.float64) for p in ctx.split(v)]

    def dot(a, b):
        if isinstance(a, list):
            return float(sum(np.vdot(x, y) for x, y in zip(a, b)))
        return float(np.vdot(a, b))

    mv = np.ones((2,) + ctx.shape) if minv is None else np.asarray(minv, dtype=np.float64)
    x = ctx.cgnr_begin(d_obs)
    st = ctx.cgnr_get_state()
    worst = 0.0
    # the initial normal residual: z0 = minv L^T d_obs
    z0 = mv * Lt(data_list(d_obs))
    e = rel(st["z"].cpu().numpy(), z0)
    worst = max(worst, e)
    assert e <= tol, ("z0", e)
    for it in range(niter):
        xk = x.cpu().numpy().astype(np.float64)
        rk = data_list(st["r"])
        pk = st["p"].cpu().numpy().astype(np.float64)
        zs = st["scalars"][0]
        w = L(pk)
        alpha = zs / dot(w, w)
        x_ref = xk + alpha * pk
        r_ref = [a - alpha * b for a, b in zip(rk, w)]
        s_ref = Lt(r_ref)
        z_ref = mv * s_ref
        beta = dot(z_ref, s_ref) / zs
        p_ref = z_ref + beta * pk
        ctx.cgnr_iterate(x)
        st = ctx.cgnr_get_state()
        errs = {"x": rel(x.cpu().numpy(), x_ref), "r": rel(st["r"].cpu().numpy(), concat(r_ref)),
                "z": rel(st["z"].cpu().numpy(), z_ref), "p": rel(st["p"].cpu().numpy(), p_ref)}
        print(f"CG step {it + 1}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
        worst = max(worst, max(errs.values()))
        assert max(errs.values()) <= tol, (it, errs)
    return worst, x
