"""Python binding of the HIP library (ctypes; argument marshalling only).

Every step of the imaging path runs in liblsrtm.so.  PyTorch provides device
memory and the HIP stream; nothing here computes on tensors.  If the library
is not built, importing the binding works but creating a Context raises.

Array conventions (same as the C ABI): physical grid arrays are torch float32
tensors of shape (nx, nz) in 2D and (ny, nx, nz) in 3D (z fastest); model
perturbations and images have a leading axis of 2 for (lnVp, lnIp); data
vectors are flat, shot s occupying nt * nrec_s values laid out [it][rec].

Streams: the library works on the context's stream.  A call made while another
stream is current orders itself after the work already queued there (the
arguments' producers) and queues the caller's later work after its own, and
the tensors it touches are kept from reuse until the context's stream is done
with them; a call made with the context's stream current adds nothing.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsrtm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lsrtm.h")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5, -6
CKPT = {"f32": 0, "f16": 1, "bf16": 2}
OPT_SHOTS_PER_LAUNCH, OPT_TILE, OPT_GRAPH, OPT_TIMING, OPT_MEM_BUDGET_MB, OPT_CKPT_PER_GROUP, OPT_FUSED, \
    OPT_PROGRESS, OPT_TILE_V, OPT_TILE_ADJ_A, OPT_REPLAY_CACHE_MB, OPT_GRAPH_CACHE = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12
NKERNEL = 8
KERNEL_NAMES = ("born_v", "born_p", "bg_v", "bg_p", "adj_a", "adj_b", "ckpt", "rec")

_c_int, _c_double, _c_ll, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_void_p


class Grid(ctypes.Structure):
    _fields_ = [("ndim", _c_int), ("n", _c_int * 3), ("h", _c_double * 3), ("npml", _c_int),
                ("pml_R", _c_double), ("pml_f0", _c_double), ("nt", _c_int), ("dt", _c_double),
                ("ckpt_every", _c_int), ("ckpt_dtype", _c_int)]


class LsrtmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lsrtm status {status}: {msg}")
        self.status = status


_lib = None

# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "lsrtm_create": (_c_int, [ctypes.POINTER(Grid), _vp, ctypes.POINTER(_vp)]),
    "lsrtm_set_model": (_c_int, [_vp, _vp, _vp]),
    "lsrtm_set_acquisition": (_c_int, [_vp, _c_int, _vp, _vp, _vp, _vp, _vp]),
    "lsrtm_forward": (_c_int, [_vp, _vp]),
    "lsrtm_born": (_c_int, [_vp, _vp, _vp]),
    "lsrtm_adjoint": (_c_int, [_vp, _vp, _vp, _c_int]),
    "lsrtm_cgnr": (_c_int, [_vp, _vp, _c_int, _vp, _vp]),
    "lsrtm_cgnr_begin": (_c_int, [_vp, _vp, _vp]),
    "lsrtm_cgnr_iterate": (_c_int, [_vp, _vp, ctypes.POINTER(_c_double)]),
    "lsrtm_cgnr_state": (_c_int, [_vp, _c_int, _vp, _vp, _vp, ctypes.POINTER(_c_double)]),
    "lsrtm_pseudo_hessian": (_c_int, [_vp, _vp, _vp, _c_double]),
    "lsrtm_set_preconditioner": (_c_int, [_vp, _vp]),
    "lsrtm_psf_images": (_c_int, [_vp, _c_int, _vp]),
    "lsrtm_wiener": (_c_int, [_vp, _vp, _vp, _vp, _c_int, _c_int, _c_double, _vp]),
    "lsrtm_mute": (_c_int, [_vp, _vp, _c_double, _c_double, _c_int]),
    "lsrtm_mute_noalloc": (_c_int, [_vp, _vp, _c_double, _c_double, _c_int]),
    "lsrtm_psf_apply": (_c_int, [_vp, _vp, _c_int, _c_int, _c_int, _vp, _vp]),
    "lsrtm_psf_cgnr": (_c_int, [_vp, _vp, _c_int, _c_int, _vp, _c_int, _vp, ctypes.POINTER(_c_double)]),
    "lsrtm_dot": (_c_int, [_vp, _vp, _vp, _c_ll, ctypes.POINTER(_c_double)]),
    "lsrtm_axpy": (_c_int, [_vp, _c_double, _vp, _vp, _c_ll]),
    "lsrtm_stream_mix": (_c_int, [_vp, _vp, _c_ll, _c_int, _c_int, ctypes.POINTER(_c_int),
                                  ctypes.POINTER(_c_double)]),
    "lsrtm_cgnr_step": (_c_int, [_vp, ctypes.POINTER(_c_double)]),
    "lsrtm_set_option": (_c_int, [_vp, _c_int, _c_ll]),
    "lsrtm_sizes": (_c_int, [_vp, ctypes.POINTER(_c_ll), _c_int]),
    "lsrtm_autotune": (_c_int, [_vp, _c_int, _c_int, ctypes.POINTER(_c_double)]),
    "lsrtm_stats": (_c_int, [_vp, ctypes.POINTER(_c_double), _c_int]),
    "lsrtm_tile_shape": (_c_int, [_c_int, _c_int, ctypes.POINTER(_c_int)]),
    "lsrtm_destroy": (None, [_vp]),
    "lsrtm_strerror": (ctypes.c_char_p, [_c_int]),
    "lsrtm_last_error": (ctypes.c_char_p, [_vp]),
}


def lib():
    """Load liblsrtm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2508_10405_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def _require_cuda(t, name, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != (dtype or torch.float32):
        raise TypeError(f"{name} must be {dtype or torch.float32}")
    return t


class Context:
    """One imaging problem on one GPU stream.

    Parameters follow lsrtm_grid: n = (nz, nx[, ny]) physical sizes,
    h = (dz, dx[, dy]), npml CPML cells, nt steps of dt seconds, CPML
    parameters pml_R and pml_f0, checkpoint interval (0 = planner) and
    checkpoint storage ("f32", "f16", "bf16").  tile_v and tile_adj_a give
    the velocity phases and the adjoint A phase tile shapes of their own
    (-1 = the stencil tile); results do not depend on them.  replay_cache_mb
    lets the plan keep the background replays of the last checkpoint segments
    across migration passes (LSRTM_OPT_REPLAY_CACHE_MB; bitwise the same
    results, 0 = off).
    """

    def __init__(self, n, h, nt, dt, npml=20, pml_R=1e-4, pml_f0=10.0, ckpt_every=0,
                 ckpt_dtype="f32", stream=None, shots_per_launch=0, tile=-1, graph=True,
                 timing=False, mem_budget_mb=0, ckpt_per_group=False, fused=False, progress=False,
                 tile_v=-1, tile_adj_a=-1, replay_cache_mb=0):
        import torch
        L = lib()
        self._torch = torch
        ndim = len(n)
        g = Grid()
        g.ndim = ndim
        for a in range(3):
            g.n[a] = int(n[a]) if a < ndim else 1
            g.h[a] = float(h[a]) if a < ndim else 1.0
        g.npml, g.pml_R, g.pml_f0 = int(npml), float(pml_R), float(pml_f0)
        g.nt, g.dt = int(nt), float(dt)
        g.ckpt_every, g.ckpt_dtype = int(ckpt_every), CKPT[ckpt_dtype]
        self.grid = g
        self.ndim, self.n, self.nt = ndim, tuple(int(x) for x in n), int(nt)
        self.shape = tuple(reversed(self.n))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._h = _vp()
        self._check(L.lsrtm_create(ctypes.byref(g), _vp(stream.cuda_stream), ctypes.byref(self._h)),
                    "create")
        self.set_option(OPT_SHOTS_PER_LAUNCH, shots_per_launch)
        self.set_option(OPT_TILE, tile)
        self.set_option(OPT_GRAPH, int(bool(graph)))
        self.set_option(OPT_TIMING, int(bool(timing)))
        self.set_option(OPT_MEM_BUDGET_MB, mem_budget_mb)
        self.set_option(OPT_CKPT_PER_GROUP, int(bool(ckpt_per_group)))
        self.set_option(OPT_FUSED, int(bool(fused)))
        self.set_option(OPT_PROGRESS, int(bool(progress)))
        self.set_option(OPT_TILE_V, tile_v)
        self.set_option(OPT_TILE_ADJ_A, tile_adj_a)
        self.set_option(OPT_REPLAY_CACHE_MB, replay_cache_mb)
        self.nrec: List[int] = []
        self._keep = []
        self._minv = None

    # -- plumbing -----------------------------------------------------------
    def _check(self, status, what):
        if status != OK:
            msg = ""
            if getattr(self, "_h", None) is not None and self._h.value:
                msg = lib().lsrtm_last_error(self._h).decode()
            raise LsrtmError(status, f"{what}: {lib().lsrtm_strerror(status).decode()} {msg}".strip())

    @contextlib.contextmanager
    def _ordered(self, *tensors):
        """Order a library call between the caller's current stream and the
        context's stream (see the module docstring)."""
        cur = self._torch.cuda.current_stream()
        other = cur != self.stream
        if other:
            self.stream.wait_stream(cur)
            for t in tensors:
                if t is not None:
                    t.record_stream(self.stream)
        yield
        if other:
            cur.wait_stream(self.stream)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lsrtm_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key, value):
        self._check(lib().lsrtm_set_option(self._h, int(key), int(value)), "set_option")

    # -- problem ------------------------------------------------------------
    def set_model(self, lnvp, lnip):
        _require_cuda(lnvp, "lnvp")
        _require_cuda(lnip, "lnip")
        if tuple(lnvp.shape) != self.shape or tuple(lnip.shape) != self.shape:
            raise ValueError(f"model shape must be {self.shape}")
        with self._ordered(lnvp, lnip):
            self._check(lib().lsrtm_set_model(self._h, _vp(_ptr(lnvp)), _vp(_ptr(lnip))), "set_model")

    def set_acquisition(self, win, src, rec: Sequence, wavelet):
        """win: per shot ((z0, z1), (x0, x1)[, (y0, y1)]); src: per shot node;
        rec: per shot int array (nrec, ndim); wavelet: CUDA float32 (nshot, nt)."""
        nd = self.ndim
        nshot = len(src)
        w = np.ascontiguousarray(np.array(win, dtype=np.int32).reshape(nshot, 2 * nd))
        s = np.ascontiguousarray(np.array(src, dtype=np.int32).reshape(nshot, nd))
        counts = [len(r) for r in rec]
        ptr = np.zeros(nshot + 1, dtype=np.int32)
        ptr[1:] = np.cumsum(counts)
        r = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int32).reshape(-1, nd) for x in rec])
                                 if ptr[-1] > 0 else np.zeros((0, nd), np.int32))
        _require_cuda(wavelet, "wavelet")
        if tuple(wavelet.shape) != (nshot, self.nt):
            raise ValueError("wavelet must have shape (nshot, nt)")
        with self._ordered(wavelet):
            self._check(lib().lsrtm_set_acquisition(
                self._h, nshot, w.ctypes.data, s.ctypes.data, ptr.ctypes.data, r.ctypes.data,
                _vp(_ptr(wavelet))), "set_acquisition")
        self.nrec = counts
        self.nshot = nshot

    # -- sizes --------------------------------------------------------------
    def autotune(self, nsteps=8, groups=False):
        out = (_c_double * 5)()
        self._check(lib().lsrtm_autotune(self._h, int(nsteps), int(bool(groups)), out), "autotune")
        return {"tile": int(out[0]), "shots_per_launch": int(out[1]), "ms_per_step": out[2],
                "tile_v": int(out[3]), "tile_adj_a": int(out[4])}

    def sizes(self):
        out = (_c_ll * 14)()
        self._check(lib().lsrtm_sizes(self._h, out, 14), "sizes")
        keys = ("data_len", "grid_points", "shots_per_launch", "ckpt_every", "groups",
                "padded_points", "plan_bytes", "tile", "ckpt_per_group", "fused", "tile_v", "tile_adj_a",
                "replay_cache_segments", "graphs")
        return dict(zip(keys, [int(x) for x in out]))

    @property
    def data_len(self) -> int:
        return self.sizes()["data_len"]

    def stats(self):
        m = 1 + 2 * NKERNEL
        out = (_c_double * m)()
        self._check(lib().lsrtm_stats(self._h, out, m), "stats")
        d = {"pass_ms": out[0]}
        for k, name in enumerate(KERNEL_NAMES):
            d[name] = (out[1 + 2 * k], int(out[2 + 2 * k]))
        return d

    def split(self, d) -> list:
        """Flat data vector -> list of per-shot (nt, nrec_s) views."""
        out, o = [], 0
        for c in self.nrec:
            out.append(d[o:o + self.nt * c].view(self.nt, c))
            o += self.nt * c
        return out

    # -- operators ----------------------------------------------------------
    def _data(self, d):
        torch = self._torch
        if d is None:
            d = torch.empty(self.data_len, dtype=torch.float32, device="cuda")
        _require_cuda(d, "d")
        if d.numel() != self.data_len:
            raise ValueError(f"data vector must have {self.data_len} values")
        return d

    def _image(self, img, name="image"):
        torch = self._torch
        if img is None:
            img = torch.empty((2,) + self.shape, dtype=torch.float32, device="cuda")
        _require_cuda(img, name)
        if tuple(img.shape) != (2,) + self.shape:
            raise ValueError(f"{name} must have shape {(2,) + self.shape}")
        return img

    def _data_in(self, d, name):
        _require_cuda(d, name)
        if d.numel() != self.data_len:
            raise ValueError(f"{name} must have {self.data_len} values")
        return d

    def _psf(self, psf):
        _require_cuda(psf, "psf")
        if tuple(psf.shape) != (2, 2) + self.shape:
            raise ValueError(f"psf must have shape {(2, 2) + self.shape}")
        return psf

    def forward(self, d=None):
        d = self._data(d)
        with self._ordered(d):
            self._check(lib().lsrtm_forward(self._h, _vp(_ptr(d))), "forward")
        return d

    def born(self, dm, d=None):
        _require_cuda(dm, "dm")
        if tuple(dm.shape) != (2,) + self.shape:
            raise ValueError(f"dm must have shape {(2,) + self.shape}")
        d = self._data(d)
        with self._ordered(dm, d):
            self._check(lib().lsrtm_born(self._h, _vp(_ptr(dm)), _vp(_ptr(d))), "born")
        return d

    def adjoint(self, d, img=None, accumulate=False):
        self._data_in(d, "d")
        img = self._image(img)
        with self._ordered(d, img):
            self._check(lib().lsrtm_adjoint(self._h, _vp(_ptr(d)), _vp(_ptr(img)), int(bool(accumulate))),
                        "adjoint")
        return img

    def cgnr(self, d_obs, niter, x=None, log=None):
        """niter CGNR iterations from x = 0; returns (x, normalised misfits).
        With log (a path), one JSON line per iteration is appended to it:
        the iteration, misfit, alpha, beta and ||L p||^2 (lsrtm_cgnr_step),
        the iteration's wall time and its Gpts/s (padded nodes x nt x 2
        passes)."""
        self._data_in(d_obs, "d_obs")
        if niter < 0:
            raise ValueError("niter must be >= 0")
        if log is None:
            x = self._image(x)
            mis = (_c_double * (niter + 1))()
            with self._ordered(d_obs, x):
                self._check(lib().lsrtm_cgnr(self._h, _vp(_ptr(d_obs)), int(niter), _vp(_ptr(x)), mis), "cgnr")
            return x, [float(v) for v in mis]
        import json
        import time
        torch = self._torch
        x = self.cgnr_begin(d_obs, x)
        mis = [1.0]
        pts = self.sizes()["padded_points"]
        with open(log, "a") as f:
            for _ in range(int(niter)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                self.cgnr_iterate(x)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                st = self.cgnr_step()
                mis.append(st["misfit"])
                f.write(json.dumps({**st, "seconds": dt, "gpts": 2.0 * pts * self.nt / dt / 1e9}) + "\n")
                f.flush()
        return x, mis

    def cgnr_step(self):
        """The last iteration's step (lsrtm_cgnr_step): k, alpha, beta,
        ||L p||^2 and the normalised misfit, as the solver computed them."""
        out = (_c_double * 5)()
        self._check(lib().lsrtm_cgnr_step(self._h, out), "cgnr_step")
        return {"iter": int(out[0]), "alpha": out[1], "beta": out[2], "ww": out[3], "misfit": out[4]}

    def cgnr_begin(self, d_obs, x=None):
        self._data_in(d_obs, "d_obs")
        x = self._image(x, "x")
        with self._ordered(d_obs, x):
            self._check(lib().lsrtm_cgnr_begin(self._h, _vp(_ptr(d_obs)), _vp(_ptr(x))), "cgnr_begin")
        return x

    def cgnr_iterate(self, x) -> float:
        self._image(x, "x")
        m = _c_double()
        with self._ordered(x):
            self._check(lib().lsrtm_cgnr_iterate(self._h, _vp(_ptr(x)), ctypes.byref(m)), "cgnr_iterate")
        return m.value

    def cgnr_get_state(self):
        torch = self._torch
        r = torch.empty(self.data_len, dtype=torch.float32, device="cuda")
        z = torch.empty((2,) + self.shape, dtype=torch.float32, device="cuda")
        p = torch.empty_like(z)
        sc = (_c_double * 4)()
        with self._ordered(r, z, p):
            self._check(lib().lsrtm_cgnr_state(self._h, 1, _vp(_ptr(r)), _vp(_ptr(z)), _vp(_ptr(p)), sc),
                        "cgnr_state")
        return {"r": r, "z": z, "p": p, "scalars": [float(v) for v in sc]}

    def cgnr_set_state(self, st):
        if len(st["scalars"]) != 4:
            raise ValueError("the CG state holds 4 scalars")
        sc = (_c_double * 4)(*st["scalars"])
        self._data_in(st["r"], "r")
        self._image(st["z"], "z")
        self._image(st["p"], "p")
        with self._ordered(st["r"], st["z"], st["p"]):
            self._check(lib().lsrtm_cgnr_state(self._h, 0, _vp(_ptr(st["r"])), _vp(_ptr(st["z"])),
                                               _vp(_ptr(st["p"])), sc), "cgnr_state")

    def cgnr_save(self, path, x):
        """Write the CG run to `path` (numpy .npz of plain arrays, nothing
        pickled): the iterate x and the solver state r, z, p in FP32 as the
        library holds them (so that a resumed run continues bit for bit), the
        scalars (<z, s>, <r0, r0>, <r, r>, k) in FP64, and the preconditioner
        in use, if any."""
        _require_cuda(x, "x")
        st = self.cgnr_get_state()
        arrays = {"x": x.cpu().numpy(), "r": st["r"].cpu().numpy(), "z": st["z"].cpu().numpy(),
                  "p": st["p"].cpu().numpy(), "scalars": np.asarray(st["scalars"], dtype=np.float64),
                  "shape": np.asarray(self.shape, dtype=np.int64),
                  "data_len": np.asarray(self.data_len, dtype=np.int64)}
        if self._minv is not None:
            arrays["minv"] = self._minv.cpu().numpy()
        with open(path, "wb") as f:
            np.savez(f, **arrays)

    def cgnr_load(self, path):
        """Resume a CG run written by cgnr_save on a context with the same grid
        and acquisition: restores its preconditioner (or none) and its solver
        state, and returns the iterate x as a device tensor for
        cgnr_iterate."""
        torch = self._torch
        with np.load(path, allow_pickle=False) as f:
            if tuple(f["shape"]) != tuple(self.shape) or int(f["data_len"]) != self.data_len:
                raise ValueError(f"{path}: CG state of another problem")
            dev = lambda k: torch.from_numpy(np.ascontiguousarray(f[k], dtype=np.float32)).cuda()
            self.set_preconditioner(dev("minv") if "minv" in f.files else None)
            self.cgnr_set_state({"r": dev("r"), "z": dev("z"), "p": dev("p"),
                                 "scalars": [float(v) for v in f["scalars"]]})
            return dev("x")

    def pseudo_hessian(self, eps_rel=1e-3, preconditioner=True):
        """Pseudo-Hessian diagonal h [shape] (lsrtm_pseudo_hessian) and, with
        preconditioner=True, minv [2, *shape] = 1 / (h + eps_rel max h)."""
        torch = self._torch
        h = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        minv = torch.empty((2,) + self.shape, dtype=torch.float32, device="cuda") if preconditioner else None
        with self._ordered(h, minv):
            self._check(lib().lsrtm_pseudo_hessian(self._h, _vp(_ptr(h)), _vp(_ptr(minv)), float(eps_rel)),
                        "pseudo_hessian")
        return h, minv

    def set_preconditioner(self, minv):
        """Diagonal preconditioner of the CGNR solver ([2, *shape]), or None."""
        if minv is not None:
            _require_cuda(minv, "minv")
            if minv.numel() != 2 * int(np.prod(self.shape)):
                raise ValueError("minv must hold 2 x grid points")
        with self._ordered(minv):
            self._check(lib().lsrtm_set_preconditioner(self._h, _vp(_ptr(minv))), "set_preconditioner")
        self._minv = None if minv is None else minv.detach().clone()

    def psf_images(self, spacing):
        """PSF images [2 (scatterer parameter), 2 (response), *shape]
        (lsrtm_psf_images)."""
        torch = self._torch
        psf = torch.empty((2, 2) + self.shape, dtype=torch.float32, device="cuda")
        with self._ordered(psf):
            self._check(lib().lsrtm_psf_images(self._h, int(spacing), _vp(_ptr(psf))), "psf_images")
        return psf

    def _psf_vec(self, v, mono, name):
        _require_cuda(v, name)
        want = (1 if mono else 2) * int(np.prod(self.shape))
        if v.numel() != want:
            raise ValueError(f"{name} must hold {want} values")

    def psf_apply(self, psf, spacing, x, transpose=False, mono=False):
        """y = H x or H^T x with the interpolated PSF Hessian (lsrtm_psf_apply)."""
        self._psf(psf)
        self._psf_vec(x, mono, "x")
        y = self._torch.empty_like(x)
        with self._ordered(psf, x, y):
            self._check(lib().lsrtm_psf_apply(self._h, _vp(_ptr(psf)), int(spacing), int(bool(mono)),
                                              int(bool(transpose)), _vp(_ptr(x)), _vp(_ptr(y))), "psf_apply")
        return y

    def psf_cgnr(self, psf, spacing, m_rtm, niter, mono=False):
        """Image-domain CGNR with the PSF Hessian; returns x and the misfit
        history (lsrtm_psf_cgnr)."""
        self._psf(psf)
        self._psf_vec(m_rtm, mono, "m_rtm")
        if niter < 0:
            raise ValueError("niter must be >= 0")
        x = self._torch.empty_like(m_rtm)
        mis = (_c_double * (niter + 1))()
        with self._ordered(psf, m_rtm, x):
            self._check(lib().lsrtm_psf_cgnr(self._h, _vp(_ptr(psf)), int(spacing), int(bool(mono)),
                                             _vp(_ptr(m_rtm)), int(niter), _vp(_ptr(x)), mis), "psf_cgnr")
        return x, [float(v) for v in mis]

    def mute(self, d, v_mute, t0=0.0, ntaper=0):
        """Top mute of a data vector in place (lsrtm_mute); returns d."""
        self._data_in(d, "d")
        with self._ordered(d):
            self._check(lib().lsrtm_mute(self._h, _vp(_ptr(d)), float(v_mute), float(t0), int(ntaper)), "mute")
        return d

    def mute_noalloc(self, d, v_mute, t0=0.0, ntaper=0):
        """The same mute without device allocations (lsrtm_mute_noalloc; at
        most 2^18 receivers); returns d."""
        self._data_in(d, "d")
        with self._ordered(d):
            self._check(lib().lsrtm_mute_noalloc(self._h, _vp(_ptr(d)), float(v_mute), float(t0), int(ntaper)),
                        "mute_noalloc")
        return d

    def wiener(self, m_ref, m_blur, m_in=None, block=64, eps_rel=1e-3):
        """Nonstationary Wiener deblurring (lsrtm_wiener) of one image or a
        stack [k, *shape]; m_in defaults to m_ref."""
        m_in = m_ref if m_in is None else m_in
        n = int(np.prod(self.shape))
        for t, name in ((m_ref, "m_ref"), (m_blur, "m_blur"), (m_in, "m_in")):
            _require_cuda(t, name)
            if t.numel() % n or t.numel() != m_ref.numel():
                raise ValueError(f"{name} must hold a whole number of images")
        out = self._torch.empty_like(m_ref)
        with self._ordered(m_ref, m_blur, m_in, out):
            self._check(lib().lsrtm_wiener(self._h, _vp(_ptr(m_ref)), _vp(_ptr(m_blur)), _vp(_ptr(m_in)),
                                           m_ref.numel() // n, int(block), float(eps_rel), _vp(_ptr(out))),
                        "wiener")
        return out

    def dot(self, a, b) -> float:
        _require_cuda(a, "a")
        _require_cuda(b, "b")
        if a.numel() != b.numel():
            raise ValueError("length mismatch")
        out = _c_double()
        with self._ordered(a, b):
            self._check(lib().lsrtm_dot(self._h, _vp(_ptr(a)), _vp(_ptr(b)), a.numel(), ctypes.byref(out)),
                        "dot")
        return out.value

    def axpy(self, alpha, x, y):
        _require_cuda(x, "x")
        _require_cuda(y, "y")
        if x.numel() != y.numel():
            raise ValueError("length mismatch")
        with self._ordered(x, y):
            self._check(lib().lsrtm_axpy(self._h, float(alpha), _vp(_ptr(x)), _vp(_ptr(y)), x.numel()), "axpy")
        return y


    def stream_mix(self, buf, n, nread, nwrite, grid=None) -> float:
        """Calibration (lsrtm_stream_mix): kernel time in ms of one streaming
        pass over nread + nwrite arrays of n floats in buf (a device float
        tensor of at least (nread + nwrite) * n elements, overwritten); grid =
        (nz, nx, ny, ldz) walks them in the 3D tiles' order."""
        _require_cuda(buf, "buf")
        if buf.numel() < (nread + nwrite) * n:
            raise ValueError("buf too small")
        g = (_c_int * 4)(*grid) if grid is not None else None
        ms = _c_double()
        with self._ordered(buf):
            self._check(lib().lsrtm_stream_mix(self._h, _vp(_ptr(buf)), int(n), int(nread), int(nwrite), g,
                                               ctypes.byref(ms)), "stream_mix")
        return ms.value


def tile_shape(ndim: int, tile_id: int):
    out = (_c_int * 2)()
    st = lib().lsrtm_tile_shape(int(ndim), int(tile_id), out)
    if st != OK:
        raise LsrtmError(st, "unknown tile id")
    return int(out[0]), int(out[1])


def context_for(w, device="cuda", **opts) -> Context:
    """Context with model and acquisition of a workload description (an object
    with h, dt, nt, npml, pml_R, pml_freq, lnvp, lnip, win, src, rec, wavelet)."""
    import torch
    n = tuple(reversed(w.lnvp.shape))
    ctx = Context(n, w.h, w.nt, w.dt, npml=w.npml, pml_R=w.pml_R, pml_f0=w.pml_freq, **opts)
    ctx.set_model(torch.from_numpy(np.ascontiguousarray(w.lnvp, np.float32)).to(device),
                  torch.from_numpy(np.ascontiguousarray(w.lnip, np.float32)).to(device))
    ctx.set_acquisition(w.win, w.src, w.rec,
                        torch.from_numpy(np.ascontiguousarray(w.wavelet, np.float32)).to(device))
    return ctx
