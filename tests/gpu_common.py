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
