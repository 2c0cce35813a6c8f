"""Oracle runs in worker processes for the GPU tests on large grids.

The FP64 oracle takes tens of seconds per shot on the full-size grids; the
tests that compare such shots start the Born and migration runs side by side
in a process pool (each worker is single-threaded numpy).  Jobs are plain
tuples of arrays and numbers so that they pickle without the test module.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
from multiprocessing import get_context

import numpy as np


def _problem(job):
    from oracle import lsrtm_oracle as O
    h, dt, nt, npml, R, f0, win, src, rec, wav = job["problem"]
    return O.Problem(h, dt, nt, npml, R, f0, win, src, rec, np.asarray(wav, dtype=np.float64))


def _run(job):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import lsrtm_oracle as O
    prob = _problem(job)
    lnvp, lnip = job["lnvp"], job["lnip"]
    if job["kind"] == "born":
        return O.born(prob, lnvp, lnip, job["dm"])
    if job["kind"] == "adjoint":
        return O.adjoint(prob, lnvp, lnip, job["ys"], ckpt_every=job.get("ckpt_every", 50))
    raise ValueError(job["kind"])


def problem_tuple(w, shots, nt):
    """Problem description of the given shots of workload w on nt steps."""
    return (tuple(w.h), w.dt, nt, w.npml, w.pml_R, w.pml_freq, [w.win[s] for s in shots],
            [w.src[s] for s in shots], [np.asarray(w.rec[s]) for s in shots],
            np.asarray(w.wavelet[list(shots), :nt], dtype=np.float64))


def born_job(w, shots, nt, dm):
    return {"kind": "born", "problem": problem_tuple(w, shots, nt),
            "lnvp": np.asarray(w.lnvp, np.float64), "lnip": np.asarray(w.lnip, np.float64),
            "dm": np.asarray(dm, np.float64)}


def adjoint_job(w, shots, nt, ys, ckpt_every=50):
    return {"kind": "adjoint", "problem": problem_tuple(w, shots, nt),
            "lnvp": np.asarray(w.lnvp, np.float64), "lnip": np.asarray(w.lnip, np.float64),
            "ys": [np.asarray(y, np.float64) for y in ys], "ckpt_every": ckpt_every}


class Running:
    """Jobs started in a pool of worker processes; results() waits for them
    (in job order).  Start them before the GPU work so that both proceed
    together."""

    def __init__(self, jobs, workers=None):
        workers = workers or min(len(jobs), 8)
        self._ex = ProcessPoolExecutor(max_workers=workers, mp_context=get_context("spawn"))
        self._futs = [self._ex.submit(_run, j) for j in jobs]

    def results(self):
        try:
            return [f.result() for f in self._futs]
        finally:
            self._ex.shutdown()


def run_all(jobs, workers=None):
    """Results of the jobs, in order, computed in parallel processes."""
    return Running(jobs, workers).results()
