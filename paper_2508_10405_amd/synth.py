"""Seeded synthetic inputs: models, perturbations, acquisition, wavelets.

This module is shared by the tests, the benchmark and the oracle-facing test
code.  It holds no arithmetic of the imaging method itself (no stencil, no
parameter map, no source scaling): it only draws inputs.  It imports nothing
from the rest of the package.

Shapes: physical arrays are (nx, nz) in 2D and (ny, nx, nz) in 3D (z is the
fastest axis); node coordinates are (iz, ix[, iy]); windows are
((z0, z1), (x0, x1)[, (y0, y1)]) half-open physical index ranges.

The paper's own models (Marmousi, Overthrust, Viking Graben) are not
available; the generators below stand in for them with the grid shapes,
spacings, velocity ranges and acquisition layouts of the benchmark
configurations (seeded faulted-layered 2D model, dipping layers plus a
Gaussian high-velocity body in 3D, Gardner density, Gaussian-smoothed
migration background).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.ndimage import gaussian_filter

F32 = np.float32


def ricker(f0: float, nt: int, dt: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet sampled at the half steps t = (n + 1/2) dt, delay 1.5/f0."""
    if t0 is None:
        t0 = 1.5 / f0
    t = (np.arange(nt) + 0.5) * dt - t0
    a = (np.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def gardner(vp: np.ndarray) -> np.ndarray:
    """Gardner's relation rho = 310 vp^0.25 (kg/m^3, vp in m/s)."""
    return 310.0 * vp ** 0.25


@dataclass
class Workload:
    """One seeded configuration: global model, perturbation, acquisition."""
    name: str
    h: tuple                 # (dz, dx[, dy]) in m
    dt: float
    nt: int
    npml: int
    f0: float
    lnvp: np.ndarray         # background ln Vp (float32, physical)
    lnip: np.ndarray         # background ln Ip
    dm: np.ndarray           # (2, *shape) true (dlnVp, dlnIp), float32
    win: list
    src: list
    rec: list
    wavelet: np.ndarray      # (nshot, nt) float32
    pml_R: float = 1e-4
    pml_f0: Optional[float] = None
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return len(self.h)

    @property
    def shape(self):
        return self.lnvp.shape

    @property
    def n(self):
        """(nz, nx[, ny])"""
        return tuple(reversed(self.lnvp.shape))

    @property
    def nshot(self) -> int:
        return len(self.src)

    @property
    def pml_freq(self) -> float:
        return self.f0 if self.pml_f0 is None else self.pml_f0

    def padded_points(self) -> int:
        tot = 0
        for w in self.win:
            pts = 1
            for lo, hi in w:
                pts *= (hi - lo) + 2 * self.npml
            tot += pts
        return tot

    def nrec_total(self) -> int:
        return int(sum(len(r) for r in self.rec))


def _logs(vp, rho):
    return np.log(vp).astype(F32), np.log(rho * vp).astype(F32)


def _full_window(n):
    return tuple((0, int(m)) for m in n)


# ---------------------------------------------------------------------------
# 2D models
# ---------------------------------------------------------------------------
def faulted_layered(nz: int, nx: int, h: float, seed: int, vmin=1500.0, vmax=5500.0,
                    nlayers: int = 12, nfaults: int = 3) -> np.ndarray:
    """Vp (nx, nz): monotone layers with undulating interfaces and normal faults."""
    rng = np.random.default_rng(seed)
    zs = np.arange(nz) * h
    xs = np.arange(nx) * h
    X, Z = np.meshgrid(xs, zs, indexing="ij")          # (nx, nz)
    zmax = nz * h
    depths = np.sort(rng.uniform(0.06 * zmax, 0.96 * zmax, nlayers - 1))
    amp = rng.uniform(0.0, 50.0, nlayers - 1)
    wlen = rng.uniform(1500.0, 6000.0, nlayers - 1)
    phase = rng.uniform(0.0, 2 * np.pi, nlayers - 1)
    vel = np.sort(rng.uniform(vmin, vmax, nlayers))
    vel[0], vel[-1] = vmin, vmax
    # faults: hanging wall (right of the plane x = xf + z / tan(dip)) dropped
    xf = np.sort(rng.uniform(0.15, 0.85, nfaults)) * nx * h
    dip = np.deg2rad(60.0 + rng.uniform(-10.0, 10.0, nfaults))
    throw = rng.uniform(50.0, 200.0, nfaults)
    Zs = Z.copy()
    for f in range(nfaults):
        hanging = X > xf[f] + Z / np.tan(dip[f])
        Zs = np.where(hanging, Zs - throw[f], Zs)
    layer = np.zeros_like(Z, dtype=np.int64)
    for k in range(nlayers - 1):
        iface = depths[k] + amp[k] * np.sin(2 * np.pi * X / wlen[k] + phase[k])
        layer += (Zs > iface).astype(np.int64)
    return vel[layer]


def _smooth_background(vp, rho, sigma):
    vp0 = gaussian_filter(vp, sigma, mode="nearest")
    rho0 = gaussian_filter(rho, sigma, mode="nearest")
    return vp0, rho0


def _perturbation(vp, rho, vp0, rho0):
    """True (dlnVp, dlnIp) = ln(true) - ln(background)."""
    dlnvp = np.log(vp) - np.log(vp0)
    dlnip = np.log(rho * vp) - np.log(rho0 * vp0)
    return np.stack([dlnvp, dlnip]).astype(F32)


def config1(seed: int = 1) -> Workload:
    """2D single shot: 100 x 200 at 10 m, linear Vp 1500->3000 m/s with depth,
    smoothed Gardner density, 5 seeded reflector rows, nt = 1000, 10 Hz."""
    nz, nx, h = 100, 200, 10.0
    rng = np.random.default_rng(seed)
    iz = np.arange(nz)
    vp = np.broadcast_to(1500.0 + 1500.0 * iz / (nz - 1), (nx, nz)).copy()
    rho = gaussian_filter(gardner(vp), 5.0, mode="nearest")
    lnvp, lnip = _logs(vp, rho)
    # 5 one-cell rows in [20, 95], at least 5 apart
    while True:
        rows = np.sort(rng.choice(np.arange(20, 96), 5, replace=False))
        if np.all(np.diff(rows) >= 5):
            break
    amps = rng.uniform(-0.1, 0.1, (2, 5))
    dm = np.zeros((2, nx, nz))
    for k, r in enumerate(rows):
        dm[:, :, r] = amps[:, k][:, None]
    nt, dt, f0 = 1000, 1e-3, 10.0
    rec = np.stack([np.full(nx, 2), np.arange(nx)], axis=1)
    return Workload("config1: 2D single shot 100x200", (h, h), dt, nt, 20, f0,
                    lnvp, lnip, dm.astype(F32), [_full_window((nz, nx))], [(2, 100)], [rec],
                    ricker(f0, nt, dt)[None].astype(F32))


def config2(seed: int = 2, nt: int = 4000) -> Workload:
    """2D LSRTM: 737 x 240 at 12.5 m faulted-layered model, 120 shots every
    6 nodes at iz = 2, 369 receivers every 2 nodes, 15 Hz, nt = 4000."""
    nz, nx, h = 240, 737, 12.5
    vp = faulted_layered(nz, nx, h, seed)
    rho = gardner(vp)
    vp0, rho0 = _smooth_background(vp, rho, 250.0 / h)
    lnvp, lnip = _logs(vp0, rho0)
    dm = _perturbation(vp, rho, vp0, rho0)
    f0, dt = 15.0, 1e-3
    src = [(2, 11 + 6 * k) for k in range(120)]
    rec1 = np.stack([np.full(369, 2), np.arange(0, 737, 2)], axis=1)
    w = ricker(f0, nt, dt).astype(F32)
    return Workload("config2: 2D 737x240, 120 shots", (h, h), dt, nt, 20, f0, lnvp, lnip, dm,
                    [_full_window((nz, nx))] * 120, src, [rec1] * 120,
                    np.tile(w, (120, 1)))


def config3(seed: int = 3, nt: int = 4000, nshot: int = 256) -> Workload:
    """Uneven apertures: the config-2 model with 256 shots, each on its own
    window of width U{200..737} centred on a seeded source position."""
    base = config2(seed=2, nt=nt)
    nz, nx = base.n
    rng = np.random.default_rng(seed)
    win, src, rec = [], [], []
    for _ in range(nshot):
        sx = int(rng.integers(0, nx))
        w = int(rng.integers(200, nx + 1))
        x0 = min(max(sx - w // 2, 0), nx - w)
        win.append(((0, nz), (x0, x0 + w)))
        src.append((2, sx))
        rx = np.arange(x0, x0 + w, 2)
        rec.append(np.stack([np.full(len(rx), 2), rx], axis=1))
    w = ricker(base.f0, nt, base.dt).astype(F32)
    return Workload("config3: 2D uneven apertures, 256 shots", base.h, base.dt, nt, 20,
                    base.f0, base.lnvp, base.lnip, base.dm, win, src, rec,
                    np.tile(w, (nshot, 1)))


def config4(seed: int = 4, nt: int = 3000) -> Workload:
    """Autograd workload: 480 x 160 at 12.5 m, 32 shots, receivers every 2nd
    node, nt = 3000, 15 Hz."""
    nz, nx, h = 160, 480, 12.5
    vp = faulted_layered(nz, nx, h, seed)
    rho = gardner(vp)
    vp0, rho0 = _smooth_background(vp, rho, 250.0 / h)
    lnvp, lnip = _logs(vp0, rho0)
    dm = _perturbation(vp, rho, vp0, rho0)
    f0, dt = 15.0, 1e-3
    xs = np.linspace(8, nx - 9, 32).round().astype(int)
    src = [(2, int(x)) for x in xs]
    rec1 = np.stack([np.full(nx // 2, 2), np.arange(0, nx, 2)], axis=1)
    w = ricker(f0, nt, dt).astype(F32)
    return Workload("config4: 2D 480x160, 32 shots", (h, h), dt, nt, 20, f0, lnvp, lnip, dm,
                    [_full_window((nz, nx))] * 32, src, [rec1] * 32, np.tile(w, (32, 1)))


def dipping_salt_3d(nz, nx, ny, h, seed, vmin=1500.0, vmax=4500.0, nlayers=8):
    """Vp (ny, nx, nz): seeded dipping layers plus a Gaussian high-velocity
    body (vmax where exp(-r^2 / 2 sigma^2) > 1/2, sigma = 600 m, centred at
    (x, y, z) = (2.5, 2.5, 1.2) km)."""
    rng = np.random.default_rng(seed)
    z = np.arange(nz) * h
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    Y, X, Z = np.meshgrid(y, x, z, indexing="ij")
    zmax = nz * h
    depths = np.sort(rng.uniform(0.05 * zmax, 0.95 * zmax, nlayers - 1))
    sx = rng.uniform(-0.1, 0.1, nlayers - 1)
    sy = rng.uniform(-0.1, 0.1, nlayers - 1)
    vel = np.sort(rng.uniform(vmin, vmax * 0.9, nlayers))
    vel[0] = vmin
    xc, yc = x.mean(), y.mean()
    layer = np.zeros(Z.shape, dtype=np.int64)
    for k in range(nlayers - 1):
        iface = depths[k] + sx[k] * (X - xc) + sy[k] * (Y - yc)
        layer += (Z > iface).astype(np.int64)
    vp = vel[layer]
    r2 = (X - 2500.0) ** 2 + (Y - 2500.0) ** 2 + (Z - 1200.0) ** 2
    vp = np.where(np.exp(-r2 / (2 * 600.0 ** 2)) > 0.5, vmax, vp)
    return vp


def config5(seed: int = 5, nt: int = 2500, n=(200, 400, 400)) -> Workload:
    """3D: 400 x 400 x 200 (x, y, z) at 12.5 m, 16 shots on a 4x4 lattice at
    iz = 2, 80 x 80 receivers every 5 nodes, 20 Hz, nt = 2500."""
    nz, nx, ny = n
    h = 12.5
    vp = dipping_salt_3d(nz, nx, ny, h, seed)
    rho = gardner(vp)
    vp0, rho0 = _smooth_background(vp, rho, 250.0 / h)
    lnvp, lnip = _logs(vp0, rho0)
    dm = _perturbation(vp, rho, vp0, rho0)
    del vp, rho, vp0, rho0
    f0, dt = 20.0, 1e-3
    lat_x = [int(round(nx * (2 * k + 1) / 8)) for k in range(4)]
    lat_y = [int(round(ny * (2 * k + 1) / 8)) for k in range(4)]
    src = [(2, ix, iy) for iy in lat_y for ix in lat_x]
    rx, ry = np.meshgrid(np.arange(0, nx, 5), np.arange(0, ny, 5), indexing="xy")
    rec1 = np.stack([np.full(rx.size, 2), rx.ravel(), ry.ravel()], axis=1)
    w = ricker(f0, nt, dt).astype(F32)
    return Workload("config5: 3D 400x400x200, 16 shots", (h, h, h), dt, nt, 20, f0,
                    lnvp, lnip, dm, [_full_window((nz, nx, ny))] * 16, src, [rec1] * 16,
                    np.tile(w, (16, 1)))


# ---------------------------------------------------------------------------
# Small seeded problems for parity and edge-case tests
# ---------------------------------------------------------------------------
def small(n, h=10.0, nt=120, dt=1e-3, npml=6, f0=15.0, seed=0, nshot=1,
          nrec=None, uneven=False, vmin=1800.0, vmax=2600.0) -> Workload:
    """A seeded random smooth medium on a small grid (2D if len(n) == 2).

    n = (nz, nx[, ny]).  Velocity and density are smooth random fields so
    that every stencil term is exercised; dm is white noise.  With uneven=True
    each shot gets its own x-window of seeded width.
    """
    rng = np.random.default_rng(seed)
    ndim = len(n)
    shape = tuple(reversed(n))
    vp = gaussian_filter(rng.standard_normal(shape), 2.0, mode="wrap")
    vp = vmin + (vmax - vmin) * (vp - vp.min()) / max(np.ptp(vp), 1e-12)
    rho = gaussian_filter(1800.0 + 400.0 * rng.standard_normal(shape), 2.0, mode="wrap")
    lnvp, lnip = _logs(vp, rho)
    dm = (0.05 * rng.standard_normal((2,) + shape)).astype(F32)
    win, src, rec = [], [], []
    for s in range(nshot):
        if uneven and ndim >= 2:
            w = int(rng.integers(max(4, n[1] // 2), n[1] + 1))
            x0 = int(rng.integers(0, n[1] - w + 1))
        else:
            w, x0 = n[1], 0
        wz = [(0, n[0]), (x0, x0 + w)] + ([(0, n[2])] if ndim == 3 else [])
        win.append(tuple(wz))
        c = [int(rng.integers(0, min(3, n[0]))), int(rng.integers(x0, x0 + w))]
        if ndim == 3:
            c.append(int(rng.integers(0, n[2])))
        src.append(tuple(c))
        m = nrec if nrec is not None else max(1, w // 2)
        rz = rng.integers(0, n[0], m)
        rx = rng.integers(x0, x0 + w, m)
        cols = [rz, rx] + ([rng.integers(0, n[2], m)] if ndim == 3 else [])
        rec.append(np.stack(cols, axis=1))
    wav = np.stack([ricker(f0 * (1 + 0.1 * s), nt, dt) for s in range(nshot)]).astype(F32)
    return Workload(f"small {n}", tuple([h] * ndim), dt, nt, npml, f0, lnvp, lnip, dm,
                    win, src, rec, wav)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
