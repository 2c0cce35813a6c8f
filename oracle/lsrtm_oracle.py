"""FP64 CPU oracle for the data-domain LSRTM hot path (lnVp-lnIp parametrisation).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
constant generator with the HIP library; both sides receive the same seeded
inputs (model logs, acquisition, wavelet samples) and nothing else.

What is computed, and where the paper defines it (Yang & Ji, "A comparative
study of data- and image-domain LSRTM under velocity-impedance
parametrization"):

* The first-order velocity-pressure system A(m)u = f (section 2, first
  equation): rho dv/dt + grad p = f_v, kappa div v + dp/dt = f_p.
* The log parameters lnrho = lnIp - lnVp, lnkappa = lnIp + lnVp (section 2,
  relation after eq. ln).
* The Born scattering system with the lnVp/lnIp secondary sources
  -(dm2 - dm1) rho dv/dt and -(dm2 + dm1) kappa div v (section 2,
  eq. scattereqln), recorded by the restriction R (section 3, misfit J).
* The adjoint L^H of Born modelling, built matrix-free by the adjoint-state
  method (appendix A, eqs. adjeq, gradlsm, gradrho, gradkappa) and mapped to
  (lnVp, lnIp) by the gradient chain rule (section 3, the pair of equations
  after eq. normal).
* CGNR on the normal equations L^H L dm = L^H dd (section 3, eq. normal and
  the CGNR paragraph), and its preconditioned form with the pseudo-Hessian
  diagonal of appendix B.
* Image-domain LSRTM with the point-spread-function Hessian (section 3,
  eq. migdeconobj; appendix C, eq. trilinear): PSF images of a scatterer
  lattice, the interpolated banded Hessian, mono- and multiparameter.
* Nonstationary Wiener deblurring (appendix D, eq. sol and the regularised
  least-squares estimate of the inverse eigenvalues): local blocks, Fourier
  transforms, overlap-add with valences.
* The nonlinear-residual data preparation (section 4.1): a top mute of the
  direct arrival on observed-minus-background data.

The paper gives the continuous equations only.  The discrete scheme below is
one explicit reading of them (all readings are listed in the design notes of
the repository): Virieux staggering with an O(2,8) half-offset stencil, a
recursive-convolution CPML, a pressure point source injected with the
midpoint rule, and the exact discrete transpose as the adjoint.  Every
operation follows the definition directly; there is no blocking, fusion or
reordering.  All arithmetic is in the dtype of the inputs (float64, or
complex128 for the complex-step check).

Array convention: physical arrays have shape (nx, nz) in 2D and (ny, nx, nz)
in 3D, so z is the fastest (last) numpy axis.  Axis index ``a`` = 0 is z,
1 is x, 2 is y; its numpy axis is ``ndim - 1 - a``.  Node coordinates are
given as (iz, ix[, iy]).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import Callable, List, Optional, Sequence

import numpy as np

HALF = 4  # half-width of the O(2,8) staggered stencil


# ---------------------------------------------------------------------------
# O(2,8) staggered first derivative
# ---------------------------------------------------------------------------
def fd_coefficients(half_width: int = HALF) -> List[Fraction]:
    """Exact coefficients c_1..c_M of the staggered first derivative.

    f'(x) ~ sum_k c_k [f(x + (k-1/2)h) - f(x - (k-1/2)h)] / h.  Matching the
    Taylor series of both sides gives sum_k c_k (2k-1) = 1 and
    sum_k c_k (2k-1)^(2m+1) = 0 for m = 1..M-1; the system is solved in exact
    rational arithmetic.
    """
    M = half_width
    A = [[Fraction(2 * k - 1) ** (2 * m + 1) for k in range(1, M + 1)] for m in range(M)]
    b = [Fraction(1 if m == 0 else 0) for m in range(M)]
    # Gauss-Jordan elimination over the rationals
    for col in range(M):
        piv = next(r for r in range(col, M) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(M):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] = b[r] - f * b[col]
    return [b[i] / A[i][i] for i in range(M)]


COEF = tuple(float(c) for c in fd_coefficients(HALF))


def _nax(ndim: int, a: int) -> int:
    return ndim - 1 - a


def _zero_pad(f: np.ndarray, ax: int, w: int) -> np.ndarray:
    pad = [(0, 0)] * f.ndim
    pad[ax] = (w, w)
    return np.pad(f, pad)


def _take(fp: np.ndarray, ax: int, start: int, n: int) -> np.ndarray:
    sl = [slice(None)] * fp.ndim
    sl[ax] = slice(start, start + n)
    return fp[tuple(sl)]


def op_G(f: np.ndarray, a: int, h: float) -> np.ndarray:
    """Forward staggered derivative along axis a, node -> half node.

    (G f)[i] = sum_k c_k (f[i+k] - f[i-k+1]) / h lives at i + 1/2; values
    outside the array are zero.
    """
    ax = _nax(f.ndim, a)
    n = f.shape[ax]
    fp = _zero_pad(f, ax, HALF)
    out = np.zeros_like(f)
    for k, c in enumerate(COEF, start=1):
        out = out + c * (_take(fp, ax, HALF + k, n) - _take(fp, ax, HALF - k + 1, n))
    return out / h


def op_D(g: np.ndarray, a: int, h: float) -> np.ndarray:
    """Backward staggered derivative along axis a, half node -> node.

    (D g)[i] = sum_k c_k (g[i+k-1] - g[i-k]) / h lives at node i; g[j] is the
    value at j + 1/2 and values outside the array are zero.
    """
    ax = _nax(g.ndim, a)
    n = g.shape[ax]
    gp = _zero_pad(g, ax, HALF)
    out = np.zeros_like(g)
    for k, c in enumerate(COEF, start=1):
        out = out + c * (_take(gp, ax, HALF + k - 1, n) - _take(gp, ax, HALF - k, n))
    return out / h


def _next_clamped(f: np.ndarray, a: int) -> np.ndarray:
    """f[min(i+1, n-1)] along axis a."""
    ax = _nax(f.ndim, a)
    n = f.shape[ax]
    idx = np.minimum(np.arange(n) + 1, n - 1)
    return np.take(f, idx, axis=ax)


def avg_half(f: np.ndarray, a: int) -> np.ndarray:
    """Mean of the two nodes around half node i+1/2 (last node clamped)."""
    return 0.5 * (f + _next_clamped(f, a))


def avg_half_T(x: np.ndarray, a: int) -> np.ndarray:
    """Exact transpose of avg_half: node i collects half of every half-node
    value that averaged it (the clamped last node collects both halves)."""
    ax = _nax(x.ndim, a)
    n = x.shape[ax]
    out = 0.5 * x
    idx = np.minimum(np.arange(n) + 1, n - 1)
    # scatter 0.5*x[i] onto node min(i+1, n-1)
    moved = np.zeros_like(x)
    xs = np.moveaxis(0.5 * x, ax, 0)
    ms = np.moveaxis(moved, ax, 0)
    for i in range(n):
        ms[idx[i]] = ms[idx[i]] + xs[i]
    return out + np.moveaxis(ms, 0, ax)


# ---------------------------------------------------------------------------
# Medium: logs -> kappa and buoyancy, CPML tables
# ---------------------------------------------------------------------------
def pad_edge(a: np.ndarray, npml: int) -> np.ndarray:
    """Physical grid -> padded grid, model values replicated into the PML."""
    return np.pad(a, npml, mode="edge")


def pad_zero(a: np.ndarray, npml: int) -> np.ndarray:
    """Physical grid -> padded grid, zero in the PML (perturbations)."""
    return np.pad(a, npml)


def log_params(lnvp: np.ndarray, lnip: np.ndarray):
    """lnrho = lnIp - lnVp, lnkappa = lnIp + lnVp (section 2)."""
    return lnip - lnvp, lnip + lnvp


@dataclass
class CPML:
    """Per-axis recursive-convolution coefficients (ac, bc) at half nodes
    (used with G p) and at nodes (used with D v), shaped to broadcast."""
    ach: list
    bch: list
    aci: list
    bci: list


def cpml_profile(n_pad: int, npml: int, h: float, dt: float, vmax: float,
                 R: float, f0: float, half: bool):
    """1D C-PML coefficients along one axis.

    xi = distance past the last physical node / (npml h), clipped to [0, 1];
    d = d0 xi^2 with d0 = -3 vmax ln(R) / (2 npml h); alpha = pi f0 (1 - xi);
    bc = exp(-(d + alpha) dt); ac = d (bc - 1) / (d + alpha), 0 where d = 0.
    """
    if npml == 0:
        return np.zeros(n_pad), np.ones(n_pad)
    pos = np.arange(n_pad, dtype=np.float64) + (0.5 if half else 0.0)
    first, last = npml, n_pad - npml - 1
    dist = np.where(pos < first, first - pos, np.where(pos > last, pos - last, 0.0))
    xi = np.clip(dist / npml, 0.0, 1.0)
    d0 = -3.0 * vmax * np.log(R) / (2.0 * npml * h)
    d = d0 * xi ** 2
    alpha = np.pi * f0 * (1.0 - xi)
    bc = np.exp(-(d + alpha) * dt)
    with np.errstate(invalid="ignore", divide="ignore"):
        ac = np.where(d > 0.0, d * (bc - 1.0) / (d + alpha), 0.0)
    return ac, bc


@dataclass
class Medium:
    """Background medium of one shot on its padded grid."""
    ndim: int
    h: tuple
    dt: float
    kappa: np.ndarray
    b: list          # buoyancy at half nodes, one array per axis
    cpml: CPML
    shape: tuple

    @property
    def cell(self) -> float:
        return float(np.prod(self.h))


def make_medium(lnvp_pad, lnip_pad, h, dt, npml, vmax, R, f0) -> Medium:
    """kappa at nodes and b_a = exp(-(lnrho_i + lnrho_{i+1})/2) at half nodes."""
    ndim = lnvp_pad.ndim
    lnr, lnk = log_params(lnvp_pad, lnip_pad)
    kappa = np.exp(lnk)
    b = [np.exp(-avg_half(lnr, a)) for a in range(ndim)]
    ach, bch, aci, bci = [], [], [], []
    for a in range(ndim):
        ax = _nax(ndim, a)
        n = lnvp_pad.shape[ax]
        shp = [1] * ndim
        shp[ax] = n
        for half, (la, lb) in ((True, (ach, bch)), (False, (aci, bci))):
            ac, bc = cpml_profile(n, npml, h[a], dt, vmax, R, f0, half)
            la.append(ac.reshape(shp))
            lb.append(bc.reshape(shp))
    return Medium(ndim, tuple(h), dt, kappa, b, CPML(ach, bch, aci, bci), lnvp_pad.shape)


# ---------------------------------------------------------------------------
# One time step of the background and scattered systems
# ---------------------------------------------------------------------------
@dataclass
class State:
    p: np.ndarray
    v: list
    psi: list   # CPML memory of G_a p (half nodes)
    phi: list   # CPML memory of D_a v_a (nodes)

    @staticmethod
    def zeros(shape, ndim, dtype=np.float64) -> "State":
        z = lambda: np.zeros(shape, dtype=dtype)
        return State(z(), [z() for _ in range(ndim)], [z() for _ in range(ndim)],
                     [z() for _ in range(ndim)])

    def copy(self) -> "State":
        return State(self.p.copy(), [x.copy() for x in self.v],
                     [x.copy() for x in self.psi], [x.copy() for x in self.phi])


def step_background(st: State, med: Medium, src_idx, src_amp):
    """Advance the background field by one step (leapfrog, section 2 first
    equation).  Returns the velocity increments dv_a and the CPML-corrected
    divergence q of this step, the two quantities the Born sources and the
    imaging condition use.

    v_a <- v_a - dt b_a (G_a p + psi_a);  p <- p - dt kappa q + dt s/cell.
    """
    dv = []
    for a in range(med.ndim):
        g = op_G(st.p, a, med.h[a])
        st.psi[a] = med.cpml.bch[a] * st.psi[a] + med.cpml.ach[a] * g
        inc = -med.dt * med.b[a] * (g + st.psi[a])
        st.v[a] = st.v[a] + inc
        dv.append(inc)
    q = 0.0
    for a in range(med.ndim):
        e = op_D(st.v[a], a, med.h[a])
        st.phi[a] = med.cpml.bci[a] * st.phi[a] + med.cpml.aci[a] * e
        q = q + e + st.phi[a]
    st.p = st.p - med.dt * med.kappa * q
    if src_idx is not None:
        st.p[src_idx] = st.p[src_idx] + med.dt * src_amp / med.cell
    return dv, q


def step_scattered(sc: State, med: Medium, dv, q, rbar, dlnk):
    """Advance the scattered field by one step with the Born sources of
    eq. scattereqln: -(dm2-dm1) rho dv/dt enters as -avg(dlnrho) * dv_a and
    -(dm2+dm1) kappa div v as dlnkappa * (-dt kappa q)."""
    for a in range(med.ndim):
        g = op_G(sc.p, a, med.h[a])
        sc.psi[a] = med.cpml.bch[a] * sc.psi[a] + med.cpml.ach[a] * g
        sc.v[a] = sc.v[a] - med.dt * med.b[a] * (g + sc.psi[a])
        sc.v[a] = sc.v[a] - rbar[a] * dv[a]
    dq = 0.0
    for a in range(med.ndim):
        e = op_D(sc.v[a], a, med.h[a])
        sc.phi[a] = med.cpml.bci[a] * sc.phi[a] + med.cpml.aci[a] * e
        dq = dq + e + sc.phi[a]
    sc.p = sc.p - med.dt * med.kappa * dq
    sc.p = sc.p + dlnk * (-med.dt * med.kappa * q)


# ---------------------------------------------------------------------------
# Single-shot operators on the padded grid
# ---------------------------------------------------------------------------
def _rec_gather(p: np.ndarray, rec_idx):
    return p[rec_idx]


def forward_shot(med: Medium, src_idx, rec_idx, wav: np.ndarray, nt: int,
                 keep_history: bool = False):
    """Background data d[n, r] = p^{n+1}(receiver r)."""
    st = State.zeros(med.shape, med.ndim, np.result_type(med.kappa, np.float64))
    nrec = len(rec_idx[0]) if rec_idx else 0
    d = np.zeros((nt, nrec), dtype=st.p.dtype)
    hist = [] if keep_history else None
    for n in range(nt):
        dv, q = step_background(st, med, src_idx, wav[n])
        if keep_history:
            hist.append((dv, q))
        d[n] = _rec_gather(st.p, rec_idx)
    return d, hist


def born_shot(med: Medium, src_idx, rec_idx, wav: np.ndarray, nt: int,
              dlnr_pad: np.ndarray, dlnk_pad: np.ndarray):
    """Born data dd = R du (section 3, L[m0] dm := R du) and background data."""
    dtype = np.result_type(med.kappa, dlnr_pad, np.float64)
    st = State.zeros(med.shape, med.ndim, dtype)
    sc = State.zeros(med.shape, med.ndim, dtype)
    rbar = [avg_half(dlnr_pad, a) for a in range(med.ndim)]
    nrec = len(rec_idx[0])
    d0 = np.zeros((nt, nrec), dtype=dtype)
    dd = np.zeros((nt, nrec), dtype=dtype)
    for n in range(nt):
        dv, q = step_background(st, med, src_idx, wav[n])
        step_scattered(sc, med, dv, q, rbar, dlnk_pad)
        d0[n] = _rec_gather(st.p, rec_idx)
        dd[n] = _rec_gather(sc.p, rec_idx)
    return dd, d0


def round_significand(x: np.ndarray, bits: int) -> np.ndarray:
    """x rounded to the nearest number with `bits` significant bits, ties to
    even (no exponent limits)."""
    m, e = np.frexp(x)
    return np.ldexp(np.rint(np.ldexp(m, bits)), e - bits)


def compress_field(x: np.ndarray, dtype: str) -> np.ndarray:
    """One stored-and-restored snapshot field (appendix A names compression
    as a way to keep the background history; the format is a reading): the
    field is divided by a per-snapshot scale s, rounded to nearest with ties
    to even, and multiplied by s again.

    f16 : s = max|x| / 2^14, IEEE binary16 (11 significant bits, spacing
          2^-24 below 2^-14), the conversion numpy implements;
    bf16: s = max|x|, 8 significant bits (bfloat16; values below 2^-126 of
          max|x|, which bfloat16 would hold as subnormals, are kept at 8 bits);
    f64 : unchanged.  A zero field stays zero."""
    if dtype in ("f64", "f32"):
        return x.copy()
    mx = float(np.max(np.abs(x))) if x.size else 0.0
    if mx == 0.0:
        return np.zeros_like(x)
    if dtype == "f16":
        s = mx / 2.0 ** 14
        return (x / s).astype(np.float16).astype(np.float64) * s
    if dtype == "bf16":
        s = mx
        return round_significand(x / s, 8) * s
    raise ValueError(dtype)


def background_history(med: Medium, src_idx, wav, nt, ckpt_every: int = 0,
                       ckpt_dtype: str = "f64"):
    """Source-side quantities (dv^n, q^n) for n = 0..nt-1, served in reverse.

    With ckpt_every = 0 the whole history is stored.  Otherwise the state is
    stored every ckpt_every steps and each segment is recomputed on demand;
    in FP64 the recomputation repeats the same operations, so it returns the
    same numbers as storing everything.  With ckpt_dtype "f16" or "bf16" the
    pressure and velocities of every stored state go through compress_field
    (the CPML memories are kept exactly), so the replayed history is that of
    compressed snapshots.
    """
    if ckpt_every <= 0:
        st = State.zeros(med.shape, med.ndim, np.result_type(med.kappa, np.float64))
        hist = []
        for n in range(nt):
            hist.append(step_background(st, med, src_idx, wav[n]))
        return lambda n: hist[n]
    ckpts = {}
    st = State.zeros(med.shape, med.ndim, np.result_type(med.kappa, np.float64))
    for n in range(nt):
        if n % ckpt_every == 0:
            c = st.copy()
            c.p = compress_field(c.p, ckpt_dtype)
            c.v = [compress_field(v, ckpt_dtype) for v in c.v]
            ckpts[n] = c
        step_background(st, med, src_idx, wav[n])
    cache = {"seg": None, "vals": None}

    def get(n):
        s0 = (n // ckpt_every) * ckpt_every
        if cache["seg"] != s0:
            s = ckpts[s0].copy()
            vals = []
            for m in range(s0, min(s0 + ckpt_every, nt)):
                vals.append(step_background(s, med, src_idx, wav[m]))
            cache["seg"], cache["vals"] = s0, vals
        return cache["vals"][n - s0]
    return get


def adjoint_shot(med: Medium, src_idx, rec_idx, wav: np.ndarray, nt: int,
                 y: np.ndarray, ckpt_every: int = 0, ckpt_dtype: str = "f64"):
    """Exact discrete transpose of born_shot, y -> (g_lnrho, g_lnkappa).

    Appendix A derives the adjoint-state gradient: the adjoint field runs
    backwards in time driven by the data (eq. adjeq) and is cross-correlated
    with the background field (eqs. gradlsm, gradrho, gradkappa).  Here every
    update of step_background/step_scattered is transposed in reverse order,
    so <L x, y> = <x, L^T y> holds to rounding; in the interior the adjoint
    recursion is the paper's compliance form (appendix A, the equation after
    eq. adjnotused) run backwards.
    """
    hist = background_history(med, src_idx, wav, nt, ckpt_every, ckpt_dtype)
    dtype = np.result_type(med.kappa, y, np.float64)
    pt = np.zeros(med.shape, dtype=dtype)            # adjoint of dp
    vt = [np.zeros(med.shape, dtype=dtype) for _ in range(med.ndim)]   # of dv_a
    chi = [np.zeros(med.shape, dtype=dtype) for _ in range(med.ndim)]  # of dpsi_a
    vphi = [np.zeros(med.shape, dtype=dtype) for _ in range(med.ndim)]  # of dphi_a
    g_rbar = [np.zeros(med.shape, dtype=dtype) for _ in range(med.ndim)]
    g_k = np.zeros(med.shape, dtype=dtype)
    for n in range(nt - 1, -1, -1):
        dv, q = hist(n)
        # transpose of the receiver restriction
        np.add.at(pt, rec_idx, y[n])
        # transpose of dp <- dp - dt kappa dq + dlnk (-dt kappa q)
        g_k = g_k + (-med.dt * med.kappa * q) * pt
        qt = -med.dt * med.kappa * pt
        # transpose of dq = sum_a (e_a + phi_a), phi_a <- bci phi_a + aci e_a,
        # e_a = D_a dv_a
        for a in range(med.ndim):
            vphi[a] = vphi[a] + qt
            et = qt + med.cpml.aci[a] * vphi[a]
            vphi[a] = med.cpml.bci[a] * vphi[a]
            vt[a] = vt[a] - op_G(et, a, med.h[a])          # D_a^T = -G_a
        # transpose of dv_a <- dv_a - dt b_a (g_a + psi_a) - rbar_a dv_a,
        # psi_a <- bch psi_a + ach g_a, g_a = G_a dp
        for a in range(med.ndim):
            g_rbar[a] = g_rbar[a] + (-dv[a]) * vt[a]
            ht = -med.dt * med.b[a] * vt[a]
            chi[a] = chi[a] + ht
            gt = ht + med.cpml.ach[a] * chi[a]
            chi[a] = med.cpml.bch[a] * chi[a]
            pt = pt - op_D(gt, a, med.h[a])                # G_a^T = -D_a
    g_r = 0.0
    for a in range(med.ndim):
        g_r = g_r + avg_half_T(g_rbar[a], a)
    return g_r, g_k


# ---------------------------------------------------------------------------
# Multi-shot problem on a global physical grid
# ---------------------------------------------------------------------------
@dataclass
class Problem:
    """Global physical grid, time axis, CPML reading and acquisition.

    win[s]   : ((z0, z1), (x0, x1)[, (y0, y1)]) physical window of shot s
    src[s]   : (iz, ix[, iy]) global physical node of the pressure source
    rec[s]   : int array (nrec_s, ndim) global physical receiver nodes
    wavelet  : (nshot, nt) source samples w((n + 1/2) dt)
    """
    h: tuple
    dt: float
    nt: int
    npml: int
    pml_R: float
    pml_f0: float
    win: list
    src: list
    rec: list
    wavelet: np.ndarray

    @property
    def ndim(self) -> int:
        return len(self.h)

    @property
    def nshot(self) -> int:
        return len(self.src)


def _window_slices(win, ndim):
    # numpy axis order is (y, x, z); win is given as (z, x[, y])
    return tuple(slice(win[a][0], win[a][1]) for a in reversed(range(ndim)))


def _np_index(coords, ndim):
    """(iz, ix[, iy]) coordinates (arrays allowed) -> numpy index tuple."""
    return tuple(coords[a] for a in reversed(range(ndim)))


def shot_setup(prob: Problem, lnvp: np.ndarray, lnip: np.ndarray, s: int,
               vmax: Optional[float] = None):
    """Medium and padded-grid source/receiver indices of shot s."""
    ndim = prob.ndim
    npml = prob.npml
    win = prob.win[s]
    sl = _window_slices(win, ndim)
    if vmax is None:
        vmax = float(np.exp(np.max(np.real(lnvp))))
    med = make_medium(pad_edge(lnvp[sl], npml), pad_edge(lnip[sl], npml),
                      prob.h, prob.dt, npml, vmax, prob.pml_R, prob.pml_f0)
    off = [win[a][0] - npml for a in range(ndim)]
    src = tuple(int(prob.src[s][a] - off[a]) for a in range(ndim))
    rec = np.asarray(prob.rec[s], dtype=np.int64).reshape(-1, ndim)
    rc = [rec[:, a] - off[a] for a in range(ndim)]
    return med, _np_index(src, ndim), _np_index(rc, ndim), sl


def forward(prob: Problem, lnvp, lnip) -> List[np.ndarray]:
    """Background data of every shot, each (nt, nrec_s)."""
    out = []
    for s in range(prob.nshot):
        med, si, ri, _ = shot_setup(prob, lnvp, lnip, s)
        out.append(forward_shot(med, si, ri, prob.wavelet[s], prob.nt)[0])
    return out


def born(prob: Problem, lnvp, lnip, dm) -> List[np.ndarray]:
    """L dm for every shot; dm = (dlnVp, dlnIp) on the physical grid,
    zero-extended into the PML."""
    out = []
    vmax = float(np.exp(np.max(np.real(lnvp))))
    for s in range(prob.nshot):
        med, si, ri, sl = shot_setup(prob, lnvp, lnip, s, vmax)
        dlnr, dlnk = log_params(dm[0][sl], dm[1][sl])
        dd, _ = born_shot(med, si, ri, prob.wavelet[s], prob.nt,
                          pad_zero(dlnr, prob.npml), pad_zero(dlnk, prob.npml))
        out.append(dd)
    return out


def adjoint(prob: Problem, lnvp, lnip, ys: Sequence[np.ndarray],
            ckpt_every: int = 0, ckpt_dtype: str = "f64") -> np.ndarray:
    """L^T y summed over shots: image (2, *physical shape) = (lnVp, lnIp).

    Per shot, g_lnrho and g_lnkappa are mapped with the gradient chain rule
    of section 3: g_lnVp = -g_lnrho + g_lnkappa, g_lnIp = g_lnrho + g_lnkappa,
    restricted to the window's physical nodes and added into the global image
    (the reduction over shots of the paper's shot-parallel layer)."""
    ndim = prob.ndim
    img = np.zeros((2,) + lnvp.shape, dtype=np.result_type(ys[0], np.float64))
    vmax = float(np.exp(np.max(np.real(lnvp))))
    inner = tuple(slice(prob.npml, -prob.npml) if prob.npml > 0 else slice(None)
                  for _ in range(ndim))
    for s in range(prob.nshot):
        med, si, ri, sl = shot_setup(prob, lnvp, lnip, s, vmax)
        g_r, g_k = adjoint_shot(med, si, ri, prob.wavelet[s], prob.nt, ys[s], ckpt_every, ckpt_dtype)
        img[0][sl] += (-g_r + g_k)[inner]
        img[1][sl] += (g_r + g_k)[inner]
    return img


# ---------------------------------------------------------------------------
# CGNR (section 3, CGNR paragraph) in FP64
# ---------------------------------------------------------------------------
def cgnr(L: Callable, Lt: Callable, d, niter: int, dot: Optional[Callable] = None):
    """Conjugate gradients on the normal equations L^T L x = L^T d, x0 = 0.

    Returns x and the normalised misfit history ||r_k||^2 / ||r_0||^2.
    The vectors may be numpy arrays or lists of arrays (per-shot data).
    """
    if dot is None:
        def dot(a, b):
            if isinstance(a, (list, tuple)):
                return float(sum(np.vdot(x, y).real for x, y in zip(a, b)))
            return float(np.vdot(a, b).real)

    def axpy(alpha, x, y):
        if isinstance(x, (list, tuple)):
            return [yy + alpha * xx for xx, yy in zip(x, y)]
        return y + alpha * x

    r = [x.copy() for x in d] if isinstance(d, (list, tuple)) else d.copy()
    z = Lt(r)
    p = z.copy()
    x = np.zeros_like(z)
    zz = dot(z, z)
    r0 = dot(r, r)
    hist = [1.0]
    for _ in range(niter):
        w = L(p)
        alpha = zz / dot(w, w)
        x = x + alpha * p
        r = axpy(-alpha, w, r)
        z = Lt(r)
        zz_new = dot(z, z)
        beta = zz_new / zz
        p = z + beta * p
        zz = zz_new
        hist.append(dot(r, r) / r0)
    return x, hist


# ---------------------------------------------------------------------------
# Pseudo-Hessian preconditioner (appendix B) and preconditioned CGNR
# ---------------------------------------------------------------------------
def _avg_sq_T(x: np.ndarray, a: int) -> np.ndarray:
    """Transpose of the squared weights of avg_half: node i collects 1/4 of
    the half-node values i - 1/2 and i + 1/2; the clamped last half node
    averages the last node with itself (weight 1, squared 1)."""
    ax = _nax(x.ndim, a)
    n = x.shape[ax]
    xs = np.moveaxis(x, ax, 0)
    out = 0.25 * xs
    out[1:] = out[1:] + 0.25 * xs[:-1]
    out[n - 1] = out[n - 1] + 0.75 * xs[n - 1]
    return np.moveaxis(out, 0, ax)


def pseudo_hessian_shot(med: Medium, src_idx, wav: np.ndarray, nt: int):
    """Pseudo-Hessian diagonal of one shot on its padded grid (appendix B).

    The paper replaces diag(L^H L) by the time-integrated energy of the Born
    secondary source that a unit perturbation creates in the incident field,
    (dA/dm u0)^H (dA/dm u0): rho^2 int |dv/dt|^2 dt for lnrho and
    kappa^2 int (div v)^2 dt for lnkappa.  Discrete reading: the sources are
    the ones of the Born step (step_scattered) -- a unit dlnrho at node i adds
    -avg_a(e_i) dv_a to the velocities, a unit dlnkappa adds -dt kappa q at
    node i to the pressure -- and the time integral of a squared rate is the
    sum over steps of the squared increment divided by dt, the velocity
    source weighted by rho^2 as in the paper:

      H_lnrho[i]   = rho_i^2 / dt * sum_n sum_a || avg_a(e_i) * dv_a^n ||^2
      H_lnkappa[i] = 1 / dt * sum_n (dt kappa_i q_i^n)^2

    Returns (H_lnrho / (rho^2 / dt), H_lnkappa) on the padded grid: the
    density entry without its rho^2 / dt factor, which the caller applies
    from the model."""
    st = State.zeros(med.shape, med.ndim, np.result_type(med.kappa, np.float64))
    s_v = [np.zeros(med.shape, dtype=st.p.dtype) for _ in range(med.ndim)]
    s_q = np.zeros(med.shape, dtype=st.p.dtype)
    for n in range(nt):
        dv, q = step_background(st, med, src_idx, wav[n])
        for a in range(med.ndim):
            s_v[a] = s_v[a] + dv[a] * dv[a]
        s_q = s_q + q * q
    h_r = 0.0
    for a in range(med.ndim):
        h_r = h_r + _avg_sq_T(s_v[a], a)
    h_k = (med.dt * med.kappa) ** 2 * s_q / med.dt
    return h_r, h_k


def pseudo_hessian(prob: Problem, lnvp, lnip) -> np.ndarray:
    """Pseudo-Hessian diagonal for (lnVp, lnIp), summed over shots (appendix
    B): the chain rule of section 3 makes both diagonal entries equal,
    H_lnVp = H_lnIp = H_lnrho + H_lnkappa.  Returns one array of the physical
    shape (the diagonal for either parameter)."""
    ndim = prob.ndim
    out = np.zeros(lnvp.shape, dtype=np.float64)
    vmax = float(np.exp(np.max(np.real(lnvp))))
    inner = tuple(slice(prob.npml, -prob.npml) if prob.npml > 0 else slice(None)
                  for _ in range(ndim))
    for s in range(prob.nshot):
        med, si, _, sl = shot_setup(prob, lnvp, lnip, s, vmax)
        h_r, h_k = pseudo_hessian_shot(med, si, prob.wavelet[s], prob.nt)
        lnr, _ = log_params(pad_edge(lnvp[sl], prob.npml), pad_edge(lnip[sl], prob.npml))
        rho2 = np.exp(2.0 * lnr)
        out[sl] += (rho2 * h_r / med.dt + h_k)[inner]
    return out


def preconditioner(h: np.ndarray, eps_rel: float = 1e-3) -> np.ndarray:
    """Diagonal inverse 1 / (H + eps) for both parameters, eps = eps_rel *
    max H (the paper leaves the stabilisation unstated; this is the reading
    used throughout).  Shape (2, *h.shape)."""
    eps = eps_rel * float(np.max(h)) if h.size else 0.0
    m = 1.0 / (h + eps)
    return np.stack([m, m])


def pcgnr(L: Callable, Lt: Callable, d, niter: int, minv, dot: Optional[Callable] = None):
    """Preconditioned CGNR (section 3: CGNR with the pseudo-Hessian
    preconditioner of appendix B): conjugate gradients on the normal
    equations L^T L x = L^T d in which the normal residual s = L^T r is
    preconditioned by the diagonal minv, x0 = 0.

      s = L^T r, z = minv * s, p = z;  per iteration: w = L p,
      alpha = <z, s> / <w, w>, x += alpha p, r -= alpha w, s = L^T r,
      z = minv * s, beta = <z, s>_new / <z, s>_old, p = z + beta p.

    With minv = 1 this is cgnr() operation for operation.  Returns x and the
    normalised misfit history ||r_k||^2 / ||r_0||^2."""
    if dot is None:
        def dot(a, b):
            if isinstance(a, (list, tuple)):
                return float(sum(np.vdot(x, y).real for x, y in zip(a, b)))
            return float(np.vdot(a, b).real)

    def axpy(alpha, x, y):
        if isinstance(x, (list, tuple)):
            return [yy + alpha * xx for xx, yy in zip(x, y)]
        return y + alpha * x

    r = [x.copy() for x in d] if isinstance(d, (list, tuple)) else d.copy()
    s_ = Lt(r)
    z = minv * s_
    p = z.copy()
    x = np.zeros_like(z)
    zs = dot(z, s_)
    r0 = dot(r, r)
    hist = [1.0]
    for _ in range(niter):
        w = L(p)
        alpha = zs / dot(w, w)
        x = x + alpha * p
        r = axpy(-alpha, w, r)
        s_ = Lt(r)
        z = minv * s_
        zs_new = dot(z, s_)
        beta = zs_new / zs
        p = z + beta * p
        zs = zs_new
        hist.append(dot(r, r) / r0)
    return x, hist


# ---------------------------------------------------------------------------
# Point-spread-function Hessian for image-domain LSRTM (appendix C)
# ---------------------------------------------------------------------------
def psf_halfwidth(spacing: int) -> int:
    """Half-width W of the window kept around each scatterer: the windows of
    neighbouring scatterers (spacing apart) do not overlap, 2W + 1 <= spacing."""
    return (spacing - 1) // 2


def psf_lattice(n_a: int, spacing: int) -> np.ndarray:
    """Scatterer coordinates along one axis of n_a physical nodes: W, W + s,
    W + 2s, ... (every s nodes, the first window inside the grid)."""
    return np.arange(psf_halfwidth(spacing), n_a, spacing)


def psf_scatterers(shape, spacing: int, q: int) -> np.ndarray:
    """Model perturbation (2, *shape) with unit spikes in parameter q (0 =
    lnVp, 1 = lnIp) on the scatterer lattice (appendix C: point scatterers
    distributed evenly, all at once)."""
    ndim = len(shape)
    dm = np.zeros((2,) + tuple(shape))
    lat = [psf_lattice(shape[ndim - 1 - a], spacing) for a in range(ndim)]
    grids = np.meshgrid(*[lat[a] for a in reversed(range(ndim))], indexing="ij")
    dm[(q,) + tuple(grids)] = 1.0
    return dm


def psf_images(prob: Problem, lnvp, lnip, spacing: int) -> np.ndarray:
    """PSF images P[q] = L^T L (scatterers in parameter q) (appendix C: one
    demigration and one migration of the scatterer image).  Shape
    (2, 2, *physical shape): P[q][p] is the response in parameter p."""
    out = []
    for q in range(2):
        dm = psf_scatterers(lnvp.shape, spacing, q)
        d = born(prob, lnvp, lnip, dm)
        out.append(adjoint(prob, lnvp, lnip, d))
    return np.stack(out)


def _psf_cell(j: np.ndarray, lat: np.ndarray):
    """Lattice corners (c0, c1) and weight w of coordinate(s) j along one
    axis: linear between neighbouring scatterers, w clamped to [0, 1]
    outside the lattice (the nearest scatterer's window is used)."""
    if len(lat) == 1:
        c = np.full_like(j, lat[0])
        return c, c, np.zeros(j.shape)
    s_ = lat[1] - lat[0]
    k = np.clip((j - lat[0]) // s_, 0, len(lat) - 2)
    c0 = lat[k]
    c1 = lat[k + 1]
    w = np.clip((j - c0) / s_, 0.0, 1.0)
    return c0, c1, w


def psf_hessian(P: np.ndarray, spacing: int, mono: bool = False):
    """Interpolated PSF Hessian (appendix C, eq. trilinear; bilinear in 2D)
    as a sparse matrix acting on (dlnVp, dlnIp) flattened in numpy order.

    Column j of block (p, q) is the window of the PSF images around the
    lattice corners of j, shifted to j and weighted with the multilinear
    weights: H_pq[j + o, j] = sum_c w_c(j) P[q][p][c + o] for every offset
    |o_a| <= W with j + o and c + o inside the grid.  mono=True keeps the
    lnIp block H_22 only (the monoparameter mode)."""
    from scipy import sparse
    shape = P.shape[2:]
    ndim = len(shape)
    N = int(np.prod(shape))
    W = psf_halfwidth(spacing)
    # coordinates (a-order) of every point j
    idx = np.indices(shape).reshape(ndim, -1)          # numpy axes
    J = [idx[ndim - 1 - a] for a in range(ndim)]        # axis a coordinate
    n = [shape[ndim - 1 - a] for a in range(ndim)]
    lat = [psf_lattice(n[a], spacing) for a in range(ndim)]
    cells = [_psf_cell(J[a], lat[a]) for a in range(ndim)]
    blocks = [(1, 1)] if mono else [(p, q) for p in range(2) for q in range(2)]
    rows, cols, vals = [], [], []
    offsets = np.array(np.meshgrid(*[np.arange(-W, W + 1)] * ndim, indexing="ij")).reshape(ndim, -1).T
    for m in range(2 ** ndim):
        C = []
        wgt = np.ones(N)
        for a in range(ndim):
            c0, c1, w = cells[a]
            bit = (m >> a) & 1
            C.append(c1 if bit else c0)
            wgt = wgt * (w if bit else 1.0 - w)
        live = wgt != 0.0
        for o in offsets:
            R = [J[a] + o[a] for a in range(ndim)]
            S = [C[a] + o[a] for a in range(ndim)]
            ok = live.copy()
            for a in range(ndim):
                ok &= (R[a] >= 0) & (R[a] < n[a]) & (S[a] >= 0) & (S[a] < n[a])
            if not ok.any():
                continue
            r_lin = np.ravel_multi_index(tuple(R[a][ok] for a in reversed(range(ndim))), shape)
            s_idx = tuple(S[a][ok] for a in reversed(range(ndim)))
            j_lin = np.flatnonzero(ok)
            for bp, (p, q) in enumerate(blocks):
                v = wgt[ok] * P[q][p][s_idx]
                ro = 0 if mono else p * N
                co = 0 if mono else q * N
                rows.append(r_lin + ro)
                cols.append(j_lin + co)
                vals.append(v)
    M = N if mono else 2 * N
    return sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(M, M))


# ---------------------------------------------------------------------------
# Nonstationary Wiener deblurring (appendix D)
# ---------------------------------------------------------------------------
def wiener_starts(n_a: int, block: int) -> np.ndarray:
    """Window origins along one axis: every block/2 nodes from -block/2, so
    that every node lies in exactly two windows."""
    h = block // 2
    return np.arange((n_a - 1) // h + 2) * h - h


def wiener_taper(block: int) -> np.ndarray:
    """sin^2 taper of one axis; shifted by block/2 the tapers of the two
    windows over a node add up to one."""
    u = np.arange(block)
    return np.sin(np.pi * (u + 0.5) / block) ** 2


def wiener_deblur(m_ref: np.ndarray, m_blur: np.ndarray, m_in: np.ndarray,
                  block: int, eps_rel: float) -> np.ndarray:
    """Nonstationary Wiener filter of appendix D on one image.

    The Hessian is taken as locally translation invariant, hence diagonal in
    the Fourier basis of each local block: with F the block's Fourier
    transform, the inverse eigenvalues minimise
    ||F m_ref - Lambda^-1 F m_blur||^2 + eps ||Lambda^-1||^2, i.e.
    Lambda^-1 = conj(F m_blur) F m_ref / (|F m_blur|^2 + eps), and the block's
    estimate is F^-1 [Lambda^-1 F m_in] (eq. sol).  Blocks are tapered
    (wiener_taper in every axis), eps = eps_rel * max |F m_blur|^2 of the
    block, and the estimates are merged with their valences:
    dm = sum_w dm_w / sum_w t_w, t_w the block's taper at the node."""
    shape = m_ref.shape
    nd = m_ref.ndim
    T = 1.0
    for _ in range(nd):
        T = np.multiply.outer(T, wiener_taper(block)) if np.ndim(T) else wiener_taper(block)
    out = np.zeros(shape)
    wsum = np.zeros(shape)
    starts = [wiener_starts(shape[k], block) for k in range(nd)]
    for origin in np.array(np.meshgrid(*starts, indexing="ij")).reshape(nd, -1).T:
        src = tuple(slice(max(o, 0), min(o + block, shape[k])) for k, o in enumerate(origin))
        dst = tuple(slice(max(o, 0) - o, min(o + block, shape[k]) - o) for k, o in enumerate(origin))
        blk = []
        for img in (m_ref, m_blur, m_in):
            b = np.zeros((block,) * nd)
            b[dst] = img[src]
            blk.append(np.fft.fftn(T * b))
        A, B, C = blk
        pw = (B * np.conj(B)).real
        mx = pw.max()
        if mx > 0:
            G = np.conj(B) * A / (pw + eps_rel * mx)
            d = np.fft.ifftn(G * C).real
            out[src] += d[dst]
        wsum[src] += T[dst]
    return out / wsum


# ---------------------------------------------------------------------------
# Data preparation: top mute (section 4.1)
# ---------------------------------------------------------------------------
def mute_weights(prob: Problem, s: int, v_mute: float, t0: float, ntaper: int) -> np.ndarray:
    """Weights (nt, nrec_s) of the top mute of shot s (the paper mutes the
    direct arrival of its nonlinear residual data without stating how):
    with D the source-receiver distance, tc = t0 + D / v_mute; a sample
    recorded at t = (n + 1) dt before tc gets 0, the next ntaper samples
    0.5 (1 - cos(pi (t - tc) / (ntaper dt))), the rest 1."""
    rec = np.asarray(prob.rec[s], dtype=np.float64).reshape(-1, prob.ndim)
    src = np.asarray(prob.src[s], dtype=np.float64)
    dist = np.sqrt(np.sum(((rec - src) * np.asarray(prob.h)) ** 2, axis=1))
    tc = t0 + dist / v_mute
    t = (np.arange(prob.nt) + 1.0)[:, None] * prob.dt
    w = np.ones((prob.nt, len(tc)))
    w[t < tc] = 0.0
    if ntaper > 0:
        ramp = (t >= tc) & (t < tc + ntaper * prob.dt)
        w = np.where(ramp, 0.5 * (1.0 - np.cos(np.pi * (t - tc) / (ntaper * prob.dt))), w)
    return w


def mute(prob: Problem, ds: Sequence[np.ndarray], v_mute: float, t0: float = 0.0,
         ntaper: int = 0) -> List[np.ndarray]:
    """Top mute of every shot's data (nt, nrec_s)."""
    return [d * mute_weights(prob, s, v_mute, t0, ntaper) for s, d in enumerate(ds)]
