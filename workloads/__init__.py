"""Seeded synthetic inputs for the superiorized band+box projection method.

This module only synthesises data: matrices from ray geometry or dose kernels,
phantoms, noise, and the bands built around noisy measurements.  It holds none
of the method's arithmetic (no projection, proximity, objective or perturbation
step), so both the FP64 oracle and the HIP library can consume its arrays
without sharing any part of the computation.

Every generator is deterministic in its seed (``numpy.random.default_rng``).
Shapes follow the workloads of the paper (Section 2.3): straight-ray seismic
travel-time tomography, parallel-beam CT, and a radiotherapy dose-influence
matrix; the datasets and toolboxes the paper used are replaced by these
synthetic stand-ins.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

OBJ_NONE, OBJ_SQNORM, OBJ_TV2D, OBJ_LINEAR, OBJ_L1 = 0, 1, 2, 3, 4
BASIC_SIMULT, BASIC_DROP, BASIC_CQ, BASIC_EL, BASIC_EMR = 0, 1, 2, 3, 4
DVC_MAX, DVC_MIN = 0, 1  # dose-volume constraint senses: D_V <= d, D_V >= d
STEP_POWER, STEP_ADAPTIVE = 0, 1  # perturbation step size: power law gamma alpha^ell, adaptive (Section 2.1.2)
OBJ_NAMES = {OBJ_NONE: "none", OBJ_SQNORM: "sqnorm", OBJ_TV2D: "tv2d", OBJ_LINEAR: "linear", OBJ_L1: "l1"}


@dataclass
class Workload:
    """One band+box feasibility problem with a secondary objective.

    Constraint rows are ``lower[i,s] <= <a_i, x_s> <= upper[i,s]`` for every slice
    ``s`` (slices share ``A``), plus ``box_lo <= x <= box_hi``.  Arrays are float32
    (the device precision); the oracle promotes them exactly to float64.
    ``lower``/``upper`` are ``[m, B]`` and ``x0`` is ``[n, B]``.
    """

    name: str
    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float32 [nnz]
    lower: np.ndarray  # float32 [m, B]
    upper: np.ndarray  # float32 [m, B]
    box_lo: np.ndarray  # float32 [n]
    box_hi: np.ndarray  # float32 [n]
    x0: np.ndarray  # float32 [n, B]
    lam: float = 1.0
    obj: int = OBJ_NONE
    tv_rows: int = 0
    tv_cols: int = 0
    tv_eps: float = 0.0
    linear_c: Optional[np.ndarray] = None  # float32 [n]
    gamma: float = 1.0
    alpha: float = 0.99
    n_red: int = 1
    restart_every: int = 0
    max_trials: int = 100
    K: int = 100
    weights: Optional[np.ndarray] = None  # float64 [m]; None means uniform 1/m
    basic: int = 0  # BASIC_*: the feasibility-seeking step
    step_rule: int = STEP_POWER  # STEP_*: the perturbation's step size
    stop: Optional[dict] = None  # stopping rules: prox, dprox, n, max_iters, dobj, var (None: fixed K)
    # dose-volume constraints: dicts with row_begin, row_end (the structure's
    # rows), sense (DVC_MAX / DVC_MIN), fraction (V) and dose (d)
    dvc: Optional[list] = None
    image: Optional[tuple] = None  # (rows, cols) when the unknowns are the pixels of an image, row-major
    x_true: Optional[np.ndarray] = None  # float32 [n, B]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def B(self) -> int:
        return int(self.lower.shape[1])

    def with_params(self, **kw) -> "Workload":
        return replace(self, **kw)

    def slice(self, s: int) -> "Workload":
        """The single-slice problem for slice ``s`` (same ``A``)."""
        return replace(
            self,
            lower=np.ascontiguousarray(self.lower[:, s : s + 1]),
            upper=np.ascontiguousarray(self.upper[:, s : s + 1]),
            x0=np.ascontiguousarray(self.x0[:, s : s + 1]),
            x_true=None if self.x_true is None else np.ascontiguousarray(self.x_true[:, s : s + 1]),
        )

    def dense(self) -> np.ndarray:
        """Dense float64 copy of A (small problems only)."""
        A = np.zeros((self.m, self.n), dtype=np.float64)
        for i in range(self.m):
            s, e = self.row_ptr[i], self.row_ptr[i + 1]
            np.add.at(A[i], self.col_idx[s:e], self.val[s:e].astype(np.float64))
        return A


def _csr_from_dense(A: np.ndarray):
    m, n = A.shape
    mask = A != 0
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    rows, cols = np.nonzero(mask)
    return row_ptr.astype(np.int32), cols.astype(np.int32), A[rows, cols].astype(np.float32)


def _csr_matvec64(row_ptr, col_idx, val, x):
    """Forward model used only to synthesise measurements (float64); x may be
    [n] or [n, k]."""
    import scipy.sparse as sp

    m = len(row_ptr) - 1
    n = int(np.max(col_idx)) + 1 if col_idx.size else 1
    n = max(n, x.shape[0])
    A = sp.csr_matrix((val.astype(np.float64), col_idx, row_ptr.astype(np.int64)), shape=(m, n))
    return A @ np.asarray(x, np.float64)


# ---------------------------------------------------------------------------
# Dense consistent problem (small CPU-scale case)
# ---------------------------------------------------------------------------

def dense_small(seed: int = 1, m: int = 256, n: int = 128, K: int = 100) -> Workload:
    """Dense N(0,1) A with a hidden x* ~ U(0,1), bands A x* +- 0.05, box [0,1].

    Consistent by construction (x* satisfies every band and the box), with the
    squared-norm objective, lambda = 1, beta_k = 0.99^k and x0 = 0.5.
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)).astype(np.float32)
    x_star = rng.uniform(0.0, 1.0, n)
    r = A.astype(np.float64) @ x_star
    row_ptr = np.arange(0, m * n + 1, n, dtype=np.int32)
    col_idx = np.tile(np.arange(n, dtype=np.int32), m)
    return Workload(
        name=f"dense{m}x{n}",
        m=m,
        n=n,
        row_ptr=row_ptr,
        col_idx=col_idx,
        val=A.reshape(-1).copy(),
        lower=(r - 0.05).astype(np.float32)[:, None],
        upper=(r + 0.05).astype(np.float32)[:, None],
        box_lo=np.zeros(n, np.float32),
        box_hi=np.ones(n, np.float32),
        x0=np.full((n, 1), 0.5, np.float32),
        lam=1.0,
        obj=OBJ_SQNORM,
        gamma=1.0,
        alpha=0.99,
        n_red=1,
        K=K,
        x_true=x_star.astype(np.float32)[:, None],
    )


# ---------------------------------------------------------------------------
# Random sparse matrices with skewed row lengths (kernel edge cases)
# ---------------------------------------------------------------------------

def random_sparse(
    m: int,
    n: int,
    mean_row: float,
    seed: int,
    B: int = 1,
    empty_frac: float = 0.05,
    long_rows: int = 0,
    long_len: Optional[int] = None,
    obj: int = OBJ_SQNORM,
    K: int = 20,
    tv_shape: Optional[tuple] = None,
    margin: float = 0.05,
) -> Workload:
    """Random CSR with geometric row lengths, some empty rows and a few long rows.

    Bands surround A x* for a hidden x* ~ U(0,1) with a relative margin, and a
    fraction of rows is made one-sided (infinite bound) or an equality band.
    """
    rng = np.random.default_rng(seed)
    lens = rng.geometric(1.0 / max(mean_row, 1.0), size=m).astype(np.int64)
    lens = np.minimum(lens, n)
    lens[rng.random(m) < empty_frac] = 0
    if long_rows:
        L = n if long_len is None else min(long_len, n)
        idx = rng.choice(m, size=min(long_rows, m), replace=False)
        lens[idx] = L
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    cols = np.empty(row_ptr[-1], np.int32)
    for i in range(m):
        s, e = row_ptr[i], row_ptr[i + 1]
        if e > s:
            c = rng.choice(n, size=e - s, replace=False)
            if rng.random() < 0.5:
                c.sort()
            cols[s:e] = c
    vals = rng.uniform(-1.0, 1.0, row_ptr[-1]).astype(np.float32)
    vals[vals == 0] = 0.5
    x_star = rng.uniform(0.0, 1.0, (n, B))
    lower = np.empty((m, B))
    upper = np.empty((m, B))
    for s in range(B):
        r = _csr_matvec64(row_ptr, cols, vals, x_star[:, s])
        scale = np.abs(r) * margin + 0.02
        lower[:, s] = r - scale
        upper[:, s] = r + scale
    kind = rng.integers(0, 5, size=m)
    lower[kind == 0, :] = -np.inf
    upper[kind == 1, :] = np.inf
    eq = kind == 2
    upper[eq, :] = lower[eq, :] = 0.5 * (lower[eq, :] + upper[eq, :])
    rows, cols_tv = (tv_shape if tv_shape is not None else (0, 0))
    if obj == OBJ_TV2D:
        assert tv_shape is not None and rows * cols_tv == n
    lin_c = None
    if obj == OBJ_LINEAR:
        lin_c = rng.uniform(0.1, 1.0, n).astype(np.float32)
    return Workload(
        name=f"rand{m}x{n}",
        m=m,
        n=n,
        image=tuple(tv_shape) if tv_shape is not None else None,
        row_ptr=row_ptr.astype(np.int32),
        col_idx=cols,
        val=vals,
        lower=lower.astype(np.float32),
        upper=upper.astype(np.float32),
        box_lo=np.full(n, -0.25, np.float32),
        box_hi=np.full(n, 1.25, np.float32),
        x0=rng.uniform(0.0, 1.0, (n, B)).astype(np.float32),
        lam=1.0,
        obj=obj,
        tv_rows=rows,
        tv_cols=cols_tv,
        tv_eps=1e-2 if obj == OBJ_TV2D else 0.0,
        linear_c=lin_c,
        gamma=0.5,
        alpha=0.95,
        n_red=2,
        restart_every=7,
        K=K,
        x_true=x_star.astype(np.float32),
    )


# ---------------------------------------------------------------------------
# Exact ray/pixel intersection lengths on a regular grid
# ---------------------------------------------------------------------------

def trace_rays(p0, p1, nx, ny, xmin, ymin, hx, hy):
    """Exact lengths of the segments p0->p1 inside each cell of an nx*ny grid.

    Cell (i, j) spans x in [xmin + j hx, xmin + (j+1) hx], y in
    [ymin + i hy, ymin + (i+1) hy] and has index ``i * nx + j``.  Returns
    ``(counts[R], cols, lengths)`` with each ray's cells in order along the ray.
    """
    p0 = np.asarray(p0, np.float64)
    p1 = np.asarray(p1, np.float64)
    R = p0.shape[0]
    d = p1 - p0
    L = np.hypot(d[:, 0], d[:, 1])
    xs = xmin + hx * np.arange(nx + 1)
    ys = ymin + hy * np.arange(ny + 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = (xs[None, :] - p0[:, 0:1]) / d[:, 0:1]
        ty = (ys[None, :] - p0[:, 1:2]) / d[:, 1:2]
    t = np.concatenate([tx, ty, np.zeros((R, 1)), np.ones((R, 1))], axis=1)
    t[~np.isfinite(t)] = np.nan
    t = np.clip(t, 0.0, 1.0)
    t.sort(axis=1)  # NaN sort last
    seg = t[:, 1:] - t[:, :-1]
    mid = 0.5 * (t[:, 1:] + t[:, :-1])
    mx = p0[:, 0:1] + mid * d[:, 0:1]
    my = p0[:, 1:2] + mid * d[:, 1:2]
    with np.errstate(invalid="ignore"):
        j = np.floor((mx - xmin) / hx)
        i = np.floor((my - ymin) / hy)
    valid = np.isfinite(seg) & (seg > 1e-12) & (j >= 0) & (j < nx) & (i >= 0) & (i < ny)
    counts = valid.sum(axis=1)
    cols = (i[valid] * nx + j[valid]).astype(np.int64)
    lens = (seg * L[:, None])[valid]
    return counts, cols, lens


def _assemble(chunks, m):
    counts = np.concatenate([c[0] for c in chunks])
    cols = np.concatenate([c[1] for c in chunks]).astype(np.int32)
    lens = np.concatenate([c[2] for c in chunks])
    assert counts.size == m
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return row_ptr.astype(np.int32), cols, lens


# ---------------------------------------------------------------------------
# Parallel-beam CT
# ---------------------------------------------------------------------------

def ellipse_phantom(N: int, seed: int, n_ellipses: int = 10) -> np.ndarray:
    """Piecewise-constant N*N phantom on the unit square, values in [0, 1]."""
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    c = -0.5 + (np.arange(N) + 0.5) * h
    Y, X = np.meshgrid(c, c, indexing="ij")  # Y varies along rows (i), X along cols (j)
    img = np.zeros((N, N))
    img[(X / 0.45) ** 2 + (Y / 0.38) ** 2 <= 1.0] = 0.2
    for _ in range(n_ellipses):
        rad = 0.35 * np.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * np.pi)
        cx, cy = rad * np.cos(ang), rad * np.sin(ang)
        a, b = rng.uniform(0.03, 0.25, 2)
        th = rng.uniform(0, np.pi)
        v = rng.uniform(0, 1)
        u = (X - cx) * np.cos(th) + (Y - cy) * np.sin(th)
        w = -(X - cx) * np.sin(th) + (Y - cy) * np.cos(th)
        img[(u / a) ** 2 + (w / b) ** 2 <= 1.0] = v
    return np.clip(img, 0.0, 1.0)


def ct_matrix(N: int, n_angles: int, n_det: int):
    """System matrix of parallel-beam CT on the unit-square field of view.

    Angles are theta_a = a*pi/n_angles, detector d sits at offset
    (d - (n_det-1)/2) * h with h = 1/N, and entries are exact intersection lengths
    (field-of-view units, so a full row sums to the chord through the square).
    Row index is ``a * n_det + d``; pixel (i, j) is column ``i * N + j``.
    """
    h = 1.0 / N
    offs = (np.arange(n_det) - (n_det - 1) / 2.0) * h
    chunks = []
    for a in range(n_angles):
        th = a * np.pi / n_angles
        nrm = np.array([np.cos(th), np.sin(th)])
        dirv = np.array([-np.sin(th), np.cos(th)])
        base = offs[:, None] * nrm[None, :]
        p0 = base - 1.0 * dirv[None, :]
        p1 = base + 1.0 * dirv[None, :]
        chunks.append(trace_rays(p0, p1, N, N, -0.5, -0.5, h, h))
    return _assemble(chunks, n_angles * n_det)


def ct(
    N: int = 256,
    n_angles: int = 180,
    n_det: Optional[int] = None,
    seed: int = 2,
    B: int = 1,
    I0: float = 1e4,
    nsigma: float = 3.0,
    K: int = 200,
    tv_eps: float = 1e-4,
    variant: str = "default",
) -> Workload:
    """Low-dose parallel-beam CT with Poisson noise and +-3 sigma bands.

    counts ~ Poisson(I0 exp(-A x_true)); b = -ln(max(counts,1)/I0);
    sigma = 1/sqrt(max(counts,1)); bands b -+ nsigma*sigma; box [0, 1];
    isotropic TV perturbation.  ``variant='paper'`` uses the CT perturbation
    parameters of the paper's first experiment (gamma 5, alpha 0.99, four
    reductions, restart every 50).
    """
    if n_det is None:
        n_det = int(np.ceil(np.sqrt(2.0) * N))
    row_ptr, cols, lens = ct_matrix(N, n_angles, n_det)
    val = lens.astype(np.float32)
    m, n = n_angles * n_det, N * N
    rng = np.random.default_rng(seed + 7919)
    lower = np.empty((m, B), np.float32)
    upper = np.empty((m, B), np.float32)
    xt = np.empty((n, B), np.float32)
    for s in range(B):
        x_true = ellipse_phantom(N, seed * 1000 + s).reshape(-1)
        p = _csr_matvec64(row_ptr, cols, val, x_true)
        counts = rng.poisson(I0 * np.exp(-p))
        cc = np.maximum(counts, 1).astype(np.float64)
        b = -np.log(cc / I0)
        sig = 1.0 / np.sqrt(cc)
        lower[:, s] = b - nsigma * sig
        upper[:, s] = b + nsigma * sig
        xt[:, s] = x_true
    params = dict(gamma=1.0, alpha=0.99, n_red=1, restart_every=0)
    if variant == "paper":
        params = dict(gamma=5.0, alpha=0.99, n_red=4, restart_every=50)
    return Workload(
        name=f"ct{N}",
        m=m,
        n=n,
        image=(N, N),
        row_ptr=row_ptr,
        col_idx=cols,
        val=val,
        lower=lower,
        upper=upper,
        box_lo=np.zeros(n, np.float32),
        box_hi=np.ones(n, np.float32),
        x0=np.zeros((n, B), np.float32),
        lam=1.0,
        obj=OBJ_TV2D,
        tv_rows=N,
        tv_cols=N,
        tv_eps=tv_eps,
        K=K,
        x_true=xt,
        meta=dict(n_angles=n_angles, n_det=n_det, I0=I0),
        **params,
    )


# ---------------------------------------------------------------------------
# Straight-ray travel-time tomography
# ---------------------------------------------------------------------------

def slowness_field(rows: int, cols: int, seed: int) -> np.ndarray:
    """Layered slowness (1.0 at the top to 0.6 at the bottom) plus four
    Gaussian anomalies of +-10 %."""
    rng = np.random.default_rng(seed)
    depth = (np.arange(rows) + 0.5) / rows
    layer = np.minimum((depth * 5).astype(int), 4)
    base = np.array([1.0, 0.9, 0.8, 0.7, 0.6])[layer]
    s = np.repeat(base[:, None], cols, axis=1)
    I, J = np.meshgrid(np.arange(rows) + 0.5, np.arange(cols) + 0.5, indexing="ij")
    bump = np.zeros_like(s)
    for _ in range(4):
        ci, cj = rng.uniform(0, rows), rng.uniform(0, cols)
        sg = rng.uniform(10, 30)
        amp = rng.choice([-0.1, 0.1])
        bump += amp * np.exp(-((I - ci) ** 2 + (J - cj) ** 2) / (2 * sg * sg))
    return s * (1.0 + bump)


def seismic_matrix(rows: int, cols: int, n_src: int, n_rec: int):
    """Straight rays from sources on the top edge to receivers on the bottom
    edge of a rows*cols grid of unit cells.  Row index is ``src * n_rec + rec``."""
    xs = (np.arange(n_src) + 0.5) * cols / n_src
    xr = (np.arange(n_rec) + 0.5) * cols / n_rec
    chunks = []
    for a in range(n_src):
        p0 = np.stack([np.full(n_rec, xs[a]), np.zeros(n_rec)], axis=1)
        p1 = np.stack([xr, np.full(n_rec, float(rows))], axis=1)
        chunks.append(trace_rays(p0, p1, cols, rows, 0.0, 0.0, 1.0, 1.0))
    return _assemble(chunks, n_src * n_rec)


def fresnel_matrix(N: int, n_src: int, n_rec: int, wavelength: float = 1.0, w0: float = 0.5):
    """Band rows of a cross-well / surface travel-time model on an N x N grid of
    unit pixels (pixel (i, j) = unknown i*N + j, centre (j + 1/2, i + 1/2)):
    sources on the right edge, receivers half on the left edge and half on the
    top edge; row ``src * n_rec + rec``.  Each ray is widened to a band around
    its segment p0 -> p1 of length L: at fraction t along it the half-width is
    w(t) = sqrt(wavelength * L * t (1 - t)) + w0 (a first-Fresnel-zone-like
    width); a pixel at distance d from the segment gets weight
    exp(-(d / w(t))^2) if d <= 2 w(t), and the row is scaled to sum to L, so a
    constant slowness s gives travel times s * L.  Returns (row_ptr, cols, vals)."""
    ys = (np.arange(n_src) + 0.5) * N / n_src
    half = n_rec // 2
    rec = np.concatenate([np.stack([np.zeros(half), (np.arange(half) + 0.5) * N / half], 1),
                          np.stack([(np.arange(n_rec - half) + 0.5) * N / (n_rec - half),
                                    np.zeros(n_rec - half)], 1)])
    counts, cols_all, vals_all = [], [], []
    for a in range(n_src):
        p0 = np.array([float(N), ys[a]])
        for b in range(n_rec):
            p1 = rec[b]
            dv = p1 - p0
            L = float(np.hypot(dv[0], dv[1]))
            u = dv / L
            wmax = np.sqrt(wavelength * L / 4.0) + w0
            reach = 2.0 * wmax
            # candidate pixels: every pixel whose centre lies within `reach` of the segment's bounding box
            lo = np.floor(np.minimum(p0, p1) - reach).astype(int)
            hi = np.ceil(np.maximum(p0, p1) + reach).astype(int)
            jj = np.arange(max(lo[0], 0), min(hi[0], N))
            ii = np.arange(max(lo[1], 0), min(hi[1], N))
            J, I = np.meshgrid(jj, ii)
            cx, cy = J.ravel() + 0.5, I.ravel() + 0.5
            t = ((cx - p0[0]) * u[0] + (cy - p0[1]) * u[1]) / L
            tc = np.clip(t, 0.0, 1.0)
            d = np.hypot(cx - (p0[0] + tc * dv[0]), cy - (p0[1] + tc * dv[1]))
            w = np.sqrt(wavelength * L * tc * (1.0 - tc)) + w0
            keep = d <= 2.0 * w
            om = np.exp(-(d[keep] / w[keep]) ** 2)
            idx = (I.ravel()[keep] * N + J.ravel()[keep]).astype(np.int64)
            order = np.argsort(idx)
            counts.append(idx.size)
            cols_all.append(idx[order])
            vals_all.append((L * om / om.sum())[order])
    row_ptr = np.zeros(len(counts) + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return row_ptr.astype(np.int32), np.concatenate(cols_all).astype(np.int32), np.concatenate(vals_all)


def with_dvc(w: "Workload", groups) -> "Workload":
    """Append one dose-volume constraint per entry of ``groups`` =
    [(rows, sense, fraction, dose), ...]: the rows ``rows`` of A are copied, in
    order, to the end of A as the structure's block, with placeholder bands
    (-inf, +inf) that the constraint replaces at every point."""
    rp = np.asarray(w.row_ptr, np.int64)
    cols, vals = [np.asarray(w.col_idx)], [np.asarray(w.val)]
    counts = [np.diff(rp)]
    dvc = list(w.dvc or [])
    m = w.m
    for rows, sense, fraction, dose in groups:
        rows = np.asarray(rows, np.int64)
        take = np.concatenate([np.arange(rp[i], rp[i + 1]) for i in rows]) if rows.size else np.zeros(0, np.int64)
        cols.append(np.asarray(w.col_idx)[take])
        vals.append(np.asarray(w.val)[take])
        counts.append(rp[rows + 1] - rp[rows])
        dvc.append(dict(row_begin=m, row_end=m + rows.size, sense=int(sense), fraction=float(fraction),
                        dose=float(dose)))
        m += rows.size
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.concatenate(counts), out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    extra = m - w.m
    pad_lo = np.full((extra, w.B), -np.inf, np.float32)
    pad_up = np.full((extra, w.B), np.inf, np.float32)
    weights = None
    if w.weights is not None:
        weights = np.concatenate([np.asarray(w.weights, np.float64),
                                  np.full(extra, float(np.mean(w.weights)))])
    return replace(w, name=w.name + "_dvc", m=m, row_ptr=row_ptr.astype(np.int32),
                   col_idx=np.concatenate(cols).astype(np.int32), val=np.concatenate(vals).astype(np.float32),
                   lower=np.concatenate([w.lower, pad_lo]), upper=np.concatenate([w.upper, pad_up]),
                   weights=weights, dvc=dvc)


def rt_with_dvc(w: "Workload", basic: int = BASIC_EMR) -> "Workload":
    """A radiotherapy workload with the dose-volume constraints of the paper's
    horseshoe plan (Section 2.3.3) on the scale of a mean target dose of 1
    (2.1 Gy): target D95% >= 0.97, target D5% <= 1.03, organ-at-risk D5% <=
    0.16; the EMR step (the paper's choice for this case) and the horseshoe's
    power law (gamma = 1, alpha = 0.7, restarts every 500 iterations)."""
    t, o = w.meta["target_rows"], w.meta["oar_rows"]
    out = with_dvc(w, [(t, DVC_MIN, 0.95, 0.97), (t, DVC_MAX, 0.05, 1.03), (o, DVC_MAX, 0.05, 0.16)])
    return out.with_params(basic=basic, gamma=1.0, alpha=0.7, restart_every=500)


def rt_plan(seed: int, K: int = 300, n_beams: int = 9) -> "Workload":
    """A radiotherapy plan of the 160 x 160 x 80 configuration's shape for a
    serving stream (one operator per plan): the beam set rotated by a seeded
    angle in [0, 2 pi / n_beams)."""
    rng = np.random.default_rng(seed)
    w = rt_large(seed=seed, K=K, n_beams=n_beams, angle_offset=float(rng.uniform(0.0, 2 * np.pi / n_beams)))
    return replace(w, name=f"rt_plan{seed}")


def synthetic_iterate(w: "Workload", seed: int, spread: float = 0.1) -> np.ndarray:
    """A seeded point of the kind an iteration passes through: the true
    solution (0.5 where none is known) times (1 + spread * N(0, 1)), clipped
    to the box; float32 [n, B]."""
    rng = np.random.default_rng(seed)
    base = np.full((w.n, w.B), 0.5) if w.x_true is None else np.asarray(w.x_true, np.float64).reshape(w.n, -1)
    x = base * (1.0 + spread * rng.standard_normal((w.n, base.shape[1])))
    x = np.clip(x, np.asarray(w.box_lo, np.float64)[:, None], np.asarray(w.box_hi, np.float64)[:, None])
    return np.ascontiguousarray(np.broadcast_to(x, (w.n, w.B)), dtype=np.float32)


def add_relative_noise(t: np.ndarray, noise: float, seed: int) -> np.ndarray:
    """Travel times t (m x B) times (1 + noise * N(0, 1)), per entry, float32."""
    rng = np.random.default_rng(seed + 7919)
    return (t * (1.0 + noise * rng.standard_normal(t.shape))).astype(np.float32)


def seismic_fresnel(
    N: int = 256,
    n_src: int = 64,
    n_rec: int = 128,
    seed: int = 6,
    B: int = 1,
    noise: float = 0.0,
    obj: int = OBJ_L1,
    basic: int = BASIC_DROP,
    K: int = 200,
) -> Workload:
    """The seismic setup at the paper's shape (Section 2.3.1: 64 sources, 128
    receivers, a 256 x 256 grid, A of 8192 x 65536) with band rows
    (:func:`fresnel_matrix`).  The system A s = b is solved as equality bands,
    noise-free (an exact solution exists) or with relative Gaussian noise (5 %
    in the paper's second case); box s >= 0; DROP with lambda = m (1/w for the
    uniform weights) and the L1, squared-norm or TV perturbation."""
    row_ptr, cols_idx, vals = fresnel_matrix(N, n_src, n_rec)
    val = vals.astype(np.float32)
    m, n = n_src * n_rec, N * N
    t = np.empty((m, B), np.float64)
    xt = np.empty((n, B), np.float32)
    for s in range(B):
        sl = slowness_field(N, N, seed * 1000 + s).reshape(-1)
        t[:, s] = _csr_matvec64(row_ptr, cols_idx, val, sl)
        xt[:, s] = sl
    b = add_relative_noise(t, noise, seed)
    return Workload(
        name=f"seismic_fresnel{N}",
        m=m,
        n=n,
        image=(N, N),
        row_ptr=row_ptr,
        col_idx=cols_idx,
        val=val,
        lower=b.copy(),
        upper=b.copy(),
        box_lo=np.zeros(n, np.float32),
        box_hi=np.full(n, np.inf, np.float32),
        x0=np.zeros((n, B), np.float32),
        lam=float(m) if basic == BASIC_DROP else 1.0,
        obj=obj,
        tv_rows=N if obj == OBJ_TV2D else 0,
        tv_cols=N if obj == OBJ_TV2D else 0,
        tv_eps=1e-4 if obj == OBJ_TV2D else 0.0,
        gamma=1.0,
        alpha=0.975,
        n_red=4,
        restart_every=50,
        K=K,
        x_true=xt,
        basic=basic,
        meta=dict(n_src=n_src, n_rec=n_rec, noise=noise, seed=seed, t_clean=t),
    )


def seismic(
    rows: int = 200,
    cols: int = 400,
    n_src: int = 100,
    n_rec: int = 200,
    seed: int = 3,
    B: int = 1,
    noise: float = 0.01,
    nsigma: float = 2.0,
    K: int = 500,
    variant: str = "default",
) -> Workload:
    """Travel-time tomography: t = A s, b = t (1 + noise*xi), bands b -+ 2 sigma
    with sigma = noise*t, box [0, inf), TV perturbation.  ``variant='paper'``
    uses the seismic perturbation parameters of the paper (gamma 1, alpha 0.975,
    four reductions, restart every 50)."""
    row_ptr, cols_idx, lens = seismic_matrix(rows, cols, n_src, n_rec)
    val = lens.astype(np.float32)
    m, n = n_src * n_rec, rows * cols
    rng = np.random.default_rng(seed + 104729)
    lower = np.empty((m, B), np.float32)
    upper = np.empty((m, B), np.float32)
    xt = np.empty((n, B), np.float32)
    smax = 0.0
    for s in range(B):
        sl = slowness_field(rows, cols, seed * 1000 + s).reshape(-1)
        smax = max(smax, float(sl.max()))
        t = _csr_matvec64(row_ptr, cols_idx, val, sl)
        b = t * (1.0 + noise * rng.standard_normal(m))
        sig = noise * t
        lower[:, s] = b - nsigma * sig
        upper[:, s] = b + nsigma * sig
        xt[:, s] = sl
    params = dict(gamma=1.0, alpha=0.99, n_red=1, restart_every=0)
    if variant == "paper":
        params = dict(gamma=1.0, alpha=0.975, n_red=4, restart_every=50)
    return Workload(
        name=f"seismic{rows}x{cols}",
        m=m,
        n=n,
        image=(rows, cols),
        row_ptr=row_ptr,
        col_idx=cols_idx,
        val=val,
        lower=lower,
        upper=upper,
        box_lo=np.zeros(n, np.float32),
        box_hi=np.full(n, np.inf, np.float32),
        x0=np.zeros((n, B), np.float32),
        lam=1.0,
        obj=OBJ_TV2D,
        tv_rows=rows,
        tv_cols=cols,
        tv_eps=1e-4 * smax,
        K=K,
        x_true=xt,
        meta=dict(n_src=n_src, n_rec=n_rec),
        **params,
    )


# ---------------------------------------------------------------------------
# Radiotherapy dose-influence matrix
# ---------------------------------------------------------------------------

def rt(
    grid=(40, 40, 20),
    n_beams: int = 9,
    beamlets=(12, 12),
    spacing: float = 2.4,
    mu: float = 0.005,
    rho: float = 2.0,
    r_cut: float = 6.4,
    seed: int = 4,
    infeasible: bool = True,
    K: int = 300,
    variant: str = "default",
    angle_offset: float = 0.0,
) -> Workload:
    """Synthetic dose-influence matrix and dose bands for fluence planning.

    Voxels of an X*Y*Z grid (unit spacing) are rows; beamlets of ``n_beams``
    coplanar beams (equal angular steps around the z axis, the first at
    ``angle_offset`` radians) on a
    ``beamlets[0] x beamlets[1]`` grid of the given spacing are columns.
    a_ij = exp(-mu * depth) * exp(-r / rho) for voxels within lateral distance
    ``r_cut`` of the beamlet axis.  The matrix is scaled so that x = 1 gives a
    mean target dose of 1.  Bands: target [0.95, 1.07], organ-at-risk voxels
    (-inf, 0.5], other voxels (-inf, 1.07].  With ``infeasible`` every voxel of an
    OAR/target overlap shell is duplicated as a second row with band
    (-inf, 0.3], which cannot hold together with the target's lower bound.
    Objective: summed dose over all voxels (a linear function of x with
    c = A^T 1).  Box x >= 0.
    """
    rng = np.random.default_rng(seed)
    X, Y, Z = grid
    nv = X * Y * Z
    ci = (np.arange(X) + 0.5) - X / 2.0
    cj = (np.arange(Y) + 0.5) - Y / 2.0
    ck = (np.arange(Z) + 0.5) - Z / 2.0
    PX, PY, PZ = np.meshgrid(ci, cj, ck, indexing="ij")
    PX, PY, PZ = PX.reshape(-1), PY.reshape(-1), PZ.reshape(-1)
    nbu, nbw = beamlets
    n = n_beams * nbu * nbw
    half = 0.5 * max(X, Y)
    # candidate beamlet offsets around the nearest beamlet
    reach = int(np.ceil(r_cut / spacing)) + 1
    offs = [(du, dw) for du in range(-reach, reach + 1) for dw in range(-reach, reach + 1)]
    per_row_cols = []
    per_row_vals = []
    for b in range(n_beams):
        th = angle_offset + 2 * np.pi * b / n_beams
        e_d = np.array([np.cos(th), np.sin(th)])  # beam travels along +e_d
        e_u = np.array([-np.sin(th), np.cos(th)])
        depth = PX * e_d[0] + PY * e_d[1] + half
        u = PX * e_u[0] + PY * e_u[1]
        w = PZ
        fu = u / spacing + (nbu - 1) / 2.0
        fw = w / spacing + (nbw - 1) / 2.0
        bu0 = np.rint(fu).astype(np.int64)
        bw0 = np.rint(fw).astype(np.int64)
        att = np.exp(-mu * np.maximum(depth, 0.0))
        for du, dw in offs:
            bu = bu0 + du
            bw = bw0 + dw
            r = spacing * np.hypot(fu - bu, fw - bw)
            ok = (bu >= 0) & (bu < nbu) & (bw >= 0) & (bw < nbw) & (r <= r_cut)
            col = np.where(ok, b * nbu * nbw + bu * nbw + bw, -1)
            v = np.where(ok, att * np.exp(-r / rho), 0.0)
            per_row_cols.append(col)
            per_row_vals.append(v)
    C = np.stack(per_row_cols, axis=1)  # [nv, n_beams*len(offs)]
    V = np.stack(per_row_vals, axis=1)
    ok = C >= 0
    # structures
    rr = np.sqrt(PX**2 + PY**2 + PZ**2)
    R_t = 0.25 * min(X, Y, 2 * Z)
    target = rr <= R_t
    oar_c = np.array([R_t * 1.1, 0.0])
    oar = (np.hypot(PX - oar_c[0], PY - oar_c[1]) <= 0.45 * R_t) & (np.abs(PZ) <= 0.8 * R_t)
    overlap = target & oar
    # scale A so that x = 1 gives a mean target dose of 1
    d1 = (V * ok).sum(axis=1)
    scale = 1.0 / max(d1[target].mean(), 1e-30)
    V = V * scale
    counts = ok.sum(axis=1)
    up = np.where(oar, 0.5, 1.07)
    lo = np.where(target, 0.95, -np.inf)
    up = np.where(target & ~oar, 1.07, up)
    row_ptr = np.zeros(nv + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols = C[ok].astype(np.int32)
    vals = V[ok].astype(np.float32)
    lower = lo.astype(np.float64)
    upper = up.astype(np.float64)
    meta = dict(n_target=int(target.sum()), n_oar=int(oar.sum()), n_overlap=int(overlap.sum()),
                target_rows=np.nonzero(target)[0], oar_rows=np.nonzero(oar)[0])
    if infeasible and overlap.any():
        dup = np.nonzero(overlap)[0]
        lower[dup] = 0.95
        upper[dup] = 1.07
        dcounts = counts[dup]
        drp = np.zeros(dup.size + 1, np.int64)
        np.cumsum(dcounts, out=drp[1:])
        dcols = np.concatenate([C[i, ok[i]] for i in dup]).astype(np.int32)
        dvals = np.concatenate([V[i, ok[i]] for i in dup]).astype(np.float32)
        row_ptr = np.concatenate([row_ptr, row_ptr[-1] + drp[1:]])
        cols = np.concatenate([cols, dcols])
        vals = np.concatenate([vals, dvals])
        lower = np.concatenate([lower, np.full(dup.size, -np.inf)])
        upper = np.concatenate([upper, np.full(dup.size, 0.3)])
    m = row_ptr.size - 1
    # summed body dose: c = A^T 1 over the voxel rows (duplicates excluded)
    c = np.zeros(n)
    np.add.at(c, C[ok], V[ok].astype(np.float32).astype(np.float64))
    params = dict(gamma=1.0, alpha=0.99, n_red=1, restart_every=0)
    if variant == "paper":
        params = dict(gamma=1.0, alpha=0.99, n_red=1, restart_every=500)
    assert row_ptr[-1] < 2**31
    return Workload(
        name=f"rt{X}x{Y}x{Z}",
        m=m,
        n=n,
        row_ptr=row_ptr.astype(np.int32),
        col_idx=cols,
        val=vals,
        lower=lower.astype(np.float32)[:, None],
        upper=upper.astype(np.float32)[:, None],
        box_lo=np.zeros(n, np.float32),
        box_hi=np.full(n, np.inf, np.float32),
        x0=np.zeros((n, 1), np.float32),
        lam=1.0,
        obj=OBJ_LINEAR,
        linear_c=c.astype(np.float32),
        K=K,
        meta=meta,
        **params,
    )


# ---------------------------------------------------------------------------
# Serving stream
# ---------------------------------------------------------------------------

def serving_mix(
    sizes=(128, 256, 512),
    n_requests: int = 64,
    slices=(8, 32),
    pool: int = 32,
    K: int = 200,
    rate_hz: float = 0.0,
    seed: int = 5,
    n_angles: int = 180,
):
    """A stream of CT solve requests for a serving run.

    One operator per image size (parallel beam, `n_angles` angles); each request
    picks a size uniformly, a slice count uniformly in `slices`, and that many
    slices (own bands and starting point) from a pool of `pool` seeded phantoms
    of that size.  Arrivals are Poisson with `rate_hz` (all at t = 0 when 0).
    Returns (operators, requests): operators map a key to a dict of CSR arrays
    and problem parameters; each request is a dict with op_key, lower [m,S],
    upper [m,S], x0 [n,S], K and t_arrival.
    """
    rng = np.random.default_rng(seed)
    ops = {}
    pools = {}
    for N in sizes:
        w = ct(N=N, n_angles=n_angles, seed=seed * 100 + N, B=pool, K=K)
        key = f"ct{N}"
        ops[key] = dict(m=w.m, n=w.n, row_ptr=w.row_ptr, col_idx=w.col_idx, val=w.val,
                        params=dict(box_lo=w.box_lo, box_hi=w.box_hi, lam=w.lam, obj=w.obj, tv_rows=w.tv_rows,
                                    tv_cols=w.tv_cols, tv_eps=w.tv_eps, gamma=w.gamma, alpha=w.alpha,
                                    n_red=w.n_red, restart_every=w.restart_every, max_trials=w.max_trials))
        pools[key] = w
    reqs = []
    t = 0.0
    for i in range(n_requests):
        key = f"ct{sizes[rng.integers(len(sizes))]}"
        S = int(rng.integers(slices[0], slices[1] + 1))
        pick = rng.choice(pool, size=S, replace=S > pool)
        w = pools[key]
        if rate_hz > 0:
            t += rng.exponential(1.0 / rate_hz)
        reqs.append(dict(rid=i, op_key=key, lower=np.ascontiguousarray(w.lower[:, pick]),
                         upper=np.ascontiguousarray(w.upper[:, pick]), x0=np.ascontiguousarray(w.x0[:, pick]),
                         K=K, t_arrival=t if rate_hz > 0 else 0.0, pool_index=pick))
    return ops, reqs, pools


# ---------------------------------------------------------------------------
# Full-size radiotherapy matrix (C++ generator, same model as rt())
# ---------------------------------------------------------------------------

_RT_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rt_gen.cpp")
_RT_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librtgen.so")


def build_rt_generator(force: bool = False) -> str:
    import subprocess

    if force or not os.path.exists(_RT_LIB):
        tmp = _RT_LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _RT_SRC])
        os.replace(tmp, _RT_LIB)
    return _RT_LIB


def rt_large(
    grid=(160, 160, 80),
    n_beams: int = 9,
    beamlets=(47, 47),
    spacing: float = 3.4,
    mu: float = 0.005,
    rho: float = 2.5,
    r_cut: float = 9.2,
    seed: int = 4,
    infeasible: bool = True,
    K: int = 300,
    variant: str = "default",
    angle_offset: float = 0.0,
) -> Workload:
    """The rt() model at full size, generated row by row in C++ (OpenMP).

    Defaults: 160 x 160 x 80 voxels (2.05M rows), 9 beams of 47 x 47 beamlets
    (19,881 columns); spacing and cutoff give about 1 % density.  Structures,
    bands, the infeasible duplicated overlap rows, the scaling to a mean target
    dose of 1 and the summed-dose objective are those of rt().
    """
    import ctypes as C

    lib = C.CDLL(build_rt_generator())

    class _P(C.Structure):
        _fields_ = [("X", C.c_int32), ("Y", C.c_int32), ("Z", C.c_int32), ("n_beams", C.c_int32),
                    ("nbu", C.c_int32), ("nbw", C.c_int32), ("spacing", C.c_double), ("mu", C.c_double),
                    ("rho", C.c_double), ("r_cut", C.c_double), ("angle0", C.c_double)]

    X, Y, Z = grid
    P = _P(X, Y, Z, n_beams, beamlets[0], beamlets[1], spacing, mu, rho, r_cut, angle_offset)
    nv = X * Y * Z
    n = n_beams * beamlets[0] * beamlets[1]
    counts = np.zeros(nv, np.int64)
    lib.rt_count(C.byref(P), counts.ctypes.data_as(C.POINTER(C.c_int64)))
    row_ptr = np.zeros(nv + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    cols = np.empty(nnz, np.int32)
    vals = np.empty(nnz, np.float64)
    lib.rt_fill(C.byref(P), row_ptr.ctypes.data_as(C.POINTER(C.c_int64)), cols.ctypes.data_as(C.POINTER(C.c_int32)),
                vals.ctypes.data_as(C.POINTER(C.c_double)))
    # structures (as in rt())
    ci = (np.arange(X) + 0.5) - X / 2.0
    cj = (np.arange(Y) + 0.5) - Y / 2.0
    ck = (np.arange(Z) + 0.5) - Z / 2.0
    PX, PY, PZ = np.meshgrid(ci, cj, ck, indexing="ij")
    PX, PY, PZ = PX.reshape(-1), PY.reshape(-1), PZ.reshape(-1)
    rr = np.sqrt(PX**2 + PY**2 + PZ**2)
    R_t = 0.25 * min(X, Y, 2 * Z)
    target = rr <= R_t
    oar = (np.hypot(PX - R_t * 1.1, PY) <= 0.45 * R_t) & (np.abs(PZ) <= 0.8 * R_t)
    overlap = target & oar
    nonempty = counts > 0
    d1 = np.zeros(nv)
    d1[nonempty] = np.add.reduceat(vals, row_ptr[:-1][nonempty])
    scale = 1.0 / max(d1[target].mean(), 1e-30)
    vals *= scale
    val32 = vals.astype(np.float32)
    del vals
    up = np.where(oar, 0.5, 1.07)
    lo = np.where(target, 0.95, -np.inf)
    up = np.where(target & ~oar, 1.07, up)
    c = np.bincount(cols, weights=val32.astype(np.float64), minlength=n)
    lower, upper = lo.astype(np.float64), up.astype(np.float64)
    meta = dict(n_target=int(target.sum()), n_oar=int(oar.sum()), n_overlap=int(overlap.sum()),
                target_rows=np.nonzero(target)[0], oar_rows=np.nonzero(oar)[0])
    if infeasible and overlap.any():
        dup = np.nonzero(overlap)[0]
        lower[dup] = 0.95
        upper[dup] = 1.07
        seg = [np.arange(row_ptr[i], row_ptr[i + 1]) for i in dup]
        take = np.concatenate(seg)
        drp = np.zeros(dup.size + 1, np.int64)
        np.cumsum(counts[dup], out=drp[1:])
        row_ptr = np.concatenate([row_ptr, row_ptr[-1] + drp[1:]])
        cols = np.concatenate([cols, cols[take]])
        val32 = np.concatenate([val32, val32[take]])
        lower = np.concatenate([lower, np.full(dup.size, -np.inf)])
        upper = np.concatenate([upper, np.full(dup.size, 0.3)])
    m = row_ptr.size - 1
    assert row_ptr[-1] < 2**31
    params = dict(gamma=1.0, alpha=0.99, n_red=1, restart_every=0)
    if variant == "paper":
        params = dict(gamma=1.0, alpha=0.99, n_red=1, restart_every=500)
    return Workload(
        name=f"rt{X}x{Y}x{Z}",
        m=m,
        n=n,
        row_ptr=row_ptr.astype(np.int32),
        col_idx=cols,
        val=val32,
        lower=lower.astype(np.float32)[:, None],
        upper=upper.astype(np.float32)[:, None],
        box_lo=np.zeros(n, np.float32),
        box_hi=np.full(n, np.inf, np.float32),
        x0=np.zeros((n, 1), np.float32),
        lam=1.0,
        obj=OBJ_LINEAR,
        linear_c=c.astype(np.float32),
        K=K,
        meta=meta,
        **params,
    )
