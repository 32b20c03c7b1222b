"""Seeded input generators: geometry checks against closed forms, size checks
against the configured workloads, reproducibility."""
import math

import numpy as np
import pytest

import workloads as W


def test_ct_row_sums_are_chords():
    """Each CT row sums to the length of its ray inside the unit square."""
    N, n_ang = 32, 12
    row_ptr, cols, lens = W.ct_matrix(N, n_ang, 46)
    h = 1.0 / N
    offs = (np.arange(46) - 45 / 2.0) * h
    sums = np.add.reduceat(lens, row_ptr[:-1].clip(max=len(lens) - 1).astype(np.int64))
    sums[np.diff(row_ptr) == 0] = 0.0
    for a in range(n_ang):
        th = a * np.pi / n_ang
        c, s = math.cos(th), math.sin(th)
        for d in range(46):
            t = offs[d]
            # chord of the line {p : p.(c,s) = t} through [-1/2, 1/2]^2 (Liang-Barsky on the box)
            p0 = np.array([t * c + s, t * s - c])
            dvec = np.array([-2 * s, 2 * c])
            lo, hi = 0.0, 1.0
            for k in range(2):
                if abs(dvec[k]) < 1e-15:
                    if not (-0.5 <= p0[k] <= 0.5):
                        lo, hi = 1.0, 0.0
                    continue
                t1, t2 = (-0.5 - p0[k]) / dvec[k], (0.5 - p0[k]) / dvec[k]
                lo, hi = max(lo, min(t1, t2)), min(hi, max(t1, t2))
            chord = max(0.0, hi - lo) * 2.0
            assert sums[a * 46 + d] == pytest.approx(chord, abs=1e-9)


def test_seismic_constant_slowness_travel_time():
    rows, cols, ns, nr = 20, 40, 5, 8
    row_ptr, ci, lens = W.seismic_matrix(rows, cols, ns, nr)
    sums = np.add.reduceat(lens, row_ptr[:-1].astype(np.int64))
    xs = (np.arange(ns) + 0.5) * cols / ns
    xr = (np.arange(nr) + 0.5) * cols / nr
    for a in range(ns):
        for b in range(nr):
            dist = math.hypot(xr[b] - xs[a], rows)
            assert 1.7 * sums[a * nr + b] == pytest.approx(1.7 * dist, rel=1e-12)


def test_sizes_match_the_configured_workloads():
    w = W.ct(N=256, seed=2)
    assert (w.m, w.n) == (180 * 363, 65536)
    assert 12e6 <= w.nnz <= 20e6  # about 15-17M
    s = W.seismic(seed=3)
    assert (s.m, s.n) == (20000, 80000)
    assert 4.8e6 <= s.nnz <= 8e6  # about 6M
    d = W.dense_small()
    assert (d.m, d.n, d.nnz) == (256, 128, 32768)


def test_generators_are_reproducible():
    a = W.ct(N=24, n_angles=10, seed=9, B=2)
    b = W.ct(N=24, n_angles=10, seed=9, B=2)
    for f in ("row_ptr", "col_idx", "val", "lower", "upper", "x0"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    c = W.ct(N=24, n_angles=10, seed=10, B=2)
    assert not np.array_equal(a.lower, c.lower)


def test_dense_case_is_consistent():
    """The hidden point satisfies every band and the box."""
    w = W.dense_small()
    r = w.dense() @ w.x_true[:, 0].astype(np.float64)
    assert np.all(r >= w.lower[:, 0] - 1e-4) and np.all(r <= w.upper[:, 0] + 1e-4)
    assert np.all((w.x_true >= 0) & (w.x_true <= 1))


@pytest.mark.parametrize("angle", [0.0, 0.37])
def test_rt_cpp_generator_matches_numpy_model(angle):
    a = W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=10, angle_offset=angle)
    b = W.rt_large(grid=(20, 20, 10), beamlets=(6, 6), spacing=2.4, rho=2.0, r_cut=6.4, angle_offset=angle)
    for f in ("row_ptr", "col_idx", "lower", "upper"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    np.testing.assert_allclose(b.val, a.val, rtol=1e-6)
    np.testing.assert_allclose(b.linear_c, a.linear_c, rtol=1e-6)
    assert a.meta.keys() == b.meta.keys()
    for k in a.meta:
        assert np.array_equal(a.meta[k], b.meta[k]), k


def test_rt_infeasible_rows_conflict():
    """Every duplicated overlap row has a band disjoint from its original row's."""
    w = W.rt(grid=(20, 20, 10), beamlets=(6, 6), seed=10)
    nv = 20 * 20 * 10
    dup_rows = np.arange(nv, w.m)
    assert dup_rows.size == w.meta["n_overlap"] > 0
    assert np.all(w.upper[dup_rows, 0] < 0.95)
    # the duplicate carries the same coefficients as some target row with lower bound 0.95
    rp = w.row_ptr
    first = dup_rows[0]
    seg = w.val[rp[first]:rp[first + 1]]
    matches = [i for i in range(nv) if rp[i + 1] - rp[i] == seg.size and np.array_equal(w.val[rp[i]:rp[i + 1]], seg)]
    assert matches and w.lower[matches[0], 0] == pytest.approx(0.95)


def test_serving_mix_shapes():
    ops, reqs, pools = W.serving_mix(sizes=(16, 24), n_requests=12, slices=(2, 4), pool=5, K=7, seed=3,
                                     n_angles=10, rate_hz=100.0)
    assert set(ops) == {"ct16", "ct24"}
    t = [r["t_arrival"] for r in reqs]
    assert t == sorted(t) and t[0] > 0
    for r in reqs:
        o = ops[r["op_key"]]
        S = r["lower"].shape[1]
        assert 2 <= S <= 4 and r["upper"].shape == (o["m"], S) and r["x0"].shape == (o["n"], S)


def test_fresnel_rows_sum_to_ray_lengths():
    """Constant slowness s gives travel times s * L, L the source-receiver
    distance (each band row is scaled to sum to its ray's length)."""
    N, ns, nr = 40, 6, 10
    rp, ci, v = W.fresnel_matrix(N, ns, nr)
    sums = np.add.reduceat(v, rp[:-1].astype(np.int64))
    ys = (np.arange(ns) + 0.5) * N / ns
    half = nr // 2
    for a in range(ns):
        for b in range(nr):
            if b < half:
                p1 = (0.0, (b + 0.5) * N / half)
            else:
                p1 = ((b - half + 0.5) * N / (nr - half), 0.0)
            L = math.hypot(p1[0] - N, p1[1] - ys[a])
            assert sums[a * nr + b] == pytest.approx(L, rel=1e-12)
    assert np.all(v > 0) and np.all((ci >= 0) & (ci < N * N))


def test_fresnel_paper_shape():
    w = W.seismic_fresnel(N=32, n_src=8, n_rec=16, K=3)
    assert (w.m, w.n) == (8 * 16, 32 * 32) and w.basic == W.BASIC_DROP and w.lam == w.m
    np.testing.assert_array_equal(w.lower, w.upper)
