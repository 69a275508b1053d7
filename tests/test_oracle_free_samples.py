"""Pins of the oracle's free-space samples (Sec. III; reading R4) and voxel
indices (readings R5/R6).

The binary32 recipe is re-derived here with numpy float32 operations (every
numpy float32 ufunc rounds once, with no fused multiply-add), which is an
implementation independent of the C oracle; equality is bit for bit.  The
geometric checks hold for any correct linear interpolation along a beam.
"""
import numpy as np
import pytest

import oracle
import scenes


def np_free_samples(xyz, label, origin, s):
    """numpy float32 restatement of reading R4."""
    f = np.float32
    o = origin.astype(np.float32)
    s = f(s)
    out, par = [], []
    for i in range(xyz.shape[0]):
        if label[i] == -1:
            continue
        v = (xyz[i] - o).astype(np.float32)
        L = np.sqrt(f(f(v[0] * v[0]) + f(v[1] * v[1])) + f(v[2] * v[2]))
        if not (L > 0 and s > 0):
            continue
        n = int(np.ceil(f(L / s))) - 1
        for j in range(1, n + 1):
            t = f(f(j) * s)
            w = f(t / L)
            q = (o + (w * v).astype(np.float32)).astype(np.float32)
            out.append(q)
            par.append(i)
    return np.array(out, dtype=np.float32).reshape(-1, 3), np.array(par, dtype=np.int64)


def test_free_samples_bit_exact_against_numpy_float32():
    sc = scenes.make_config(0).scans[0]
    sel = slice(0, 300)
    xyz, lab = sc.xyz[sel].copy(), sc.label[sel].copy()
    lab[::37] = -1                                   # dropped beams (reading R10)
    q, par = oracle.free_samples(xyz, lab, sc.origin, 0.1, 4)
    q2, par2 = np_free_samples(xyz, lab, sc.origin, 0.1)
    assert q.shape == q2.shape
    assert np.array_equal(par, par2)
    assert np.array_equal(q.view(np.uint32), q2.view(np.uint32))


def test_free_samples_lie_on_the_beam_at_even_spacing():
    rng = np.random.default_rng(7)
    o = np.array([3.25, -40.5, 1.73], np.float32)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rng_len = rng.uniform(0.05, 50.0, size=200)
    xyz = (o + d * rng_len[:, None]).astype(np.float32)
    lab = np.ones(200, np.int32)
    s = 0.3
    q, par = oracle.free_samples(xyz, lab, o, s, 2)
    counts = np.bincount(par, minlength=200)
    L = np.linalg.norm(xyz.astype(np.float64) - o, axis=1)
    # n = ceil(L/s) - 1 samples strictly inside the beam (exact-multiple cases aside)
    assert np.all(np.abs(counts - (np.ceil(L / s) - 1)) <= 1)
    for i in np.flatnonzero(counts)[:50]:
        pts = q[par == i].astype(np.float64)
        t = np.linalg.norm(pts - o, axis=1)
        np.testing.assert_allclose(t, s * np.arange(1, counts[i] + 1), rtol=0, atol=2e-5)
        # distance from the line o + t d
        u = (xyz[i].astype(np.float64) - o) / L[i]
        perp = (pts - o) - np.outer((pts - o) @ u, u)
        assert np.abs(perp).max() < 2e-5
        assert np.all(t < L[i] + 1e-5)


def test_free_sample_count_edge_cases():
    o = np.zeros(3, np.float32)
    # exact multiple: L = 1.0, s = 0.25 -> samples at 0.25, 0.5, 0.75 (the hit is not one)
    xyz = np.array([[1.0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0.5, 0], [0, 0, 2.0]], np.float32)
    lab = np.array([1, 1, 1, -1, 1], np.int32)
    counts, tot = oracle.free_counts(xyz, lab, o, 0.25, 2)
    assert counts.tolist() == [3, 0, 0, 0, 7]      # L < s -> 0 ; L = 0 -> 0 ; label -1 -> 0
    assert tot == 10
    # free_step <= 0 -> no samples
    counts, tot = oracle.free_counts(xyz, lab, o, 0.0, 2)
    assert tot == 0


def test_free_samples_input_errors():
    o = np.zeros(3, np.float32)
    xyz = np.array([[1.0, 0, 0]], np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.free_counts(xyz, np.array([5], np.int32), o, 0.1, 4)
    assert e.value.code == oracle.E_INPUT
    with pytest.raises(oracle.OracleError):
        oracle.free_counts(np.array([[np.nan, 0, 0]], np.float32), np.array([1], np.int32), o, 0.1, 4)
    # more than 2^20 samples on one beam
    with pytest.raises(oracle.OracleError):
        oracle.free_counts(np.array([[2.0e5, 0, 0]], np.float32), np.array([1], np.int32), o, 0.1, 4)


def test_voxel_coords_are_float32_floor_of_quotient():
    rng = np.random.default_rng(3)
    xyz = rng.uniform(-60, 60, size=(5000, 3)).astype(np.float32)
    xyz[:10] = np.float32(0.3) * np.arange(10, dtype=np.float32)[:, None]   # near cell faces
    xyz[10:20] = -xyz[:10]
    res = np.float32(0.1)
    ijk = oracle.voxel_coords(xyz, res)
    expect = np.floor((xyz / res).astype(np.float32)).astype(np.int32)
    assert np.array_equal(ijk, expect)
    # negative coordinates floor downward
    assert oracle.voxel_coords(np.array([[-0.05, -0.1, -1e-9]], np.float32), 0.1).tolist() == [[-1, -1, -1]]
    # out of range index (|i| >= 2^20) is an error
    with pytest.raises(oracle.OracleError) as e:
        oracle.voxel_coords(np.array([[2.0e5, 0, 0]], np.float32), 0.1)
    assert e.value.code == oracle.E_RANGE


def test_training_set_order_and_labels():
    sc = scenes.make_config(0).scans[0]
    lab = sc.label.copy()
    lab[5] = -1
    tx, ty, par = oracle.training_set(sc.xyz, lab, sc.origin, 0.1, 4, free_class=0)
    nh = int((lab != -1).sum())
    assert np.array_equal(tx[:nh], sc.xyz[lab != -1])
    assert np.array_equal(ty[:nh], lab[lab != -1])
    assert np.all(ty[nh:] == 0)
    assert np.all(np.diff(par[nh:]) >= 0) and 5 not in par
