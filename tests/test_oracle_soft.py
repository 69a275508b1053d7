"""Pins of the oracle's soft-measurement update (Sec. VI: a hit carries a
vector of class weights instead of one label; each class adds its weight times
the kernel of Eq. (8), the linear-pooling reading).

The pins tie the soft update to the hard one, which the other oracle tests pin
to brute force and closed forms, and to closed forms of its own:
  - a one-hot weight vector is the hard update, bit for bit (all-zero = label -1);
  - the update is linear in the weights, with no renormalisation;
  - a single hit on a voxel centre gives alpha0 + sigma0 f(|D| / 3) p_k;
  - negative or non-finite weights are input errors.
"""
import numpy as np
import pytest

import oracle
import scenes


def one_hot(label, K):
    p = np.zeros((label.shape[0], K), np.float32)
    keep = label >= 0
    p[np.nonzero(keep)[0], label[keep]] = 1.0
    return p


@pytest.mark.parametrize("kw", [{}, {"scsm": True}, {"face_blocks": True}])
def test_one_hot_weights_are_the_hard_update(kw):
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    xyz, lab = s.xyz[:500], s.label[:500].copy()
    lab[::17] = -1                                   # dropped hits and beams
    hard = oracle.OracleMap.from_params(p, **kw)
    hard.insert_scan(xyz, lab, s.origin, p.free_step, p.free_class)
    soft = oracle.OracleMap.from_params(p, **kw)
    soft.insert_scan_soft(xyz, one_hot(lab, p.K), s.origin, p.free_step, p.free_class)
    ih, ah, nh, bh = hard.export()
    i_s, a_s, n_s, b_s = soft.export()
    np.testing.assert_array_equal(ih, i_s)
    np.testing.assert_array_equal(ah, a_s)
    np.testing.assert_array_equal(nh, n_s)
    np.testing.assert_array_equal(bh, b_s)


@pytest.mark.parametrize("scsm", [False, True])
def test_soft_update_is_linear_in_the_weights(scsm):
    # No free samples (a step longer than every beam): the map's increment is
    # c (increment of labels y) + d (increment of labels z), for any c, d >= 0.
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    rng = np.random.default_rng(5)
    xyz = s.xyz[:400]
    y = rng.integers(0, p.K, size=400).astype(np.int32)
    z = rng.integers(0, p.K, size=400).astype(np.int32)
    c, d = np.float32(0.25), np.float32(1.5)          # weights need not sum to one
    probs = np.zeros((400, p.K), np.float32)
    probs[np.arange(400), y] += c
    probs[np.arange(400), z] += d
    far = 1.0e6
    maps = {}
    for name, kind in (("y", y), ("z", z), ("soft", None)):
        m = oracle.OracleMap.from_params(p, scsm=scsm)
        if kind is None:
            m.insert_scan_soft(xyz, probs, s.origin, far, p.free_class)
        else:
            m.insert_scan(xyz, kind, s.origin, far, p.free_class)
        maps[name] = m
    ijk, a_soft, _, _ = maps["soft"].export()
    a0 = np.float64(np.float32(p.alpha0))
    ay = maps["y"].lookup(ijk) - a0
    az = maps["z"].lookup(ijk) - a0
    np.testing.assert_allclose(a_soft - a0, float(c) * ay + float(d) * az, rtol=1e-12, atol=1e-15)
    assert len(maps["soft"]) == len(maps["y"]) == len(maps["z"])   # same positions, same voxels


def test_single_soft_hit_on_a_voxel_centre():
    # res = 1/8, l = 3/8, the hit on the centre of voxel (5, -3, 7): a voxel at
    # integer offset D with |D|^2 <= 8 gets alpha0 + sigma0 f(|D| / 3) p_k.
    sigma0 = 0.5
    m = oracle.OracleMap(K=3, res=0.125, block_size=8, l=0.375, sigma0=sigma0, alpha0=0.001)
    hit = np.array([[(5 + 0.5) * 0.125, (-3 + 0.5) * 0.125, (7 + 0.5) * 0.125]], np.float32)
    pk = np.array([[0.0, 0.25, 0.75]], np.float32)
    m.insert_scan_soft(hit, pk, origin=(0.0, 0.0, 0.0), free_step=0.0, free_class=0)
    ijk, a, nv, _ = m.export()
    n2 = ((ijk - np.array([5, -3, 7])) ** 2).sum(1)
    inside = nv > 0
    assert inside.sum() == 93 and np.all(nv[inside] == 2)   # one row per positive weight
    a0 = float(np.float32(0.001))
    np.testing.assert_array_equal(a[:, 0], a0)       # weight 0: no row, no change
    for n, f in [(0, 1.0), (1, 1 / 3 + np.sqrt(3) / (4 * np.pi)),
                 (4, 1 / 6 - np.sqrt(3) / (4 * np.pi))]:
        sel = inside & (n2 == n)
        np.testing.assert_allclose(a[sel, 1], a0 + sigma0 * 0.25 * f, rtol=1e-14)
        np.testing.assert_allclose(a[sel, 2], a0 + sigma0 * 0.75 * f, rtol=1e-14)


@pytest.mark.parametrize("bad", [-1.0e-3, np.nan, np.inf, -np.inf])
def test_negative_or_non_finite_weights_are_input_errors(bad):
    m = oracle.OracleMap(K=3, res=0.1, block_size=8, l=0.3, sigma0=1.0, alpha0=0.001)
    xyz = np.array([[1.0, 2.0, 0.5], [1.5, 2.5, 0.5]], np.float32)
    probs = np.array([[0.5, 0.5, 0.0], [0.2, bad, 0.8]], np.float32)
    with pytest.raises(oracle.OracleError):
        m.insert_scan_soft(xyz, probs, (0.0, 0.0, 1.0), 0.3)
    assert len(m) == 0


def test_weighted_gather_form_matches_brute_force_and_the_soft_map():
    # The gather form with row weights against an all-pairs numpy evaluation
    # (independent of the C code, f from the oracle), and against the map's soft
    # insert of the same scan (scatter form) on a tiny scene.
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    sel = slice(0, 150)
    probs = scenes.soft_measurements(s.label[sel], p.K, seed=2)
    tx, ty, tw = oracle.training_set_soft(s.xyz[sel], probs, s.origin, p.free_step, p.K,
                                          p.free_class)
    # the rows: one per positive weight, in (hit, class) order, then weight-1 free rows
    nz = np.nonzero(probs > 0)
    nh = nz[0].shape[0]
    np.testing.assert_array_equal(ty[:nh], nz[1])
    np.testing.assert_array_equal(tw[:nh], probs[nz].astype(np.float64))
    np.testing.assert_array_equal(tx[:nh], s.xyz[sel][nz[0]])
    assert np.all(ty[nh:] == p.free_class) and np.all(tw[nh:] == 1.0)
    kept = probs.sum(1) > 0
    fx, _ = oracle.free_samples(s.xyz[sel], np.where(kept, 1, -1).astype(np.int32), s.origin,
                                p.free_step, p.K)
    np.testing.assert_array_equal(tx[nh:], fx)
    m = oracle.OracleMap.from_params(p)
    m.insert_scan_soft(s.xyz[sel], probs, s.origin, p.free_step, p.free_class)
    ijk, a_map, _, _ = m.export()
    rng = np.random.default_rng(0)
    q = ijk[rng.choice(ijk.shape[0], 300, replace=False)]
    a_g, _, _ = oracle.alpha_at_voxels(tx, ty, q, p.res, p.K, p.l, p.sigma0, p.alpha0, weights=tw)
    np.testing.assert_allclose(a_g, m.lookup(q), rtol=1e-12)
    c = (q.astype(np.float64) + 0.5) * np.float64(p.res)
    d = np.linalg.norm(c[:, None, :] - tx.astype(np.float64)[None, :, :], axis=2)
    L = np.float64(p.l)
    kv = np.where(d < L, np.float64(p.sigma0) * oracle.kernel_f(np.minimum(d / L, 1.0)), 0.0)
    a_bf = np.full((q.shape[0], p.K), np.float64(p.alpha0))
    for k in range(p.K):
        a_bf[:, k] += (kv[:, ty == k] * tw[ty == k][None, :]).sum(1)
    np.testing.assert_allclose(a_g, a_bf, rtol=1e-12)
