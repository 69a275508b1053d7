"""Pins of the oracle's map update: Eq. (7) at grid centroids (Sec. IV),
Eq. (2) (S-CSM) and the readout of Eq. (3)-(4).

What fixes the expected values:
  * brute force: an all-pairs numpy evaluation written here, on tiny inputs;
  * a worked example whose voxel count is combinatorial (one measurement on a
    voxel centre, binary-exact geometry);
  * invariants of Eq. (7): the K = 2 reduction of Sec. III, linearity in
    sigma0, additivity over scans (the recursive update), permutation and
    whole-block translation invariance, locality;
  * the Dirichlet moments (mean sums to one, variance bound).
"""
import json
import os

import numpy as np
import pytest

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_alpha_numpy(tx, ty, ijk, res, K, l, sigma0, alpha0):
    """All pairs in numpy (double), independent of the C code; f from the oracle."""
    c = (ijk.astype(np.float64) + 0.5) * np.float64(np.float32(res))
    d = np.linalg.norm(c[:, None, :] - tx.astype(np.float64)[None, :, :], axis=2)
    L = np.float64(np.float32(l))
    w = np.where(d < L, np.float64(np.float32(sigma0)) * oracle.kernel_f(np.minimum(d / L, 1.0)), 0.0)
    a = np.full((ijk.shape[0], K), np.float64(np.float32(alpha0)))
    for k in range(K):
        a[:, k] += w[:, ty == k].sum(axis=1)
    return a, (d < L).sum(axis=1)


def region_voxels(xyz, res, pad):
    lo = np.floor(xyz.min(0) / res).astype(int) - pad
    hi = np.floor(xyz.max(0) / res).astype(int) + pad
    g = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
    I, J, K = np.meshgrid(*g, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], 1).astype(np.int32)


def test_map_matches_brute_force_on_tiny_inputs():
    for seed in range(3):
        sc = scenes.random_points_scene(seed, 60, K=3, extent=0.45, centre=(-0.3, 0.12, 5.07))
        p = sc.params.f32()
        xyz, lab = sc.scans[0].xyz, sc.scans[0].label
        m = oracle.OracleMap.from_params(p)
        m.insert_training(xyz, lab)
        vox = region_voxels(xyz, p.res, 4)
        a_bf, n_bf = brute_alpha_numpy(xyz, lab, vox, p.res, p.K, p.l, p.sigma0, p.alpha0)
        a_map = m.lookup(vox)
        np.testing.assert_allclose(a_map, a_bf, rtol=1e-13, atol=0)
        # the map stores exactly the voxels with an in-support point (+ band-only rows)
        ijk, a, nv, nb = m.export()
        assert set(map(tuple, ijk[nv > 0])) == set(map(tuple, vox[n_bf > 0]))
        # the gather form (C, all training points per voxel) agrees as well
        a_g, n_g, _ = oracle.alpha_at_voxels(xyz, lab, vox, p.res, p.K, p.l, p.sigma0, p.alpha0)
        np.testing.assert_allclose(a_g, a_bf, rtol=1e-13)
        assert np.array_equal(n_g, n_bf)


def test_single_measurement_worked_example():
    # res = 1/8, l = 3/8 are binary-exact, and so is a hit on a voxel centre:
    # voxels at integer offset D with |D|^2 <= 8 get alpha0 + sigma0 f(|D|/3);
    # shells |D|^2 = 0..8 hold 1, 6, 12, 8, 6, 24, 24, 0, 12 voxels -> 93 in
    # support; |D|^2 = 9 (r = 1 exactly, 30 voxels) is outside (d < l strictly).
    m = oracle.OracleMap(K=3, res=0.125, block_size=8, l=0.375, sigma0=1.0, alpha0=0.001)
    hit = np.array([[(5 + 0.5) * 0.125, (-3 + 0.5) * 0.125, (7 + 0.5) * 0.125]], np.float32)
    m.insert_training(hit, np.array([2], np.int32))
    ijk, a, nv, nb = m.export()
    D = ijk - np.array([5, -3, 7])
    n2 = (D ** 2).sum(1)
    inside = nv > 0
    assert inside.sum() == 93
    assert np.bincount(n2[inside], minlength=9).tolist() == [1, 6, 12, 8, 6, 24, 24, 0, 12]
    assert (nb > 0).sum() == 30 and np.all(n2[nb > 0] == 9) and np.all(nv[nb > 0] == 0)
    a0 = float(np.float32(0.001))                  # the prior arrives as binary32
    np.testing.assert_array_equal(a[:, 0], a0)
    np.testing.assert_array_equal(a[:, 1], a0)
    # closed forms at |D| = 0, 1, 2: f = 1, 1/3 + sqrt3/(4 pi), 1/6 - sqrt3/(4 pi)
    for n, f in [(0, 1.0), (1, 1 / 3 + np.sqrt(3) / (4 * np.pi)), (4, 1 / 6 - np.sqrt(3) / (4 * np.pi))]:
        np.testing.assert_allclose(a[inside & (n2 == n), 2], a0 + f, rtol=1e-14)


def test_k2_reduction_to_binary_counting_model():
    # Sec. III: with K = 2 (free, occupied) the semantic model reverts to the
    # binary one.  A K-class map and a 2-class map of the same scan with every
    # occupied label mapped to 1 agree: free alpha equal, occupied alpha = sum of
    # the occupied classes minus the extra priors.
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    sel = slice(0, 400)
    mK = oracle.OracleMap.from_params(p)
    mK.insert_scan(s.xyz[sel], s.label[sel], s.origin, p.free_step)
    m2 = oracle.OracleMap(2, p.res, p.block_size, p.l, p.sigma0, p.alpha0)
    m2.insert_scan(s.xyz[sel], np.minimum(s.label[sel], 1), s.origin, p.free_step)
    ijk, aK, nvK, _ = mK.export()
    ijk2, a2, nv2, _ = m2.export()
    assert np.array_equal(ijk, ijk2) and np.array_equal(nvK, nv2)
    np.testing.assert_allclose(a2[:, 0], aK[:, 0], rtol=1e-15)
    np.testing.assert_allclose(a2[:, 1], aK[:, 1:].sum(1) - (p.K - 2) * p.alpha0, rtol=1e-12)
    # a scene with a single occupied class leaves the other classes at alpha0
    m1 = oracle.OracleMap.from_params(p)
    only = s.label[sel] == 2
    m1.insert_scan(s.xyz[sel][only], s.label[sel][only], s.origin, p.free_step)
    _, a1, _, _ = m1.export()
    assert np.all(a1[:, 1] == np.float32(p.alpha0)) and np.all(a1[:, 3] == np.float32(p.alpha0))


def test_linear_in_sigma0_and_additive_over_scans():
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    A, B = slice(0, 250), slice(250, 600)
    m1 = oracle.OracleMap(p.K, p.res, 8, p.l, 1.0, p.alpha0)
    m2 = oracle.OracleMap(p.K, p.res, 8, p.l, 2.0, p.alpha0)
    for m in (m1, m2):
        m.insert_scan(s.xyz[A], s.label[A], s.origin, p.free_step)
    _, a1, _, _ = m1.export()
    _, a2, _, _ = m2.export()
    np.testing.assert_allclose(a2 - p.alpha0, 2 * (a1 - p.alpha0), rtol=1e-13, atol=1e-18)
    # recursive update (Sec. IV): insert(A); insert(B) == insert(A u B)
    mab = oracle.OracleMap.from_params(p)
    mab.insert_scan(s.xyz[A], s.label[A], s.origin, p.free_step)
    mab.insert_scan(s.xyz[B], s.label[B], s.origin, p.free_step)
    mu = oracle.OracleMap.from_params(p)
    mu.insert_scan(s.xyz[:600], s.label[:600], s.origin, p.free_step)
    i1, x1, n1, _ = mab.export()
    i2, x2, n2, _ = mu.export()
    assert np.array_equal(i1, i2) and np.array_equal(n1, n2)
    np.testing.assert_allclose(x1, x2, rtol=1e-12)


def test_permutation_and_block_translation_invariance():
    sc = scenes.random_points_scene(11, 400, K=4, extent=0.7, res=0.125, l=0.375)
    p = sc.params.f32()
    xyz, lab = sc.scans[0].xyz, sc.scans[0].label
    # xyz on a 2^-12 grid so that whole-metre shifts are exact in binary32
    xyz = (np.round(xyz * 4096) / 4096).astype(np.float32)
    m = oracle.OracleMap.from_params(p)
    m.insert_training(xyz, lab)
    perm = np.random.default_rng(0).permutation(xyz.shape[0])
    mp = oracle.OracleMap.from_params(p)
    mp.insert_training(xyz[perm], lab[perm])
    i1, a1, n1, _ = m.export()
    i2, a2, n2, _ = mp.export()
    assert np.array_equal(i1, i2) and np.array_equal(n1, n2)
    np.testing.assert_allclose(a1, a2, rtol=1e-13)
    shift = np.array([3.0, -5.0, 1.0], np.float32)           # 24, -40, 8 voxels = 3, -5, 1 blocks
    mt = oracle.OracleMap.from_params(p)
    mt.insert_training((xyz + shift).astype(np.float32), lab)
    i3, a3, n3, _ = mt.export()
    assert np.array_equal(i3, i1 + np.array([24, -40, 8]))
    np.testing.assert_allclose(a3, a1, rtol=1e-12)


def test_locality_and_counts_against_brute_force_on_tiny_scene():
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    m = oracle.OracleMap.from_params(p)
    m.insert_scan(s.xyz, s.label, s.origin, p.free_step)
    ijk, a, nv, nb = m.export()
    tx, ty, _ = oracle.training_set(s.xyz, s.label, s.origin, p.free_step, p.K)
    # voxels of the 32^3 query grid: the map's values equal Eq. (7) by definition
    q = sc.query_ijk
    ag, ng, _ = oracle.alpha_at_voxels(tx, ty, q, p.res, p.K, p.l, p.sigma0, p.alpha0)
    np.testing.assert_allclose(m.lookup(q), ag, rtol=1e-12)
    # voxels farther than l from every training point keep alpha0 exactly
    far = ng == 0
    assert far.sum() > 0 and np.all(m.lookup(q[far]) == np.float32(p.alpha0))


def test_scsm_counts_are_exact_integers():
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    m = oracle.OracleMap(p.K, p.res, 8, p.l, p.sigma0, p.alpha0, scsm=True)
    m.insert_scan(s.xyz, s.label, s.origin, p.free_step)
    ijk, a, nv, _ = m.export()
    tx, ty, _ = oracle.training_set(s.xyz, s.label, s.origin, p.free_step, p.K)
    cells = np.floor((tx / np.float32(p.res)).astype(np.float32)).astype(np.int64)
    key = {}
    for c, y in zip(map(tuple, cells), ty):
        key.setdefault(c, np.zeros(p.K, np.int64))[y] += 1
    assert len(key) == ijk.shape[0]
    for c, alpha in zip(map(tuple, ijk), a):
        np.testing.assert_array_equal(alpha - np.float32(p.alpha0), key[c].astype(np.float64))


def test_readout_moments():
    rng = np.random.default_rng(5)
    a = rng.uniform(0.001, 4.0, size=(1000, 5))
    a[0] = [2.0, 2.0, 1.0, 0.5, 0.5]            # tie: lowest index wins (reading R11)
    r = oracle.readout(a, free_class=0)
    np.testing.assert_allclose(r["mean"].sum(1), 1.0, rtol=1e-14)
    S = a.sum(1)
    assert np.all(r["var"] >= 0) and np.all(r["var"] <= 0.25 / (S[:, None] + 1) + 1e-17)
    assert np.array_equal(r["label"], np.argmax(a, axis=1)) and r["label"][0] == 0
    np.testing.assert_allclose(r["p_occ"], 1 - a[:, 0] / S, rtol=1e-13)
    allgt1 = np.all(a > 1, axis=1)
    assert np.all(np.isnan(r["mode"][~allgt1]))
    np.testing.assert_allclose(r["mode"][allgt1].sum(1), 1.0, rtol=1e-12)
    # variance of the winning class falls as measurements of that class are added
    v = [oracle.readout(np.array([[0.001, 0.001 + n, 0.001]]))["var"][0, 1] for n in range(1, 6)]
    assert np.all(np.diff(v) < 0)


def test_table1_hyperparameters_are_what_the_street_workloads_use():
    g = json.load(open(os.path.join(GOLDEN, "table1_hyperparameters.json")))
    for n in (1,):
        p = scenes.make_config(n).params
        assert (p.l, p.sigma0, p.alpha0, p.res) == (g["l_m"], g["sigma0"], g["alpha0"], g["res_m"])


def test_extended_block_selection_single_hit_at_a_block_corner():
    # The paper's implementation trains each block on its own rows and those of
    # the six face-adjacent blocks (Sec. IV).  One hit on the centre of voxel
    # (7, 7, 7), the corner voxel of block (0, 0, 0) with B = 8: of the 93 voxels
    # in support, those whose block differs from (0, 0, 0) along two or three
    # axes are not reached; the others keep exactly the exact-support value.
    kw = dict(K=3, res=0.125, block_size=8, l=0.375, sigma0=1.0, alpha0=0.001)
    hit = np.array([[(7 + 0.5) * 0.125] * 3], np.float32)
    lab = np.array([1], np.int32)
    exact = oracle.OracleMap(**kw)
    face = oracle.OracleMap(**kw, face_blocks=True)
    exact.insert_training(hit, lab)
    face.insert_training(hit, lab)
    ie, ae, nve, _ = exact.export()
    i_f, af, nvf, _ = face.export()
    D = ie - 7
    off_axes = (D >= 1).sum(1)                     # axes on which the voxel left block 0
    keep = (nve > 0) & (off_axes <= 1)
    # expected count from the offsets alone: |D|^2 <= 8 and at most one axis with D >= 1
    grid = np.stack(np.meshgrid(*[np.arange(-3, 4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    n2 = (grid ** 2).sum(1)
    expect = int(((n2 <= 8) & ((grid >= 1).sum(1) <= 1)).sum())
    assert int((nvf > 0).sum()) == expect == int(keep.sum())
    got = {tuple(v): a for v, a, n in zip(i_f, af, nvf) if n > 0}
    for v, a in zip(ie[keep], ae[keep]):
        np.testing.assert_array_equal(got[tuple(v)], a)
    # every voxel reached under the selection is reached without it, never with more
    assert set(got) <= {tuple(v) for v, n in zip(ie, nve) if n > 0}


def test_extended_block_selection_equals_exact_support_inside_blocks():
    # Rows whose support stays inside their own block see no difference.
    rng = np.random.default_rng(3)
    centres = (rng.integers(-4, 4, size=(40, 3)) * 8 + 4).astype(np.float64)   # block centres (voxels)
    xyz = ((centres + rng.uniform(-1.0, 1.0, size=centres.shape)) * 0.1).astype(np.float32)
    lab = rng.integers(0, 3, size=40).astype(np.int32)
    kw = dict(K=3, res=0.1, block_size=8, l=0.25, sigma0=0.7, alpha0=0.001)
    exact, face = oracle.OracleMap(**kw), oracle.OracleMap(**kw, face_blocks=True)
    exact.insert_training(xyz, lab)
    face.insert_training(xyz, lab)
    ie, ae, _, _ = exact.export()
    i_f, af, _, _ = face.export()
    np.testing.assert_array_equal(ie, i_f)
    np.testing.assert_array_equal(ae, af)


def test_extended_block_selection_is_a_lower_bound_on_a_scene():
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    exact = oracle.OracleMap.from_params(p)
    face = oracle.OracleMap.from_params(p, face_blocks=True)
    for m in (exact, face):
        m.insert_scan(s.xyz[:500], s.label[:500], s.origin, p.free_step)
    ie, ae, _, _ = exact.export()
    af = face.lookup(ie)
    assert np.all(af <= ae * (1 + 1e-15))
    assert np.any(af < ae * (1 - 1e-6))          # the selection does drop rows here


def test_voxel_key_format_worked_values():
    # key = (i + 2^20) << 42 | (j + 2^20) << 21 | (k + 2^20): 21 bits per axis,
    # biased by 2^20, written out here with Python integers
    lim = 1 << 20
    ijk = np.array([[0, 0, 0], [-lim, -lim, -lim], [lim - 1, lim - 1, lim - 1], [3, -7, 12],
                    [-1, 0, 1], [lim - 1, -lim, 5]], np.int32)
    want = [((int(i) + lim) << 42) | ((int(j) + lim) << 21) | (int(k) + lim) for i, j, k in ijk]
    got = oracle.pack_keys(ijk)
    assert [int(v) for v in got] == want
    assert int(got[1]) == 0 and int(got[2]) == (1 << 63) - 1
    # the key order is the lexicographic (i, j, k) order of the voxel indices
    rng = np.random.default_rng(3)
    v = rng.integers(-lim, lim, size=(500, 3)).astype(np.int32)
    v[250:] = v[:250] + rng.integers(-1, 2, size=(250, 3))
    v = np.clip(v, -lim, lim - 1).astype(np.int32)
    lex = np.lexsort((v[:, 2], v[:, 1], v[:, 0]))
    by_key = np.argsort(oracle.pack_keys(v), kind="stable")
    assert np.array_equal(v[lex], v[by_key])


def test_map_insert_does_not_depend_on_the_thread_count():
    # the insert splits the voxels over column tiles; each voxel still sums its
    # rows in row order, so any thread count gives the same bits
    sc = scenes.random_points_scene(11, 4000, K=4, extent=6.0, res=0.1, l=0.3, free_step=0.2,
                                    origin=(0.3, -0.2, 0.5))
    p = sc.params.f32()
    s = sc.scans[0]
    out = []
    for th in (1, 3, 8):
        oracle.set_num_threads(th)
        m = oracle.OracleMap.from_params(p)
        m.insert_scan(s.xyz, s.label, s.origin, p.free_step, p.free_class)
        m.insert_scan(s.xyz[::3], s.label[::3], (s.origin + np.float32(0.5)).astype(np.float32),
                      p.free_step, p.free_class)
        out.append(m.export())
    oracle.set_num_threads(max(1, os.cpu_count() or 1))
    for o in out[1:]:
        for x, y in zip(out[0], o):
            assert np.array_equal(x, y)


def test_last_insert_counts_against_brute_force():
    sc = scenes.random_points_scene(2, 80, K=3, extent=0.5, centre=(1.1, -2.3, 0.4))
    p = sc.params.f32()
    xyz, lab = sc.scans[0].xyz, sc.scans[0].label
    m = oracle.OracleMap.from_params(p)
    m.insert_training(xyz, lab)
    vox = region_voxels(xyz, p.res, 4)
    _, n_bf = brute_alpha_numpy(xyz, lab, vox, p.res, p.K, p.l, p.sigma0, p.alpha0)
    c = m.last_insert()
    assert c["V"] == int((n_bf > 0).sum()) and c["P"] == int(n_bf.sum())
    # a second insert of half the rows: its own counts, not the map's totals
    m.insert_training(xyz[:40], lab[:40])
    _, n2 = brute_alpha_numpy(xyz[:40], lab[:40], vox, p.res, p.K, p.l, p.sigma0, p.alpha0)
    c2 = m.last_insert()
    assert c2["V"] == int((n2 > 0).sum()) and c2["P"] == int(n2.sum())
    # the counting model counts rows and the voxels holding them
    ms = oracle.OracleMap.from_params(p, scsm=True)
    ms.insert_training(xyz, lab)
    cs = ms.last_insert()
    assert cs["P"] == xyz.shape[0]
    assert cs["V"] == len({tuple(v) for v in oracle.voxel_coords(xyz, p.res)})


def test_failed_insert_leaves_the_oracle_map_unchanged():
    sc = scenes.random_points_scene(4, 200, K=3, extent=0.5)
    p = sc.params.f32()
    xyz, lab = sc.scans[0].xyz, sc.scans[0].label
    m = oracle.OracleMap.from_params(p)
    m.insert_training(xyz[:100], lab[:100])
    before = m.export()
    bad = lab[100:].copy()
    bad[-1] = 7
    with pytest.raises(oracle.OracleError):
        m.insert_training(xyz[100:], bad)
    far = xyz[100:].copy()
    far[-1, 0] = 1.0e6          # voxel index beyond 2^20
    with pytest.raises(oracle.OracleError):
        m.insert_training(far, lab[100:])
    after = m.export()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
