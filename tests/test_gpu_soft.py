"""GPU parity of the soft-measurement update (Sec. VI: per-hit class-weight
vectors, linear pooling) against the oracle's soft insert, through the C ABI.

Bars: concentrations within 1e-5 relative of the float64 oracle (weights
multiply float32 kernel values, one rounding per pair more than the one-hot
path); a one-hot weight vector reproduces the hard update bit for bit; hit-row
counts exact; invalid weights rejected with the map unchanged.
"""
import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import ALPHA_RTOL, check_counts, compare_map, cuda, gpu_map_of, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    import torch
    from paper_1909_04631_amd import _lib
    _lib.lib()   # raises if the HIP library is missing: no fallback
    torch.cuda.init()


def _print_case(name):
    print(f"[case] {name}", flush=True)


def soft_of(scene, seed=7, **kw):
    return [scenes.soft_measurements(s.label, scene.params.K, seed=seed + i, **kw)
            for i, s in enumerate(scene.scans)]


def gpu_soft_map(scene, probs, scans=None, **kw):
    import torch
    from paper_1909_04631_amd import SemanticMap
    p = scene.params
    m = SemanticMap.from_params(p, **kw)
    for s, pr in zip(scene.scans if scans is None else scans, probs):
        m.insert_scan_soft(cuda(s.xyz), cuda(pr), s.origin, p.free_step)
    torch.cuda.synchronize()
    return m


def oracle_soft_map(scene, probs, scans=None, scsm=False, face_blocks=False):
    p = scene.params.f32()
    m = oracle.OracleMap.from_params(p, scsm=scsm, face_blocks=face_blocks)
    for s, pr in zip(scene.scans if scans is None else scans, probs):
        m.insert_scan_soft(s.xyz, pr, s.origin, p.free_step, p.free_class)
    return m


@pytest.mark.parametrize("top", [1, 3, 20])
def test_soft_tiny_scene_matches_the_oracle(top):
    sc = scenes.make_config(0)
    p = sc.params
    probs = soft_of(sc, top=top)
    _print_case(f"soft tiny top={top}")
    gm = gpu_soft_map(sc, probs)
    om = oracle_soft_map(sc, probs)
    worst, (ijk, a_ref, nv, nb) = compare_map(gm, om, p.K)
    st = gm.stats()
    assert st["n_hits"] == int((probs[-1] > 0).sum())   # one hit row per positive weight
    check_counts(st, nv, nb)
    print(f"soft tiny top={top}: {ijk.shape[0]} voxels, max rel err {worst:.2e}", flush=True)


def test_one_hot_weights_reproduce_the_hard_update_bit_for_bit():
    sc = scenes.make_config(0)
    p = sc.params
    lab = [s.label.copy() for s in sc.scans]
    for l_ in lab:
        l_[::13] = -1
    scans = [scenes.Scan(s.xyz, l_, s.origin) for s, l_ in zip(sc.scans, lab)]
    probs = []
    for l_ in lab:
        pr = np.zeros((l_.shape[0], p.K), np.float32)
        keep = l_ >= 0
        pr[np.nonzero(keep)[0], l_[keep]] = 1.0
        probs.append(pr)
    _print_case("soft one-hot vs hard")
    hard = gpu_map_of(sc, scans=scans)
    soft = gpu_soft_map(sc, probs, scans=scans)
    ijk, _, _, _ = oracle_soft_map(sc, probs, scans=scans).export()
    q = cuda(ijk.astype(np.int32))
    a_h = hard.query(q)["alpha"].cpu().numpy()
    a_s = soft.query(q)["alpha"].cpu().numpy()
    np.testing.assert_array_equal(a_h, a_s)
    sh, ss = hard.stats(), soft.stats()
    assert {k: v for k, v in sh.items() if not k.endswith("_ms")} == \
        {k: v for k, v in ss.items() if not k.endswith("_ms")}


def test_soft_recursive_update_and_reach():
    # two soft scans one after the other, block size 4 and the largest reach
    sc = scenes.random_points_scene(5, 3000, K=5, extent=1.3, centre=(-7.3, 12.9, -0.4),
                                    res=0.2, l=0.89, sigma0=0.4, free_step=0.25,
                                    origin=(-6.0, 11.0, 0.5))
    sc.params.block_size = 4
    s = sc.scans[0]
    A = scenes.Scan(s.xyz[:1700], s.label[:1700], s.origin)
    B = scenes.Scan(s.xyz[1700:], s.label[1700:], s.origin)
    probs = [scenes.soft_measurements(x.label, 5, seed=11 + i, top=4) for i, x in enumerate((A, B))]
    _print_case("soft two scans B=4 l=0.89")
    compare_map(gpu_soft_map(sc, probs, scans=[A, B]), oracle_soft_map(sc, probs, scans=[A, B]),
                sc.params.K)


def test_soft_small_stencil_two_rows_per_step():
    # l / res = 1.5: a stencil of 29 offsets, so the splat takes two rows per
    # step, each half with its own row's weight; two scans, several classes per hit
    sc = scenes.random_points_scene(7, 3000, K=6, extent=1.3, centre=(3.1, -2.2, 0.6),
                                    res=0.2, l=0.3, sigma0=0.7, free_step=0.25,
                                    origin=(1.5, -1.0, 1.2))
    sc.params.block_size = 4
    s = sc.scans[0]
    A = scenes.Scan(s.xyz[:1300], s.label[:1300], s.origin)
    B = scenes.Scan(s.xyz[1300:], s.label[1300:], s.origin)
    probs = [scenes.soft_measurements(x.label, 6, seed=21 + i, top=3) for i, x in enumerate((A, B))]
    _print_case("soft two rows per step")
    compare_map(gpu_soft_map(sc, probs, scans=[A, B]), oracle_soft_map(sc, probs, scans=[A, B]),
                sc.params.K)


def test_soft_counting_model_and_extended_block_selection():
    sc = scenes.make_config(0)
    p = sc.params
    probs = soft_of(sc)
    _print_case("soft S-CSM")
    gm = gpu_soft_map(sc, probs, model="scsm")
    om = oracle_soft_map(sc, probs, scsm=True)
    compare_map(gm, om, p.K)
    _print_case("soft extended block")
    compare_map(gpu_soft_map(sc, probs, selection="face_blocks"),
                oracle_soft_map(sc, probs, face_blocks=True), p.K)


def test_invalid_weights_leave_the_map_unchanged():
    import torch
    from paper_1909_04631_amd import SmkiError
    sc = scenes.make_config(0)
    p = sc.params
    s = sc.scans[0]
    pr = scenes.soft_measurements(s.label, p.K, seed=3)
    gm = gpu_soft_map(sc, [pr[:500]], scans=[scenes.Scan(s.xyz[:500], s.label[:500], s.origin)])
    before = gm.export()
    for bad in (-0.25, np.nan, np.inf):
        b = pr[500:900].copy()
        b[17, 3] = bad
        with pytest.raises(SmkiError) as e:
            gm.insert_scan_soft(cuda(s.xyz[500:900]), cuda(b), s.origin, p.free_step)
        assert e.value.status == -5
    with pytest.raises(ValueError):   # one row of K weights per hit
        gm.insert_scan_soft(cuda(s.xyz[500:900]), cuda(pr[500:900, :p.K - 1]), s.origin, p.free_step)
    # all-zero rows drop their hits and beams: an all-zero scan changes nothing
    gm.insert_scan_soft(cuda(s.xyz[500:900]), cuda(np.zeros((400, p.K), np.float32)), s.origin,
                        p.free_step)
    gm.insert_scan_soft(cuda(s.xyz[:0]), cuda(pr[:0]), s.origin, p.free_step)
    torch.cuda.synchronize()
    after = gm.export()
    assert all(torch.equal(x, y) for x, y in zip(before, after))


def test_soft_lidar_scan_full_size_sampled():
    sc = scenes.make_config(1)
    p = sc.params.f32()
    s = sc.scans[0]
    pr = scenes.soft_measurements(s.label, p.K, seed=1)
    _print_case(f"soft lidar full size n={s.xyz.shape[0]}")
    gm = gpu_soft_map(sc, [pr])
    st = gm.stats()
    print("soft lidar stats", st, flush=True)
    tx, ty, tw = oracle.training_set_soft(s.xyz, pr, s.origin, p.free_step, p.K, p.free_class)
    nh = int((pr > 0).sum())
    assert st["n_hits"] == nh and st["n_free"] == tx.shape[0] - nh
    rng = np.random.default_rng(0)
    vh = oracle.voxel_coords(s.xyz[rng.choice(s.xyz.shape[0], 120, replace=False)], p.res)
    vs = oracle.voxel_coords((s.origin + rng.uniform(-1.5, 1.5, size=(60, 3))).astype(np.float32),
                             p.res)
    vr = oracle.voxel_coords(tx[rng.choice(tx.shape[0], 120, replace=False)], p.res)
    q = np.concatenate([vh, vs, vr]).astype(np.int32)
    a_ref, _, _ = oracle.alpha_at_voxels(tx, ty, q, p.res, p.K, p.l, p.sigma0, p.alpha0,
                                         weights=tw)
    a = gm.query(cuda(q))["alpha"].cpu().numpy()
    err = rel_err(a, a_ref)
    print(f"soft lidar sampled max rel err {err.max():.2e}", flush=True)
    assert err.max() <= ALPHA_RTOL
