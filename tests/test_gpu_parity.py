"""GPU parity of the S-BKI map update against the float64 CPU oracle.

Every call goes through the C ABI (libsmki.so) via the thin binding.  Bars:
bit-exact for free-sample positions, voxel keys, cell counts and cell id sets;
float32 concentrations within 1e-5 relative of the oracle; updated-voxel and
pair counts exact up to pairs inside the rounding band of the support edge.
"""
import os

import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import ALPHA_RTOL, check_counts, compare_map, cuda, gpu_map_of, oracle_map_of, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    import torch
    from paper_1909_04631_amd import _lib
    _lib.lib()   # raises if the HIP library is missing: no fallback
    torch.cuda.init()


def _print_case(name):
    print(f"[case] {name}", flush=True)


# ---------------------------------------------------------------------------
# free samples and bucketing: integer / bit-exact work
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg,step,sub", [(0, 0.1, None), (1, 0.3, slice(0, None, 7))])
def test_free_samples_bit_exact(cfg, step, sub):
    from paper_1909_04631_amd import free_samples
    sc = scenes.make_config(cfg)
    s = sc.scans[0]
    xyz, lab = (s.xyz, s.label) if sub is None else (s.xyz[sub], s.label[sub])
    lab = lab.copy()
    lab[::101] = -1
    _print_case(f"free samples cfg={cfg} n={xyz.shape[0]}")
    q_ref, par_ref = oracle.free_samples(xyz, lab, s.origin, step, sc.params.K)
    q, par = free_samples(cuda(xyz), cuda(lab), s.origin, step, sc.params.K)
    q, par = q.cpu().numpy(), par.cpu().numpy()
    assert q.shape == q_ref.shape
    assert np.array_equal(par, par_ref)
    assert np.array_equal(q.view(np.uint32), q_ref.view(np.uint32))


def test_free_samples_edge_cases():
    from paper_1909_04631_amd import free_samples, SmkiError
    o = np.zeros(3, np.float32)
    xyz = np.array([[1.0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0.5, 0]], np.float32)
    lab = np.array([1, 1, 1, -1], np.int32)
    q, par = free_samples(cuda(xyz), cuda(lab), o, 0.25, 2)
    assert par.cpu().tolist() == [0, 0, 0]
    q, par = free_samples(cuda(xyz[:0]), cuda(lab[:0]), o, 0.25, 2)
    assert q.shape[0] == 0
    with pytest.raises(SmkiError) as e:
        free_samples(cuda(xyz), cuda(np.array([1, 1, 7, 1], np.int32)), o, 0.25, 2)
    assert e.value.status == -5


def test_cell_table_capacity_error_for_huge_boxes():
    from paper_1909_04631_amd import SmkiError, bucket_cells
    xyz = np.array([[0.0, 0.0, 0.0], [900.0, -900.0, 900.0]], np.float32)
    with pytest.raises(SmkiError) as e:
        bucket_cells(cuda(xyz), 0.2, 4)
    assert e.value.status == -3


@pytest.mark.parametrize("case", ["tiny_training_set", "negative_and_far"])
def test_cell_table_bit_exact(case):
    from paper_1909_04631_amd import bucket_cells
    if case == "tiny_training_set":
        sc = scenes.make_config(0)
        s = sc.scans[0]
        xyz, _, _ = oracle.training_set(s.xyz, s.label, s.origin, 0.1, 4)
        res, B = 0.1, 8
    else:
        rng = np.random.default_rng(9)
        xyz = rng.uniform(-3.0, 3.0, size=(20000, 3)).astype(np.float32)
        xyz[:5000, 0] += np.float32(-812.3)
        xyz[5000:5100] = np.float32(0.2) * np.round(xyz[5000:5100] / np.float32(0.2))  # on faces
        res, B = 0.2, 4
    _print_case(f"cells {case} n={xyz.shape[0]}")
    keys, start, count, order = bucket_cells(cuda(xyz), res, B)
    keys = keys.cpu().numpy().view(np.uint64)
    start, count, order = start.cpu().numpy(), count.cpu().numpy(), order.cpu().numpy()
    ref_ijk = oracle.voxel_coords(xyz, res)
    ref_keys = oracle.pack_keys(ref_ijk)
    uk, cnt = np.unique(ref_keys, return_counts=True)
    srt = np.argsort(keys, kind="stable")
    assert np.array_equal(keys[srt], uk)
    assert np.array_equal(count[srt], cnt)
    assert np.array_equal(np.sort(order), np.arange(xyz.shape[0]))
    for c in range(0, keys.shape[0], max(1, keys.shape[0] // 500)):
        ids = order[start[c]:start[c] + count[c]]
        assert np.all(ref_keys[ids] == keys[c])
    # rows of one cell keep their input order (stable sort)
    assert all(np.all(np.diff(order[start[c]:start[c] + count[c]]) > 0) for c in range(min(2000, keys.shape[0])))


# ---------------------------------------------------------------------------
# the map update (Eq. 7-8 at grid centroids)
# ---------------------------------------------------------------------------
def test_tiny_scene_alpha_counts_and_readout():
    import torch
    sc = scenes.make_config(0)
    _print_case("tiny scene insert")
    om = oracle_map_of(sc)
    gm = gpu_map_of(sc)
    far = np.array([[40, 40, 40], [-100, 3, 2], [0, 0, -60]], np.int32)
    worst, (ijk, a_ref, nv, nb) = compare_map(gm, om, sc.params.K, extra_ijk=far)
    print(f"tiny: V={int((nv > 0).sum())} max rel err {worst:.2e}", flush=True)
    check_counts(gm.stats(), nv, nb)
    # the 32^3 query grid, and the readout of Eq. (3)-(4)
    q = sc.query_ijk
    out = gm.query(cuda(q))
    ref = oracle.readout(om.lookup(q), free_class=0)
    a = out["alpha"].cpu().numpy()
    assert rel_err(a, om.lookup(q)).max() <= ALPHA_RTOL
    np.testing.assert_allclose(out["mean"].cpu().numpy(), ref["mean"], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(out["var"].cpu().numpy(), ref["var"], rtol=5e-5, atol=1e-9)
    np.testing.assert_allclose(out["p_occ"].cpu().numpy(), ref["p_occ"], rtol=2e-5, atol=1e-6)
    # argmax: equal where the oracle's top two classes are apart by more than the tolerance
    lab = out["label"].cpu().numpy()
    srt = np.sort(om.lookup(q), axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 4 * ALPHA_RTOL * srt[:, -1]
    assert np.array_equal(lab[clear], ref["label"][clear])
    # voxels the scan cannot reach keep alpha0 bit for bit
    a_far = gm.query(cuda(far))["alpha"].cpu().numpy()
    assert np.all(a_far == np.float32(sc.params.alpha0))


@pytest.mark.parametrize("K", [3, 12, 40, 150])
def test_readout_at_several_class_counts(K):
    # the readout serves a query with K lanes (K <= 32) or 64 lanes holding
    # several classes each; labels spread over all K classes, the free class last
    import dataclasses
    sc = scenes.make_config(0)
    rng = np.random.default_rng(K)
    p = dataclasses.replace(sc.params, K=K, free_class=K - 1)
    scans = []
    for s in sc.scans:
        lab = rng.integers(0, K, size=s.label.shape[0]).astype(np.int32)
        lab[s.label < 0] = -1
        scans.append(scenes.Scan(s.xyz, lab, s.origin))
    sck = dataclasses.replace(sc, params=p, scans=scans)
    _print_case(f"readout K={K}")
    om = oracle_map_of(sck)
    gm = gpu_map_of(sck)
    ijk, a_ref, _, _ = om.export()
    q = np.concatenate([ijk[::3], sc.query_ijk[::5]]).astype(np.int32)
    out = gm.query(cuda(q))
    a_o = om.lookup(q)
    ref = oracle.readout(a_o, free_class=K - 1)
    assert rel_err(out["alpha"].cpu().numpy(), a_o).max() <= ALPHA_RTOL
    np.testing.assert_allclose(out["mean"].cpu().numpy(), ref["mean"], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(out["var"].cpu().numpy(), ref["var"], rtol=5e-5, atol=1e-9)
    np.testing.assert_allclose(out["p_occ"].cpu().numpy(), ref["p_occ"], rtol=2e-5, atol=1e-6)
    lab = out["label"].cpu().numpy()
    srt = np.sort(a_o, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 4 * ALPHA_RTOL * srt[:, -1]
    assert clear.sum() > 0
    assert np.array_equal(lab[clear], ref["label"][clear])
    # where every class holds alpha0 the label is class 0 (lowest index on ties)
    unreached = np.all(a_o == a_o[:, :1], axis=1)
    assert np.all(lab[unreached] == 0)


def test_deterministic_across_runs():
    sc = scenes.make_config(0)
    _print_case("determinism")
    a = [gpu_map_of(sc).query(cuda(sc.query_ijk))["alpha"].cpu().numpy() for _ in range(2)]
    assert np.array_equal(a[0].view(np.uint32), a[1].view(np.uint32))


def test_recursive_update_and_batched_equal_the_oracle():
    import torch
    sc = scenes.make_config(0)
    s = sc.scans[0]
    p = sc.params
    A = scenes.Scan(s.xyz[:900], s.label[:900], s.origin)
    B = scenes.Scan(s.xyz[900:], s.label[900:], (s.origin + np.float32(0.35)).astype(np.float32))
    _print_case("two scans sequential + batched")
    om = oracle_map_of(sc, scans=[A, B])
    gseq = gpu_map_of(sc, scans=[A, B])
    compare_map(gseq, om, p.K)
    from paper_1909_04631_amd import SemanticMap
    gb = SemanticMap.from_params(p)
    xyz = np.concatenate([A.xyz, B.xyz])
    lab = np.concatenate([A.label, B.label])
    gb.insert_scans(cuda(xyz), cuda(lab), [0, 900, xyz.shape[0]], [A.origin, B.origin], p.free_step)
    torch.cuda.synchronize()
    compare_map(gb, om, p.K)


def test_batched_many_small_scans_with_empty_ones():
    # 400 scans of 0..9 hits each, every one from its own origin: the per-hit
    # scan lookup, empty scans, and a first-phase header larger than usual
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(0)
    s = sc.scans[0]
    p = sc.params
    rng = np.random.default_rng(9)
    sizes = rng.integers(0, 10, size=400)
    sizes[::37] = 0
    offs = np.concatenate([[0], np.cumsum(sizes)])
    n = int(offs[-1])
    xyz, lab = s.xyz[:n], s.label[:n]
    origins = (s.origin + rng.uniform(-0.3, 0.3, size=(400, 3))).astype(np.float32)
    scans = [scenes.Scan(xyz[offs[i]:offs[i + 1]], lab[offs[i]:offs[i + 1]], origins[i])
             for i in range(400)]
    _print_case(f"400 small scans, {n} hits")
    om = oracle_map_of(sc, scans=scans)
    gb = SemanticMap.from_params(p)
    gb.insert_scans(cuda(xyz), cuda(lab), [int(o) for o in offs], [tuple(o) for o in origins],
                    p.free_step)
    torch.cuda.synchronize()
    compare_map(gb, om, p.K)


def test_single_row_insert():
    # one hit closer to the sensor than one free step: a single training row
    # (the bucketing then runs no radix pass)
    sc = scenes.make_config(0)
    p = sc.params
    xyz = np.array([[0.05, 0.02, 0.01]], np.float32)
    lab = np.array([1], np.int32)
    scan = scenes.Scan(xyz, lab, np.zeros(3, np.float32))
    _print_case("single row")
    om = oracle_map_of(sc, scans=[scan])
    gm = gpu_map_of(sc, scans=[scan])
    assert gm.stats()["n_free"] == 0
    compare_map(gm, om, p.K)


def test_invalid_input_leaves_map_unchanged():
    import torch
    from paper_1909_04631_amd import SmkiError
    sc = scenes.make_config(0)
    s = sc.scans[0]
    gm = gpu_map_of(sc, scans=[scenes.Scan(s.xyz[:500], s.label[:500], s.origin)])
    before = gm.export()
    bad = s.label[500:900].copy()
    bad[17] = 9                      # label outside {-1..K-1}
    with pytest.raises(SmkiError) as e:
        gm.insert_scan(cuda(s.xyz[500:900]), cuda(bad), s.origin, sc.params.free_step)
    assert e.value.status == -5
    nanx = s.xyz[500:900].copy()
    nanx[3, 1] = np.nan
    with pytest.raises(SmkiError):
        gm.insert_scan(cuda(nanx), cuda(s.label[500:900]), s.origin, sc.params.free_step)
    far = s.xyz[500:900].copy()
    far[0] = [2.0e5, 0, 0]           # voxel index beyond 2^20
    with pytest.raises(SmkiError) as e:
        gm.insert_scan(cuda(far), cuda(s.label[500:900]), s.origin, sc.params.free_step)
    assert e.value.status == -6
    after = gm.export()
    assert all(torch.equal(x, y) for x, y in zip(before, after))
    # an empty scan and an all-dropped scan change nothing
    gm.insert_scan(cuda(s.xyz[:0]), cuda(s.label[:0]), s.origin, 0.1)
    gm.insert_scan(cuda(s.xyz[:50]), cuda(np.full(50, -1, np.int32)), s.origin, 0.1)
    assert all(torch.equal(x, y) for x, y in zip(before, gm.export()))


def test_export_import_round_trip_resumes():
    import torch
    sc = scenes.make_config(0)
    s = sc.scans[0]
    p = sc.params
    A = scenes.Scan(s.xyz[:1000], s.label[:1000], s.origin)
    B = scenes.Scan(s.xyz[1000:], s.label[1000:], s.origin)
    g1 = gpu_map_of(sc, scans=[A])
    ijk, alpha = g1.export()
    from paper_1909_04631_amd import SemanticMap
    g2 = SemanticMap.from_params(p)
    g2.import_(ijk, alpha)
    for g in (g1, g2):
        g.insert_scan(cuda(B.xyz), cuda(B.label), B.origin, p.free_step)
    torch.cuda.synchronize()
    e1, e2 = g1.export(), g2.export()
    assert torch.equal(e1[0], e2[0]) and torch.equal(e1[1], e2[1])
    compare_map(g2, oracle_map_of(sc, scans=[A, B]), p.K)


def test_single_class_scene_and_k2_reduction():
    import torch
    sc = scenes.make_config(0)
    s = sc.scans[0]
    p = sc.params
    from paper_1909_04631_amd import SemanticMap
    sel = slice(0, 700)
    g4 = gpu_map_of(sc, scans=[scenes.Scan(s.xyz[sel], s.label[sel], s.origin)])
    g2 = SemanticMap(p.res, p.block_size, p.l, p.sigma0, 2, p.alpha0)
    g2.insert_scan(cuda(s.xyz[sel]), cuda(np.minimum(s.label[sel], 1)), s.origin, p.free_step)
    torch.cuda.synchronize()
    q = cuda(sc.query_ijk)
    a4 = g4.query(q)["alpha"].cpu().numpy().astype(np.float64)
    a2 = g2.query(q)["alpha"].cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(a2[:, 0], a4[:, 0])
    np.testing.assert_allclose(a2[:, 1], a4[:, 1:].sum(1) - 2 * np.float32(p.alpha0), rtol=3e-6,
                               atol=1e-7)


@pytest.mark.parametrize("chunk,B", [(64, 8), (300, 8), (64, 4), (300, 4)])
def test_split_work_units_agree(chunk, B):
    # small chunks split every busy (class, block) into several splat units whose
    # partial sums the merge adds in chunk order (at B = 4 the reach of 3
    # exceeds half the block: up to 27 regions over a voxel)
    sc = scenes.make_config(0)
    sc.params.block_size = B
    _print_case(f"chunk {chunk} B {B}")
    gm = gpu_map_of(sc, unit_budget=chunk)
    om = oracle_map_of(sc)
    worst, (ijk, a_ref, nv, nb) = compare_map(gm, om, sc.params.K)
    st = gm.stats()
    assert st["n_units"] > st["n_point_blocks"]
    check_counts(st, nv, nb)


@pytest.mark.parametrize("B,l", [(2, 0.3), (4, 0.3), (8, 0.3), (16, 0.3), (4, 0.6), (4, 0.89),
                                 (8, 0.89), (16, 0.89)])
def test_block_sizes_and_reach(B, l):
    # res 0.2: l = 0.3 reaches 2 voxels past a row's voxel, l = 0.6 reaches 3,
    # l = 0.89 reaches 4, the largest supported reach (equal to the block edge
    # for B = 4, as 2 is for B = 2; 2R > B puts up to 27 regions over a voxel);
    # B = 16 merges four voxels per thread
    sc = scenes.random_points_scene(5, 3000, K=5, extent=1.3, centre=(-7.3, 12.9, -0.4),
                                    res=0.2, l=l, sigma0=0.4, free_step=0.25,
                                    origin=(-6.0, 11.0, 0.5))
    sc.params.block_size = B
    _print_case(f"block size {B} l {l}")
    compare_map(gpu_map_of(sc), oracle_map_of(sc), sc.params.K)


def test_reach_beyond_limit_is_rejected_and_map_unchanged():
    import torch
    from paper_1909_04631_amd import SemanticMap, SmkiError
    sc = scenes.random_points_scene(6, 500, K=3, extent=0.5, res=0.1, l=0.3)
    p = sc.params
    s = sc.scans[0]
    # reach 3 > B = 2; and S-BKI at block sizes 1 and 32
    for B, l in ((2, 0.3), (1, 0.3), (32, 0.3), (1, 0.04)):
        m = SemanticMap(p.res, B, l, p.sigma0, p.K, p.alpha0)
        with pytest.raises(SmkiError, match="CAPACITY"):
            m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, 0.0)
        assert m.num_blocks() == 0
    m = SemanticMap(p.res, 8, 0.46, p.sigma0, p.K, p.alpha0)   # l / res = 4.6 voxels
    with pytest.raises(SmkiError, match="CAPACITY"):
        m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, 0.0)
    assert m.num_blocks() == 0
    ok = SemanticMap(p.res, 8, 0.44, p.sigma0, p.K, p.alpha0)   # 4.4 voxels: supported
    ok.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, 0.0)
    torch.cuda.synchronize()
    assert ok.num_blocks() > 0


# ---------------------------------------------------------------------------
# full-size LiDAR scan: sampled voxels by brute force, counts by the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K", [20, 2])
def test_lidar_scan_full_size_sampled(K):
    # K = 20: 29-bit row keys, four 8-bit radix passes; K = 2: 26-bit keys,
    # three 9-bit passes
    import dataclasses
    sc = scenes.make_config(1)
    if K != sc.params.K:
        s0 = sc.scans[0]
        lab = np.where(s0.label < 0, s0.label, s0.label % K).astype(np.int32)
        sc = dataclasses.replace(sc, params=dataclasses.replace(sc.params, K=K),
                                 scans=[scenes.Scan(s0.xyz, lab, s0.origin)])
    p = sc.params.f32()
    s = sc.scans[0]
    _print_case(f"lidar full size n={s.xyz.shape[0]} K={K}")
    gm = gpu_map_of(sc)
    st = gm.stats()
    print("lidar stats", st, flush=True)
    tx, ty, _ = oracle.training_set(s.xyz, s.label, s.origin, p.free_step, p.K)
    assert st["n_hits"] == s.xyz.shape[0] and st["n_free"] == tx.shape[0] - s.xyz.shape[0]
    rng = np.random.default_rng(0)
    # sample voxels near hits (dense), near the sensor (dense free space), and anywhere in the box
    vh = oracle.voxel_coords(s.xyz[rng.choice(s.xyz.shape[0], 120, replace=False)], p.res)
    vs = oracle.voxel_coords((s.origin + rng.uniform(-1.5, 1.5, size=(60, 3))).astype(np.float32), p.res)
    vr = oracle.voxel_coords(tx[rng.choice(tx.shape[0], 120, replace=False)], p.res)
    q = np.concatenate([vh, vs, vr]).astype(np.int32)
    a_ref, n_in, _ = oracle.alpha_at_voxels(tx, ty, q, p.res, p.K, p.l, p.sigma0, p.alpha0)
    a = gm.query(cuda(q))["alpha"].cpu().numpy()
    err = rel_err(a, a_ref)
    print(f"lidar sampled max rel err {err.max():.2e}, max n_in {n_in.max()}", flush=True)
    assert err.max() <= ALPHA_RTOL


# ---------------------------------------------------------------------------
# the paper's extended-block selection (a voxel trains on rows of its block and
# the six face-adjacent blocks)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B", [4, 8])
def test_extended_block_selection_matches_the_oracle(B):
    sc = scenes.make_config(0)
    sc.params.block_size = B
    _print_case(f"face blocks B={B}")
    gm = gpu_map_of(sc, selection="face_blocks")
    om = oracle_map_of(sc, face_blocks=True)
    worst, (ijk, a_ref, nv, nb) = compare_map(gm, om, sc.params.K)
    st = gm.stats()
    v_strict = int((nv > 0).sum())
    assert abs(st["n_updated_voxels"] - v_strict) <= int((nb > 0).sum())
    # voxels the exact support reaches but the selection does not stay at alpha0
    ex = oracle_map_of(sc)
    ie, ae, nve, _ = ex.export()
    dropped = np.array([tuple(v) not in set(map(tuple, ijk[nv > 0])) for v in ie]) & (nve > 0)
    if dropped.any():
        a = gm.query(cuda(ie[dropped].astype(np.int32)))["alpha"].cpu().numpy()
        ref = om.lookup(ie[dropped])
        assert rel_err(a, ref).max() <= ALPHA_RTOL


def test_kernel_times_and_reset():
    import torch
    sc = scenes.make_config(0)
    p = sc.params
    s = sc.scans[0]
    _print_case("kernel times and reset")
    gm = gpu_map_of(sc)
    for _ in range(2):
        gm.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    sp, mg = gm.kernel_times(10)
    assert len(sp) == len(mg) == 3 and min(sp) > 0 and min(mg) > 0
    assert len(gm.kernel_times(2)[0]) == 2
    gm.reset()                      # empties the map without synchronising
    assert gm.num_blocks() == 0
    gm.set_kernel_timing(False)     # an insert without events: same map, no new times
    gm.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    torch.cuda.synchronize()
    assert gm.kernel_times(10)[0] == sp
    st = gm.stats()
    assert st["n_new_blocks"] == gm.num_blocks() > 0 and st["splat_ms"] == 0.0
    compare_map(gm, oracle_map_of(sc), p.K)
    gm.set_kernel_timing(True)
    gm.reset()
    gm.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    assert len(gm.kernel_times(10)[0]) == 4 and gm.stats()["splat_ms"] > 0
