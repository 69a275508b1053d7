"""GPU parity of the S-BKI map update at the workloads' full sizes and at the
edges of the key and offset ranges (Eq. (7)-(8) at grid centroids, Sec. IV,
applied recursively scan after scan).

Every comparison is against the float64 CPU oracle, whose map insert is split
over voxel-column tiles with the serial sum order; voxel counts V and pair
counts P come from the oracle's own per-insert counters.  Bars as elsewhere:
float32 concentrations within 1e-5 relative; V and P exact up to the pairs in
the rounding band |d^2/l^2 - 1| <= 1e-5.
"""
import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import ALPHA_RTOL, compare_map, cuda, oracle_map_of, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    import torch
    from paper_1909_04631_amd import _lib
    _lib.lib()   # raises if the HIP library is missing: no fallback
    torch.cuda.init()


def _print_case(name):
    print(f"[case] {name}", flush=True)


def _tuned(workload):
    """The autotuner's (block size, unit budget) for a workload (defaults when untuned)."""
    from paper_1909_04631_amd import autotune
    s = autotune.settings(workload)
    return {"block_size": s[0], "unit_budget": s[1]} if s else {"block_size": 8, "unit_budget": 0}


def _counts_agree(gpu_stats, ora, what):
    """V and P of one insert: exact up to band pairs."""
    dv = abs(gpu_stats["n_updated_voxels"] - ora["V"])
    dp = abs(gpu_stats["n_pairs"] - ora["P"])
    assert dv <= ora["V_band"], (what, gpu_stats["n_updated_voxels"], ora)
    assert dp <= ora["P_band"], (what, gpu_stats["n_pairs"], ora)


def _sample_voxels(rng, xyz, res, n, jitter=0.4):
    """Voxels at and around randomly chosen points (inside and near the support)."""
    pick = xyz[rng.choice(xyz.shape[0], size=min(n, xyz.shape[0]), replace=False)]
    pick = pick + rng.uniform(-jitter, jitter, size=pick.shape).astype(np.float32)
    return oracle.voxel_coords(pick.astype(np.float32), res)


# ---------------------------------------------------------------------------
# the LiDAR scan: every voxel the oracle updates
# ---------------------------------------------------------------------------
def test_lidar_scan_whole_map():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(1)
    p = sc.params
    s = sc.scans[0]
    _print_case(f"lidar whole map n={s.xyz.shape[0]}")
    om = oracle_map_of(sc)
    ora = om.last_insert()
    t = _tuned("lidar")   # the settings the benchmark runs at
    gm = SemanticMap(p.res, t["block_size"], p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                     unit_budget=t["unit_budget"])
    gm.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    torch.cuda.synchronize()
    st = gm.stats()
    print(f"lidar: gpu V={st['n_updated_voxels']} P={st['n_pairs']}; oracle {ora}", flush=True)
    _counts_agree(st, ora, "lidar")
    worst, (ijk, a_ref, nv, nb) = compare_map(gm, om, p.K)
    print(f"lidar whole map: {ijk.shape[0]} voxels, max rel err {worst:.2e}", flush=True)
    assert ijk.shape[0] >= ora["V"]


# ---------------------------------------------------------------------------
# the batched town: 64 uneven scans, sequential and batched
# ---------------------------------------------------------------------------
@pytest.mark.timeout(600)
def test_batched_town_counts_and_sampled_alpha():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(3)
    p = sc.params
    _print_case(f"town: {len(sc.scans)} scans, {sum(x.xyz.shape[0] for x in sc.scans)} hits")
    om = oracle.OracleMap.from_params(p.f32())
    gs = SemanticMap.from_params(p, initial_blocks=1 << 18)
    pf = p.f32()
    for i, s in enumerate(sc.scans):
        om.insert_scan(s.xyz, s.label, s.origin, pf.free_step, pf.free_class)
        gs.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
        torch.cuda.synchronize()
        _counts_agree(gs.stats(), om.last_insert(), f"town scan {i}")
    print(f"town: per-scan V and P agree over {len(sc.scans)} scans", flush=True)
    # the batched insert of all 64 scans into a fresh map
    xyz = np.concatenate([s.xyz for s in sc.scans])
    lab = np.concatenate([s.label for s in sc.scans])
    offs = np.concatenate([[0], np.cumsum([s.xyz.shape[0] for s in sc.scans])])
    t = _tuned("town")   # the batched insert at the settings the benchmark runs at
    gb = SemanticMap(p.res, t["block_size"], p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                     unit_budget=t["unit_budget"], initial_blocks=1 << 18)
    gb.insert_scans(cuda(xyz), cuda(lab), [int(o) for o in offs], [s.origin for s in sc.scans],
                    p.free_step)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    q = [_sample_voxels(rng, s.xyz, p.res, 600) for s in sc.scans]
    # free space near every sensor, and voxels more than 100 m from the origin
    q.append(oracle.voxel_coords(np.concatenate(
        [(s.origin + rng.uniform(-3, 3, size=(40, 3))).astype(np.float32) for s in sc.scans]), p.res))
    far = xyz[np.hypot(xyz[:, 0], xyz[:, 1]) > 100.0]
    assert far.shape[0] > 1000
    q.append(_sample_voxels(rng, far, p.res, 3000))
    q = np.unique(np.concatenate(q), axis=0).astype(np.int32)
    a_ref = om.lookup(q)
    assert (np.hypot(q[:, 0], q[:, 1]) * p.res > 100.0).sum() > 1000
    for name, g in (("sequential", gs), ("batched", gb)):
        a = g.query(cuda(q), mean=False, var=False, label=False, p_occ=False)["alpha"].cpu().numpy()
        err = rel_err(a, a_ref)
        print(f"town {name}: {q.shape[0]} sampled voxels, max rel err {err.max():.2e}", flush=True)
        assert err.max() <= ALPHA_RTOL


# ---------------------------------------------------------------------------
# the stereo sequence: the first scans into one persistent map
# ---------------------------------------------------------------------------
def test_stereo_scans_into_one_map():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(2, first=3, workers=8)
    p = sc.params
    _print_case(f"stereo: {len(sc.scans)} scans of {[s.xyz.shape[0] for s in sc.scans]} hits")
    om = oracle.OracleMap.from_params(p.f32())
    t = _tuned("stereo")
    gm = SemanticMap(p.res, t["block_size"], p.l, p.sigma0, p.K, p.alpha0, p.free_class,
                     unit_budget=t["unit_budget"], initial_blocks=1 << 15)
    pf = p.f32()
    for i, s in enumerate(sc.scans):
        om.insert_scan(s.xyz, s.label, s.origin, pf.free_step, pf.free_class)
        gm.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
        torch.cuda.synchronize()
        _counts_agree(gm.stats(), om.last_insert(), f"stereo scan {i}")
    rng = np.random.default_rng(2)
    q = [_sample_voxels(rng, s.xyz, p.res, 4000) for s in sc.scans]
    q += [oracle.voxel_coords((s.origin + rng.uniform(-0.5, 8, size=(2000, 3)) *
                               np.array([3, 1, 0.3])).astype(np.float32), p.res) for s in sc.scans]
    q = np.unique(np.concatenate(q), axis=0).astype(np.int32)
    a = gm.query(cuda(q), mean=False, var=False, label=False, p_occ=False)["alpha"].cpu().numpy()
    err = rel_err(a, om.lookup(q))
    print(f"stereo: {q.shape[0]} sampled voxels, max rel err {err.max():.2e}", flush=True)
    assert err.max() <= ALPHA_RTOL


# ---------------------------------------------------------------------------
# key and offset ranges
# ---------------------------------------------------------------------------
def _key_bits(vlo, vhi, B, K):
    """Bits of the library's row keys for a voxel box (classes x grid blocks x
    voxels of a block), written out from the key layout: the box is grown by
    one voxel, blocks are floor(v / B)."""
    lo = (np.asarray(vlo) - 1) // B
    hi = (np.asarray(vhi) + 1) // B
    n = int(np.prod(hi - lo + 1)) * K
    return int(np.ceil(np.log2(n))) + 3 * int(np.log2(B))


def test_sparse_wide_scan_takes_64_bit_keys():
    # a few thousand hits over 150 x 150 x 10 m at 0.1 m voxels and K = 20:
    # the row keys need more than 32 bits (64-bit sort and key path)
    rng = np.random.default_rng(21)
    n = 3000
    xyz = np.stack([rng.uniform(-75, 75, n), rng.uniform(-75, 75, n), rng.uniform(0, 10, n)],
                   1).astype(np.float32)
    xyz[:400] = (xyz[:1] + rng.normal(0, 0.3, size=(400, 3))).astype(np.float32)   # one dense spot
    lab = rng.integers(1, 20, n).astype(np.int32)
    origin = np.array([1.5, -2.0, 1.7], np.float32)
    sc = scenes.Scene("wide", scenes.Params(res=0.1, block_size=8, l=0.3, sigma0=0.1, alpha0=0.001,
                                            K=20, free_class=0, free_step=0.0),
                      [scenes.Scan(xyz, lab, origin)])
    v = oracle.voxel_coords(xyz, 0.1)
    assert _key_bits(v.min(0), v.max(0), 8, 20) > 32
    _print_case("64-bit keys")
    from gpu_cases import gpu_map_of
    om = oracle_map_of(sc)
    gm = gpu_map_of(sc)
    _counts_agree(gm.stats(), om.last_insert(), "wide keys")
    compare_map(gm, om, 20)
    # the same hits with free samples from one origin (rows along 100 m beams)
    sc.params.free_step = 0.5
    sub = scenes.Scan(xyz[::10], lab[::10], origin)
    om2 = oracle_map_of(sc, scans=[sub])
    gm2 = gpu_map_of(sc, scans=[sub])
    _counts_agree(gm2.stats(), om2.last_insert(), "wide keys with beams")
    compare_map(gm2, om2, 20)


@pytest.mark.parametrize("centre", [(612.3, -540.7, 23.1), (-1843.9, 2210.35, -96.2)])
def test_far_from_the_origin(centre):
    # coordinates hundreds of metres out: float32 positions keep ~1e-4 m, the
    # voxel-relative records and the centroid distances must not lose more
    sc = scenes.random_points_scene(31, 2500, K=6, extent=2.5, centre=centre, res=0.1, l=0.3,
                                    sigma0=0.1, free_step=0.3,
                                    origin=tuple(np.asarray(centre) + np.array([3.0, -4.0, 1.0])))
    _print_case(f"far from the origin {centre}")
    from gpu_cases import gpu_map_of
    om = oracle_map_of(sc)
    gm = gpu_map_of(sc)
    _counts_agree(gm.stats(), om.last_insert(), "far")
    worst, _ = compare_map(gm, om, sc.params.K)
    print(f"far {centre}: max rel err {worst:.2e}", flush=True)


def test_wide_partial_sum_offsets():
    # the merge's 64-bit addressing (used above 4 GiB of partial sums), forced
    # on a small case: the same sums as the 32-bit form, bit for bit
    sc = scenes.make_config(0)
    _print_case("wide offsets")
    from gpu_cases import gpu_map_of
    gw = gpu_map_of(sc, wide_offsets=True, unit_budget=96)
    gn = gpu_map_of(sc, unit_budget=96)
    compare_map(gw, oracle_map_of(sc), sc.params.K)
    a = gw.query(cuda(sc.query_ijk))["alpha"].cpu().numpy()
    b = gn.query(cuda(sc.query_ijk))["alpha"].cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_import_rejects_bad_blocks_and_leaves_the_map_unchanged():
    import torch
    from paper_1909_04631_amd import SemanticMap, SmkiError
    from gpu_cases import gpu_map_of
    sc = scenes.make_config(0)
    s = sc.scans[0]
    p = sc.params
    gm = gpu_map_of(sc, scans=[scenes.Scan(s.xyz[:600], s.label[:600], s.origin)])
    before = gm.export()
    ijk, alpha = before
    dup = ijk.clone()
    dup[-1] = dup[0]
    with pytest.raises(SmkiError) as e:
        gm.import_(dup, alpha)
    assert e.value.status == -5
    far = ijk.clone()
    far[1, 0] = (1 << 20) // p.block_size       # its voxels leave [-2^20, 2^20)
    with pytest.raises(SmkiError) as e:
        gm.import_(far, alpha)
    assert e.value.status == -6
    after = gm.export()
    assert all(torch.equal(x, y) for x, y in zip(before, after))
    # the map still updates correctly after the rejected imports
    gm.insert_scan(cuda(s.xyz[600:]), cuda(s.label[600:]), s.origin, p.free_step)
    torch.cuda.synchronize()
    compare_map(gm, oracle_map_of(sc, scans=[scenes.Scan(s.xyz[:600], s.label[:600], s.origin),
                                             scenes.Scan(s.xyz[600:], s.label[600:], s.origin)]),
                p.K)
    # a valid import into a map that already holds other blocks replaces them
    g2 = SemanticMap.from_params(p)
    g2.insert_scan(cuda(s.xyz[1500:]), cuda(s.label[1500:]), s.origin, p.free_step)
    g2.import_(ijk, alpha)
    e2 = g2.export()
    assert torch.equal(e2[0], ijk) and torch.equal(e2[1], alpha)
