"""The batched insert recorded as one HIP graph (smki_batch_capture / replay).

Eq. (7) is additive over training rows (the recursive update of Sec. IV), so S
scans go in one pass; the recording reads every count on the device and runs
with no host synchronisation.  Checked here: every replay equals the ordinary
(uncaptured) batched insert bit for bit and the float64 oracle within 1e-5,
across replays with eager work between them; new data of the same shape;
replays on top of earlier ones; and the failure paths (capacity overflow, rows
outside the recorded voxel box, moved map storage) leave the map unchanged.
"""
import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import compare_map, cuda, oracle_map_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    import torch
    from paper_1909_04631_amd import _lib
    _lib.lib()   # raises if the HIP library is missing: no fallback
    torch.cuda.init()


def _print_case(name):
    print(f"[case] {name}", flush=True)


def _split(sc, n_scans, seed, spread=0.4):
    """The tiny scene's hits as n_scans scans of uneven size, each from its own origin."""
    s = sc.scans[0]
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, s.xyz.shape[0]), n_scans - 1, replace=False))
    offs = np.concatenate([[0], cuts, [s.xyz.shape[0]]]).astype(np.int64)
    origins = (s.origin + rng.uniform(-spread, spread, size=(n_scans, 3))).astype(np.float32)
    scans = [scenes.Scan(s.xyz[offs[i]:offs[i + 1]], s.label[offs[i]:offs[i + 1]], origins[i])
             for i in range(n_scans)]
    return s.xyz, s.label, offs, origins, scans


def _bits_equal(m1, m2):
    a, b = m1.export(), m2.export()
    return a[0].shape == b[0].shape and bool((a[0] == b[0]).all()) and \
        np.array_equal(a[1].cpu().numpy().view(np.uint32), b[1].cpu().numpy().view(np.uint32))


def test_replays_equal_the_uncaptured_insert_and_the_oracle():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(0)
    p = sc.params
    xyz, lab, offs, origins, scans = _split(sc, 6, 1)
    _print_case("capture: tiny scene in 6 scans")
    ref = SemanticMap.from_params(p)
    ref.insert_scans(cuda(xyz), cuda(lab), offs, origins, p.free_step)
    om = oracle_map_of(sc, scans=scans)
    m = SemanticMap.from_params(p)
    tx, tl = cuda(xyz), cuda(lab)
    b = m.batch_capture(tx, tl, offs, origins, p.free_step)   # inserts once, uncaptured
    torch.cuda.synchronize()
    assert _bits_equal(m, ref)
    st_ref = ref.stats()
    for rep in range(3):
        m.reset()
        b.replay(offs, origins)
        m.sync()
        assert _bits_equal(m, ref), f"replay {rep}"
        st = m.stats()
        for k in ("n_hits", "n_free", "n_point_blocks", "n_units", "n_updated_voxels", "n_pairs",
                  "n_new_blocks", "n_new_class_blocks"):
            assert st[k] == st_ref[k], (rep, k, st[k], st_ref[k])
        # eager work between replays
        _ = m.query(cuda(sc.query_ijk))
        torch.cuda.synchronize()
    compare_map(m, om, p.K)
    # a replay on top of the map: every scan twice
    b.replay(offs, origins)
    m.sync()
    compare_map(m, oracle_map_of(sc, scans=scans + scans), p.K)
    b.close()


def test_replay_of_new_data_of_the_same_shape():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(0)
    p = sc.params
    xyz, lab, offs, origins, scans = _split(sc, 5, 2)
    tx, tl = cuda(xyz), cuda(lab)
    m = SemanticMap.from_params(p)
    b = m.batch_capture(tx, tl, offs, origins, p.free_step, margin=0.5)
    # the same buffers now hold other hits (jittered, relabelled), other origins
    rng = np.random.default_rng(7)
    xyz2 = (xyz + rng.normal(0, 0.02, size=xyz.shape)).astype(np.float32)
    lab2 = np.where(lab < 0, lab, rng.integers(1, p.K, size=lab.shape)).astype(np.int32)
    origins2 = (origins + np.float32(0.05)).astype(np.float32)
    tx.copy_(cuda(xyz2))
    tl.copy_(cuda(lab2))
    _print_case("replay of new data")
    m.reset()
    b.replay(offs, origins2)
    m.sync()
    ref = SemanticMap.from_params(p)
    ref.insert_scans(cuda(xyz2), cuda(lab2), offs, origins2, p.free_step)
    torch.cuda.synchronize()
    assert _bits_equal(m, ref)
    scans2 = [scenes.Scan(xyz2[offs[i]:offs[i + 1]], lab2[offs[i]:offs[i + 1]], origins2[i])
              for i in range(len(offs) - 1)]
    compare_map(m, oracle_map_of(sc, scans=scans2), p.K)
    b.close()


def test_failed_replays_leave_the_map_unchanged():
    import torch
    from paper_1909_04631_amd import SemanticMap, SmkiError
    sc = scenes.make_config(0)
    p = sc.params
    xyz, lab, offs, origins, scans = _split(sc, 4, 3)
    tx, tl = cuda(xyz), cuda(lab)
    m = SemanticMap.from_params(p)
    b = m.batch_capture(tx, tl, offs, origins, p.free_step, margin=0.0)
    torch.cuda.synchronize()
    before = m.export()
    # (1) far more free samples than recorded: origins 1.2 m away lengthen every beam
    far = (origins + np.array([1.2, 0.0, 0.0], np.float32)).astype(np.float32)
    _print_case("replay beyond the row capacity")
    b.replay(offs, far)
    with pytest.raises(SmkiError) as e:
        m.sync()
    print(f"overflow replay: status {e.value.status}", flush=True)
    assert e.value.status in (-3, -6)
    after = m.export()
    assert all(torch.equal(x, y) for x, y in zip(before, after))
    # (2) hits moved outside the recorded voxel box
    _print_case("replay outside the voxel box")
    tx.copy_(cuda((xyz + np.array([30.0, 0, 0], np.float32)).astype(np.float32)))
    b.replay(offs, (origins + np.array([30.0, 0, 0], np.float32)).astype(np.float32))
    with pytest.raises(SmkiError) as e:
        m.sync()
    assert e.value.status in (-3, -6)
    after = m.export()
    assert all(torch.equal(x, y) for x, y in zip(before, after))
    # (3) the original data replays correctly after the failures
    tx.copy_(cuda(xyz))
    b.replay(offs, origins)
    m.sync()
    compare_map(m, oracle_map_of(sc, scans=scans + scans), p.K)
    # (4) an ordinary insert that grows the map's storage invalidates the recording
    big = scenes.random_points_scene(9, 6000, K=p.K, extent=9.0, centre=(40.0, 40.0, 3.0),
                                     res=p.res, l=p.l)
    s9 = big.scans[0]
    m.insert_scan(cuda(s9.xyz), cuda(s9.label), s9.origin, 0.0)
    with pytest.raises(SmkiError) as e:
        b.replay(offs, origins)
    assert e.value.status == -3
    b.close()


@pytest.mark.timeout(600)
def test_town_replay_equals_the_uncaptured_batched_insert():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(3)
    p = sc.params
    xyz, lab, offs, org = sc.concat()
    _print_case(f"town capture: {len(sc.scans)} scans, {xyz.shape[0]} hits")
    tx, tl = cuda(xyz), cuda(lab)
    ref = SemanticMap.from_params(p, initial_blocks=1 << 18)
    ref.insert_scans(tx, tl, offs, org, p.free_step)
    torch.cuda.synchronize()
    st_ref = ref.stats()
    m = SemanticMap.from_params(p, initial_blocks=1 << 18)
    b = m.batch_capture(tx, tl, offs, org, p.free_step)
    for rep in range(2):
        m.reset()
        b.replay(offs, org)
        m.sync()
        st = m.stats()
        assert st["n_updated_voxels"] == st_ref["n_updated_voxels"]
        assert st["n_pairs"] == st_ref["n_pairs"]
        assert st["n_new_class_blocks"] == st_ref["n_new_class_blocks"]
    # every hit's voxel and its neighbours: identical concentrations
    v = oracle.voxel_coords(xyz, p.res)
    q = np.unique(np.concatenate([v, v + np.array([1, 0, 0]), v - np.array([0, 1, 1])]),
                  axis=0).astype(np.int32)
    a = m.query(cuda(q), mean=False, var=False, label=False, p_occ=False)["alpha"]
    r = ref.query(cuda(q), mean=False, var=False, label=False, p_occ=False)["alpha"]
    assert torch.equal(a.view(torch.int32), r.view(torch.int32))
    print(f"town replay: {q.shape[0]} voxels identical", flush=True)
    b.close()
