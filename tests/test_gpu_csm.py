"""GPU parity of the counting model (S-CSM, Eq. (2)) against the oracle's
counting map: every voxel's per-class count alpha - alpha0 is an integer and
must match exactly; the concentration itself within 1e-5 relative."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import ALPHA_RTOL, cuda, gpu_map_of, oracle_map_of, rel_err

pytestmark = pytest.mark.gpu


def _compare_counts(gm, om, p, single_insert=True):
    ijk, a_ref, nv, _ = om.export()
    out = gm.query(cuda(ijk.astype(np.int32)))
    a = out["alpha"].cpu().numpy().astype(np.float64)
    counts_gpu = np.rint(a - np.float32(p.alpha0)).astype(np.int64)
    counts_ref = np.rint(a_ref - np.float32(p.alpha0)).astype(np.int64)
    np.testing.assert_array_equal(counts_gpu, counts_ref)
    assert rel_err(a, a_ref).max() <= ALPHA_RTOL
    if single_insert:   # the stats describe the last insert only
        assert gm.stats()["n_updated_voxels"] == ijk.shape[0]
    return ijk, out


def test_counting_model_tiny_scene_exact():
    sc = scenes.make_config(0)
    p = sc.params
    gm = gpu_map_of(sc, model="scsm")
    om = oracle_map_of(sc, scsm=True)
    ijk, out = _compare_counts(gm, om, p)
    st = gm.stats()
    assert st["n_pairs"] == st["n_hits"] + st["n_free"]   # every row counts once
    # untouched voxels read alpha0, readout sums to one
    far = cuda(np.array([[1000, 1000, 1000]], np.int32))
    assert float(gm.query(far)["alpha"].max()) == pytest.approx(np.float32(p.alpha0))
    np.testing.assert_allclose(out["mean"].sum(1).cpu().numpy(), 1.0, rtol=1e-5)


def test_counting_model_recursive_and_batched():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(0)
    p = sc.params
    s = sc.scans[0]
    A = scenes.Scan(s.xyz[:900], s.label[:900], s.origin)
    Bs = scenes.Scan(s.xyz[900:], s.label[900:], s.origin)
    seq = gpu_map_of(sc, scans=[A, Bs], model="scsm")
    bat = SemanticMap.from_params(p, model="scsm")
    bat.insert_scans(cuda(s.xyz), cuda(s.label), [0, 900, s.xyz.shape[0]], [s.origin, s.origin],
                     p.free_step)
    torch.cuda.synchronize()
    om = oracle_map_of(sc, scans=[A, Bs], scsm=True)
    _compare_counts(seq, om, p, single_insert=False)
    ijk, a_ref, _, _ = om.export()
    a_bat = bat.query(cuda(ijk.astype(np.int32)))["alpha"].cpu().numpy()
    a_seq = seq.query(cuda(ijk.astype(np.int32)))["alpha"].cpu().numpy()
    # integer counts are order-free and exact; alpha0 + count rounds once per insert
    a0 = np.float32(p.alpha0)
    np.testing.assert_array_equal(np.rint(a_bat - a0), np.rint(a_seq - a0))
    assert rel_err(a_bat, a_seq).max() <= 2.4e-7


def test_counting_model_lidar_scan_full_size():
    sc = scenes.make_config(1)
    p = sc.params
    gm = gpu_map_of(sc, model="scsm")
    om = oracle_map_of(sc, scsm=True)
    ijk, _ = _compare_counts(gm, om, p)
    print(f"lidar S-CSM: {ijk.shape[0]} voxels, stats {gm.stats()}", flush=True)


@pytest.mark.parametrize("B", [1, 2, 16, 32])
def test_counting_model_at_every_block_depth(B):
    # block depth d: 2^(d-1) voxels per block edge (depth 1: a block is one
    # voxel, the setting the paper runs the counting model at); counts exact
    sc = scenes.make_config(0)
    sc.params.block_size = B
    p = sc.params
    print(f"[case] S-CSM block size {B}", flush=True)
    gm = gpu_map_of(sc, model="scsm")
    om = oracle_map_of(sc, scsm=True)
    _compare_counts(gm, om, p)
    ijk, alpha = gm.export()
    assert alpha.shape[2:] == (B, B, B)
