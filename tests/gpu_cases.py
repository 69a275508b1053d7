"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np

import oracle

ALPHA_RTOL = 1e-5   # relative tolerance of float32 concentrations against the float64 oracle


def cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def oracle_map_of(scene, scans=None, scsm=False, face_blocks=False):
    p = scene.params.f32()
    m = oracle.OracleMap.from_params(p, scsm=scsm, face_blocks=face_blocks)
    for s in (scene.scans if scans is None else scans):
        m.insert_scan(s.xyz, s.label, s.origin, p.free_step, p.free_class)
    return m


def gpu_map_of(scene, scans=None, **kw):
    import torch
    from paper_1909_04631_amd import SemanticMap
    p = scene.params
    m = SemanticMap.from_params(p, **kw)
    for s in (scene.scans if scans is None else scans):
        m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    torch.cuda.synchronize()
    return m


def rel_err(a_gpu, a_ref):
    a_ref = np.asarray(a_ref, np.float64)
    return np.abs(np.asarray(a_gpu, np.float64) - a_ref) / np.abs(a_ref)


def compare_map(gm, om, K, extra_ijk=None, rtol=ALPHA_RTOL):
    """Every voxel the oracle updated, plus extra voxels: GPU alpha within rtol.
    Returns (max relative error, oracle export)."""
    ijk, a_ref, nv, nb = om.export()
    q = ijk if extra_ijk is None else np.concatenate([ijk, extra_ijk])
    ref = a_ref if extra_ijk is None else np.concatenate([a_ref, om.lookup(extra_ijk)])
    out = gm.query(cuda(q.astype(np.int32)), mean=False, var=False, label=False, p_occ=False)
    a = out["alpha"].cpu().numpy()
    err = rel_err(a, ref)
    worst = float(err.max()) if err.size else 0.0
    assert worst <= rtol, f"max relative alpha error {worst:.3e} > {rtol:.1e} at voxel {q[np.unravel_index(err.argmax(), err.shape)[0]]}"
    return worst, (ijk, a_ref, nv, nb)


def check_counts(stats, nv, nb):
    """V and P_s: exact up to pairs in the rounding band |d^2/l^2 - 1| <= 1e-5."""
    v_strict = int((nv > 0).sum())
    band_vox = int((nb > 0).sum())
    assert abs(stats["n_updated_voxels"] - v_strict) <= band_vox, (stats, v_strict, band_vox)
    assert abs(stats["n_pairs"] - int(nv.sum())) <= int(nb.sum()), (stats, int(nv.sum()), int(nb.sum()))
