"""GPU parity of per-class kernel parameters (l_k, sigma0_k per class) against
the float64 oracle, through the C ABI: the map update and the predictive loss
with its per-class adjoint.

Bars: concentrations within 1e-5 relative; counts exact up to band pairs; the
loss within 1e-5 relative; gradients within 1e-4 relative per gradient vector
(the 2K kernel parameters compared in log units, as one vector).
"""
import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import ALPHA_RTOL, check_counts, compare_map, cuda, rel_err

pytestmark = pytest.mark.gpu

LK = np.array([0.3, 0.17, 0.41, 0.25], np.float32)
SK = np.array([1.0, 0.6, 1.7, 0.35], np.float32)


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    import torch
    from paper_1909_04631_amd import _lib
    _lib.lib()   # raises if the HIP library is missing: no fallback
    torch.cuda.init()


def _print_case(name):
    print(f"[case] {name}", flush=True)


def gpu_map(sc, lk, sk, scans=None, **kw):
    import torch
    from paper_1909_04631_amd import SemanticMap
    p = sc.params
    m = SemanticMap.from_params(p, **kw)
    m.set_class_params(lk, sk)
    for s in (sc.scans if scans is None else scans):
        m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    torch.cuda.synchronize()
    return m


def oracle_map(sc, lk, sk, scans=None, face_blocks=False):
    p = sc.params.f32()
    m = oracle.OracleMap.from_params(p, face_blocks=face_blocks)
    m.set_class_params(lk, sk)
    for s in (sc.scans if scans is None else scans):
        m.insert_scan(s.xyz, s.label, s.origin, p.free_step, p.free_class)
    return m


@pytest.mark.parametrize("B", [4, 8])
def test_per_class_map_tiny_scene(B):
    sc = scenes.make_config(0)
    sc.params.block_size = B
    _print_case(f"per-class map B={B}")
    gm = gpu_map(sc, LK, SK)
    worst, (ijk, _, nv, nb) = compare_map(gm, oracle_map(sc, LK, SK), sc.params.K)
    check_counts(gm.stats(), nv, nb)
    print(f"per-class B={B}: {ijk.shape[0]} voxels, max rel err {worst:.2e}", flush=True)


def test_per_class_map_two_scans_and_extended_block():
    sc = scenes.make_config(0)
    s = sc.scans[0]
    A = scenes.Scan(s.xyz[:1100], s.label[:1100], s.origin)
    B = scenes.Scan(s.xyz[1100:], s.label[1100:], s.origin)
    _print_case("per-class two scans")
    compare_map(gpu_map(sc, LK, SK, scans=[A, B]), oracle_map(sc, LK, SK, scans=[A, B]),
                sc.params.K)
    _print_case("per-class extended block")
    compare_map(gpu_map(sc, LK, SK, selection="face_blocks"),
                oracle_map(sc, LK, SK, face_blocks=True), sc.params.K)


def test_equal_class_params_are_the_single_kernel_map():
    from gpu_cases import gpu_map_of
    sc = scenes.make_config(0)
    p = sc.params
    _print_case("per-class equal params")
    a = gpu_map_of(sc)
    b = gpu_map(sc, np.full(p.K, p.l, np.float32), np.full(p.K, p.sigma0, np.float32))
    ijk, _, _, _ = oracle_map(sc, np.full(p.K, p.l, np.float32),
                              np.full(p.K, p.sigma0, np.float32)).export()
    q = cuda(ijk.astype(np.int32))
    np.testing.assert_array_equal(a.query(q)["alpha"].cpu().numpy(),
                                  b.query(q)["alpha"].cpu().numpy())


def test_invalid_class_params_and_reach_limit():
    import torch
    from paper_1909_04631_amd import SemanticMap, SmkiError
    sc = scenes.random_points_scene(6, 500, K=3, extent=0.5, res=0.1, l=0.3)
    p = sc.params
    s = sc.scans[0]
    m = SemanticMap(p.res, 8, p.l, p.sigma0, p.K, p.alpha0)
    for lk, sk in (([0.3, 0.0, 0.3], [1, 1, 1]), ([0.3, 0.3, 0.3], [1, float("nan"), 1])):
        with pytest.raises(SmkiError, match="INVALID"):
            m.set_class_params(lk, sk)
    with pytest.raises(ValueError):
        m.set_class_params([0.3, 0.3], [1, 1])
    m.set_class_params([0.3, 0.46, 0.2], [1, 1, 1])      # one class reaches 4.6 voxels
    with pytest.raises(SmkiError, match="CAPACITY"):
        m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, 0.0)
    assert m.num_blocks() == 0
    m.set_class_params([0.3, 0.44, 0.2], [1, 1, 1])      # 4.4 voxels: supported
    m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, 0.0)
    torch.cuda.synchronize()
    om = oracle.OracleMap.from_params(p.f32())
    om.set_class_params(np.array([0.3, 0.44, 0.2], np.float32), np.ones(3, np.float32))
    om.insert_scan(s.xyz, s.label, s.origin, 0.0, p.free_class)
    compare_map(m, om, p.K)


def test_per_class_lidar_scan_full_size_sampled():
    # Reference by columns: column k of a per-class map is column k of the
    # single-kernel map (l_k, sigma0_k) over the rows of class k (an oracle pin).
    sc = scenes.make_config(1)
    p = sc.params.f32()
    s = sc.scans[0]
    rng = np.random.default_rng(3)
    lk = rng.choice(np.array([0.2, 0.25, 0.3, 0.35, 0.4], np.float32), p.K).astype(np.float32)
    sk = rng.choice(np.array([0.05, 0.1, 0.2], np.float32), p.K).astype(np.float32)
    _print_case(f"per-class lidar full size n={s.xyz.shape[0]}")
    gm = gpu_map(sc, lk, sk)
    print("per-class lidar stats", gm.stats(), flush=True)
    tx, ty, _ = oracle.training_set(s.xyz, s.label, s.origin, p.free_step, p.K)
    vh = oracle.voxel_coords(s.xyz[rng.choice(s.xyz.shape[0], 120, replace=False)], p.res)
    vs = oracle.voxel_coords((s.origin + rng.uniform(-1.5, 1.5, size=(60, 3))).astype(np.float32),
                             p.res)
    vr = oracle.voxel_coords(tx[rng.choice(tx.shape[0], 120, replace=False)], p.res)
    q = np.concatenate([vh, vs, vr]).astype(np.int32)
    ref = np.empty((q.shape[0], p.K))
    for k in range(p.K):
        sel = ty == k
        a_k, _, _ = oracle.alpha_at_voxels(tx[sel], ty[sel], q, p.res, p.K, float(lk[k]),
                                           float(sk[k]), p.alpha0)
        ref[:, k] = a_k[:, k]
    a = gm.query(cuda(q))["alpha"].cpu().numpy()
    err = rel_err(a, ref)
    print(f"per-class lidar sampled max rel err {err.max():.2e}", flush=True)
    assert err.max() <= ALPHA_RTOL


def loss_rows():
    sc = scenes.make_config(4)
    p = sc.params.f32()
    tr = sc.scans[0]
    tx, ty, _ = oracle.training_set(tr.xyz, tr.label, tr.origin, p.free_step, p.K)
    return p, tx, ty, sc.holdout.xyz, sc.holdout.label


def gpu_loss_grads(tx, ty, qx, qy, lk, sk, a0, K):
    import torch
    from paper_1909_04631_amd import predictive_loss_classes
    txt = cuda(tx).requires_grad_(True)
    qxt = cuda(qx).requires_grad_(True)
    lt = torch.tensor(lk, dtype=torch.float32, device="cuda", requires_grad=True)
    st = torch.tensor(sk, dtype=torch.float32, device="cuda", requires_grad=True)
    L = predictive_loss_classes(txt, cuda(ty), qxt, cuda(qy), lt, st, a0, K)
    L.backward()
    return (float(L), lt.grad.cpu().numpy().astype(np.float64),
            st.grad.cpu().numpy().astype(np.float64),
            txt.grad.cpu().numpy().astype(np.float64), qxt.grad.cpu().numpy().astype(np.float64))


def vec_rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("which", ["distinct", "equal"])
def test_per_class_loss_and_gradient(which):
    from paper_1909_04631_amd import loss_forward_classes
    p, tx, ty, qx, qy = loss_rows()
    if which == "distinct":
        lk, sk = LK.astype(np.float64), SK.astype(np.float64)
    else:
        lk, sk = np.full(p.K, p.l), np.full(p.K, p.sigma0)
    _print_case(f"per-class loss {which}")
    ref = oracle.loss_classes(tx, ty, qx, qy, p.K, lk, sk, p.alpha0)
    loss, aq = loss_forward_classes(cuda(tx), cuda(ty), cuda(qx), cuda(qy), lk, sk, p.alpha0, p.K)
    assert np.max(np.abs(aq.cpu().numpy() - ref["alpha_q"]) / ref["alpha_q"]) <= 1e-5
    assert abs(float(loss.cpu()) - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    L, gl, gs, gt, gq = gpu_loss_grads(tx, ty, qx, qy, lk, sk, p.alpha0, p.K)
    assert abs(L - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    g_ref = np.concatenate([lk * ref["grad_l"], sk * ref["grad_sigma0"]])
    g_gpu = np.concatenate([lk * gl, sk * gs])
    assert vec_rel(g_gpu, g_ref) <= 1e-4, (g_gpu, g_ref)
    assert vec_rel(gt, ref["grad_train"]) <= 1e-4
    assert vec_rel(gq, ref["grad_query"]) <= 1e-4
    if which == "equal":   # the per-class gradients sum to the single-kernel gradient
        single = oracle.loss(tx, ty, qx, qy, p.K, p.l, p.sigma0, p.alpha0)
        assert abs(gl.sum() - single["grad_l"]) <= 1e-4 * abs(single["grad_l"])
        assert abs(gs.sum() - single["grad_sigma0"]) <= 1e-4 * abs(single["grad_sigma0"])


def test_per_class_gradient_descent_teacher_forced():
    # 30 steps of gradient descent on (ln l_k, ln sigma0_k), eta = 0.1, from the
    # single-kernel values: the oracle's trajectory is the reference, and at
    # each of its iterates the GPU gradient agrees to 1e-4.
    import torch
    from paper_1909_04631_amd import predictive_loss_classes
    p, tx, ty, qx, qy = loss_rows()
    K = p.K
    th = np.log(np.concatenate([np.full(K, 0.3), np.full(K, 1.0)]))
    txt, tyt, qxt, qyt = cuda(tx), cuda(ty), cuda(qx), cuda(qy)
    losses = []
    for it in range(30):
        v = np.exp(th).astype(np.float32).astype(np.float64)
        lk, sk = v[:K], v[K:]
        ref = oracle.loss_classes(tx, ty, qx, qy, K, lk, sk, p.alpha0)
        lt = torch.tensor(lk, dtype=torch.float32, device="cuda", requires_grad=True)
        st = torch.tensor(sk, dtype=torch.float32, device="cuda", requires_grad=True)
        L = predictive_loss_classes(txt, tyt, qxt, qyt, lt, st, p.alpha0, K)
        L.backward()
        g_ref = np.concatenate([lk * ref["grad_l"], sk * ref["grad_sigma0"]])
        g_gpu = np.concatenate([lk * lt.grad.cpu().numpy(), sk * st.grad.cpu().numpy()])
        assert np.linalg.norm(g_gpu - g_ref) <= 1e-4 * np.linalg.norm(g_ref), (it, g_gpu, g_ref)
        losses.append(ref["loss"])
        th = th - 0.1 * g_ref
    assert losses[-1] < losses[0]
    print(f"per-class descent: loss {losses[0]:.5f} -> {losses[-1]:.5f}", flush=True)
