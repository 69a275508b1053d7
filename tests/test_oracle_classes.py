"""Pins of the oracle's per-class kernel parameters (reading R23: rows of class
k use their own length-scale l_k and scale sigma0_k, as the paper suggests
for its class-independent l and sigma0).

  - map: column k of a per-class map equals column k of a map built with the
    single kernel (l_k, sigma0_k), bit for bit; equal parameters reproduce the
    single-kernel map bit for bit;
  - loss: the per-class gradient against central differences of the loss in
    every l_k, sigma0_k and a few coordinates; with equal parameters the loss
    equals the single-kernel loss and the per-class gradients sum to its
    gradient; the sigma0_k derivative in closed form.
"""
import numpy as np
import pytest

import oracle
import scenes


def test_per_class_map_columns_are_single_kernel_maps():
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    sel = slice(0, 400)
    lk = np.array([0.3, 0.17, 0.41, 0.25], np.float32)
    sk = np.array([1.0, 0.6, 1.7, 0.35], np.float32)
    m = oracle.OracleMap.from_params(p)
    m.set_class_params(lk, sk)
    m.insert_scan(s.xyz[sel], s.label[sel], s.origin, p.free_step, p.free_class)
    ijk, a, _, _ = m.export()
    for k in range(p.K):
        mk = oracle.OracleMap(p.K, p.res, p.block_size, float(lk[k]), float(sk[k]), p.alpha0)
        mk.insert_scan(s.xyz[sel], s.label[sel], s.origin, p.free_step, p.free_class)
        ik, ak, _, _ = mk.export()
        np.testing.assert_array_equal(m.lookup(ik)[:, k], ak[:, k])
        # and the other way round: every voxel of the per-class map
        np.testing.assert_array_equal(a[:, k], mk.lookup(ijk)[:, k])


def test_equal_class_params_reproduce_the_single_kernel_map():
    sc = scenes.make_config(0)
    p = sc.params.f32()
    s = sc.scans[0]
    m1 = oracle.OracleMap.from_params(p)
    m2 = oracle.OracleMap.from_params(p)
    m2.set_class_params(np.full(p.K, p.l, np.float32), np.full(p.K, p.sigma0, np.float32))
    for m in (m1, m2):
        m.insert_scan(s.xyz[:600], s.label[:600], s.origin, p.free_step, p.free_class)
    for x, y in zip(m1.export(), m2.export()):
        np.testing.assert_array_equal(x, y)


def test_invalid_class_params_are_rejected():
    m = oracle.OracleMap(K=3, res=0.1, block_size=8, l=0.3, sigma0=1.0, alpha0=0.001)
    for lk, sk in (([0.3, 0.0, 0.3], [1, 1, 1]), ([0.3, 0.3, 0.3], [1, -1, 1]),
                   ([0.3, np.nan, 0.3], [1, 1, 1])):
        with pytest.raises(oracle.OracleError):
            m.set_class_params(np.array(lk, np.float32), np.array(sk, np.float32))
    with pytest.raises(ValueError):
        m.set_class_params(np.ones(2, np.float32), np.ones(2, np.float32))


def small_problem(seed, n_train=150, n_query=30, K=4, extent=0.35):
    rng = np.random.default_rng(seed)
    c = np.array([1.3, -0.4, 0.8])
    tx = rng.uniform(-extent, extent, size=(n_train, 3)) + c
    ty = rng.integers(0, K, size=n_train).astype(np.int32)
    qx = rng.uniform(-extent, extent, size=(n_query, 3)) + c
    qy = rng.integers(0, K, size=n_query).astype(np.int32)
    return tx, ty, qx, qy, K


@pytest.mark.parametrize("seed", [0, 1])
def test_per_class_gradient_matches_central_differences(seed):
    tx, ty, qx, qy, K = small_problem(seed)
    lk = np.array([0.3, 0.22, 0.37, 0.27])
    sk = np.array([0.7, 1.3, 0.45, 0.9])
    a0 = 0.001
    g = oracle.loss_classes(tx, ty, qx, qy, K, lk, sk, a0)

    def Lf(lk_, sk_, tx_=tx, qx_=qx):
        return oracle.loss_classes(tx_, ty, qx_, qy, K, lk_, sk_, a0)["loss"]

    h = 1e-6
    for k in range(K):
        e = np.zeros(K)
        e[k] = 1.0
        fd_l = (Lf(lk * (1 + h * e), sk) - Lf(lk * (1 - h * e), sk)) / (2 * lk[k] * h)
        fd_s = (Lf(lk, sk * (1 + h * e)) - Lf(lk, sk * (1 - h * e))) / (2 * sk[k] * h)
        assert g["grad_l"][k] == pytest.approx(fd_l, rel=1e-6, abs=1e-9)
        assert g["grad_sigma0"][k] == pytest.approx(fd_s, rel=1e-6, abs=1e-9)
    rng = np.random.default_rng(100 + seed)
    for t in rng.choice(tx.shape[0], 6, replace=False):
        for a in range(3):
            tp, tm = tx.copy(), tx.copy()
            tp[t, a] += h
            tm[t, a] -= h
            fd = (Lf(lk, sk, tx_=tp) - Lf(lk, sk, tx_=tm)) / (2 * h)
            assert g["grad_train"][t, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    for q in rng.choice(qx.shape[0], 4, replace=False):
        for a in range(3):
            qp, qm = qx.copy(), qx.copy()
            qp[q, a] += h
            qm[q, a] -= h
            fd = (Lf(lk, sk, qx_=qp) - Lf(lk, sk, qx_=qm)) / (2 * h)
            assert g["grad_query"][q, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_per_class_loss_identities():
    tx, ty, qx, qy, K = small_problem(3)
    l, s0, a0 = 0.3, 0.7, 0.001
    single = oracle.loss(tx, ty, qx, qy, K, l, s0, a0)
    pc = oracle.loss_classes(tx, ty, qx, qy, K, np.full(K, l), np.full(K, s0), a0)
    assert pc["loss"] == pytest.approx(single["loss"], rel=1e-14)
    np.testing.assert_allclose(pc["alpha_q"], single["alpha_q"], rtol=1e-14)
    assert pc["grad_l"].sum() == pytest.approx(single["grad_l"], rel=1e-12)
    assert pc["grad_sigma0"].sum() == pytest.approx(single["grad_sigma0"], rel=1e-12)
    np.testing.assert_allclose(pc["grad_train"], single["grad_train"], rtol=1e-12, atol=1e-15)
    # closed form: dL/dsigma0_k = sum_h G_hk (alpha_hk - alpha0) / sigma0_k with
    # G_hk = -(1/H)([k = y_h] / alpha_hk - 1/S_h)
    lk = np.array([0.3, 0.22, 0.37, 0.27])
    sk = np.array([0.7, 1.3, 0.45, 0.9])
    g = oracle.loss_classes(tx, ty, qx, qy, K, lk, sk, a0)
    A = g["alpha_q"]
    H = A.shape[0]
    G = np.zeros_like(A)
    G[np.arange(H), qy] = 1.0 / A[np.arange(H), qy]
    G = -(G - 1.0 / A.sum(1, keepdims=True)) / H
    np.testing.assert_allclose(g["grad_sigma0"], (G * (A - a0)).sum(0) / sk, rtol=1e-12)
