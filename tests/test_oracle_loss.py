"""Pins of the oracle's differentiable form (readings R14-R16).

The analytic gradient is checked against double-precision central finite
differences of the oracle's own loss (a different computation: only the
forward pass), and against identities that Eq. (7)-(8) impose on any correct
gradient: the sigma0 derivative in closed form, scale invariance of the
predictive as alpha0 -> 0, Euler's relation for a kernel that depends on d/l
only, and translation invariance.
"""
import numpy as np
import pytest

import oracle


def small_problem(seed, n_train=120, n_query=25, K=4, extent=0.35):
    rng = np.random.default_rng(seed)
    tx = rng.uniform(-extent, extent, size=(n_train, 3)) + np.array([1.3, -0.4, 0.8])
    ty = rng.integers(0, K, size=n_train).astype(np.int32)
    qx = rng.uniform(-extent, extent, size=(n_query, 3)) + np.array([1.3, -0.4, 0.8])
    qy = rng.integers(0, K, size=n_query).astype(np.int32)
    return tx, ty, qx, qy, K


def L(tx, ty, qx, qy, K, l, s0, a0):
    return oracle.loss(tx, ty, qx, qy, K, l, s0, a0)["loss"]


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    tx, ty, qx, qy, K = small_problem(seed)
    l, s0, a0 = 0.3, 0.7, 0.001
    g = oracle.loss(tx, ty, qx, qy, K, l, s0, a0)
    h = 1e-6
    fd_l = (L(tx, ty, qx, qy, K, l * (1 + h), s0, a0) - L(tx, ty, qx, qy, K, l * (1 - h), s0, a0)) / (2 * l * h)
    fd_s = (L(tx, ty, qx, qy, K, l, s0 * (1 + h), a0) - L(tx, ty, qx, qy, K, l, s0 * (1 - h), a0)) / (2 * s0 * h)
    assert g["grad_l"] == pytest.approx(fd_l, rel=1e-6)
    assert g["grad_sigma0"] == pytest.approx(fd_s, rel=1e-6)
    rng = np.random.default_rng(100 + seed)
    for t in rng.choice(tx.shape[0], 8, replace=False):
        for a in range(3):
            tp, tm = tx.copy(), tx.copy()
            tp[t, a] += h
            tm[t, a] -= h
            fd = (L(tp, ty, qx, qy, K, l, s0, a0) - L(tm, ty, qx, qy, K, l, s0, a0)) / (2 * h)
            assert g["grad_train"][t, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)
    for q in rng.choice(qx.shape[0], 5, replace=False):
        for a in range(3):
            qp, qm = qx.copy(), qx.copy()
            qp[q, a] += h
            qm[q, a] -= h
            fd = (L(tx, ty, qp, qy, K, l, s0, a0) - L(tx, ty, qm, qy, K, l, s0, a0)) / (2 * h)
            assert g["grad_query"][q, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_gradient_identities():
    tx, ty, qx, qy, K = small_problem(3)
    l, s0, a0 = 0.3, 0.7, 0.001
    g = oracle.loss(tx, ty, qx, qy, K, l, s0, a0)
    A = g["alpha_q"]
    H = qx.shape[0]
    S = A.sum(1, keepdims=True)
    G = -((np.arange(K)[None, :] == qy[:, None]) / A - 1 / S) / H
    # sigma0 derivative in closed form: alpha - alpha0 is linear in sigma0
    assert g["grad_sigma0"] == pytest.approx((G * (A - a0)).sum() / s0, rel=1e-12)
    # Euler: the kernel depends on d/l only
    euler = l * g["grad_l"] + (tx * g["grad_train"]).sum() + (qx * g["grad_query"]).sum()
    scale = abs(l * g["grad_l"]) + np.abs(tx * g["grad_train"]).sum()
    assert abs(euler) <= 1e-12 * scale
    # translation invariance
    tot = g["grad_train"].sum(0) + g["grad_query"].sum(0)
    assert np.abs(tot).max() <= 1e-12 * np.abs(g["grad_train"]).sum()
    # as alpha0 -> 0 the predictive of a query with an in-support point of its
    # own class is invariant to sigma0; a query without one contributes
    # -(1/H) d log(alpha0 / S)/d log sigma0 -> 1/H
    g0 = oracle.loss(tx, ty, qx, qy, K, l, s0, 1e-12)
    lonely = np.sum(g0["alpha_q"][np.arange(H), qy] == 1e-12)
    assert s0 * g0["grad_sigma0"] == pytest.approx(lonely / H, abs=1e-8)


def test_loss_value_by_hand_single_pair():
    # one training point of class 1 at distance l/2 from one query of class 1:
    # alpha = (a0, a0 + s0 f(1/2)) with f(1/2) = 1/6
    tx = np.array([[0.0, 0.0, 0.0]])
    qx = np.array([[0.15, 0.0, 0.0]])
    g = oracle.loss(tx, np.array([1], np.int32), qx, np.array([1], np.int32), 2, 0.3, 1.2, 0.01)
    a1 = 0.01 + 1.2 / 6
    assert g["loss"] == pytest.approx(-np.log(a1 / (a1 + 0.01)), rel=1e-14)
