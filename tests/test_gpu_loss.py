"""GPU parity of the differentiable form (predictive loss and adjoint) against
the float64 oracle, on the tiny scene with 20 % of its hits held out.

Bars: alpha at the queries and the loss within 1e-5 relative; gradients within
1e-4 relative per gradient vector (l and sigma0 compared in log-parameter
units against the norm of (l dL/dl, sigma0 dL/dsigma0)).
"""
import numpy as np
import pytest

import oracle
import scenes
from gpu_cases import cuda

pytestmark = pytest.mark.gpu


def rows(sc):
    p = sc.params.f32()
    tr = sc.scans[0]
    tx, ty, _ = oracle.training_set(tr.xyz, tr.label, tr.origin, p.free_step, p.K)
    return p, tx, ty, sc.holdout.xyz, sc.holdout.label


def gpu_grads(tx, ty, qx, qy, l, s0, a0, K):
    import torch
    from paper_1909_04631_amd import predictive_loss
    txt = cuda(tx).requires_grad_(True)
    qxt = cuda(qx).requires_grad_(True)
    lt = torch.tensor(float(l), device="cuda", requires_grad=True)
    st = torch.tensor(float(s0), device="cuda", requires_grad=True)
    L = predictive_loss(txt, cuda(ty), qxt, cuda(qy), lt, st, a0, K)
    L.backward()
    return (float(L), float(lt.grad), float(st.grad), txt.grad.cpu().numpy().astype(np.float64),
            qxt.grad.cpu().numpy().astype(np.float64))


def vec_rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_forward_alpha_and_loss():
    from paper_1909_04631_amd import loss_forward
    sc = scenes.make_config(4)
    p, tx, ty, qx, qy = rows(sc)
    ref = oracle.loss(tx, ty, qx, qy, p.K, p.l, p.sigma0, p.alpha0)
    loss, aq = loss_forward(cuda(tx), cuda(ty), cuda(qx), cuda(qy), p.l, p.sigma0, p.alpha0, p.K)
    aq = aq.cpu().numpy()
    assert np.max(np.abs(aq - ref["alpha_q"]) / ref["alpha_q"]) <= 1e-5
    assert abs(float(loss.cpu()) - ref["loss"]) <= 1e-5 * abs(ref["loss"])


@pytest.mark.parametrize("l,s0", [(0.3, 1.0), (0.42, 0.25)])
def test_backward_matches_oracle_gradient(l, s0):
    sc = scenes.make_config(4)
    p, tx, ty, qx, qy = rows(sc)
    l32, s32 = float(np.float32(l)), float(np.float32(s0))
    ref = oracle.loss(tx, ty, qx, qy, p.K, l32, s32, p.alpha0)
    L, gl, gs, gt, gq = gpu_grads(tx, ty, qx, qy, l32, s32, p.alpha0, p.K)
    assert abs(L - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    scale = np.hypot(l32 * ref["grad_l"], s32 * ref["grad_sigma0"])
    assert abs(l32 * gl - l32 * ref["grad_l"]) <= 1e-4 * scale
    assert abs(s32 * gs - s32 * ref["grad_sigma0"]) <= 1e-4 * scale
    assert vec_rel(gt, ref["grad_train"]) <= 1e-4
    assert vec_rel(gq, ref["grad_query"]) <= 1e-4


def test_gradient_descent_teacher_forced():
    # 50 steps of gradient descent on (ln l, ln sigma0), eta = 0.1, from (0.3, 1.0):
    # the oracle's trajectory is the reference; at each of its iterates the GPU
    # gradient must agree to 1e-4 (teacher forcing).
    import torch
    from paper_1909_04631_amd import predictive_loss
    sc = scenes.make_config(4)
    p, tx, ty, qx, qy = rows(sc)
    th = np.log([0.3, 1.0])
    txt, tyt, qxt, qyt = cuda(tx), cuda(ty), cuda(qx), cuda(qy)
    losses = []
    for it in range(50):
        l32, s32 = (float(np.float32(v)) for v in np.exp(th))
        ref = oracle.loss(tx, ty, qx, qy, p.K, l32, s32, p.alpha0)
        lt = torch.tensor(l32, device="cuda", requires_grad=True)
        st = torch.tensor(s32, device="cuda", requires_grad=True)
        L = predictive_loss(txt, tyt, qxt, qyt, lt, st, p.alpha0, p.K)
        L.backward()
        g_ref = np.array([l32 * ref["grad_l"], s32 * ref["grad_sigma0"]])
        g_gpu = np.array([l32 * float(lt.grad), s32 * float(st.grad)])
        assert np.linalg.norm(g_gpu - g_ref) <= 1e-4 * np.linalg.norm(g_ref), (it, g_gpu, g_ref)
        losses.append(ref["loss"])
        th = th - 0.1 * g_ref
    assert losses[-1] < losses[0]
