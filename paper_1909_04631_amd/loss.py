"""Differentiable form: predictive loss of held-out labels and its adjoint.

Binding of smki_loss_forward / smki_loss_backward and their per-class forms
(argument marshalling only).
The backward recomputes kernel weights in the library; it stores nothing per
pair.  l and sigma0 are taken as 0-d tensors (or floats) so that gradient
descent on them can run through autograd.
"""
import ctypes as C

import torch

from ._lib import check, lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _rows(xyz, lab, name):
    if not (xyz.is_cuda and lab.is_cuda):
        raise ValueError(f"{name} tensors must be on the GPU")
    if xyz.dtype != torch.float32 or lab.dtype != torch.int32 or xyz.dim() != 2 or xyz.shape[1] != 3:
        raise ValueError(f"{name}: xyz must be float32 [n,3] and labels int32 [n]")
    return xyz.contiguous(), lab.contiguous()


def workspace(n_train, n_query, K, device=None):
    """A device workspace (uint8 tensor) for loss_forward / loss_backward of these
    sizes (smki_loss_workspace_bytes); without one, every call allocates its own."""
    nb = int(lib().smki_loss_workspace_bytes(int(n_train), int(n_query), int(K)))
    return torch.empty((nb,), dtype=torch.uint8, device=device or torch.cuda.current_device())


def _ws(ws):
    return (_ptr(ws), ws.numel()) if ws is not None else (None, 0)


def loss_forward(train_xyz, train_label, query_xyz, query_label, l, sigma0, alpha0, K,
                 keep_alpha=True, ws=None):
    """(loss float32 [1], alpha_q float32 [H, K] or None when keep_alpha is False)."""
    tx, ty = _rows(train_xyz, train_label, "train")
    qx, qy = _rows(query_xyz, query_label, "query")
    loss = torch.empty((1,), dtype=torch.float32, device=qx.device)
    aq = (torch.empty((qx.shape[0], int(K)), dtype=torch.float32, device=qx.device)
          if keep_alpha else None)
    check(lib().smki_loss_forward(_ptr(tx), _ptr(ty), tx.shape[0], _ptr(qx), _ptr(qy), qx.shape[0],
                                  float(l), float(sigma0), float(alpha0), int(K), _stream(),
                                  *_ws(ws), _ptr(loss), _ptr(aq)), "smki_loss_forward")
    return loss, aq


def loss_backward(train_xyz, train_label, query_xyz, query_label, l, sigma0, alpha0, K, alpha_q,
                  grad_loss, need_train=True, need_query=True, ws=None):
    """(grad_l [1], grad_sigma0 [1], grad_train [N,3] or None, grad_query [H,3] or None)."""
    tx, ty = _rows(train_xyz, train_label, "train")
    qx, qy = _rows(query_xyz, query_label, "query")
    dev = qx.device
    gl = torch.empty((1,), dtype=torch.float32, device=dev)
    gs = torch.empty((1,), dtype=torch.float32, device=dev)
    gt = torch.empty((tx.shape[0], 3), dtype=torch.float32, device=dev) if need_train else None
    gq = torch.empty((qx.shape[0], 3), dtype=torch.float32, device=dev) if need_query else None
    g = grad_loss.reshape(1).to(torch.float32).contiguous()
    check(lib().smki_loss_backward(_ptr(tx), _ptr(ty), tx.shape[0], _ptr(qx), _ptr(qy),
                                   qx.shape[0], float(l), float(sigma0), float(alpha0), int(K),
                                   _stream(), *_ws(ws), _ptr(alpha_q.contiguous()), _ptr(g),
                                   _ptr(gl), _ptr(gs), _ptr(gt), _ptr(gq)), "smki_loss_backward")
    return gl, gs, gt, gq


def _class_params(l, sigma0, K):
    lk = [float(v) for v in (l.detach().reshape(-1).cpu().tolist() if torch.is_tensor(l) else l)]
    sk = [float(v) for v in (sigma0.detach().reshape(-1).cpu().tolist() if torch.is_tensor(sigma0)
                             else sigma0)]
    if len(lk) != K or len(sk) != K:
        raise ValueError(f"per-class l and sigma0 must hold K = {K} values")
    return (C.c_float * K)(*lk), (C.c_float * K)(*sk)


def loss_forward_classes(train_xyz, train_label, query_xyz, query_label, l, sigma0, alpha0, K):
    """Per-class kernels (l, sigma0: K values each): (loss [1], alpha_q [H, K])."""
    tx, ty = _rows(train_xyz, train_label, "train")
    qx, qy = _rows(query_xyz, query_label, "query")
    lk, sk = _class_params(l, sigma0, int(K))
    loss = torch.empty((1,), dtype=torch.float32, device=qx.device)
    aq = torch.empty((qx.shape[0], int(K)), dtype=torch.float32, device=qx.device)
    check(lib().smki_loss_forward_classes(_ptr(tx), _ptr(ty), tx.shape[0], _ptr(qx), _ptr(qy),
                                          qx.shape[0], lk, sk, float(alpha0), int(K), _stream(),
                                          None, 0, _ptr(loss), _ptr(aq)),
          "smki_loss_forward_classes")
    return loss, aq


def loss_backward_classes(train_xyz, train_label, query_xyz, query_label, l, sigma0, alpha0, K,
                          alpha_q, grad_loss, need_train=True, need_query=True):
    """(grad_l [K], grad_sigma0 [K], grad_train [N,3] or None, grad_query [H,3] or None)."""
    tx, ty = _rows(train_xyz, train_label, "train")
    qx, qy = _rows(query_xyz, query_label, "query")
    lk, sk = _class_params(l, sigma0, int(K))
    dev = qx.device
    gl = torch.empty((int(K),), dtype=torch.float32, device=dev)
    gs = torch.empty((int(K),), dtype=torch.float32, device=dev)
    gt = torch.empty((tx.shape[0], 3), dtype=torch.float32, device=dev) if need_train else None
    gq = torch.empty((qx.shape[0], 3), dtype=torch.float32, device=dev) if need_query else None
    g = grad_loss.reshape(1).to(torch.float32).contiguous()
    check(lib().smki_loss_backward_classes(_ptr(tx), _ptr(ty), tx.shape[0], _ptr(qx), _ptr(qy),
                                           qx.shape[0], lk, sk, float(alpha0), int(K), _stream(),
                                           None, 0, _ptr(alpha_q.contiguous()), _ptr(g), _ptr(gl),
                                           _ptr(gs), _ptr(gt), _ptr(gq)),
          "smki_loss_backward_classes")
    return gl, gs, gt, gq


class PredictiveLossClasses(torch.autograd.Function):
    """The predictive loss with per-class kernels: l, sigma0 tensors of K values."""

    @staticmethod
    def forward(ctx, train_xyz, query_xyz, l, sigma0, train_label, query_label, alpha0, K):
        loss, aq = loss_forward_classes(train_xyz, train_label, query_xyz, query_label, l, sigma0,
                                        alpha0, K)
        ctx.save_for_backward(train_xyz, query_xyz, train_label, query_label, aq, l, sigma0)
        ctx.hp = (float(alpha0), int(K))
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad):
        tx, qx, ty, qy, aq, l, sigma0 = ctx.saved_tensors
        a0, K = ctx.hp
        gl, gs, gt, gq = loss_backward_classes(tx, ty, qx, qy, l, sigma0, a0, K, aq, grad,
                                               need_train=ctx.needs_input_grad[0],
                                               need_query=ctx.needs_input_grad[1])
        return gt, gq, gl.reshape(l.shape), gs.reshape(sigma0.shape), None, None, None, None


def predictive_loss_classes(train_xyz, train_label, query_xyz, query_label, l, sigma0, alpha0, K):
    """l, sigma0: tensors of K values (per-class kernels), differentiable."""
    if not torch.is_tensor(l):
        l = torch.tensor(l, dtype=torch.float32, device=query_xyz.device)
    if not torch.is_tensor(sigma0):
        sigma0 = torch.tensor(sigma0, dtype=torch.float32, device=query_xyz.device)
    return PredictiveLossClasses.apply(train_xyz, query_xyz, l, sigma0, train_label, query_label,
                                       alpha0, K)


class PredictiveLoss(torch.autograd.Function):
    """loss(train_xyz, query_xyz, l, sigma0) = -(1/H) sum_h log(alpha_h^{y_h} / S_h)."""

    @staticmethod
    def forward(ctx, train_xyz, query_xyz, l, sigma0, train_label, query_label, alpha0, K):
        lv, sv = float(l), float(sigma0)
        loss, aq = loss_forward(train_xyz, train_label, query_xyz, query_label, lv, sv, alpha0, K)
        ctx.save_for_backward(train_xyz, query_xyz, train_label, query_label, aq)
        ctx.hp = (lv, sv, float(alpha0), int(K))
        ctx.l_shape = l.shape if torch.is_tensor(l) else None
        ctx.s_shape = sigma0.shape if torch.is_tensor(sigma0) else None
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad):
        tx, qx, ty, qy, aq = ctx.saved_tensors
        lv, sv, a0, K = ctx.hp
        gl, gs, gt, gq = loss_backward(tx, ty, qx, qy, lv, sv, a0, K, aq, grad,
                                       need_train=ctx.needs_input_grad[0],
                                       need_query=ctx.needs_input_grad[1])
        g_l = gl.reshape(ctx.l_shape) if ctx.l_shape is not None else None
        g_s = gs.reshape(ctx.s_shape) if ctx.s_shape is not None else None
        return gt, gq, g_l, g_s, None, None, None, None


def predictive_loss(train_xyz, train_label, query_xyz, query_label, l, sigma0, alpha0, K):
    return PredictiveLoss.apply(train_xyz, query_xyz, l, sigma0, train_label, query_label, alpha0, K)
