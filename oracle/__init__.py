"""CPU correctness oracle for the S-BKI map update (Gan et al., arXiv 1909.04631).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU path.  The arithmetic lives in ``smki_oracle.c`` (plain C, double
precision; see the header of that file for the equations followed and the
readings taken where the paper is silent); this module only marshals numpy
arrays through ctypes.

Functions mirror the paper's steps:
  kernel_f / kernel_df           Eq. (8) (reading R1), its derivative
  free_counts / free_samples     free-space points along each beam (Sec. III)
  training_set                   hits + free samples of one scan
  voxel_coords                   floor_f32(x / res) per axis
  alpha_at / alpha_at_voxels     Eq. (7) by definition (all training points)
  OracleMap                      Eq. (7) at every grid centroid, scan after scan;
                                 Eq. (2) (S-CSM) with scsm=True
  readout                        Eq. (3)-(4)
  loss                           predictive loss and its analytic gradient
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsmki_oracle.so")
_lib = None

OK = 0
E_ARG, E_OOM, E_INPUT, E_RANGE = -1, -2, -5, -6


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        f32p, f64p = C.POINTER(C.c_float), C.POINTER(C.c_double)
        i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        u64p = C.POINTER(C.c_uint64)
        L.oracle_kernel_f.restype = C.c_double
        L.oracle_kernel_f.argtypes = [C.c_double]
        L.oracle_kernel_df.restype = C.c_double
        L.oracle_kernel_df.argtypes = [C.c_double]
        L.oracle_kernel_df_over_r.restype = C.c_double
        L.oracle_kernel_df_over_r.argtypes = [C.c_double]
        L.oracle_free_counts.argtypes = [f32p, i32p, C.c_int64, f32p, C.c_float, C.c_int32, i64p, i64p]
        L.oracle_free_samples.argtypes = [f32p, i32p, C.c_int64, f32p, C.c_float, C.c_int32, f32p, i64p]
        L.oracle_voxel_coords.argtypes = [f32p, C.c_int64, C.c_float, i32p]
        L.oracle_pack_keys.argtypes = [i32p, C.c_int64, u64p]
        L.oracle_alpha_at.argtypes = [f32p, i32p, C.c_int64, f64p, C.c_int64, C.c_int32, C.c_float,
                                      C.c_float, C.c_float, f64p, i64p, i64p]
        L.oracle_alpha_at_voxels.argtypes = [f32p, i32p, C.c_int64, i32p, C.c_int64, C.c_float,
                                             C.c_int32, C.c_float, C.c_float, C.c_float, f64p,
                                             i64p, i64p]
        L.oracle_alpha_at_voxels_w.argtypes = [f32p, i32p, f64p, C.c_int64, i32p, C.c_int64,
                                               C.c_float, C.c_int32, C.c_float, C.c_float,
                                               C.c_float, f64p, i64p, i64p]
        L.oracle_voxel_centres.argtypes = [i32p, C.c_int64, C.c_float, f64p]
        L.oracle_training_set_soft.argtypes = [f32p, f32p, C.c_int64, f32p, C.c_float, C.c_int32,
                                               C.c_int32, i64p, f32p, i32p, f64p]
        L.oracle_training_set.argtypes = [f32p, i32p, C.c_int64, f32p, C.c_float, C.c_int32,
                                          C.c_int32, i64p, f32p, i32p, i64p]
        L.oracle_map_create.restype = C.c_void_p
        L.oracle_map_create.argtypes = [C.c_int32, C.c_float, C.c_int32, C.c_float, C.c_float,
                                        C.c_float, C.c_int32, C.c_int32]
        L.oracle_map_destroy.argtypes = [C.c_void_p]
        L.oracle_map_insert_training.argtypes = [C.c_void_p, f32p, i32p, C.c_int64]
        L.oracle_map_insert_scan.argtypes = [C.c_void_p, f32p, i32p, C.c_int64, f32p, C.c_float,
                                             C.c_int32]
        L.oracle_map_insert_scan_soft.argtypes = [C.c_void_p, f32p, f32p, C.c_int64, f32p,
                                                  C.c_float, C.c_int32]
        L.oracle_map_set_class_params.argtypes = [C.c_void_p, f32p, f32p]
        L.oracle_loss_classes.argtypes = [f64p, i32p, C.c_int64, f64p, i32p, C.c_int64, C.c_int32,
                                          f64p, f64p, C.c_double, f64p, f64p, f64p, f64p, f64p,
                                          f64p]
        L.oracle_map_last_insert.argtypes = [C.c_void_p, i64p]
        L.oracle_map_size.restype = C.c_int64
        L.oracle_map_size.argtypes = [C.c_void_p]
        L.oracle_map_export.argtypes = [C.c_void_p, i32p, f64p, i64p, i64p]
        L.oracle_map_lookup.argtypes = [C.c_void_p, i32p, C.c_int64, f64p]
        L.oracle_readout.argtypes = [f64p, C.c_int64, C.c_int32, C.c_int32, f64p, f64p, f64p, i32p,
                                     f64p]
        L.oracle_loss.argtypes = [f64p, i32p, C.c_int64, f64p, i32p, C.c_int64, C.c_int32,
                                  C.c_double, C.c_double, C.c_double, f64p, f64p, f64p, f64p,
                                  f64p, f64p]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _chk(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def _f32x3(a):
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1, 3)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32).reshape(-1)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the map insert (its results do not depend on the count)."""
    _chk(lib().oracle_set_num_threads(int(n)), "set_num_threads")


def kernel_f(r) -> np.ndarray:
    """f(r) of Eq. (8) (reading R1), elementwise; k = sigma0 f(d/l)."""
    r = np.asarray(r, dtype=np.float64)
    f = lib().oracle_kernel_f
    return np.vectorize(lambda x: f(float(x)), otypes=[np.float64])(r)


def kernel_df(r) -> np.ndarray:
    r = np.asarray(r, dtype=np.float64)
    f = lib().oracle_kernel_df
    return np.vectorize(lambda x: f(float(x)), otypes=[np.float64])(r)


def free_counts(xyz, label, origin, free_step, K):
    xyz, label = _f32x3(xyz), _i32(label)
    o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
    n = xyz.shape[0]
    counts = np.zeros(n, dtype=np.int64)
    tot = np.zeros(1, dtype=np.int64)
    _chk(lib().oracle_free_counts(_p(xyz, C.c_float), _p(label, C.c_int32), n, _p(o, C.c_float),
                                  C.c_float(free_step), K, _p(counts, C.c_int64),
                                  _p(tot, C.c_int64)), "free_counts")
    return counts, int(tot[0])


def free_samples(xyz, label, origin, free_step, K):
    """Free samples (float32 [Nf,3]) and their parent hit index (int64 [Nf])."""
    xyz, label = _f32x3(xyz), _i32(label)
    o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
    _, tot = free_counts(xyz, label, o, free_step, K)
    out = np.zeros((tot, 3), dtype=np.float32)
    par = np.zeros(tot, dtype=np.int64)
    _chk(lib().oracle_free_samples(_p(xyz, C.c_float), _p(label, C.c_int32), xyz.shape[0],
                                   _p(o, C.c_float), C.c_float(free_step), K,
                                   _p(out, C.c_float), _p(par, C.c_int64)), "free_samples")
    return out, par


def training_set(xyz, label, origin, free_step, K, free_class=0):
    """Rows of one scan's training set: kept hits (input order) then free samples."""
    xyz, label = _f32x3(xyz), _i32(label)
    o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
    n_out = np.zeros(1, dtype=np.int64)
    L = lib()
    args = (_p(xyz, C.c_float), _p(label, C.c_int32), xyz.shape[0], _p(o, C.c_float),
            C.c_float(free_step), K, free_class)
    _chk(L.oracle_training_set(*args, _p(n_out, C.c_int64), None, None, None), "training_set")
    nt = int(n_out[0])
    tx = np.zeros((nt, 3), dtype=np.float32)
    ty = np.zeros(nt, dtype=np.int32)
    par = np.zeros(nt, dtype=np.int64)
    _chk(L.oracle_training_set(*args, _p(n_out, C.c_int64), _p(tx, C.c_float),
                               _p(ty, C.c_int32), _p(par, C.c_int64)), "training_set")
    return tx, ty, par


def training_set_soft(xyz, probs, origin, free_step, K, free_class=0):
    """Rows of one scan of soft measurements: (xyz, class, weight) -- one row per
    positive class weight of each hit, then the free samples (weight 1)."""
    xyz = _f32x3(xyz)
    probs = np.ascontiguousarray(probs, dtype=np.float32)
    if probs.shape != (xyz.shape[0], K):
        raise ValueError(f"probs must have shape [n, {K}]")
    o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
    n_out = np.zeros(1, dtype=np.int64)
    L = lib()
    args = (_p(xyz, C.c_float), _p(probs, C.c_float), xyz.shape[0], _p(o, C.c_float),
            C.c_float(free_step), K, free_class)
    _chk(L.oracle_training_set_soft(*args, _p(n_out, C.c_int64), None, None, None),
         "training_set_soft")
    nt = int(n_out[0])
    tx = np.zeros((nt, 3), dtype=np.float32)
    ty = np.zeros(nt, dtype=np.int32)
    tw = np.zeros(nt, dtype=np.float64)
    _chk(L.oracle_training_set_soft(*args, _p(n_out, C.c_int64), _p(tx, C.c_float),
                                    _p(ty, C.c_int32), _p(tw, C.c_double)), "training_set_soft")
    return tx, ty, tw


def voxel_coords(xyz, res):
    xyz = _f32x3(xyz)
    out = np.zeros((xyz.shape[0], 3), dtype=np.int32)
    _chk(lib().oracle_voxel_coords(_p(xyz, C.c_float), xyz.shape[0], C.c_float(res),
                                   _p(out, C.c_int32)), "voxel_coords")
    return out


def pack_keys(ijk):
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(ijk.shape[0], dtype=np.uint64)
    lib().oracle_pack_keys(_p(ijk, C.c_int32), ijk.shape[0], _p(out, C.c_uint64))
    return out


def voxel_centres(ijk, res):
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((ijk.shape[0], 3), dtype=np.float64)
    lib().oracle_voxel_centres(_p(ijk, C.c_int32), ijk.shape[0], C.c_float(res),
                               _p(out, C.c_double))
    return out


def alpha_at(train_xyz, train_label, query_xyz, K, l, sigma0, alpha0):
    """Eq. (7) at arbitrary (double) query points: (alpha [Q,K], n_in [Q], n_band [Q])."""
    tx, ty = _f32x3(train_xyz), _i32(train_label)
    q = np.ascontiguousarray(query_xyz, dtype=np.float64).reshape(-1, 3)
    nq = q.shape[0]
    a = np.zeros((nq, K), dtype=np.float64)
    nin = np.zeros(nq, dtype=np.int64)
    nb = np.zeros(nq, dtype=np.int64)
    _chk(lib().oracle_alpha_at(_p(tx, C.c_float), _p(ty, C.c_int32), tx.shape[0],
                               _p(q, C.c_double), nq, K, C.c_float(l), C.c_float(sigma0),
                               C.c_float(alpha0), _p(a, C.c_double), _p(nin, C.c_int64),
                               _p(nb, C.c_int64)), "alpha_at")
    return a, nin, nb


def alpha_at_voxels(train_xyz, train_label, ijk, res, K, l, sigma0, alpha0, weights=None):
    """Eq. (7) at the centroids of voxels ijk: (alpha [Q,K], n_in [Q], n_band [Q]).
    weights (float64 per row, optional): each row's kernel value is scaled by its
    weight (soft measurements)."""
    tx, ty = _f32x3(train_xyz), _i32(train_label)
    v = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    nq = v.shape[0]
    a = np.zeros((nq, K), dtype=np.float64)
    nin = np.zeros(nq, dtype=np.int64)
    nb = np.zeros(nq, dtype=np.int64)
    tail = (_p(v, C.c_int32), nq, C.c_float(res), K, C.c_float(l), C.c_float(sigma0),
            C.c_float(alpha0), _p(a, C.c_double), _p(nin, C.c_int64), _p(nb, C.c_int64))
    if weights is None:
        _chk(lib().oracle_alpha_at_voxels(_p(tx, C.c_float), _p(ty, C.c_int32), tx.shape[0],
                                          *tail), "alpha_at_voxels")
    else:
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        if w.shape[0] != tx.shape[0]:
            raise ValueError("weights must hold one value per training row")
        _chk(lib().oracle_alpha_at_voxels_w(_p(tx, C.c_float), _p(ty, C.c_int32),
                                            _p(w, C.c_double), tx.shape[0], *tail),
             "alpha_at_voxels_w")
    return a, nin, nb


class OracleMap:
    """Eq. (7) at every grid centroid, accumulated scan after scan (Sec. IV);
    with scsm=True the counting model of Eq. (2) instead.  face_blocks=True
    restricts a voxel's training rows to its block and the six blocks sharing a
    face with it (the extended block of the paper's implementation, Sec. IV)."""

    def __init__(self, K, res, block_size, l, sigma0, alpha0, scsm=False, face_blocks=False):
        self.K = int(K)
        self._h = lib().oracle_map_create(K, C.c_float(res), block_size, C.c_float(l),
                                          C.c_float(sigma0), C.c_float(alpha0), int(bool(scsm)),
                                          int(bool(face_blocks)))
        if not self._h:
            raise OracleError(E_ARG, "map_create")

    @classmethod
    def from_params(cls, p, scsm=False, face_blocks=False):
        return cls(p.K, p.res, p.block_size, p.l, p.sigma0, p.alpha0, scsm=scsm,
                   face_blocks=face_blocks)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_map_destroy(h)
            self._h = None

    def insert_training(self, xyz, label):
        xyz, label = _f32x3(xyz), _i32(label)
        _chk(lib().oracle_map_insert_training(self._h, _p(xyz, C.c_float),
                                              _p(label, C.c_int32), xyz.shape[0]),
             "map_insert_training")

    def insert_scan(self, xyz, label, origin, free_step, free_class=0):
        xyz, label = _f32x3(xyz), _i32(label)
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        _chk(lib().oracle_map_insert_scan(self._h, _p(xyz, C.c_float), _p(label, C.c_int32),
                                          xyz.shape[0], _p(o, C.c_float), C.c_float(free_step),
                                          free_class), "map_insert_scan")

    def set_class_params(self, l, sigma0):
        """Per-class kernels (float32 [K] each): rows of class k use l[k], sigma0[k]."""
        lk = np.ascontiguousarray(l, dtype=np.float32).reshape(-1)
        sk = np.ascontiguousarray(sigma0, dtype=np.float32).reshape(-1)
        if lk.shape[0] != self.K or sk.shape[0] != self.K:
            raise ValueError(f"l and sigma0 must hold {self.K} values")
        _chk(lib().oracle_map_set_class_params(self._h, _p(lk, C.c_float), _p(sk, C.c_float)),
             "map_set_class_params")

    def insert_scan_soft(self, xyz, probs, origin, free_step, free_class=0):
        """One scan of soft measurements: probs[i] holds non-negative class
        weights of hit i (all zero drops the hit and its beam); each positive
        weight adds weight x kernel to its class (Sec. VI, linear pooling)."""
        xyz = _f32x3(xyz)
        probs = np.ascontiguousarray(probs, dtype=np.float32)
        if probs.shape != (xyz.shape[0], self.K):
            raise ValueError(f"probs must have shape [n, {self.K}]")
        o = np.ascontiguousarray(origin, dtype=np.float32).reshape(3)
        _chk(lib().oracle_map_insert_scan_soft(self._h, _p(xyz, C.c_float), _p(probs, C.c_float),
                                               xyz.shape[0], _p(o, C.c_float),
                                               C.c_float(free_step), free_class),
             "map_insert_scan_soft")

    def __len__(self):
        return int(lib().oracle_map_size(self._h))

    def last_insert(self):
        """Counters of the last insert: V (voxels with at least one row within
        l; S-CSM: voxels holding a row), P (in-support pairs; S-CSM: rows), and
        the voxels and pairs in the rounding band |d^2/l^2 - 1| <= 1e-5."""
        out = np.zeros(4, dtype=np.int64)
        _chk(lib().oracle_map_last_insert(self._h, _p(out, C.c_int64)), "map_last_insert")
        return {"V": int(out[0]), "P": int(out[1]), "V_band": int(out[2]), "P_band": int(out[3])}

    def export(self):
        """(ijk int32 [V,3], alpha [V,K], n_in [V], n_band [V]) sorted by voxel key."""
        n = len(self)
        ijk = np.zeros((n, 3), dtype=np.int32)
        a = np.zeros((n, self.K), dtype=np.float64)
        nv = np.zeros(n, dtype=np.int64)
        nb = np.zeros(n, dtype=np.int64)
        _chk(lib().oracle_map_export(self._h, _p(ijk, C.c_int32), _p(a, C.c_double),
                                     _p(nv, C.c_int64), _p(nb, C.c_int64)), "map_export")
        return ijk, a, nv, nb

    def lookup(self, ijk):
        v = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        a = np.zeros((v.shape[0], self.K), dtype=np.float64)
        lib().oracle_map_lookup(self._h, _p(v, C.c_int32), v.shape[0], _p(a, C.c_double))
        return a


def readout(alpha, free_class=0):
    """Eq. (3)-(4): dict(mean, var, mode, label, p_occ)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    n, K = a.shape
    mean = np.zeros_like(a)
    var = np.zeros_like(a)
    mode = np.zeros_like(a)
    lab = np.zeros(n, dtype=np.int32)
    pocc = np.zeros(n, dtype=np.float64)
    lib().oracle_readout(_p(a, C.c_double), n, K, free_class, _p(mean, C.c_double),
                         _p(var, C.c_double), _p(mode, C.c_double), _p(lab, C.c_int32),
                         _p(pocc, C.c_double))
    return {"mean": mean, "var": var, "mode": mode, "label": lab, "p_occ": pocc}


def loss(train_xyz, train_label, query_xyz, query_label, K, l, sigma0, alpha0):
    """Predictive loss and analytic gradient (double throughout).

    Returns dict(loss, alpha_q [H,K], grad_l, grad_sigma0, grad_train [N,3],
    grad_query [H,3])."""
    tx = np.ascontiguousarray(train_xyz, dtype=np.float64).reshape(-1, 3)
    ty = _i32(train_label)
    qx = np.ascontiguousarray(query_xyz, dtype=np.float64).reshape(-1, 3)
    qy = _i32(query_label)
    H, N = qx.shape[0], tx.shape[0]
    out = np.zeros(1)
    aq = np.zeros((H, K))
    gl = np.zeros(1)
    gs = np.zeros(1)
    gt = np.zeros((N, 3))
    gq = np.zeros((H, 3))
    _chk(lib().oracle_loss(_p(tx, C.c_double), _p(ty, C.c_int32), N, _p(qx, C.c_double),
                           _p(qy, C.c_int32), H, K, float(l), float(sigma0), float(alpha0),
                           _p(out, C.c_double), _p(aq, C.c_double), _p(gl, C.c_double),
                           _p(gs, C.c_double), _p(gt, C.c_double), _p(gq, C.c_double)), "loss")
    return {"loss": float(out[0]), "alpha_q": aq, "grad_l": float(gl[0]),
            "grad_sigma0": float(gs[0]), "grad_train": gt, "grad_query": gq}


def loss_classes(train_xyz, train_label, query_xyz, query_label, K, l, sigma0, alpha0):
    """Predictive loss with per-class kernels (l, sigma0: [K]) and its gradient.

    Returns dict(loss, alpha_q [H,K], grad_l [K], grad_sigma0 [K], grad_train [N,3],
    grad_query [H,3])."""
    tx = np.ascontiguousarray(train_xyz, dtype=np.float64).reshape(-1, 3)
    ty = _i32(train_label)
    qx = np.ascontiguousarray(query_xyz, dtype=np.float64).reshape(-1, 3)
    qy = _i32(query_label)
    lk = np.ascontiguousarray(l, dtype=np.float64).reshape(-1)
    sk = np.ascontiguousarray(sigma0, dtype=np.float64).reshape(-1)
    if lk.shape[0] != K or sk.shape[0] != K:
        raise ValueError(f"l and sigma0 must hold {K} values")
    H, N = qx.shape[0], tx.shape[0]
    out = np.zeros(1)
    aq = np.zeros((H, K))
    gl = np.zeros(K)
    gs = np.zeros(K)
    gt = np.zeros((N, 3))
    gq = np.zeros((H, 3))
    _chk(lib().oracle_loss_classes(_p(tx, C.c_double), _p(ty, C.c_int32), N, _p(qx, C.c_double),
                                   _p(qy, C.c_int32), H, K, _p(lk, C.c_double),
                                   _p(sk, C.c_double), float(alpha0), _p(out, C.c_double),
                                   _p(aq, C.c_double), _p(gl, C.c_double), _p(gs, C.c_double),
                                   _p(gt, C.c_double), _p(gq, C.c_double)), "loss_classes")
    return {"loss": float(out[0]), "alpha_q": aq, "grad_l": gl, "grad_sigma0": gs,
            "grad_train": gt, "grad_query": gq}
