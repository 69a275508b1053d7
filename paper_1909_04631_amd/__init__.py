"""MI355X (gfx950) semantic map update by Bayesian spatial kernel smoothing
(S-BKI; Gan et al., arXiv 1909.04631).

Thin Python binding of libsmki (include/smki.h): argument marshalling only,
with torch providing device memory and the current HIP stream.  Every step of
the map update runs in the library's HIP kernels; there is no CPU path.

    m = SemanticMap(res=0.1, block_size=8, l=0.3, sigma0=0.1, K=20, alpha0=1e-3)
    m.insert_scan(xyz_cuda_f32, label_cuda_i32, origin=(0, 0, 1.73), free_step=0.3)
    out = m.query(ijk_cuda_i32)          # alpha, mean, var, label, p_occ
"""
import ctypes as C

import torch

from ._lib import (ALLOC_FN, FLAG_WIDE_OFFSETS, MODELS, RELEASE_FN, SELECTIONS, SmkiError,
                   ScanStats, Options, check, lib)

__all__ = ["SemanticMap", "SmkiError", "free_samples", "bucket_cells", "loss_forward",
           "loss_backward", "PredictiveLoss", "predictive_loss", "loss_forward_classes",
           "loss_backward_classes", "PredictiveLossClasses", "predictive_loss_classes"]


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_tensor(t, dtype, shape_tail, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    return t.contiguous()


def _f3(v):
    a = (C.c_float * 3)(*[float(x) for x in v])
    return a


def _scan_tables(offsets, origins):
    offs = [int(o) for o in offsets]
    S = len(offs) - 1
    org = [float(v) for o in origins for v in o]
    if len(org) != 3 * S:
        raise ValueError("origins must hold one (x, y, z) per scan")
    return (C.c_int64 * (S + 1))(*offs), (C.c_float * (3 * S))(*org), S


class Batch:
    """A batched insert recorded as one HIP graph (smki_batch_capture).  The
    tensors it was captured with stay referenced; replay() inserts their
    current contents with the given scan offsets and origins, asynchronously."""

    def __init__(self, m, h, keep, S):
        self._m, self._h, self._keep, self.S = m, h, keep, S

    def replay(self, offsets, origins):
        offs, org, S = _scan_tables(offsets, origins)
        if S != self.S:
            raise ValueError(f"the batch was captured for {self.S} scans")
        self._m._bind_stream()
        check(lib().smki_batch_replay(self._h, offs, org), "smki_batch_replay")

    def close(self):
        if getattr(self, "_h", None):
            lib().smki_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SemanticMap:
    """A persistent semantic occupancy map on one GPU (the device current at creation)."""

    def __init__(self, res, block_size, l, sigma0, K, alpha0=1e-3, free_class=0,
                 unit_budget=0, initial_blocks=0, model="sbki", selection="exact",
                 wide_offsets=False, allocator="torch"):
        """model: "sbki" (Eq. 7-8, the default) or "scsm" (counting model, Eq. 2).
        selection: "exact" (every row within l) or "face_blocks" (rows of the
        voxel's block and its six face neighbours, the paper's extended block).
        wide_offsets: address partial sums with 64-bit offsets at any size
        (SMKI_FLAG_WIDE_OFFSETS).  allocator: "torch" (the map's growable
        buffers come from torch's caching allocator, smki_set_allocator) or
        None (hipMalloc)."""
        if allocator not in ("torch", None):
            raise ValueError('allocator must be "torch" or None')
        if model not in MODELS:
            raise ValueError(f"model must be one of {sorted(MODELS)}")
        if selection not in SELECTIONS:
            raise ValueError(f"selection must be one of {sorted(SELECTIONS)}")
        self.model = model
        self.K, self.B = int(K), int(block_size)
        self.res, self.l, self.sigma0, self.alpha0 = float(res), float(l), float(sigma0), float(alpha0)
        self.free_class = int(free_class)
        self.device = torch.device("cuda", torch.cuda.current_device())
        opt = Options(int(initial_blocks), int(unit_budget), MODELS[model], SELECTIONS[selection],
                      FLAG_WIDE_OFFSETS if wide_offsets else 0)
        h = C.c_void_p()
        check(lib().smki_create_map(res, block_size, l, sigma0, K, alpha0, free_class,
                                    C.byref(opt), C.byref(h)), "smki_create_map")
        self._h = h
        self._alloc = None
        if allocator == "torch":
            dev = self.device

            def _alloc(nbytes, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(
                        int(nbytes), dev, torch.cuda.current_stream(dev))
                except Exception:
                    return None

            def _release(ptr, ctx):
                try:
                    torch.cuda.caching_allocator_delete(int(ptr))
                except Exception:
                    pass

            # (the callback objects must outlive the map)
            self._alloc = (ALLOC_FN(_alloc), RELEASE_FN(_release))
            check(lib().smki_set_allocator(self._h, self._alloc[0], self._alloc[1], None),
                  "smki_set_allocator")

    @classmethod
    def from_params(cls, p, **kw):
        return cls(p.res, p.block_size, p.l, p.sigma0, p.K, p.alpha0, p.free_class, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().smki_destroy_map(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        check(lib().smki_set_stream(self._h, _stream()), "smki_set_stream")

    def insert_scan(self, xyz, label, origin, free_step):
        xyz = _dev_tensor(xyz, torch.float32, (3,), "xyz")
        label = _dev_tensor(label, torch.int32, (), "label")
        self._bind_stream()
        check(lib().smki_insert_scan(self._h, _ptr(xyz), _ptr(label), xyz.shape[0], _f3(origin),
                                     float(free_step)), "smki_insert_scan")

    def set_class_params(self, l, sigma0):
        """Per-class kernels: l, sigma0 sequences of K floats (see smki_set_class_params)."""
        lk = [float(v) for v in l]
        sk = [float(v) for v in sigma0]
        if len(lk) != self.K or len(sk) != self.K:
            raise ValueError(f"l and sigma0 must hold {self.K} values")
        check(lib().smki_set_class_params(self._h, (C.c_float * self.K)(*lk),
                                          (C.c_float * self.K)(*sk)), "smki_set_class_params")

    def insert_scan_soft(self, xyz, probs, origin, free_step):
        """One scan of soft measurements: probs [n, K] float32, the class weights
        of each hit (Sec. VI); see smki_insert_scan_soft."""
        xyz = _dev_tensor(xyz, torch.float32, (3,), "xyz")
        probs = _dev_tensor(probs, torch.float32, (self.K,), "probs")
        if probs.shape[0] != xyz.shape[0]:
            raise ValueError("probs must have one row per hit")
        self._bind_stream()
        check(lib().smki_insert_scan_soft(self._h, _ptr(xyz), _ptr(probs), xyz.shape[0],
                                          _f3(origin), float(free_step)), "smki_insert_scan_soft")

    def insert_scans(self, xyz, label, offsets, origins, free_step):
        xyz = _dev_tensor(xyz, torch.float32, (3,), "xyz")
        label = _dev_tensor(label, torch.int32, (), "label")
        offs, org, S = _scan_tables(offsets, origins)
        self._bind_stream()
        check(lib().smki_insert_scans(self._h, _ptr(xyz), _ptr(label), offs, org, S,
                                      float(free_step)), "smki_insert_scans")

    def batch_capture(self, xyz, label, offsets, origins, free_step, margin=0.25):
        """Insert S scans (as insert_scans) and record that insert as a HIP graph
        for these tensors; returns a Batch whose replay() inserts what the
        tensors hold then (see smki_batch_capture)."""
        xyz = _dev_tensor(xyz, torch.float32, (3,), "xyz")
        label = _dev_tensor(label, torch.int32, (), "label")
        offs, org, S = _scan_tables(offsets, origins)
        self._bind_stream()
        h = C.c_void_p()
        check(lib().smki_batch_capture(self._h, _ptr(xyz), _ptr(label), offs, org, S,
                                       float(free_step), float(margin), C.byref(h)),
              "smki_batch_capture")
        return Batch(self, h, (xyz, label), S)

    def query(self, ijk, alpha=True, mean=True, var=True, label=True, p_occ=True):
        ijk = _dev_tensor(ijk, torch.int32, (3,), "ijk")
        M = ijk.shape[0]
        dev = ijk.device
        out = {}
        if alpha:
            out["alpha"] = torch.empty((M, self.K), dtype=torch.float32, device=dev)
        if mean:
            out["mean"] = torch.empty((M, self.K), dtype=torch.float32, device=dev)
        if var:
            out["var"] = torch.empty((M, self.K), dtype=torch.float32, device=dev)
        if label:
            out["label"] = torch.empty((M,), dtype=torch.int32, device=dev)
        if p_occ:
            out["p_occ"] = torch.empty((M,), dtype=torch.float32, device=dev)
        self._bind_stream()
        check(lib().smki_query(self._h, _ptr(ijk), M, _ptr(out.get("alpha")), _ptr(out.get("mean")),
                               _ptr(out.get("var")), _ptr(out.get("label")), _ptr(out.get("p_occ"))),
              "smki_query")
        return out

    def num_blocks(self):
        n = C.c_int64()
        check(lib().smki_num_blocks(self._h, C.byref(n)), "smki_num_blocks")
        return int(n.value)

    def export(self):
        """(block_ijk int32 [n,3], alpha float32 [n,K,B,B,B]) in ascending key order."""
        self._bind_stream()
        n = C.c_int64()
        check(lib().smki_export(self._h, 0, C.byref(n), None, None), "smki_export")
        nb = int(n.value)
        ijk = torch.empty((nb, 3), dtype=torch.int32, device=self.device)
        a = torch.empty((nb, self.K, self.B, self.B, self.B), dtype=torch.float32, device=self.device)
        if nb:
            check(lib().smki_export(self._h, nb, C.byref(n), _ptr(ijk), _ptr(a)), "smki_export")
        return ijk, a

    def import_(self, block_ijk, alpha):
        block_ijk = _dev_tensor(block_ijk, torch.int32, (3,), "block_ijk")
        alpha = _dev_tensor(alpha, torch.float32, (self.K, self.B, self.B, self.B), "alpha")
        self._bind_stream()
        check(lib().smki_import(self._h, block_ijk.shape[0], _ptr(block_ijk), _ptr(alpha)),
              "smki_import")

    def reset(self):
        """Empty the map (every voxel back to alpha0); capacity is kept."""
        self._bind_stream()
        check(lib().smki_import(self._h, 0, None, None), "smki_import")

    def stats(self):
        s = ScanStats()
        check(lib().smki_last_scan_stats(self._h, C.byref(s)), "smki_last_scan_stats")
        return s.as_dict()

    def kernel_times(self, last=64):
        """(splat_ms, merge_ms) lists of the last inserts, oldest first."""
        sp = (C.c_float * last)()
        mg = (C.c_float * last)()
        n = C.c_int32(0)
        check(lib().smki_kernel_times(self._h, int(last), sp, mg, C.byref(n)), "smki_kernel_times")
        return list(sp[:n.value]), list(mg[:n.value])

    def set_kernel_timing(self, on=True):
        """Record (or not) the HIP events behind kernel_times() in later inserts."""
        check(lib().smki_set_kernel_timing(self._h, 1 if on else 0), "smki_set_kernel_timing")

    def sync(self):
        check(lib().smki_sync(self._h), "smki_sync")


def free_samples(xyz, label, origin, free_step, K):
    """Free-space samples of one scan: (xyz float32 [Nf,3], parent int64 [Nf])."""
    xyz = _dev_tensor(xyz, torch.float32, (3,), "xyz")
    label = _dev_tensor(label, torch.int32, (), "label")
    n = C.c_int64()
    L = lib()
    check(L.smki_free_samples(_ptr(xyz), _ptr(label), xyz.shape[0], _f3(origin), float(free_step),
                              int(K), _stream(), C.byref(n), None, None), "smki_free_samples")
    out = torch.empty((int(n.value), 3), dtype=torch.float32, device=xyz.device)
    par = torch.empty((int(n.value),), dtype=torch.int64, device=xyz.device)
    if n.value:
        check(L.smki_free_samples(_ptr(xyz), _ptr(label), xyz.shape[0], _f3(origin),
                                  float(free_step), int(K), _stream(), C.byref(n), _ptr(out),
                                  _ptr(par)), "smki_free_samples")
    return out, par


def bucket_cells(xyz, res, block_size):
    """Voxel-cell table: (keys int64 [C] (packed voxel index), start int32 [C],
    count int32 [C], order int32 [n])."""
    xyz = _dev_tensor(xyz, torch.float32, (3,), "xyz")
    n = C.c_int64()
    L = lib()
    check(L.smki_bucket_cells(_ptr(xyz), xyz.shape[0], float(res), int(block_size), _stream(),
                              C.byref(n), None, None, None, None), "smki_bucket_cells")
    nc = int(n.value)
    keys = torch.empty((nc,), dtype=torch.int64, device=xyz.device)
    start = torch.empty((nc,), dtype=torch.int32, device=xyz.device)
    count = torch.empty((nc,), dtype=torch.int32, device=xyz.device)
    order = torch.empty((xyz.shape[0],), dtype=torch.int32, device=xyz.device)
    if nc:
        check(L.smki_bucket_cells(_ptr(xyz), xyz.shape[0], float(res), int(block_size), _stream(),
                                  C.byref(n), _ptr(keys), _ptr(start), _ptr(count), _ptr(order)),
              "smki_bucket_cells")
    return keys, start, count, order


from .loss import (PredictiveLoss, PredictiveLossClasses, loss_backward,  # noqa: E402
                   loss_backward_classes, loss_forward, loss_forward_classes, predictive_loss,
                   predictive_loss_classes)
