"""ctypes declarations of libsmki.so (the C ABI in include/smki.h).

The library is built in-tree by ``paper_1909_04631_amd.build``.  There is no
fallback: if the shared library is missing or fails to load, every entry
point raises.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmki.so")

SMKI_OK = 0
STATUS_NAMES = {
    0: "SMKI_OK", -1: "SMKI_E_INVALID_ARG", -2: "SMKI_E_OOM", -3: "SMKI_E_CAPACITY",
    -4: "SMKI_E_DEVICE", -5: "SMKI_E_BAD_INPUT", -6: "SMKI_E_RANGE",
}

# every symbol include/smki.h declares
EXPORTED = [
    "smki_status_string", "smki_create_map", "smki_destroy_map", "smki_set_class_params",
    "smki_set_stream", "smki_set_allocator", "smki_insert_scan", "smki_insert_scan_soft", "smki_insert_scans",
    "smki_query", "smki_num_blocks", "smki_export", "smki_import", "smki_kernel_times", "smki_set_kernel_timing", "smki_last_scan_stats", "smki_sync", "smki_free_samples", "smki_bucket_cells",
    "smki_loss_workspace_bytes", "smki_loss_forward", "smki_loss_backward",
    "smki_loss_forward_classes", "smki_loss_backward_classes", "smki_loss_forward_noalloc",
    "smki_batch_capture", "smki_batch_replay", "smki_batch_destroy",
]


class SmkiError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = int(status)
        name = STATUS_NAMES.get(self.status, str(self.status))
        msg = ""
        try:
            msg = lib().smki_status_string(self.status).decode()
        except Exception:
            pass
        super().__init__(f"{what}: {name} ({msg})")


class Options(C.Structure):
    _fields_ = [("initial_blocks", C.c_int64), ("unit_budget", C.c_int32), ("model", C.c_int32),
                ("selection", C.c_int32), ("flags", C.c_int32)]


FLAG_WIDE_OFFSETS = 1

# smki_alloc_fn / smki_release_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


MODELS = {"sbki": 0, "scsm": 1}
SELECTIONS = {"exact": 0, "face_blocks": 1}


class ScanStats(C.Structure):
    _fields_ = [("n_hits", C.c_int64), ("n_free", C.c_int64), ("n_point_blocks", C.c_int64),
                ("n_target_blocks", C.c_int64), ("n_new_blocks", C.c_int64),
                ("n_new_class_blocks", C.c_int64),
                ("n_units", C.c_int64), ("n_updated_voxels", C.c_int64), ("n_pairs", C.c_int64),
                ("n_candidates", C.c_int64), ("n_lane_slots", C.c_int64), ("splat_ms", C.c_double),
                ("merge_ms", C.c_double)]

    def as_dict(self):
        return {f: (float if f.endswith("_ms") else int)(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1909_04631_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, f, i32, i64 = C.c_void_p, C.c_float, C.c_int32, C.c_int64
    st = C.c_int32
    L.smki_status_string.restype = C.c_char_p
    L.smki_status_string.argtypes = [st]
    L.smki_create_map.restype = st
    L.smki_create_map.argtypes = [f, i32, f, f, i32, f, i32, C.POINTER(Options), C.POINTER(vp)]
    L.smki_destroy_map.restype = st
    L.smki_destroy_map.argtypes = [vp]
    L.smki_set_stream.restype = st
    L.smki_set_stream.argtypes = [vp, vp]
    L.smki_set_allocator.restype = st
    L.smki_set_allocator.argtypes = [vp, ALLOC_FN, RELEASE_FN, vp]
    L.smki_kernel_times.restype = st
    L.smki_kernel_times.argtypes = [vp, i32, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                    C.POINTER(C.c_int32)]
    L.smki_set_class_params.restype = st
    L.smki_set_class_params.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.smki_insert_scan.restype = st
    L.smki_insert_scan.argtypes = [vp, vp, vp, i64, C.POINTER(C.c_float), f]
    L.smki_insert_scan_soft.restype = st
    L.smki_insert_scan_soft.argtypes = [vp, vp, vp, i64, C.POINTER(C.c_float), f]
    L.smki_insert_scans.restype = st
    L.smki_insert_scans.argtypes = [vp, vp, vp, C.POINTER(C.c_int64), C.POINTER(C.c_float), i32, f]
    L.smki_query.restype = st
    L.smki_query.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    L.smki_num_blocks.restype = st
    L.smki_num_blocks.argtypes = [vp, C.POINTER(C.c_int64)]
    L.smki_export.restype = st
    L.smki_export.argtypes = [vp, i64, C.POINTER(C.c_int64), vp, vp]
    L.smki_import.restype = st
    L.smki_import.argtypes = [vp, i64, vp, vp]
    L.smki_last_scan_stats.restype = st
    L.smki_last_scan_stats.argtypes = [vp, C.POINTER(ScanStats)]
    L.smki_sync.restype = st
    L.smki_sync.argtypes = [vp]
    L.smki_set_kernel_timing.restype = st
    L.smki_set_kernel_timing.argtypes = [vp, i32]
    L.smki_free_samples.restype = st
    L.smki_free_samples.argtypes = [vp, vp, i64, C.POINTER(C.c_float), f, i32, vp,
                                    C.POINTER(C.c_int64), vp, vp]
    L.smki_bucket_cells.restype = st
    L.smki_bucket_cells.argtypes = [vp, i64, f, i32, vp, C.POINTER(C.c_int64), vp, vp, vp, vp]
    L.smki_loss_workspace_bytes.restype = C.c_size_t
    L.smki_loss_workspace_bytes.argtypes = [i64, i64, i32]
    L.smki_loss_forward.restype = st
    L.smki_loss_forward.argtypes = [vp, vp, i64, vp, vp, i64, f, f, f, i32, vp, vp, C.c_size_t,
                                    vp, vp]
    L.smki_loss_backward.restype = st
    L.smki_loss_backward.argtypes = [vp, vp, i64, vp, vp, i64, f, f, f, i32, vp, vp, C.c_size_t,
                                     vp, vp, vp, vp, vp, vp]
    fp = C.POINTER(C.c_float)
    L.smki_loss_forward_classes.restype = st
    L.smki_loss_forward_classes.argtypes = [vp, vp, i64, vp, vp, i64, fp, fp, f, i32, vp, vp,
                                            C.c_size_t, vp, vp]
    L.smki_loss_backward_classes.restype = st
    L.smki_loss_backward_classes.argtypes = [vp, vp, i64, vp, vp, i64, fp, fp, f, i32, vp, vp,
                                             C.c_size_t, vp, vp, vp, vp, vp, vp]
    L.smki_batch_capture.restype = st
    L.smki_batch_capture.argtypes = [vp, vp, vp, C.POINTER(C.c_int64), C.POINTER(C.c_float), i32,
                                     f, f, C.POINTER(vp)]
    L.smki_batch_replay.restype = st
    L.smki_batch_replay.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_float)]
    L.smki_batch_destroy.restype = st
    L.smki_batch_destroy.argtypes = [vp]
    L.smki_loss_forward_noalloc.restype = st
    L.smki_loss_forward_noalloc.argtypes = [vp, vp, i64, vp, vp, i64, f, f, f, i32, vp, vp, vp]
    _lib = L
    return L


def check(status, what):
    if status != SMKI_OK:
        raise SmkiError(status, what)
