"""ctypes declarations of liblma.so (mirrors include/lma.h)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblma.so")

LMA_OK, LMA_ERR_ARG, LMA_ERR_OOM, LMA_ERR_DEVICE, LMA_ERR_STATE, LMA_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
LMA_BASIS_PROBE, LMA_BASIS_GAUSSIAN, LMA_BASIS_TRIGPOLY = 0, 1, 2
LMA_GEMM_FP32, LMA_GEMM_SPLIT_BF16 = 0, 1
LMA_PTR_DEVICE, LMA_ACCUMULATE, LMA_HOST_ONLY, LMA_CONTRACT_PER_PIXEL, LMA_OWN_STREAM = 1, 2, 4, 8, 16
LMA_AUTOTUNE, LMA_GRAPH = 32, 64
LMA_REQ_BUILD, LMA_REQ_IMAGE, LMA_REQ_EDIT, LMA_REQ_PLAIN, LMA_REQ_RELEASE = 1, 2, 3, 4, 5


class lma_optics(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("lx", C.c_double), ("ly", C.c_double),
                ("wavelength", C.c_double), ("sigma", C.c_double), ("dz", C.c_double),
                ("bandlimit", C.c_double), ("alpha_max", C.c_double), ("defocus", C.c_double),
                ("cs", C.c_double)]


class lma_lattice(C.Structure):
    _fields_ = [("px", C.c_int32), ("py", C.c_int32), ("rx", C.c_int32), ("ry", C.c_int32),
                ("f", C.c_int32), ("offset_x", C.c_double), ("offset_y", C.c_double), ("L", C.c_int32),
                ("basis_kind", C.c_int32), ("precision", C.c_int32), ("window", C.c_int32 * 4),
                ("batch", C.c_int32), ("hbm_budget_bytes", C.c_int64), ("basis_param", C.c_double),
                ("prop_nx", C.c_int32), ("prop_ny", C.c_int32)]


class lma_detectors(C.Structure):
    _fields_ = [("n", C.c_int32), ("inner", C.POINTER(C.c_double)), ("outer", C.POINTER(C.c_double))]


class lma_info(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_translates", C.c_int32), ("rfx", C.c_int32),
                ("rfy", C.c_int32), ("n_sets", C.c_int32), ("ncls_x", C.c_int32), ("ncls_y", C.c_int32),
                ("L", C.c_int32), ("n_det", C.c_int32), ("n_pix", C.c_int32), ("n_probes", C.c_int32),
                ("n_rows", C.c_int32), ("batch", C.c_int32), ("n_aperture", C.c_int32),
                ("basis_valid", C.c_int32), ("host_only", C.c_int32), ("max_residual", C.c_double),
                ("device_bytes", C.c_int64), ("contract_kernel", C.c_int32), ("contract_k", C.c_int32),
                ("partitioned", C.c_int32), ("n_parts", C.c_int32), ("part_w", C.c_int32), ("part_h", C.c_int32),
                ("resident_rows", C.c_int64), ("multislice_calls", C.c_int64), ("tile_width", C.c_int32),
                ("graphs", C.c_int32), ("prop_nx", C.c_int32), ("prop_ny", C.c_int32),
                ("gap_lo", C.c_int32), ("gap_hi", C.c_int32), ("input_gap_lo", C.c_int32),
                ("input_gap_hi", C.c_int32), ("radix_schedule", C.c_int32)]


class lma_tuning(C.Structure):
    _fields_ = [("tile_width", C.c_int32), ("batch", C.c_int32), ("us_per_wave_slice", C.c_double),
                ("candidates", C.c_int32), ("radix_schedule", C.c_int32)]


class lma_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("specimen", C.c_int32), ("optics", C.POINTER(lma_optics)),
                ("lattice", C.POINTER(lma_lattice)), ("detectors", C.POINTER(lma_detectors)),
                ("potential", C.c_void_p), ("nslices", C.c_int32), ("image", C.c_void_p), ("flags", C.c_int32),
                ("weight", C.c_double), ("bbox", C.c_int32 * 4), ("radius", C.c_double)]


class lma_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


# every symbol declared in include/lma.h, with its ctypes signature
P = C.c_void_p
SIGNATURES = {
    "lma_electron_constants": (C.c_int, [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lma_build_basis": (C.c_int, [C.POINTER(lma_optics), C.POINTER(lma_lattice), C.POINTER(lma_detectors),
                                  P, C.c_int32, C.POINTER(P)]),
    "lma_propagate": (C.c_int, [P, P, C.c_int32, C.c_int32]),
    "lma_probe_image": (C.c_int, [P, P, C.c_int32, C.c_double]),
    "lma_plain_image": (C.c_int, [P, P, C.c_int32, P, C.c_int32, C.c_double]),
    "lma_plain_image_noalloc": (C.c_int, [P, P, C.c_int32, P, C.c_int32, C.c_double]),
    "lma_image": (C.c_int, [P, P, C.c_int32, P, C.c_int32, C.c_double]),
    "lma_probe_patterns": (C.c_int, [P, P, C.c_int32]),
    "lma_probe_radial": (C.c_int, [P, C.c_double, C.c_int32, P, C.c_int32, C.c_double]),
    "lma_plain_patterns": (C.c_int, [P, P, C.c_int32, P, C.c_int32]),
    "lma_recompute_local": (C.c_int, [P, P, C.c_int32, C.POINTER(C.c_int32), C.c_double, P,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lma_footprint": (C.c_int, [C.POINTER(lma_optics), C.POINTER(lma_lattice), C.POINTER(lma_detectors),
                                C.c_int32, C.POINTER(C.c_int64)]),
    "lma_plan_info": (C.c_int, [P, C.POINTER(lma_info)]),
    "lma_get_translates": (C.c_int, [P, P]),
    "lma_get_coefficients": (C.c_int, [P, P, P]),
    "lma_get_detector_pixels": (C.c_int, [P, P, P]),
    "lma_get_probe_spectrum": (C.c_int, [P, P]),
    "lma_get_input_wave_spectrum": (C.c_int, [P, P]),
    "lma_get_window_spectrum": (C.c_int, [P, P]),
    "lma_get_basis_rows": (C.c_int, [P, C.c_int32, C.c_int32, P]),
    "lma_save_basis": (C.c_int, [P, C.c_char_p]),
    "lma_load_basis": (C.c_int, [P, C.c_char_p]),
    "lma_get_rows": (C.c_int, [P, P]),
    "lma_set_timing": (C.c_int, [P, C.c_int32]),
    "lma_get_timing": (C.c_int, [P, C.POINTER(lma_kernel_time), C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
    "lma_destroy": (None, [P]),
    "lma_synchronize": (C.c_int, [P]),
    "lma_autotune": (C.c_int, [C.c_int32, C.c_int32, C.c_int64, P, C.POINTER(lma_tuning)]),
    "lma_batch_create": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(C.c_int32), P, C.POINTER(P)]),
    "lma_batch_propagate": (C.c_int, [P, C.POINTER(P), C.c_int32]),
    "lma_batch_destroy": (None, [P]),
    "lma_batch_create_grouped": (C.c_int, [C.POINTER(P), C.c_int32, C.POINTER(C.c_int32), P, C.c_int64, C.POINTER(P)]),
    "lma_server_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int64, C.POINTER(P)]),
    "lma_server_submit": (C.c_int, [P, C.POINTER(lma_request), C.POINTER(C.c_int64)]),
    "lma_server_wait": (C.c_int, [P, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lma_server_plan": (C.c_int, [P, C.c_int32, C.POINTER(P)]),
    "lma_server_in_use": (C.c_int, [P, C.POINTER(C.c_int64)]),
    "lma_server_destroy": (None, [P]),
    "lma_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads liblma.so. Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2310_16829_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname. Loading it first makes this
    # library bind to that copy, so the process holds one HIP runtime and torch streams and
    # allocations are valid here; loading ours first would map two runtimes.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
