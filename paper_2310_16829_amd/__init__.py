"""Python binding of liblma.so: the MI355X hot path of the Lattice Multislice Algorithm.

Argument marshalling only: every step of the simulation runs in the library (host planner
in C++, kernels in HIP for gfx950). Host data are numpy arrays; device data are torch
tensors on the GPU (passed by pointer with LMA_PTR_DEVICE). The library is loaded from
this directory and there is no fallback when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _lib
from ._lib import (LMA_ACCUMULATE, LMA_AUTOTUNE, LMA_BASIS_GAUSSIAN, LMA_BASIS_PROBE, LMA_BASIS_TRIGPOLY, LMA_CONTRACT_PER_PIXEL,
                   LMA_GEMM_FP32, LMA_GEMM_SPLIT_BF16, LMA_GRAPH, LMA_HOST_ONLY, LMA_OWN_STREAM, LMA_PTR_DEVICE,
                   LMA_REQ_BUILD, LMA_REQ_EDIT, LMA_REQ_IMAGE, LMA_REQ_PLAIN, LMA_REQ_RELEASE, lma_detectors,
                   lma_info, lma_kernel_time, lma_lattice, lma_optics, lma_request, lma_tuning)

__all__ = ["LmaError", "Plan", "electron_constants", "footprint", "optics", "lattice", "detectors",
           "LMA_ACCUMULATE", "LMA_PTR_DEVICE", "LMA_HOST_ONLY", "LMA_GEMM_FP32", "LMA_GEMM_SPLIT_BF16",
           "LMA_BASIS_PROBE", "LMA_BASIS_GAUSSIAN", "LMA_BASIS_TRIGPOLY", "LMA_CONTRACT_PER_PIXEL", "LMA_OWN_STREAM", "LMA_AUTOTUNE",
           "LMA_GRAPH", "Server", "Batch", "autotune", "lib"]


class LmaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liblma status {status}: {msg}")
        self.status = status


def lib():
    return _lib.load()


def _check(status):
    if status != 0:
        raise LmaError(status, lib().lma_last_error().decode())


def electron_constants(kv: float):
    lam, sig = C.c_double(), C.c_double()
    _check(lib().lma_electron_constants(float(kv), C.byref(lam), C.byref(sig)))
    return lam.value, sig.value


def optics(nx, ny, lx, ly, wavelength, sigma, dz, bandlimit, alpha_max, defocus=0.0, cs=0.0) -> lma_optics:
    return lma_optics(int(nx), int(ny), float(lx), float(ly), float(wavelength), float(sigma), float(dz),
                      float(bandlimit), float(alpha_max), float(defocus), float(cs))


def lattice(px, py, rx, ry, f=1, offset=(0.5, 0.5), L=1, precision=LMA_GEMM_FP32, window=(0, 0, 0, 0),
            batch=0, hbm_budget_bytes=0, basis_kind=LMA_BASIS_PROBE, basis_param=0.0,
            prop_window=(0, 0)) -> lma_lattice:
    lat = lma_lattice()
    lat.px, lat.py, lat.rx, lat.ry, lat.f = int(px), int(py), int(rx), int(ry), int(f)
    lat.offset_x, lat.offset_y = float(offset[0]), float(offset[1])
    lat.L, lat.basis_kind, lat.precision = int(L), int(basis_kind), int(precision)
    for i in range(4):
        lat.window[i] = int(window[i])
    lat.batch, lat.hbm_budget_bytes = int(batch), int(hbm_budget_bytes)
    lat.basis_param = float(basis_param)
    lat.prop_nx, lat.prop_ny = int(prop_window[0]), int(prop_window[1])
    return lat


class _Detectors:
    """lma_detectors plus the arrays it points into."""

    def __init__(self, rings):
        rings = list(rings)
        self.inner = (C.c_double * len(rings))(*[float(a) for a, _ in rings])
        self.outer = (C.c_double * len(rings))(*[float(b) for _, b in rings])
        self.s = lma_detectors(len(rings), self.inner, self.outer)


def detectors(rings) -> _Detectors:
    """rings: sequence of (inner_rad, outer_rad)."""
    return _Detectors(rings)


def footprint(opt: lma_optics, lat: lma_lattice, det: _Detectors, nslices: int) -> int:
    b = C.c_int64()
    _check(lib().lma_footprint(C.byref(opt), C.byref(lat), C.byref(det.s), int(nslices), C.byref(b)))
    return b.value


def autotune(nx: int, ny: int, max_bytes: int = 0, stream=None) -> dict:
    """lma_autotune: the fastest (tile width, batch, radix schedule) of the slice passes for an
    nx x ny grid."""
    t = lma_tuning()
    st = _current_stream() if stream is None else C.c_void_p(stream)
    _check(lib().lma_autotune(int(nx), int(ny), int(max_bytes), st, C.byref(t)))
    return dict(tile_width=t.tile_width, batch=t.batch, us_per_wave_slice=t.us_per_wave_slice,
                candidates=t.candidates, radix_schedule=t.radix_schedule)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, flags) of a host numpy array or a device torch tensor."""
    if _is_torch(x):
        import torch
        want = {np.float32: torch.float32, np.float64: torch.float64}[dtype]
        if not x.is_cuda or x.dtype != want or not x.is_contiguous():
            raise ValueError("device tensors must be contiguous, on the GPU, of the expected dtype")
        return C.c_void_p(x.data_ptr()), LMA_PTR_DEVICE
    if not isinstance(x, np.ndarray) or x.dtype != dtype or not x.flags.c_contiguous:
        raise ValueError(f"host arrays must be C-contiguous numpy {np.dtype(dtype).name}")
    return C.c_void_p(x.ctypes.data), 0


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(None)


class Plan:
    """An lma_plan. Methods carry the names of the C entry points without the prefix."""

    def __init__(self, opt: lma_optics, lat: lma_lattice, det: _Detectors, flags: int = 0, stream=None):
        self._h = C.c_void_p()
        self._det = det
        self.host_only = bool(flags & LMA_HOST_ONLY)
        st = C.c_void_p(None) if self.host_only else (_current_stream() if stream is None else C.c_void_p(stream))
        _check(lib().lma_build_basis(C.byref(opt), C.byref(lat), C.byref(det.s), st, int(flags), C.byref(self._h)))
        self.nx, self.ny = opt.nx, opt.ny
        i = self.info()
        self.n_det, self.n_pix, self.n_rows = i.n_det, i.n_pix, i.n_rows
        w = list(lat.window)
        self.window = (0, 0, lat.px, lat.py) if w == [0, 0, 0, 0] else tuple(w)

    # --- lifetime ----------------------------------------------------------------------
    def close(self):
        if self._h:
            lib().lma_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- hot path ----------------------------------------------------------------------
    def image_shape(self):
        return (self.n_det, self.window[3], self.window[2])

    def _image_out(self, image, like_device):
        if image is None:
            if like_device:
                import torch
                image = torch.zeros(self.image_shape(), dtype=torch.float64, device="cuda")
            else:
                image = np.zeros(self.image_shape(), dtype=np.float64)
        return image

    def propagate(self, potential, flags: int = 0):
        p, f = _ptr(potential, np.float32)
        _check(lib().lma_propagate(self._h, p, int(potential.shape[0]), int(flags) | f))

    def probe_image(self, image=None, flags: int = 0, weight: float = 1.0, device: bool = False):
        image = self._image_out(image, device)
        p, f = _ptr(image, np.float64)
        _check(lib().lma_probe_image(self._h, p, int(flags) | f, float(weight)))
        return image

    def image(self, potential, image=None, flags: int = 0, weight: float = 1.0, device: bool = False):
        pp, fp = _ptr(potential, np.float32)
        image = self._image_out(image, device)
        pi, fi = _ptr(image, np.float64)
        if fp != fi:
            raise ValueError("potential and image must both be host or both be device")
        _check(lib().lma_image(self._h, pp, int(potential.shape[0]), pi, int(flags) | fi, float(weight)))
        return image

    def plain_image(self, potential, image=None, flags: int = 0, weight: float = 1.0, device: bool = False):
        pp, fp = _ptr(potential, np.float32)
        image = self._image_out(image, device)
        pi, fi = _ptr(image, np.float64)
        if fp != fi:
            raise ValueError("potential and image must both be host or both be device")
        _check(lib().lma_plain_image(self._h, pp, int(potential.shape[0]), pi, int(flags) | fi, float(weight)))
        return image

    def plain_image_noalloc(self, potential, image, flags: int = 0, weight: float = 1.0):
        """lma_plain_image_noalloc: device tensors only, no allocation by the library."""
        pp, fp = _ptr(potential, np.float32)
        pi, fi = _ptr(image, np.float64)
        if not (fp and fi):
            raise ValueError("lma_plain_image_noalloc takes device tensors")
        _check(lib().lma_plain_image_noalloc(self._h, pp, int(potential.shape[0]), pi, int(flags) | fi, float(weight)))
        return image

    def _pattern_out(self, out, device):
        shape = (self.window[3], self.window[2], self.n_pix)
        if out is None:
            if device:
                import torch
                out = torch.zeros(shape, dtype=torch.float32, device="cuda")
            else:
                out = np.zeros(shape, dtype=np.float32)
        return out

    def probe_patterns(self, out=None, flags: int = 0, device: bool = False):
        """4-D STEM: [wh][ww][D] float32 at the plan's detector pixels."""
        out = self._pattern_out(out, device)
        p, f = _ptr(out, np.float32)
        _check(lib().lma_probe_patterns(self._h, p, int(flags) | f))
        return out

    def plain_patterns(self, potential, out=None, flags: int = 0, device: bool = False):
        pp, fp = _ptr(potential, np.float32)
        out = self._pattern_out(out, device)
        po, fo = _ptr(out, np.float32)
        if fp != fo:
            raise ValueError("potential and output must both be host or both be device")
        _check(lib().lma_plain_patterns(self._h, pp, int(potential.shape[0]), po, int(flags) | fo))
        return out

    def probe_radial(self, width: float, nbins: int, image=None, flags: int = 0, weight: float = 1.0,
                     device: bool = False):
        """3-D STEM: [nbins][wh][ww] float64 sums over annuli a*width <= lambda|k| < (a+1)*width."""
        shape = (int(nbins), self.window[3], self.window[2])
        if image is None:
            if device:
                import torch
                image = torch.zeros(shape, dtype=torch.float64, device="cuda")
            else:
                image = np.zeros(shape, dtype=np.float64)
        p, f = _ptr(image, np.float64)
        _check(lib().lma_probe_radial(self._h, float(width), int(nbins), p, int(flags) | f, float(weight)))
        return image

    def recompute_local(self, potential_new, bbox, radius: float, image):
        pp, fp = _ptr(potential_new, np.float32)
        pi, fi = _ptr(image, np.float64)
        if fp or fi:
            raise ValueError("recompute_local takes host arrays")
        bb = (C.c_int32 * 4)(*[int(x) for x in bbox])
        nt, npr = C.c_int32(), C.c_int32()
        _check(lib().lma_recompute_local(self._h, pp, int(potential_new.shape[0]), bb, float(radius), pi,
                                         C.byref(nt), C.byref(npr)))
        return nt.value, npr.value

    # --- inspection --------------------------------------------------------------------
    def info(self) -> lma_info:
        i = lma_info()
        _check(lib().lma_plan_info(self._h, C.byref(i)))
        return i

    def translates(self) -> np.ndarray:
        out = np.zeros((self.info().n_translates, 2))
        _check(lib().lma_get_translates(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def coefficients(self):
        i = self.info()
        t = np.zeros((i.n_sets, i.L), dtype=np.int32)
        a = np.zeros((i.n_sets, i.L, 2))
        _check(lib().lma_get_coefficients(self._h, C.c_void_p(t.ctypes.data), C.c_void_p(a.ctypes.data)))
        return t, a[..., 0] + 1j * a[..., 1]

    def detector_pixels(self):
        n = self.info().n_pix
        flat = np.zeros(n, dtype=np.int32)
        mask = np.zeros(n, dtype=np.uint32)
        _check(lib().lma_get_detector_pixels(self._h, C.c_void_p(flat.ctypes.data), C.c_void_p(mask.ctypes.data)))
        return flat, mask

    def input_wave_spectrum(self) -> np.ndarray:
        out = np.zeros((self.ny, self.nx, 2))
        _check(lib().lma_get_input_wave_spectrum(self._h, C.c_void_p(out.ctypes.data)))
        return out[..., 0] + 1j * out[..., 1]

    def window_spectrum(self) -> np.ndarray:
        i = self.info()
        out = np.zeros((i.prop_ny, i.prop_nx, 2))
        _check(lib().lma_get_window_spectrum(self._h, C.c_void_p(out.ctypes.data)))
        return out[..., 0] + 1j * out[..., 1]

    def probe_spectrum(self) -> np.ndarray:
        out = np.zeros((self.ny, self.nx, 2))
        _check(lib().lma_get_probe_spectrum(self._h, C.c_void_p(out.ctypes.data)))
        return out[..., 0] + 1j * out[..., 1]

    def rows(self) -> np.ndarray:
        out = np.zeros(self.info().n_rows, dtype=np.int32)
        _check(lib().lma_get_rows(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def save_basis(self, path: str):
        """Writes the resident basis to `path` (lma_save_basis)."""
        _check(lib().lma_save_basis(self._h, os.fsencode(path)))

    def load_basis(self, path: str):
        """Reads a basis written by a plan of the same layout (lma_load_basis)."""
        _check(lib().lma_load_basis(self._h, os.fsencode(path)))

    def basis_rows(self, first: int, count: int) -> np.ndarray:
        out = np.zeros((count, self.n_pix, 2), dtype=np.float32)
        _check(lib().lma_get_basis_rows(self._h, int(first), int(count), C.c_void_p(out.ctypes.data)))
        return out[..., 0].astype(np.complex128) + 1j * out[..., 1]

    def set_timing(self, enable: bool):
        _check(lib().lma_set_timing(self._h, int(bool(enable))))

    def timing(self, reset: bool = False) -> dict:
        arr = (lma_kernel_time * 32)()
        n = C.c_int32()
        _check(lib().lma_get_timing(self._h, arr, 32, C.byref(n), int(bool(reset))))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}


class Batch:
    """An lma_batch: the translate propagation of several plans as one graph launch. With
    grouped=True (lma_batch_create_grouped) plans of one transform-length class share their row
    and column pass launches; max_group_bytes bounds each class's wave buffer (0: 32 GiB)."""

    def __init__(self, plans, nslices, stream=None, grouped: bool = False, max_group_bytes: int = 0):
        self._plans = list(plans)
        n = len(self._plans)
        hs = (C.c_void_p * n)(*[p._h.value for p in self._plans])
        ns = (C.c_int32 * n)(*[int(x) for x in nslices])
        self._h = C.c_void_p()
        st = C.c_void_p(None) if stream is None else C.c_void_p(stream)
        if grouped:
            _check(lib().lma_batch_create_grouped(hs, n, ns, st, int(max_group_bytes), C.byref(self._h)))
        else:
            _check(lib().lma_batch_create(hs, n, ns, st, C.byref(self._h)))

    def propagate(self, potentials, flags: int = 0):
        ptrs, fl = [], set()
        for v in potentials:
            p, f = _ptr(v, np.float32)
            ptrs.append(p.value)
            fl.add(f)
        if len(fl) != 1:
            raise ValueError("potentials must all be host or all be device")
        if fl == {LMA_PTR_DEVICE}:
            import torch
            torch.cuda.current_stream().synchronize()
        arr = (C.c_void_p * len(ptrs))(*ptrs)
        _check(lib().lma_batch_propagate(self._h, arr, int(flags) | fl.pop()))

    def close(self):
        if self._h:
            lib().lma_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """An lma_server: requests on resident specimens, run by `slots` worker threads of the
    library with continuous batching (see include/lma.h). Every buffer a request names is
    kept referenced here until its ticket has been waited for. Device tensors are made ready
    (the current torch stream is synchronised) before a request that reads them is queued."""

    def __init__(self, slots: int, max_specimens: int, budget_bytes: int):
        self._h = C.c_void_p()
        _check(lib().lma_server_create(int(slots), int(max_specimens), int(budget_bytes), C.byref(self._h)))
        self._keep = {}

    def _submit(self, req, keep):
        t = C.c_int64()
        _check(lib().lma_server_submit(self._h, C.byref(req), C.byref(t)))
        self._keep[t.value] = (req, keep)
        return t.value

    @staticmethod
    def _ready(*xs):
        if any(_is_torch(x) for x in xs):
            import torch
            torch.cuda.current_stream().synchronize()

    def build(self, specimen: int, opt: lma_optics, lat: lma_lattice, det: "_Detectors", nslices: int,
              flags: int = 0) -> int:
        r = lma_request()
        r.kind, r.specimen, r.nslices, r.flags = LMA_REQ_BUILD, int(specimen), int(nslices), int(flags)
        r.optics, r.lattice, r.detectors = C.pointer(opt), C.pointer(lat), C.pointer(det.s)
        return self._submit(r, (opt, lat, det))

    def _image_request(self, kind, specimen, potential, image, flags, weight):
        pp, fp = _ptr(potential, np.float32)
        pi, fi = _ptr(image, np.float64)
        if fp != fi:
            raise ValueError("potential and image must both be host or both be device")
        self._ready(potential, image)
        r = lma_request()
        r.kind, r.specimen, r.nslices = kind, int(specimen), int(potential.shape[0])
        r.potential, r.image, r.flags, r.weight = pp.value, pi.value, int(flags) | fi, float(weight)
        return self._submit(r, (potential, image))

    def image(self, specimen: int, potential, image, flags: int = 0, weight: float = 1.0) -> int:
        return self._image_request(LMA_REQ_IMAGE, specimen, potential, image, flags, weight)

    def plain(self, specimen: int, potential, image, flags: int = 0, weight: float = 1.0) -> int:
        return self._image_request(LMA_REQ_PLAIN, specimen, potential, image, flags, weight)

    def edit(self, specimen: int, potential: np.ndarray, bbox, radius: float, image: np.ndarray) -> int:
        pp, fp = _ptr(potential, np.float32)
        pi, fi = _ptr(image, np.float64)
        if fp or fi:
            raise ValueError("an edit takes a host potential and patches a host image")
        r = lma_request()
        r.kind, r.specimen, r.nslices = LMA_REQ_EDIT, int(specimen), int(potential.shape[0])
        r.potential, r.image, r.radius = pp.value, pi.value, float(radius)
        for i in range(4):
            r.bbox[i] = int(bbox[i])
        return self._submit(r, (potential, image))

    def release(self, specimen: int) -> int:
        r = lma_request()
        r.kind, r.specimen = LMA_REQ_RELEASE, int(specimen)
        return self._submit(r, ())

    def wait(self, ticket: int):
        """(latency_ms, service_ms) of a completed request; raises LmaError if it failed."""
        lat, svc = C.c_double(), C.c_double()
        try:
            _check(lib().lma_server_wait(self._h, int(ticket), C.byref(lat), C.byref(svc)))
        finally:
            self._keep.pop(int(ticket), None)
        return lat.value, svc.value

    def plan_info(self, specimen: int) -> lma_info:
        h = C.c_void_p()
        _check(lib().lma_server_plan(self._h, int(specimen), C.byref(h)))
        if not h.value:
            raise LmaError(_lib.LMA_ERR_STATE, f"specimen {specimen} is not resident")
        i = lma_info()
        _check(lib().lma_plan_info(h, C.byref(i)))
        return i

    def in_use(self) -> int:
        b = C.c_int64()
        _check(lib().lma_server_in_use(self._h, C.byref(b)))
        return b.value

    def close(self):
        if self._h:
            lib().lma_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
