"""Python binding of the MI355X SFFT image-differencing library.

Thin ctypes marshalling over the C ABI in include/sfft.h: the same entry
points (sfft_build_system, sfft_solve, sfft_subtract, ...) taking torch
device tensors for memory and the current HIP stream. Every step of the path
runs in the library's HIP kernels; there is no CPU fallback, and importing
the compute entry points fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfft_mi355x.so")

SFFT_OK = 0
SFFT_ERR_INVALID_ARG = 1
SFFT_ERR_UNSUPPORTED = 2
SFFT_ERR_WORKSPACE = 3
SFFT_ERR_NONFINITE = 4
SFFT_ERR_NOT_SPD = 5
SFFT_ERR_HIP = 6
SFFT_ERR_INTERNAL = 7

SFFT_F32, SFFT_F64 = 0, 1
SFFT_COMPUTE_FP64, SFFT_COMPUTE_FP32 = 0, 1


class SfftError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Desc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("ld", ctypes.c_int64),
        ("L", ctypes.c_int32),
        ("dk", ctypes.c_int32),
        ("db", ctypes.c_int32),
        ("image_dtype", ctypes.c_int32),
        ("compute", ctypes.c_int32),
        ("convention", ctypes.c_int32),
        ("ref_pedestal", ctypes.c_double),
        ("sci_pedestal", ctypes.c_double),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("failed_pivot", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("nonfinite", ctypes.c_int32),
        ("backward_err", ctypes.c_double),
        ("min_pivot", ctypes.c_double),
        ("max_pivot", ctypes.c_double),
    ]


SOLVE_INFO_BYTES = ctypes.sizeof(SolveInfo)


class BatchKnobs(ctypes.Structure):
    """sfft_batch_knobs: the batched form's launch configuration."""
    _fields_ = [("rows_per_block", ctypes.c_int32), ("radix_order", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("team", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("desc", Desc),
        ("ref", ctypes.c_void_p),
        ("sci", ctypes.c_void_p),
        ("diff", ctypes.c_void_p),
        ("G", ctypes.c_void_p),
        ("h", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
        ("info", ctypes.c_void_p),
        ("chi2", ctypes.c_void_p),
        ("ws", ctypes.c_void_p),
        ("ws_bytes", ctypes.c_size_t),
    ]

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "sfft_create": (ctypes.c_int, [ctypes.POINTER(_P)]),
    "sfft_destroy": (ctypes.c_int, [_P]),
    "sfft_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sfft_num_unknowns": (ctypes.c_int64, [ctypes.POINTER(Desc)]),
    "sfft_validate": (ctypes.c_int, [ctypes.POINTER(Desc)]),
    "sfft_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]),
    "sfft_build_system": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "sfft_build_system_masked": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, ctypes.c_int64, _P, _P, _P,
                                                ctypes.c_size_t, _P]),
    "sfft_solve": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, ctypes.c_int32, _P, _P,
                                  ctypes.c_size_t, _P]),
    "sfft_subtract": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "sfft_set_solve_team": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sfft_get_solve_team": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "sfft_set_radix_order": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sfft_get_radix_order": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "sfft_median_combine": (ctypes.c_int, [_P, ctypes.POINTER(Desc), ctypes.POINTER(_P), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_double), ctypes.c_double, _P, _P]),
    "sfft_difference_multi": (ctypes.c_int, [_P, ctypes.POINTER(Desc), ctypes.POINTER(_P), _P, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_double, ctypes.c_int32, _P, _P, _P, _P, _P,
                                             ctypes.POINTER(_P), _P, _P, ctypes.c_size_t, _P]),
    "sfft_aperture_flux": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, ctypes.c_int32, ctypes.c_double, _P,
                                          _P]),
    "sfft_limiting_magnitude": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "sfft_forced_photometry": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, ctypes.c_int32, ctypes.c_double,
                                              ctypes.c_double, _P, _P, _P, _P, _P]),
    "sfft_rb_num_params": (ctypes.c_int64, []),
    "sfft_rb_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "sfft_rb_extract": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, _P, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _P, _P]),
    "sfft_rb_score": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P]),
    "sfft_subtract_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, _P, _P, _P]),
    "sfft_refit_background": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                             _P]),
    "sfft_stamps_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(Desc), ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "sfft_build_system_stamps": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, ctypes.c_int32,
                                                ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P]),
    "sfft_profile_events": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "sfft_batch_create": (ctypes.c_int, [_P, ctypes.POINTER(BatchItem), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(_P)]),
    "sfft_batch_run": (ctypes.c_int, [_P, _P]),
    "sfft_batch_run_graph": (ctypes.c_int, [_P, _P]),
    "sfft_batch_tune": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "sfft_batch_plan": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "sfft_batch_set_knobs": (ctypes.c_int, [_P, ctypes.POINTER(BatchKnobs)]),
    "sfft_batch_get_knobs": (ctypes.c_int, [_P, ctypes.POINTER(BatchKnobs)]),
    "sfft_batch_set_pedestals": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                                ctypes.POINTER(ctypes.c_double)]),
    "sfft_batch_destroy": (ctypes.c_int, [_P]),
    "sfft_surrogate_num_params": (ctypes.c_int64, [ctypes.c_int32]),
    "sfft_surrogate_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.POINTER(ctypes.c_size_t)]),
    "sfft_extract_stamps": (ctypes.c_int, [_P, ctypes.POINTER(Desc), _P, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "sfft_surrogate_forward": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]),
    "sfft_surrogate_grad": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           _P, _P, _P, ctypes.c_size_t, _P]),
    "sfft_surrogate_adam": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                           ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "sfft_surrogate_destandardize": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
}

SFFT_NET_FP32, SFFT_NET_BF16 = 0, 1

# sfft_prof_slot
SFFT_PROF_ROW_PASS, SFFT_PROF_COL_PASS, SFFT_PROF_XINV, SFFT_PROF_SUBTRACT = 1, 2, 3, 4
SFFT_PROF_SOLVE, SFFT_PROF_BUILD, SFFT_PROF_STAMP_GRAM = 5, 6, 7

_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"SFFT HIP library not built ({LIB_PATH}); run __graft_entry__.build()")
        # torch ships its own HIP runtime: load it first so that this library
        # binds to the same runtime instance (one per process)
        import torch  # noqa: F401
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().sfft_status_string(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def _check(status: int, where: str):
    if status != SFFT_OK:
        raise SfftError(status, where)


SFFT_CONV_INPUT_PIXEL, SFFT_CONV_OUTPUT_PIXEL = 0, 1


def make_desc(width, height, L, dk, db, *, ld=None, image_dtype=SFFT_F32, compute=SFFT_COMPUTE_FP64,
              ref_pedestal=0.0, sci_pedestal=0.0, convention=SFFT_CONV_INPUT_PIXEL) -> Desc:
    return Desc(int(width), int(height), int(width if ld is None else ld), int(L), int(dk), int(db),
                int(image_dtype), int(compute), int(convention), float(ref_pedestal), float(sci_pedestal))


def sfft_num_unknowns(desc: Desc) -> int:
    return int(lib().sfft_num_unknowns(ctypes.byref(desc)))


def sfft_validate(desc: Desc) -> int:
    return int(lib().sfft_validate(ctypes.byref(desc)))


class Handle:
    """Owns an sfft_handle (plan tables) bound to the current device."""

    def __init__(self):
        h = _P()
        _check(lib().sfft_create(ctypes.byref(h)), "sfft_create")
        self._h = h

    @property
    def ptr(self):
        return self._h

    def close(self):
        """Release the handle's device tables now (idempotent)."""
        if self._h:
            lib().sfft_destroy(self._h)
            self._h = _P()

    def __del__(self, _finalizing=sys.is_finalizing):
        # During interpreter shutdown the HIP runtime and torch's allocator may
        # already be finalising: leave the tables to process exit rather than
        # call into HIP from a finaliser. Explicit close() is the normal path.
        # (The check is bound at definition: module globals such as `sys` may
        # already be cleared when a finaliser runs at shutdown.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return _P(s.cuda_stream)


def _dp(t):
    return None if t is None else _P(t.data_ptr())


def sfft_workspace_size(handle: Handle, desc: Desc) -> int:
    n = ctypes.c_size_t()
    _check(lib().sfft_workspace_size(handle.ptr, ctypes.byref(desc), ctypes.byref(n)), "sfft_workspace_size")
    return int(n.value)


def sfft_build_system(handle: Handle, desc: Desc, ref, sci, G, h, ws, stream=None):
    _check(lib().sfft_build_system(handle.ptr, ctypes.byref(desc), _dp(ref), _dp(sci), _dp(G), _dp(h),
                                   _dp(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_build_system")


def sfft_build_system_masked(handle: Handle, desc: Desc, ref, sci, mask, G, h, ws, stream=None):
    """mask: uint8 (H, W) device tensor, nonzero = the pixel enters the fit."""
    _check(lib().sfft_build_system_masked(handle.ptr, ctypes.byref(desc), _dp(ref), _dp(sci), _dp(mask),
                                          int(mask.stride(0)), _dp(G), _dp(h), _dp(ws),
                                          ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_build_system_masked")


def sfft_solve(handle: Handle, desc: Desc, G, h, coef, info, ws, max_refine=2, stream=None):
    _check(lib().sfft_solve(handle.ptr, ctypes.byref(desc), _dp(G), _dp(h), _dp(coef), int(max_refine),
                            _dp(info), _dp(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_solve")


def sfft_set_solve_team(handle: Handle, team: int):
    _check(lib().sfft_set_solve_team(handle.ptr, int(team)), "sfft_set_solve_team")


def sfft_get_solve_team(handle: Handle) -> int:
    t = ctypes.c_int32(0)
    _check(lib().sfft_get_solve_team(handle.ptr, ctypes.byref(t)), "sfft_get_solve_team")
    return int(t.value)


def sfft_set_radix_order(handle: Handle, order: int):
    _check(lib().sfft_set_radix_order(handle.ptr, int(order)), "sfft_set_radix_order")


def sfft_get_radix_order(handle: Handle) -> int:
    o = ctypes.c_int32(0)
    _check(lib().sfft_get_radix_order(handle.ptr, ctypes.byref(o)), "sfft_get_radix_order")
    return int(o.value)


def sfft_subtract(handle: Handle, desc: Desc, ref, sci, coef, diff, chi2, ws, stream=None):
    _check(lib().sfft_subtract(handle.ptr, ctypes.byref(desc), _dp(ref), _dp(sci), _dp(coef), _dp(diff),
                               _dp(chi2), _dp(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_subtract")


def sfft_subtract_noalloc(handle: Handle, desc: Desc, ref, sci, coef, diff, chi2, stream=None):
    _check(lib().sfft_subtract_noalloc(handle.ptr, ctypes.byref(desc), _dp(ref), _dp(sci), _dp(coef), _dp(diff),
                                       _dp(chi2), _stream_ptr(stream)),
           "sfft_subtract_noalloc")


def sfft_stamps_workspace_size(handle: Handle, desc: Desc, n_stamps: int, size: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().sfft_stamps_workspace_size(handle.ptr, ctypes.byref(desc), int(n_stamps), int(size),
                                            ctypes.byref(n)), "sfft_stamps_workspace_size")
    return int(n.value)


def sfft_build_system_stamps(handle: Handle, desc: Desc, ref, sci, centers, size, G, h, ws, stream=None):
    """centers: device int32 tensor (n, 2) of (x, y)."""
    _check(lib().sfft_build_system_stamps(handle.ptr, ctypes.byref(desc), _dp(ref), _dp(sci), _dp(centers),
                                          int(centers.shape[0]), int(size), _dp(G), _dp(h), _dp(ws),
                                          ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_build_system_stamps")


def sfft_profile_events(handle: Handle, slot: int, start_event, stop_event):
    """Bracket every launch of `slot` with the given hipEvent_t handles (ints or None)."""
    _check(lib().sfft_profile_events(handle.ptr, int(slot), _P(start_event), _P(stop_event)),
           "sfft_profile_events")


def read_info(info_tensor) -> SolveInfo:
    """Copy a device sfft_solve_info (uint8 tensor) to the host."""
    raw = bytes(info_tensor.cpu().numpy().tobytes())
    return SolveInfo.from_buffer_copy(raw[:SOLVE_INFO_BYTES])


@dataclass
class Buffers:
    G: object
    h: object
    coef: object
    info: object
    diff: object
    chi2: object
    ws: object


class Differencer:
    """Reusable device buffers + handle for one image shape and fit."""

    def __init__(self, width, height, L, dk, db, *, image_dtype="float32", compute="fp64",
                 ref_pedestal=0.0, sci_pedestal=0.0, device="cuda", stamps=None, convention="input",
                 solve_team=0, radix_order=0):
        import torch
        self.torch = torch
        self.dtype = torch.float32 if image_dtype in ("float32", torch.float32) else torch.float64
        self.desc = make_desc(width, height, L, dk, db,
                              image_dtype=SFFT_F32 if self.dtype == torch.float32 else SFFT_F64,
                              compute=SFFT_COMPUTE_FP32 if compute == "fp32" else SFFT_COMPUTE_FP64,
                              ref_pedestal=ref_pedestal, sci_pedestal=sci_pedestal,
                              convention=SFFT_CONV_OUTPUT_PIXEL if convention == "output" else SFFT_CONV_INPUT_PIXEL)
        self.handle = Handle()
        if solve_team:
            sfft_set_solve_team(self.handle, solve_team)
        if radix_order:
            sfft_set_radix_order(self.handle, radix_order)
        self.N = sfft_num_unknowns(self.desc)
        # stamps = (n_stamps, size): size the workspace for the stamp build as well
        self.stamps = stamps
        if stamps is None:
            st = sfft_validate(self.desc)
            if st != SFFT_OK:
                raise SfftError(st, "sfft_validate")
            nbytes = sfft_workspace_size(self.handle, self.desc)
        else:
            nbytes = sfft_stamps_workspace_size(self.handle, self.desc, stamps[0], stamps[1])
            if sfft_validate(self.desc) == SFFT_OK:
                nbytes = max(nbytes, sfft_workspace_size(self.handle, self.desc))
        dev = torch.device(device)
        N = self.N
        self.buf = Buffers(
            G=torch.empty((N, N), dtype=torch.float64, device=dev),
            h=torch.empty((N,), dtype=torch.float64, device=dev),
            coef=torch.empty((N,), dtype=torch.float64, device=dev),
            info=torch.zeros((64,), dtype=torch.uint8, device=dev),
            diff=torch.empty((height, width), dtype=self.dtype, device=dev),
            chi2=torch.zeros((1,), dtype=torch.float64, device=dev),
            ws=torch.empty((nbytes + 255) // 256 * 256, dtype=torch.uint8, device=dev),
        )

    def set_pedestals(self, ref_pedestal, sci_pedestal):
        self.desc.ref_pedestal = float(ref_pedestal)
        self.desc.sci_pedestal = float(sci_pedestal)

    def build(self, ref, sci, stream=None, mask=None):
        """Normal equations (mask: optional uint8 device image, the masked fit)."""
        b = self.buf
        if mask is None:
            sfft_build_system(self.handle, self.desc, ref, sci, b.G, b.h, b.ws, stream)
        else:
            sfft_build_system_masked(self.handle, self.desc, ref, sci, mask, b.G, b.h, b.ws, stream)

    def refit_background(self, ref, sci, coef=None, stream=None):
        """Overwrite the background part of coef with the least-squares
        background for its kernel part (sfft_refit_background)."""
        b = self.buf
        c = b.coef if coef is None else coef
        _check(lib().sfft_refit_background(self.handle.ptr, ctypes.byref(self.desc), _dp(ref), _dp(sci), _dp(c),
                                           _dp(b.G), _dp(b.h), _dp(b.ws), b.ws.numel() * b.ws.element_size(),
                                           _stream_ptr(stream)),
               "sfft_refit_background")

    def build_stamps(self, ref, sci, centers, size, stream=None):
        b = self.buf
        sfft_build_system_stamps(self.handle, self.desc, ref, sci, centers, size, b.G, b.h, b.ws, stream)

    def solve(self, max_refine=2, stream=None):
        b = self.buf
        sfft_solve(self.handle, self.desc, b.G, b.h, b.coef, b.info, b.ws, max_refine, stream)

    def subtract(self, ref, sci, coef=None, chi2=True, stream=None):
        b = self.buf
        sfft_subtract(self.handle, self.desc, ref, sci, b.coef if coef is None else coef, b.diff,
                      b.chi2 if chi2 else None, b.ws, stream)

    def run(self, ref, sci, max_refine=2, stream=None, mask=None):
        """build + solve + subtract (+ chi2) on the stream; asynchronous."""
        self.build(ref, sci, stream, mask)
        self.solve(max_refine, stream)
        self.subtract(ref, sci, stream=stream)
        return self.buf

    def info(self) -> SolveInfo:
        return read_info(self.buf.info)

    def close(self):
        """Release the handle now; the torch buffers go with the object."""
        self.handle.close()


class PairPipeline:
    """Several CCD pairs in flight on one GPU: `depth` slots, each a
    Differencer (its own handle, workspace and result buffers) with its own
    HIP stream; pair k goes to slot k % depth. A slot's work is ordered on its
    stream, so pair k + depth overwrites the results of pair k in that slot:
    read or copy them first (wait(slot) or the slot's stream).

    The solve of one pair is a persistent kernel bound by its diagonal
    Cholesky chain; with a smaller team (`solve_team` workgroups) it leaves
    CUs to the builds and subtracts of the other pairs in flight. Each pair's
    results equal those of a single Differencer with the same solve_team."""

    def __init__(self, width, height, L, dk, db, *, depth=3, solve_team=32, **kw):
        import torch
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.torch = torch
        self.depth = depth
        self.slots = [Differencer(width, height, L, dk, db, solve_team=solve_team, **kw) for _ in range(depth)]
        self.streams = [torch.cuda.Stream() for _ in range(depth)]
        self.count = 0

    def submit(self, ref, sci, max_refine=2, mask=None, pedestals=None) -> int:
        """Queue build + solve + subtract of one pair (pedestals: optional
        (ref, sci) pedestals of this pair); returns its slot. The slot's
        stream first waits for the caller's current stream (where the inputs
        were produced)."""
        torch = self.torch
        k = self.count % self.depth
        self.count += 1
        if pedestals is not None:
            self.slots[k].set_pedestals(*pedestals)
        s = self.streams[k]
        s.wait_stream(torch.cuda.current_stream())
        for t in (ref, sci) + (() if mask is None else (mask,)):
            t.record_stream(s)
        self.slots[k].run(ref, sci, max_refine=max_refine, stream=s, mask=mask)
        return k

    def wait(self, slot=None):
        """Block until the slot's queued work (or every slot's) is done."""
        for k in (range(self.depth) if slot is None else (slot,)):
            self.streams[k].synchronize()

    def buffers(self, slot) -> Buffers:
        return self.slots[slot].buf

    def info(self, slot) -> SolveInfo:
        return self.slots[slot].info()

    def close(self):
        for d in self.slots:
            d.close()


# ---------------------------------------------------------------------------
# multi-template differencing and aperture photometry
# ---------------------------------------------------------------------------

MAX_TEMPLATES = 16


def _ptr_array(ts):
    return (_P * len(ts))(*[_P(t.data_ptr()) for t in ts])


def _dbl_array(v):
    v = [float(x) for x in v]
    return (ctypes.c_double * len(v))(*v)


def image_desc(img) -> Desc:
    """Descriptor of a 2-D torch image for the photometry and combine calls
    (only width, height, pitch and element type are used)."""
    import torch
    H, W = img.shape
    dt = SFFT_F32 if img.dtype == torch.float32 else SFFT_F64
    return make_desc(W, H, 1, 0, 0, ld=img.stride(0), image_dtype=dt)


def sfft_median_combine(handle: Handle, desc: Desc, diffs, zps, zp_common, out, stream=None):
    _check(lib().sfft_median_combine(handle.ptr, ctypes.byref(desc), _ptr_array(diffs), len(diffs),
                                     _dbl_array(zps), float(zp_common), _dp(out), _stream_ptr(stream)),
           "sfft_median_combine")


def sfft_difference_multi(handle: Handle, desc: Desc, refs, sci, zps, zp_common, G, h, coefs, infos, chi2s,
                          diffs, combined, ws, max_refine=2, ref_pedestals=None, stream=None):
    peds = None if ref_pedestals is None else _dbl_array(ref_pedestals)
    _check(lib().sfft_difference_multi(handle.ptr, ctypes.byref(desc), _ptr_array(refs), _dp(sci), len(refs), peds,
                                       _dbl_array(zps), float(zp_common), int(max_refine), _dp(G), _dp(h),
                                       _dp(coefs), _dp(infos), _dp(chi2s), _ptr_array(diffs), _dp(combined),
                                       _dp(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_difference_multi")


def sfft_aperture_flux(handle: Handle, desc: Desc, image, xy, radius, flux, stream=None):
    _check(lib().sfft_aperture_flux(handle.ptr, ctypes.byref(desc), _dp(image), _dp(xy), int(xy.shape[0]),
                                    float(radius), _dp(flux), _stream_ptr(stream)), "sfft_aperture_flux")


def sfft_limiting_magnitude(handle: Handle, desc: Desc, image, xy, radius, zp, flux, result, nsigma=5.0,
                            stream=None):
    _check(lib().sfft_limiting_magnitude(handle.ptr, ctypes.byref(desc), _dp(image), _dp(xy), int(xy.shape[0]),
                                         float(radius), float(zp), float(nsigma), _dp(flux), _dp(result),
                                         _stream_ptr(stream)), "sfft_limiting_magnitude")


def sfft_forced_photometry(handle: Handle, desc: Desc, image, xy, radius, zp, sigma, flux, mag=None, mag_err=None,
                           stream=None):
    _check(lib().sfft_forced_photometry(handle.ptr, ctypes.byref(desc), _dp(image), _dp(xy), int(xy.shape[0]),
                                        float(radius), float(zp), _dp(sigma), _dp(flux), _dp(mag), _dp(mag_err),
                                        _stream_ptr(stream)), "sfft_forced_photometry")


def sfft_rb_num_params() -> int:
    return int(lib().sfft_rb_num_params())


def sfft_rb_workspace_size(n: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().sfft_rb_workspace_size(int(n), ctypes.byref(b)), "sfft_rb_workspace_size")
    return int(b.value)


def _flt3(v):
    return (ctypes.c_float * 3)(*[float(x) for x in v])


def sfft_rb_extract(handle: Handle, desc: Desc, sci, ref, diff, centers, offsets, scales, stamps, stream=None):
    _check(lib().sfft_rb_extract(handle.ptr, ctypes.byref(desc), _dp(sci), _dp(ref), _dp(diff), _dp(centers),
                                 int(centers.shape[0]), _flt3(offsets), _flt3(scales), _dp(stamps),
                                 _stream_ptr(stream)), "sfft_rb_extract")


def sfft_rb_score(handle: Handle, params, stamps, logits, probs, ws, stream=None):
    _check(lib().sfft_rb_score(handle.ptr, _dp(params), _dp(stamps), int(stamps.shape[0]), _dp(logits), _dp(probs),
                               _dp(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)), "sfft_rb_score")


class MultiDifferencer:
    """One science image against n templates (sfft_difference_multi): every
    difference image, its coefficients, solve info and chi2, and the
    zero-point-normalised median combine, in caller-owned torch buffers."""

    def __init__(self, width, height, L, dk, db, n_templates, *, image_dtype="float32", compute="fp64",
                 sci_pedestal=0.0, device="cuda", solve_team=0):
        import torch
        self.torch = torch
        self.dtype = torch.float32 if image_dtype in ("float32", torch.float32) else torch.float64
        self.desc = make_desc(width, height, L, dk, db,
                              image_dtype=SFFT_F32 if self.dtype == torch.float32 else SFFT_F64,
                              compute=SFFT_COMPUTE_FP32 if compute == "fp32" else SFFT_COMPUTE_FP64,
                              sci_pedestal=sci_pedestal)
        st = sfft_validate(self.desc)
        if st != SFFT_OK:
            raise SfftError(st, "sfft_validate")
        self.handle = Handle()
        if solve_team:
            sfft_set_solve_team(self.handle, solve_team)
        self.n = int(n_templates)
        self.N = N = sfft_num_unknowns(self.desc)
        dev = torch.device(device)
        nbytes = sfft_workspace_size(self.handle, self.desc)
        self.G = torch.empty((N, N), dtype=torch.float64, device=dev)
        self.h = torch.empty((N,), dtype=torch.float64, device=dev)
        self.coefs = torch.empty((self.n, N), dtype=torch.float64, device=dev)
        self.infos = torch.zeros((self.n, SOLVE_INFO_BYTES), dtype=torch.uint8, device=dev)
        self.chi2s = torch.zeros((self.n,), dtype=torch.float64, device=dev)
        self.diffs = [torch.empty((height, width), dtype=self.dtype, device=dev) for _ in range(self.n)]
        self.combined = torch.empty((height, width), dtype=self.dtype, device=dev)
        self.ws = torch.empty((nbytes + 255) // 256 * 256, dtype=torch.uint8, device=dev)

    def run(self, refs, sci, zps, zp_common, max_refine=2, ref_pedestals=None, stream=None):
        assert len(refs) == self.n
        sfft_difference_multi(self.handle, self.desc, refs, sci, zps, zp_common, self.G, self.h, self.coefs,
                              self.infos, self.chi2s, self.diffs, self.combined, self.ws, max_refine,
                              ref_pedestals, stream)
        return self.combined

    def info(self, t) -> SolveInfo:
        return read_info(self.infos[t])

    def close(self):
        self.handle.close()


# ---------------------------------------------------------------------------
# learned form
# ---------------------------------------------------------------------------


def sfft_surrogate_num_params(n_out: int) -> int:
    return int(lib().sfft_surrogate_num_params(int(n_out)))


def sfft_surrogate_workspace_size(n_pairs: int, n_stamps: int, n_out: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().sfft_surrogate_workspace_size(int(n_pairs), int(n_stamps), int(n_out), ctypes.byref(n)),
           "sfft_surrogate_workspace_size")
    return int(n.value)


def sfft_extract_stamps(handle: Handle, desc: Desc, ref, sci, centers, stamps, pos, stream=None):
    _check(lib().sfft_extract_stamps(handle.ptr, ctypes.byref(desc), _dp(ref), _dp(sci), _dp(centers),
                                     int(centers.shape[0]), _dp(stamps), _dp(pos), _stream_ptr(stream)),
           "sfft_extract_stamps")


def sfft_surrogate_forward(handle: Handle, params, stamps, pos, n_pairs, n_stamps, n_out, precision, pred, ws,
                           stream=None):
    _check(lib().sfft_surrogate_forward(handle.ptr, _dp(params), _dp(stamps), _dp(pos), int(n_pairs),
                                        int(n_stamps), int(n_out), int(precision), _dp(pred), _dp(ws),
                                        ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_surrogate_forward")


def sfft_surrogate_grad(handle: Handle, params, stamps, pos, target, n_pairs, n_stamps, n_out, grads, loss, ws,
                        stream=None):
    _check(lib().sfft_surrogate_grad(handle.ptr, _dp(params), _dp(stamps), _dp(pos), _dp(target), int(n_pairs),
                                     int(n_stamps), int(n_out), _dp(grads), _dp(loss), _dp(ws),
                                     ws.numel() * ws.element_size(), _stream_ptr(stream)),
           "sfft_surrogate_grad")


def sfft_surrogate_adam(handle: Handle, params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                        stream=None):
    _check(lib().sfft_surrogate_adam(handle.ptr, _dp(params), _dp(grads), _dp(m), _dp(v), int(params.numel()),
                                     int(step), float(lr), float(beta1), float(beta2), float(eps),
                                     _stream_ptr(stream)),
           "sfft_surrogate_adam")


def sfft_surrogate_destandardize(handle: Handle, pred, mean, scale, n_pairs, n_out, coef, stream=None):
    _check(lib().sfft_surrogate_destandardize(handle.ptr, _dp(pred), _dp(mean), _dp(scale), int(n_pairs),
                                              int(n_out), _dp(coef), _stream_ptr(stream)),
           "sfft_surrogate_destandardize")


class Surrogate:
    """Device state of the learned form: parameters, Adam moments and a
    workspace sized for batches of up to `max_pairs` pairs of `n_stamps` stamps."""

    def __init__(self, params, n_out, n_stamps=64, max_pairs=32, handle=None, device="cuda"):
        import torch
        self.torch = torch
        self.handle = handle or Handle()
        self.n_out, self.n_stamps, self.max_pairs = int(n_out), int(n_stamps), int(max_pairs)
        n = sfft_surrogate_num_params(self.n_out)
        p = torch.as_tensor(params, dtype=torch.float32)
        assert p.numel() == n, (p.numel(), n)
        dev = torch.device(device)
        self.params = p.to(dev).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.loss = torch.zeros((1,), dtype=torch.float64, device=dev)
        self.step = 0
        nb = sfft_surrogate_workspace_size(self.max_pairs, self.n_stamps, self.n_out)
        self.ws = torch.empty((nb + 255) // 256 * 256, dtype=torch.uint8, device=dev)

    def forward(self, stamps, pos, n_pairs, precision=SFFT_NET_FP32, out=None, stream=None):
        out = out if out is not None else self.torch.empty((n_pairs, self.n_out), dtype=self.torch.float32,
                                                             device=self.params.device)
        sfft_surrogate_forward(self.handle, self.params, stamps, pos, n_pairs, self.n_stamps, self.n_out,
                               precision, out, self.ws, stream)
        return out

    def grad(self, stamps, pos, target, n_pairs, stream=None):
        sfft_surrogate_grad(self.handle, self.params, stamps, pos, target, n_pairs, self.n_stamps, self.n_out,
                            self.grads, self.loss, self.ws, stream)
        return self.grads, self.loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        sfft_surrogate_adam(self.handle, self.params, self.grads, self.m, self.v, self.step, lr, beta1, beta2,
                            eps, stream)

    def train_step(self, stamps, pos, target, n_pairs, lr, stream=None):
        self.grad(stamps, pos, target, n_pairs, stream)
        self.adam(lr, stream=stream)
        return self.loss


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------


class Batch:
    """Device buffers and an sfft_batch for a list of pair shapes.

    shapes: list of (width, height, L); dk, db common; FP32 images and
    FP32 spectra (the batched form's precision)."""

    def __init__(self, shapes, dk=2, db=2, max_refine=1, handle=None, device="cuda"):
        import torch
        self.torch = torch
        self._own_handle = handle is None
        self.handle = handle or Handle()
        dev = torch.device(device)
        self.items = []
        self.peds = [(0.0, 0.0)] * len(shapes)
        self._peds_dirty = False
        self.bufs = []
        arr = (BatchItem * len(shapes))()
        for k, (W, H, L) in enumerate(shapes):
            desc = make_desc(W, H, L, dk, db, image_dtype=SFFT_F32, compute=SFFT_COMPUTE_FP32)
            N = sfft_num_unknowns(desc)
            nb = sfft_workspace_size(self.handle, desc)
            b = Buffers(G=torch.empty((N, N), dtype=torch.float64, device=dev),
                        h=torch.empty((N,), dtype=torch.float64, device=dev),
                        coef=torch.empty((N,), dtype=torch.float64, device=dev),
                        info=torch.zeros((64,), dtype=torch.uint8, device=dev),
                        diff=torch.empty((H, W), dtype=torch.float32, device=dev),
                        chi2=torch.zeros((1,), dtype=torch.float64, device=dev),
                        ws=torch.empty((nb + 255) // 256 * 256, dtype=torch.uint8, device=dev))
            b.ref = torch.zeros((H, W), dtype=torch.float32, device=dev)
            b.sci = torch.zeros((H, W), dtype=torch.float32, device=dev)
            b.desc = desc
            self.bufs.append(b)
            it = arr[k]
            it.desc = desc
            it.ref, it.sci, it.diff = b.ref.data_ptr(), b.sci.data_ptr(), b.diff.data_ptr()
            it.G, it.h, it.coef = b.G.data_ptr(), b.h.data_ptr(), b.coef.data_ptr()
            it.info, it.chi2 = b.info.data_ptr(), b.chi2.data_ptr()
            it.ws, it.ws_bytes = b.ws.data_ptr(), b.ws.numel()
        self._arr = arr
        ptr = _P()
        _check(lib().sfft_batch_create(self.handle.ptr, arr, len(shapes), int(max_refine), ctypes.byref(ptr)),
               "sfft_batch_create")
        self._b = ptr

    def load(self, k, ref, sci, pedestals=True):
        """Copy pair k's images into the batch's resident input buffers. With
        pedestals, the item's pedestals become the FP64 means of its two
        images (the precision form's reading; applied before the next run)."""
        self.bufs[k].ref.copy_(ref)
        self.bufs[k].sci.copy_(sci)
        if pedestals:
            import math
            t = self.torch
            pr = float(self.bufs[k].ref.to(t.float64).mean())
            ps = float(self.bufs[k].sci.to(t.float64).mean())
            # a non-finite pixel makes the mean non-finite: keep 0 and let the
            # build flag the pixel (the item then reports SFFT_ERR_NONFINITE)
            self.peds[k] = (pr if math.isfinite(pr) else 0.0, ps if math.isfinite(ps) else 0.0)
            self._peds_dirty = True

    def set_pedestals(self, peds):
        """peds: one (ref, sci) pair per item (sfft_batch_set_pedestals)."""
        self.peds = [(float(a), float(b)) for a, b in peds]
        n = len(self.peds)
        ra = (ctypes.c_double * n)(*[p[0] for p in self.peds])
        sa = (ctypes.c_double * n)(*[p[1] for p in self.peds])
        _check(lib().sfft_batch_set_pedestals(self._b, ra, sa), "sfft_batch_set_pedestals")
        for b, (pr, ps) in zip(self.bufs, self.peds):
            b.desc.ref_pedestal, b.desc.sci_pedestal = pr, ps
        self._peds_dirty = False

    def _sync(self):
        if self._peds_dirty:
            self.set_pedestals(self.peds)

    def run(self, stream=None):
        self._sync()
        _check(lib().sfft_batch_run(self._b, _stream_ptr(stream)), "sfft_batch_run")

    def run_graph(self, stream=None):
        self._sync()
        _check(lib().sfft_batch_run_graph(self._b, _stream_ptr(stream)), "sfft_batch_run_graph")

    def tune(self, stream=None):
        self._sync()
        rpb, team = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().sfft_batch_tune(self._b, _stream_ptr(stream), ctypes.byref(rpb), ctypes.byref(team)),
               "sfft_batch_tune")
        return int(rpb.value), int(team.value)

    def plan(self, rows_per_block, team):
        """Fixed rows per workgroup and solve team (team 0: one solve team per
        item); the other knobs keep their values."""
        _check(lib().sfft_batch_plan(self._b, int(rows_per_block), int(team)), "sfft_batch_plan")

    def knobs(self) -> dict:
        """The whole launch configuration in use (team resolved)."""
        k = BatchKnobs()
        _check(lib().sfft_batch_get_knobs(self._b, ctypes.byref(k)), "sfft_batch_get_knobs")
        return k.as_dict()

    def set_knobs(self, rows_per_block=4, radix_order=0, tile_rows=32, team=0):
        self._sync()
        k = BatchKnobs(int(rows_per_block), int(radix_order), int(tile_rows), int(team))
        _check(lib().sfft_batch_set_knobs(self._b, ctypes.byref(k)), "sfft_batch_set_knobs")

    def info(self, k) -> SolveInfo:
        return read_info(self.bufs[k].info)

    def close(self):
        """Destroy the batch (tables, captured graph) and its handle if owned."""
        if getattr(self, "_b", None):
            lib().sfft_batch_destroy(self._b)
            self._b = None
        if getattr(self, "_own_handle", False):
            self.handle.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
