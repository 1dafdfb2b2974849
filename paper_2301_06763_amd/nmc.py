"""Thin ctypes binding of libnmc (argument marshalling only).

Every step of the nested solve runs in the HIP library; PyTorch supplies
device memory and the current stream.  There is no fallback: if libnmc.so is
missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# NMC_LIBRARY may point at another build of the same library (A/B timing).
LIB_PATH = os.environ.get("NMC_LIBRARY") or os.path.join(HERE, "libnmc.so")

NMC_F64, NMC_F32 = 0, 1
NMC_OK, NMC_EINVAL, NMC_ENOMEM, NMC_EDEVICE, NMC_EUNSUPPORTED, NMC_EAGAIN = 0, -1, -2, -3, -4, -5
NMC_NO_RESTRICT = 1 << 0
NMC_PROLONG_TRILINEAR = 1 << 1
NMC_F32_UNCOMPENSATED = 1 << 2
NMC_NO_GRAPH = 1 << 3
NMC_ONE_STREAM = 1 << 4
NMC_NO_FUSED_PLANES = 1 << 5
NMC_MODIFIED = 1 << 6  # the dipole-preserving method of Sect. 7 / Appendix B
NMC_MODIFIED3 = 1 << 7  # ... with Appendix B's three-level scheme
NMC_SCRATCH_BYTES = 64 << 20  # largest workspace of solve_noalloc

_CODES = {NMC_EINVAL: "EINVAL", NMC_ENOMEM: "ENOMEM", NMC_EDEVICE: "EDEVICE",
          NMC_EUNSUPPORTED: "EUNSUPPORTED", NMC_EAGAIN: "EAGAIN"}


class NmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nmc {_CODES.get(code, code)}: {msg}")
        self.code = code


class Request(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("N", ctypes.c_int),
                ("L", ctypes.c_int), ("h0", ctypes.c_double), ("G", ctypes.c_double),
                ("p", ctypes.c_int), ("flags", ctypes.c_uint)]


class PassStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


NUM_PASSES = 13


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("inflight", ctypes.c_uint64),
                ("inflight_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t),
                ("peak_inflight_bytes", ctypes.c_size_t), ("green_cache_bytes", ctypes.c_size_t),
                ("arena_bytes", ctypes.c_size_t)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnmc.so (built in-tree by paper_2301_06763_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2301_06763_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, u, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_size_t
    sig = {
        "nmc_create": (i, [ctypes.POINTER(vp), i, sz]),
        "nmc_destroy": (None, [vp]),
        "nmc_last_error": (ctypes.c_char_p, [vp]),
        "nmc_footprint_bytes": (i, [i, i, i, ctypes.POINTER(sz)]),
        "nmc_footprint_bytes_flags": (i, [i, i, i, ctypes.c_uint, ctypes.POINTER(sz)]),
        "nmc_solve": (i, [vp, vp, vp, i, i, d, i, d, i, u, vp]),
        "nmc_solve_noalloc": (i, [vp, vp, vp, i, i, d, i, d, i, u, vp]),
        "nmc_solve_batch": (i, [vp, ctypes.POINTER(Request), i, vp]),
        "nmc_serve_submit": (i, [vp, ctypes.POINTER(Request), vp, ctypes.POINTER(ctypes.c_uint64)]),
        "nmc_serve_tick": (i, [vp, ctypes.POINTER(i)]),
        "nmc_serve_poll": (i, [vp, ctypes.c_uint64, ctypes.POINTER(i)]),
        "nmc_serve_stats_get": (i, [vp, ctypes.POINTER(ServeStats)]),
        "nmc_serve_drain": (i, [vp]),
        "nmc_serve_take_completed": (i, [vp, ctypes.POINTER(ctypes.c_uint64), i, ctypes.POINTER(i)]),
        "nmc_acceleration": (i, [vp, vp, vp, i, i, d, i, vp]),
        "nmc_green_spectrum": (i, [vp, i, i, vp, vp]),
        "nmc_period": (i, [i]),
        "nmc_fft_lines": (i, [vp, vp, vp, i, i, i, i, vp]),
        "nmc_profile_enable": (i, [vp, i]),
        "nmc_profile_read": (i, [vp, ctypes.POINTER(PassStat)]),
        "nmc_pass_name": (ctypes.c_char_p, [i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def period(N: int) -> int:
    return lib().nmc_period(N)


def precision_of(dtype: torch.dtype) -> int:
    if dtype == torch.float64:
        return NMC_F64
    if dtype == torch.float32:
        return NMC_F32
    raise TypeError(f"unsupported dtype {dtype} (float64 or float32)")


def footprint_bytes(N: int, L: int, dtype=torch.float64, flags: int = 0) -> int:
    out = ctypes.c_size_t()
    rc = lib().nmc_footprint_bytes_flags(N, L, precision_of(dtype), flags, ctypes.byref(out))
    if rc:
        raise NmcError(rc, f"footprint of N={N} L={L} flags={flags}")
    return out.value


def _stream_ptr(stream, device) -> int:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return s.cuda_stream


def _check_levels(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 4 or t.shape[1] != t.shape[2] or t.shape[2] != t.shape[3]:
        raise ValueError(f"{name} must have shape [L, N, N, N]")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class Ticket:
    id: int
    rho: torch.Tensor
    phi: torch.Tensor


class Context:
    """An libnmc context on one device: Green-spectrum cache, workspace pool,
    serving queue."""

    def __init__(self, device=None, budget_bytes: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libnmc needs a HIP GPU; none is available")
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           torch.device(device).index or 0)
        self.device = dev
        h = ctypes.c_void_p()
        rc = lib().nmc_create(ctypes.byref(h), dev.index, budget_bytes)
        if rc:
            raise NmcError(rc, "nmc_create failed")
        self._h = h
        self._tickets: dict[int, Ticket] = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().nmc_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc, what):
        msg = lib().nmc_last_error(self._h).decode()
        raise NmcError(rc, f"{what}: {msg}")

    # -- solve ---------------------------------------------------------------
    def solve(self, rho: torch.Tensor, h0: float, G: float = 1.0, flags: int = 0,
              out: torch.Tensor | None = None, stream=None, refine: int = 2) -> torch.Tensor:
        """Potential on every level of a nested mesh; rho [L, N, N, N] on the device."""
        _check_levels(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        _check_levels(out, "out")
        L, N = rho.shape[0], rho.shape[1]
        rc = lib().nmc_solve(self._h, rho.data_ptr(), out.data_ptr(), N, L, float(h0), refine,
                             float(G), precision_of(rho.dtype), flags, _stream_ptr(stream, self.device))
        if rc:
            self._err(rc, "nmc_solve")
        return out

    def solve_noalloc(self, rho: torch.Tensor, h0: float, G: float = 1.0, flags: int = 0,
                      out: torch.Tensor | None = None, stream=None, refine: int = 2) -> torch.Tensor:
        """nmc_solve_noalloc: the solve on the library's static per-device
        scratch, without any device allocation by the library (the Green
        tables of this N must be resident; `out` is the caller's)."""
        _check_levels(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        _check_levels(out, "out")
        L, N = rho.shape[0], rho.shape[1]
        rc = lib().nmc_solve_noalloc(self._h, rho.data_ptr(), out.data_ptr(), N, L, float(h0), refine,
                                     float(G), precision_of(rho.dtype), flags, _stream_ptr(stream, self.device))
        if rc:
            self._err(rc, "nmc_solve_noalloc")
        return out

    def acceleration(self, phi: torch.Tensor, h0: float, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
        """g = -grad Phi on every level of a solved potential phi [L, N, N, N];
        returns [L, 3, N, N, N] (components x, y, z)."""
        _check_levels(phi, "phi")
        L, N = phi.shape[0], phi.shape[1]
        if out is None:
            out = torch.empty((L, 3, N, N, N), dtype=phi.dtype, device=phi.device)
        if out.shape != (L, 3, N, N, N) or out.dtype != phi.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous [L, 3, N, N, N] tensor of phi's dtype")
        rc = lib().nmc_acceleration(self._h, phi.data_ptr(), out.data_ptr(), N, L, float(h0),
                                    precision_of(phi.dtype), _stream_ptr(stream, self.device))
        if rc:
            self._err(rc, "nmc_acceleration")
        return out

    def _request(self, rho, h0, G, flags, out) -> Request:
        _check_levels(rho, "rho")
        _check_levels(out, "out")
        if out.dtype != rho.dtype or out.shape != rho.shape:
            raise ValueError("out must match rho in shape and dtype")
        return Request(rho.data_ptr(), out.data_ptr(), rho.shape[1], rho.shape[0], float(h0),
                       float(G), precision_of(rho.dtype), flags)

    def solve_batch(self, items, stream=None) -> list:
        """items: iterable of (rho, h0[, G[, flags]]).  Returns the potentials."""
        outs, reqs = [], []
        for it in items:
            rho, h0 = it[0], it[1]
            G = it[2] if len(it) > 2 else 1.0
            flags = it[3] if len(it) > 3 else 0
            out = torch.empty_like(rho)
            reqs.append(self._request(rho, h0, G, flags, out))
            outs.append(out)
        arr = (Request * len(reqs))(*reqs)
        rc = lib().nmc_solve_batch(self._h, arr, len(reqs), _stream_ptr(stream, self.device))
        if rc:
            self._err(rc, "nmc_solve_batch")
        return outs

    # -- serving ---------------------------------------------------------------
    def submit(self, rho: torch.Tensor, h0: float, G: float = 1.0, flags: int = 0,
               out: torch.Tensor | None = None, stream=None) -> Ticket:
        """Queue a request for the serving loop; the solve is ordered after the
        work enqueued so far on `stream` (default: the current stream)."""
        if out is None:
            out = torch.empty_like(rho)
        req = self._request(rho, h0, G, flags, out)
        t = ctypes.c_uint64()
        rc = lib().nmc_serve_submit(self._h, ctypes.byref(req), _stream_ptr(stream, self.device),
                                    ctypes.byref(t))
        if rc:
            self._err(rc, "nmc_serve_submit")
        tk = Ticket(t.value, rho, out)
        self._tickets[t.value] = tk
        return tk

    def tick(self) -> int:
        n = ctypes.c_int()
        rc = lib().nmc_serve_tick(self._h, ctypes.byref(n))
        if rc:
            self._err(rc, "nmc_serve_tick")
        return n.value

    def poll(self, ticket: Ticket | int) -> bool:
        tid = ticket.id if isinstance(ticket, Ticket) else ticket
        d = ctypes.c_int()
        rc = lib().nmc_serve_poll(self._h, tid, ctypes.byref(d))
        if rc:
            self._err(rc, "nmc_serve_poll")
        if d.value:
            self._tickets.pop(tid, None)
        return bool(d.value)

    def take_completed(self, cap: int = 4096) -> list:
        """Ticket ids completed since the last call (the context forgets them)."""
        buf = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int()
        rc = lib().nmc_serve_take_completed(self._h, buf, cap, ctypes.byref(n))
        if rc:
            self._err(rc, "nmc_serve_take_completed")
        done = [buf[k] for k in range(n.value)]
        for t in done:
            self._tickets.pop(t, None)
        return done

    def drain(self):
        rc = lib().nmc_serve_drain(self._h)
        if rc:
            self._err(rc, "nmc_serve_drain")
        self._tickets.clear()

    def stats(self) -> dict:
        s = ServeStats()
        rc = lib().nmc_serve_stats_get(self._h, ctypes.byref(s))
        if rc:
            self._err(rc, "nmc_serve_stats_get")
        return {k: getattr(s, k) for k, _ in ServeStats._fields_}

    # -- profiling -------------------------------------------------------------
    def profile(self, on: bool = True):
        rc = lib().nmc_profile_enable(self._h, 1 if on else 0)
        if rc:
            self._err(rc, "nmc_profile_enable")

    def profile_read(self) -> dict:
        """{pass name: {launches, total_ms, bytes}} since the last enable/read."""
        arr = (PassStat * NUM_PASSES)()
        rc = lib().nmc_profile_read(self._h, arr)
        if rc:
            self._err(rc, "nmc_profile_read")
        return {lib().nmc_pass_name(k).decode(): dict(launches=arr[k].launches, total_ms=arr[k].total_ms,
                                                       bytes=arr[k].bytes) for k in range(NUM_PASSES)}

    # -- diagnostics -------------------------------------------------------------
    def green_spectrum(self, N: int, dtype=torch.float64, stream=None) -> torch.Tensor:
        P = period(N)
        if not P:
            raise NmcError(NMC_EINVAL, f"unsupported N={N}")
        H = P // 2 + 1
        out = torch.empty((H, H, H), dtype=dtype, device=self.device)
        rc = lib().nmc_green_spectrum(self._h, N, precision_of(dtype), out.data_ptr(),
                                      _stream_ptr(stream, self.device))
        if rc:
            self._err(rc, "nmc_green_spectrum")
        return out

    def fft_lines(self, x: torch.Tensor, direction: int = -1, stream=None) -> torch.Tensor:
        """Batched 1-D FFT of the rows of a complex [nlines, P] device tensor."""
        if x.dtype not in (torch.complex128, torch.complex64) or x.dim() != 2 or not x.is_contiguous():
            raise ValueError("x must be a contiguous complex [nlines, P] tensor")
        p = NMC_F64 if x.dtype == torch.complex128 else NMC_F32
        out = torch.empty_like(x)
        rc = lib().nmc_fft_lines(self._h, x.data_ptr(), out.data_ptr(), x.shape[1], x.shape[0],
                                 direction, p, _stream_ptr(stream, self.device))
        if rc:
            self._err(rc, "nmc_fft_lines")
        return out


_contexts: dict = {}


def context(device=None) -> Context:
    """Process-wide default context per device."""
    key = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    if key not in _contexts:
        _contexts[key] = Context(torch.device("cuda", key))
    return _contexts[key]


def solve(rho: torch.Tensor, h0: float, G: float = 1.0, flags: int = 0, out=None, stream=None):
    """Potential on every level of a nested mesh (see include/nmc.h, nmc_solve)."""
    return context(rho.device).solve(rho, h0, G, flags, out, stream)
