"""Python binding of libdmimo (ctypes).

Argument marshalling only: every step runs in the HIP kernels of
libdmimo.so.  Arrays are torch tensors on the GPU (device memory), and calls
are ordered on the current torch stream unless ``stream`` is given.  There is
no CPU fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmimo.so")

# precision / model / precoder / points enums (include/dmimo.h)
F64, F32, MIX_F16X3, MIX_BF16X3 = 0, 1, 2, 3
CH_LOS, CH_RICIAN = 0, 1
MR, ZF, MR_PHASE, PA = 0, 1, 2, 3
PTS_GRID, PTS_LIST = 0, 1
CALL_CHANNEL, CALL_GRAM, CALL_BEAMFORM_MR, CALL_BEAMFORM_ZF, CALL_POWERMAP, CALL_PA_PRECODER = \
    0, 1, 2, 3, 4, 5
K_MAX = 32

PRECISIONS = {"f64": F64, "f32": F32, "f16x3": MIX_F16X3, "bf16x3": MIX_BF16X3}
PRECODERS = {"mr": MR, "zf": ZF, "mr_phase": MR_PHASE, "pa": PA}

STATUS = {0: "DMIMO_OK", 1: "DMIMO_E_ARG", 2: "DMIMO_E_SHAPE", 3: "DMIMO_E_DTYPE",
          4: "DMIMO_E_WORKSPACE", 5: "DMIMO_E_HIP", 6: "DMIMO_E_UNSUPPORTED",
          7: "DMIMO_E_BUSY", 8: "DMIMO_E_NOMEM", 9: "DMIMO_E_NOTFOUND"}


class DmimoError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class ChannelParams(ctypes.Structure):
    _fields_ = [("freq_hz", ctypes.c_double), ("model", ctypes.c_int32),
                ("kappa_lin", ctypes.c_double), ("d_min_m", ctypes.c_double)]


class Points(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("z", ctypes.c_double),
                ("xyz", ctypes.c_void_p), ("n", ctypes.c_int32)]


_vp, _i32, _f64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "dmimo_channel": [ctypes.POINTER(ChannelParams), _i32, _i32, _vp, ctypes.POINTER(Points),
                      _vp, _i32, _vp, _vp],
    "dmimo_gram": [_i32, _i32, _i32, _vp, _i32, _vp, _vp],
    "dmimo_beamform": [_i32, _i32, _i32, _i32, _vp, _vp, _f64, _f64, _i32, _vp, _vp, _vp, _vp,
                       _vp, _vp, _vp, _sz, _vp],
    "dmimo_beamform_batched": [_i32, ctypes.POINTER(ChannelParams), _i32, _i32, _i32, _vp, _vp, _vp,
                               _vp, _f64, _f64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "dmimo_beamform_noalloc": [_i32, _i32, _i32, _i32, _vp, _vp, _f64, _f64, _i32, _vp, _vp, _vp,
                               _vp, _vp, _vp, _vp],
    "dmimo_powermap": [ctypes.POINTER(ChannelParams), _i32, _vp, _i32, _vp,
                       ctypes.POINTER(Points), _f64, _i32, _vp, _vp, _vp, _vp, _vp],
    "dmimo_beamform_multi": [_i32, _vp, _i32, _i32, _i32, _vp, _vp, _f64, _f64, _i32, _vp, _vp,
                             _vp, _vp, _vp, _vp, _vp, _sz, _vp],
    "dmimo_beamform_multi_workspace_size": [_i32, _vp, _i32, _i32, _i32, _i32],
    "dmimo_beamform_users": [_i32, _vp, ctypes.POINTER(ChannelParams), _i32, _i32, _i32, _vp, _vp,
                             _vp, _f64, _f64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                             _vp],
    "dmimo_powermap_batch": [ctypes.POINTER(ChannelParams), _i32, _vp, _i32, _i32, _vp,
                             ctypes.POINTER(Points), _f64, _i32, _vp, _vp, _vp, _vp, _vp],
    "dmimo_workspace_size": [_i32, _i32, _i32, _i32, _i32, _i32],
    "dmimo_pgd": [_i32, _i32, _i32, _vp, _vp, _f64, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp],
    "dmimo_pa_precoder": [_i32, _i32, _i32, _vp, _vp, _f64, _i32, _vp, _vp, _i32, _vp, _vp, _vp,
                          _vp, _vp, _vp, _sz, _vp],
    "dmimo_ufpgd_workspace_size": [_i32, _i32, _i32, _i32],
    "dmimo_ufpgd_grad": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _f64, _f64, _i32, _vp, _vp, _i32,
                         _vp, _vp, _vp, _vp, _sz, _vp],
    "dmimo_ufpgd_train": [_i32, _i32, _i32, _vp, _vp, _f64, _f64, _i32, _vp, _vp, _vp, _vp,
                          ctypes.c_int64, ctypes.c_void_p, _i32, _i32, _vp, _vp, _i32, _vp, _sz,
                          _vp],
    "dmimo_server_create": [_i32, _sz, _i32, ctypes.POINTER(ctypes.c_void_p)],
    "dmimo_server_add_deployment": [_vp, ctypes.POINTER(ChannelParams), _i32, _vp,
                                    ctypes.POINTER(_i32)],
    "dmimo_server_submit": [_vp, _i32, _i32, _vp, _i32, ctypes.POINTER(Points), _f64, _f64, _i32,
                            _vp, _vp, ctypes.POINTER(ctypes.c_uint64)],
    "dmimo_server_poll": [_vp, ctypes.c_uint64, ctypes.POINTER(_i32), ctypes.POINTER(_f64),
                          ctypes.POINTER(_f64)],
    "dmimo_server_wait": [_vp, ctypes.c_uint64, _f64, ctypes.POINTER(_i32)],
    "dmimo_server_release": [_vp, ctypes.c_uint64],
    "dmimo_server_cancel": [_vp, ctypes.c_uint64],
    "dmimo_server_set_queue_timeout": [_vp, _f64],
    "dmimo_server_query_info": [_vp, ctypes.c_uint64, ctypes.POINTER(_i32)],
    "dmimo_server_set_pa_schedule": [_vp, _i32, _vp, _vp, _f64],
    "dmimo_server_stats": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_i32),
                           ctypes.POINTER(_i32)],
    "dmimo_server_destroy": [_vp],
    "dmimo_status_string": [_i32],
    "dmimo_last_error": [],
    "dmimo_version": [],
}
_RESTYPES = {"dmimo_workspace_size": _sz, "dmimo_beamform_multi_workspace_size": _sz, "dmimo_ufpgd_workspace_size": _sz, "dmimo_status_string": ctypes.c_char_p,
             "dmimo_last_error": ctypes.c_char_p, "dmimo_version": ctypes.c_char_p}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libdmimo.so not built ({path}); run python -m paper_2304_12745_amd.build")
    lib = ctypes.CDLL(path)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _RESTYPES.get(name, _i32)
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(status: int, where: str):
    if status != 0:
        detail = lib().dmimo_last_error().decode()
        raise DmimoError(status, where, detail)


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def channel_params(freq_hz: float, model: int = CH_LOS, kappa_lin: float = 0.0,
                   d_min_m: float = 0.0) -> ChannelParams:
    return ChannelParams(float(freq_hz), int(model), float(kappa_lin), float(d_min_m))


def grid_points(grid) -> Points:
    """Descriptor of a regular grid (an object with x0, y0, dx, dy, z, nx, ny)."""
    return Points(PTS_GRID, int(grid.nx), int(grid.ny), float(grid.x0), float(grid.y0),
                  float(grid.dx), float(grid.dy), float(grid.z), None, 0)


def list_points(xyz, n: int) -> Points:
    """Descriptor of an explicit device point list (FP64 tensor [.., n, 3]).

    The descriptor holds a reference to ``xyz``, so the device memory stays
    alive as long as the descriptor does.
    """
    p = Points(PTS_LIST, 0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, _ptr(xyz), int(n))
    p._keep = xyz
    return p


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _cdtype(prec: int):
    import torch
    return torch.complex128 if prec == F64 else torch.complex64


def _rdtype(prec: int):
    import torch
    return torch.float64 if prec == F64 else torch.float32


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def channel(params: ChannelParams, ap_xyz, points: Points, nlos=None, prec="f32", out=None,
            B: Optional[int] = None, N: Optional[int] = None, stream=None):
    """H[b][n][m] (dmimo_channel).  ap_xyz: float64 [B][M][3] on the GPU."""
    import torch
    prec = _prec(prec)
    B = ap_xyz.shape[0] if B is None else B
    M = ap_xyz.shape[1]
    if N is None:
        N = points.nx * points.ny if points.kind == PTS_GRID else points.n
    if out is None:
        out = torch.empty((B, N, M), dtype=_cdtype(prec), device=ap_xyz.device)
    _check(lib().dmimo_channel(ctypes.byref(params), B, M, _ptr(ap_xyz), ctypes.byref(points),
                               _ptr(nlos), prec, _ptr(out), _stream(stream)), "dmimo_channel")
    return out


def gram(H, prec="f32", out=None, stream=None):
    """G[b] = H[b] H[b]^H (dmimo_gram).  H: complex [B][K][M] on the GPU."""
    import torch
    prec = _prec(prec)
    B, K, M = H.shape
    if out is None:
        out = torch.empty((B, K, K), dtype=_cdtype(prec), device=H.device)
    _check(lib().dmimo_gram(B, K, M, _ptr(H), prec, _ptr(out), _stream(stream)), "dmimo_gram")
    return out


def workspace_size(call: int, B: int, K: int, M: int, N: int, prec) -> int:
    return int(lib().dmimo_workspace_size(call, B, K, M, N, _prec(prec)))


@dataclass
class BeamformResult:
    W: object
    p_ant: object
    l21: object
    sinr: object
    rsum: object
    info: object


def beamform_outputs(B: int, K: int, M: int, prec="f32", device=None, outputs=True,
                     precoder="zf") -> BeamformResult:
    """Allocate the outputs of beamform() once, for reuse through ``out=``.

    The workspace of a ZF call (``ws``) is allocated here too.
    """
    import torch
    prec = _prec(prec)
    W = torch.empty((B, K, M), dtype=_cdtype(prec), device=device)
    r = BeamformResult(
        W,
        torch.empty((B, M), dtype=torch.float64, device=device) if outputs else None,
        torch.empty((B,), dtype=torch.float64, device=device) if outputs else None,
        torch.empty((B, K), dtype=torch.float64, device=device) if outputs else None,
        torch.empty((B,), dtype=torch.float64, device=device) if outputs else None,
        torch.empty((B,), dtype=torch.int32, device=device) if outputs else None)
    pc = PRECODERS[precoder] if isinstance(precoder, str) else int(precoder)
    need = workspace_size(CALL_BEAMFORM_ZF if pc == ZF else CALL_BEAMFORM_MR, B, K, M, 0, prec)
    r.ws = torch.empty((need,), dtype=torch.uint8, device=device) if need else None
    return r


def beamform(H, precoder="zf", gamma_lin=None, sigma2=1.0, p_total=0.0, prec="f32",
             outputs=True, ws=None, stream=None, out: Optional[BeamformResult] = None
             ) -> BeamformResult:
    """Precoder + epilogues (dmimo_beamform).  H: complex [B][K][M] on the GPU.

    ``out`` (from beamform_outputs) reuses preallocated outputs and workspace.
    """
    prec = _prec(prec)
    pc = PRECODERS[precoder] if isinstance(precoder, str) else int(precoder)
    B, K, M = H.shape
    if out is None:
        out = beamform_outputs(B, K, M, prec, H.device, outputs, pc)
    if ws is None:
        ws = getattr(out, "ws", None)
    g = None
    if gamma_lin is not None:
        g = (ctypes.c_double * K)(*[float(x) for x in gamma_lin])
    _check(lib().dmimo_beamform(pc, B, K, M, _ptr(H), g, float(sigma2), float(p_total), prec,
                                _ptr(out.W), _ptr(out.p_ant), _ptr(out.l21), _ptr(out.sinr),
                                _ptr(out.rsum), _ptr(out.info), _ptr(ws),
                                ws.numel() if ws is not None else 0, _stream(stream)),
           "dmimo_beamform")
    return out


def beamform_batched(params: ChannelParams, ap_xyz, user_xyz, nlos=None, precoder="zf",
                     gamma_lin=None, sigma2=1.0, p_total=0.0, prec="f32", want_H=False,
                     want_W=True, out: Optional[BeamformResult] = None,
                     stream=None) -> BeamformResult:
    """dmimo_beamform_batched: the users' channels (LoS, or Rician with
    ``nlos`` complex64 [B][K][M]) and their MR / ZF precoder with epilogues,
    for many small deployments in one launch (K <= 16, M <= 256).
    ap_xyz float64 [B][M][3], user_xyz float64 [B][K][3].  H (``out.H``) and
    W are written when asked for."""
    import torch
    prec = _prec(prec)
    pc = PRECODERS[precoder] if isinstance(precoder, str) else int(precoder)
    B, M = ap_xyz.shape[0], ap_xyz.shape[1]
    K = user_xyz.shape[1]
    if tuple(user_xyz.shape) != (B, K, 3) or tuple(ap_xyz.shape) != (B, M, 3):
        raise ValueError("beamform_batched: ap_xyz [B][M][3] and user_xyz [B][K][3]")
    if not (ap_xyz.is_contiguous() and user_xyz.is_contiguous()):
        raise ValueError("beamform_batched: contiguous coordinates required")
    dev = ap_xyz.device
    if out is None:
        f64 = dict(dtype=torch.float64, device=dev)
        out = BeamformResult(
            torch.empty((B, K, M), dtype=torch.complex64, device=dev) if want_W else None,
            torch.empty((B, M), **f64), torch.empty((B,), **f64), torch.empty((B, K), **f64),
            torch.empty((B,), **f64), torch.empty((B,), dtype=torch.int32, device=dev))
        out.H = torch.empty((B, K, M), dtype=torch.complex64, device=dev) if want_H else None
    g = None
    if gamma_lin is not None:
        g = (ctypes.c_double * K)(*[float(x) for x in gamma_lin])
    _check(lib().dmimo_beamform_batched(pc, ctypes.byref(params), B, K, M, _ptr(ap_xyz),
                                        _ptr(user_xyz), _ptr(nlos), g, float(sigma2),
                                        float(p_total), prec, _ptr(getattr(out, "H", None)),
                                        _ptr(out.W), _ptr(out.p_ant), _ptr(out.l21),
                                        _ptr(out.sinr), _ptr(out.rsum), _ptr(out.info),
                                        _stream(stream)),
           "dmimo_beamform_batched")
    return out


# bytes of the static scratch array of dmimo_beamform_noalloc (DMIMO_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 8 << 20


def beamform_noalloc(H, precoder="zf", gamma_lin=None, sigma2=1.0, p_total=0.0, prec="f32",
                     out: Optional[BeamformResult] = None, stream=None) -> BeamformResult:
    """dmimo_beamform_noalloc: dmimo_beamform with the scratch in the library's
    static device array (no workspace argument, nothing allocated by the
    call).  ``out`` (from beamform_outputs) reuses preallocated outputs."""
    prec = _prec(prec)
    pc = PRECODERS[precoder] if isinstance(precoder, str) else int(precoder)
    B, K, M = H.shape
    if out is None:
        out = beamform_outputs(B, K, M, prec, H.device, True, pc)
    g = None
    if gamma_lin is not None:
        g = (ctypes.c_double * K)(*[float(x) for x in gamma_lin])
    _check(lib().dmimo_beamform_noalloc(pc, B, K, M, _ptr(H), g, float(sigma2), float(p_total),
                                        prec, _ptr(out.W), _ptr(out.p_ant), _ptr(out.l21),
                                        _ptr(out.sinr), _ptr(out.rsum), _ptr(out.info),
                                        _stream(stream)),
           "dmimo_beamform_noalloc")
    return out


def beamform_multi(H, precoders=("mr", "zf"), gamma_lin=None, sigma2=1.0, p_total=0.0,
                   prec="f32", outputs=True, out: Optional[BeamformResult] = None, ws=None,
                   stream=None) -> BeamformResult:
    """Several precoders of the same channels (dmimo_beamform_multi): every
    output gains a leading [P] dimension (W [P][B][K][M]); the results equal
    one beamform() per precoder bit for bit."""
    import torch
    prec = _prec(prec)
    pcs = [PRECODERS[p] if isinstance(p, str) else int(p) for p in precoders]
    P = len(pcs)
    B, K, M = H.shape
    dev = H.device
    arr = (ctypes.c_int32 * max(P, 1))(*pcs)
    if out is None:
        f64 = dict(dtype=torch.float64, device=dev)
        out = BeamformResult(
            torch.empty((P, B, K, M), dtype=_cdtype(prec), device=dev),
            torch.empty((P, B, M), **f64) if outputs else None,
            torch.empty((P, B), **f64) if outputs else None,
            torch.empty((P, B, K), **f64) if outputs else None,
            torch.empty((P, B), **f64) if outputs else None,
            torch.empty((P, B), dtype=torch.int32, device=dev) if outputs else None)
    need = lib().dmimo_beamform_multi_workspace_size(P, arr, B, K, M, prec)
    if ws is None:
        ws = getattr(out, "ws", None)
    if need and (ws is None or ws.numel() < need):
        ws = torch.empty((need,), dtype=torch.uint8, device=dev)
    out.ws = ws
    g = None
    if gamma_lin is not None:
        g = (ctypes.c_double * K)(*[float(x) for x in gamma_lin])
    _check(lib().dmimo_beamform_multi(P, arr, B, K, M, _ptr(H), g, float(sigma2), float(p_total),
                                      prec, _ptr(out.W), _ptr(out.p_ant), _ptr(out.l21),
                                      _ptr(out.sinr), _ptr(out.rsum), _ptr(out.info), _ptr(ws),
                                      ws.numel() if ws is not None else 0, _stream(stream)),
           "dmimo_beamform_multi")
    return out


def beamform_users(params: ChannelParams, ap_xyz, user_xyz, precoders=("mr", "zf"),
                   gamma_lin=None, sigma2=1.0, p_total=0.0, prec="f32", outputs=True,
                   out: Optional[BeamformResult] = None, H=None, ws=None,
                   stream=None) -> BeamformResult:
    """The users' LoS channels and several precoders of them
    (dmimo_beamform_users): ap_xyz float64 [B][M][3], user_xyz float64
    [B][K][3]; H [B][K][M] is written to ``H`` (allocated if None) and kept
    as ``out.H``.  The results equal channel() followed by beamform_multi()
    bit for bit."""
    import torch
    prec = _prec(prec)
    pcs = [PRECODERS[p] if isinstance(p, str) else int(p) for p in precoders]
    P = len(pcs)
    B, M = ap_xyz.shape[0], ap_xyz.shape[1]
    K = user_xyz.shape[1]
    if tuple(user_xyz.shape) != (B, K, 3) or tuple(ap_xyz.shape) != (B, M, 3):
        raise ValueError("beamform_users: ap_xyz [B][M][3] and user_xyz [B][K][3]")
    if not (ap_xyz.is_contiguous() and user_xyz.is_contiguous()):
        raise ValueError("beamform_users: contiguous coordinates required")
    dev = ap_xyz.device
    arr = (ctypes.c_int32 * max(P, 1))(*pcs)
    if H is None:
        H = getattr(out, "H", None)
    if H is None:
        H = torch.empty((B, K, M), dtype=_cdtype(prec), device=dev)
    if out is None:
        f64 = dict(dtype=torch.float64, device=dev)
        out = BeamformResult(
            torch.empty((P, B, K, M), dtype=_cdtype(prec), device=dev),
            torch.empty((P, B, M), **f64) if outputs else None,
            torch.empty((P, B), **f64) if outputs else None,
            torch.empty((P, B, K), **f64) if outputs else None,
            torch.empty((P, B), **f64) if outputs else None,
            torch.empty((P, B), dtype=torch.int32, device=dev) if outputs else None)
    out.H = H
    need = lib().dmimo_beamform_multi_workspace_size(P, arr, B, K, M, prec)
    if ws is None:
        ws = getattr(out, "ws", None)
    if need and (ws is None or ws.numel() < need):
        ws = torch.empty((need,), dtype=torch.uint8, device=dev)
    out.ws = ws
    g = None
    if gamma_lin is not None:
        g = (ctypes.c_double * K)(*[float(x) for x in gamma_lin])
    _check(lib().dmimo_beamform_users(P, arr, ctypes.byref(params), B, K, M, _ptr(ap_xyz),
                                      _ptr(user_xyz), g, float(sigma2), float(p_total), prec,
                                      _ptr(H), _ptr(out.W), _ptr(out.p_ant), _ptr(out.l21),
                                      _ptr(out.sinr), _ptr(out.rsum), _ptr(out.info), _ptr(ws),
                                      ws.numel() if ws is not None else 0, _stream(stream)),
           "dmimo_beamform_users")
    return out


@dataclass
class MapResult:
    power: object
    sinr: object
    best_k: object
    per_stream: object


def powermap(params: ChannelParams, ap_xyz, W, points: Points, sigma2=1e-12, prec="f32",
             want_sinr=True, want_best=True, want_per_stream=False, out=None,
             stream=None) -> MapResult:
    """Fused synthesis + coherent sums (dmimo_powermap).  ap_xyz float64 [M][3], W [K][M]."""
    import torch
    prec = _prec(prec)
    K, M = W.shape
    N = points.nx * points.ny if points.kind == PTS_GRID else points.n
    dev = W.device
    rd = _rdtype(prec)
    if out is None:
        out = MapResult(
            torch.empty((N,), dtype=rd, device=dev),
            torch.empty((N,), dtype=rd, device=dev) if want_sinr else None,
            torch.empty((N,), dtype=torch.int32, device=dev) if want_best else None,
            torch.empty((N, K), dtype=rd, device=dev) if want_per_stream else None)
    _check(lib().dmimo_powermap(ctypes.byref(params), M, _ptr(ap_xyz), K, _ptr(W),
                                ctypes.byref(points), float(sigma2), prec, _ptr(out.power),
                                _ptr(out.sinr), _ptr(out.best_k), _ptr(out.per_stream),
                                _stream(stream)), "dmimo_powermap")
    return out


def powermap_batch(params: ChannelParams, ap_xyz, W, points: Points, sigma2=1e-12, prec="f32",
                   want_sinr=True, want_best=True, want_per_stream=False, out=None,
                   stream=None) -> MapResult:
    """The maps of several precoders over the same points in one launch
    (dmimo_powermap_batch).  W [P][K][M]; outputs [P][N] ([P][N][K] per stream)."""
    import torch
    prec = _prec(prec)
    P, K, M = W.shape
    if not W.is_contiguous():
        raise ValueError("powermap_batch: W must be contiguous [P][K][M]")
    N = points.nx * points.ny if points.kind == PTS_GRID else points.n
    dev = W.device
    rd = _rdtype(prec)
    if out is None:
        out = MapResult(
            torch.empty((P, N), dtype=rd, device=dev),
            torch.empty((P, N), dtype=rd, device=dev) if want_sinr else None,
            torch.empty((P, N), dtype=torch.int32, device=dev) if want_best else None,
            torch.empty((P, N, K), dtype=rd, device=dev) if want_per_stream else None)
    _check(lib().dmimo_powermap_batch(ctypes.byref(params), M, _ptr(ap_xyz), P, K, _ptr(W),
                                      ctypes.byref(points), float(sigma2), prec, _ptr(out.power),
                                      _ptr(out.sinr), _ptr(out.best_k), _ptr(out.per_stream),
                                      _stream(stream)), "dmimo_powermap_batch")
    return out


@dataclass
class PgdResult:
    W: object
    l21: object
    rsum: object


def pgd(H, lambdas, etas, gamma_lin=None, sigma2=1.0, W0=None, prec="f32", out=None,
        want_l21=True, want_rsum=True, stream=None) -> PgdResult:
    """PGD / unfolded PGD (dmimo_pgd).  H complex64 [B][K][M]; lambdas, etas:
    per-layer values (sequences or FP64 device tensors of length I)."""
    import torch
    B, K, M = H.shape
    dev = H.device
    lam = lambdas if torch.is_tensor(lambdas) else torch.tensor(list(lambdas), dtype=torch.float64)
    eta = etas if torch.is_tensor(etas) else torch.tensor(list(etas), dtype=torch.float64)
    lam = lam.to(device=dev, dtype=torch.float64).contiguous()
    eta = eta.to(device=dev, dtype=torch.float64).contiguous()
    if lam.numel() != eta.numel():
        raise ValueError("lambdas and etas need the same length")
    if out is None:
        out = PgdResult(torch.empty((B, K, M), dtype=torch.complex64, device=dev),
                        torch.empty((B,), dtype=torch.float64, device=dev) if want_l21 else None,
                        torch.empty((B,), dtype=torch.float64, device=dev) if want_rsum else None)
    g = None
    if gamma_lin is not None:
        g = (ctypes.c_double * K)(*[float(x) for x in gamma_lin])
    out._keep = (lam, eta)
    _check(lib().dmimo_pgd(B, K, M, _ptr(H), g, float(sigma2), lam.numel(), _ptr(lam), _ptr(eta),
                           _ptr(W0), _prec(prec), _ptr(out.W), _ptr(out.l21), _ptr(out.rsum),
                           _stream(stream)), "dmimo_pgd")
    return out


@dataclass
class PaResult:
    W: object       # [B][K][M] complex64
    p_ant: object   # [B][M] FP64
    l21: object     # [B]
    sinr: object    # [B][K]
    rsum: object    # [B]


def pa_precoder(H, lambdas, eta_rel, gamma_lin=None, sigma2=1.0, out=None, ws=None,
                stream=None, prec="f32") -> PaResult:
    """PA-aware precoder of deployments with channels of any scale
    (dmimo_pa_precoder).  H complex64 [B][K][M] on the GPU; lambdas, eta_rel
    per layer (steps relative to 1 / lambda_max of the normalised Gram)."""
    import torch
    B, K, M = H.shape
    dev = H.device
    lam = _f64_dev(lambdas, dev)
    er = _f64_dev(eta_rel, dev)
    if lam.numel() != er.numel():
        raise ValueError("lambdas and eta_rel need the same length")
    if out is None:
        f64 = dict(dtype=torch.float64, device=dev)
        out = PaResult(torch.empty((B, K, M), dtype=torch.complex64, device=dev),
                       torch.empty((B, M), **f64), torch.empty((B,), **f64),
                       torch.empty((B, K), **f64), torch.empty((B,), **f64))
    nbytes = workspace_size(CALL_PA_PRECODER, B, K, M, 0, F32)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty((max(nbytes, 1),), dtype=torch.uint8, device=dev)
    out._keep = (lam, er, ws)
    _check(lib().dmimo_pa_precoder(B, K, M, _ptr(H), _gamma(gamma_lin, K), float(sigma2),
                                   lam.numel(), _ptr(lam), _ptr(er), _prec(prec), _ptr(out.W),
                                   _ptr(out.p_ant), _ptr(out.l21), _ptr(out.sinr),
                                   _ptr(out.rsum), _ptr(ws), nbytes, _stream(stream)),
           "dmimo_pa_precoder")
    return out


# ---------------------------------------------------------------------------
# unsupervised training of the unfolded network
# ---------------------------------------------------------------------------

LAM_COST = 1.0 / 15.0     # the cost's lambda in the paper's simulations


class AdamParams(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


def ufpgd_workspace_size(B: int, K: int, M: int, layers: int) -> int:
    return int(lib().dmimo_ufpgd_workspace_size(B, K, M, layers))


def _gamma(gamma_lin, K):
    if gamma_lin is None:
        return None
    return (ctypes.c_double * K)(*[float(x) for x in gamma_lin])


def _f64_dev(x, dev):
    import torch
    t = x if torch.is_tensor(x) else torch.tensor(list(x), dtype=torch.float64)
    return t.to(device=dev, dtype=torch.float64).contiguous()


@dataclass
class UfpgdGrad:
    cost: object     # [B]
    dlam: object     # [B][I] or None
    deta: object


def ufpgd_grad(H, lambdas, etas, gamma_lin=None, sigma2=1.0, lam_c=LAM_COST, idx=None,
               want_grad=True, ws=None, stream=None) -> UfpgdGrad:
    """Per-channel cost and gradients of the unfolded network (dmimo_ufpgd_grad).
    H complex64 [n][K][M]; idx optional device int32 [B] selecting channels."""
    import torch
    n, K, M = H.shape
    dev = H.device
    B = n if idx is None else idx.numel()
    lam = _f64_dev(lambdas, dev)
    eta = _f64_dev(etas, dev)
    I = lam.numel()
    if eta.numel() != I:
        raise ValueError("lambdas and etas need the same length")
    out = UfpgdGrad(torch.empty((B,), dtype=torch.float64, device=dev),
                    torch.empty((B, I), dtype=torch.float64, device=dev) if want_grad else None,
                    torch.empty((B, I), dtype=torch.float64, device=dev) if want_grad else None)
    nbytes = 0
    if want_grad:
        nbytes = ufpgd_workspace_size(max(B, 1), K, M, I)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty((max(nbytes, 1),), dtype=torch.uint8, device=dev)
    out._keep = (lam, eta, ws, idx)
    _check(lib().dmimo_ufpgd_grad(B, n, K, M, _ptr(H), _ptr(idx), _gamma(gamma_lin, K),
                                  float(sigma2), float(lam_c), I, _ptr(lam), _ptr(eta), F32,
                                  _ptr(out.cost), _ptr(out.dlam), _ptr(out.deta),
                                  _ptr(ws) if want_grad else None, nbytes,
                                  _stream(stream)), "dmimo_ufpgd_grad")
    return out


class UfpgdState:
    """Trainable parameters lambda_i, eta_i and the Adam moments, on the device."""

    def __init__(self, lambdas, etas, device):
        import torch
        self.lambdas = _f64_dev(lambdas, device)
        self.etas = _f64_dev(etas, device)
        I = self.lambdas.numel()
        if self.etas.numel() != I:
            raise ValueError("lambdas and etas need the same length")
        self.m = torch.zeros(2 * I, dtype=torch.float64, device=device)
        self.v = torch.zeros(2 * I, dtype=torch.float64, device=device)
        self.t = 0

    @property
    def layers(self) -> int:
        return self.lambdas.numel()

    def clone(self) -> "UfpgdState":
        c = UfpgdState(self.lambdas.clone(), self.etas.clone(), self.lambdas.device)
        c.m.copy_(self.m)
        c.v.copy_(self.v)
        c.t = self.t
        return c


def ufpgd_train(H, state: UfpgdState, idx, gamma_lin=None, sigma2=1.0, lam_c=LAM_COST, lr=1e-3,
                beta1=0.9, beta2=0.999, eps=1e-8, batch_cost=None, ws=None, stream=None):
    """Run idx.shape[0] Adam steps (dmimo_ufpgd_train); idx device int32
    [steps][batch].  Updates `state` in place; returns the per-step mean batch cost."""
    import torch
    n, K, M = H.shape
    dev = H.device
    steps, batch = idx.shape
    idx = idx.to(device=dev, dtype=torch.int32).contiguous()
    if batch_cost is None:
        batch_cost = torch.empty((steps,), dtype=torch.float64, device=dev)
    nbytes = ufpgd_workspace_size(batch, K, M, state.layers)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty((max(nbytes, 1),), dtype=torch.uint8, device=dev)
    opt = AdamParams(lr, beta1, beta2, eps)
    _check(lib().dmimo_ufpgd_train(n, K, M, _ptr(H), _gamma(gamma_lin, K), float(sigma2),
                                   float(lam_c), state.layers, _ptr(state.lambdas),
                                   _ptr(state.etas), _ptr(state.m), _ptr(state.v), state.t,
                                   ctypes.addressof(opt), batch, steps, _ptr(idx),
                                   _ptr(batch_cost), F32, _ptr(ws), nbytes, _stream(stream)),
           "dmimo_ufpgd_train")
    state.t += steps
    state._keep = (idx, ws, batch_cost)
    return batch_cost


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

Q_QUEUED, Q_RUNNING, Q_DONE, Q_FAILED, Q_CANCELLED, Q_TIMED_OUT = 0, 1, 2, 3, 4, 5


class Server:
    """Continuous-batching power-map server (dmimo_server_*).

    Output tensors passed to submit() are kept referenced until the ticket is
    released, so their device memory outlives the query.
    """

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 64, device: int = 0):
        self._h = ctypes.c_void_p()
        self._keep = {}
        _check(lib().dmimo_server_create(int(device), int(hbm_budget_bytes), int(max_inflight),
                                         ctypes.byref(self._h)), "dmimo_server_create")

    def add_deployment(self, params: ChannelParams, ap_xyz_host) -> int:
        import numpy as np
        ap = np.ascontiguousarray(ap_xyz_host, dtype=np.float64)
        dep = _i32()
        _check(lib().dmimo_server_add_deployment(self._h, ctypes.byref(params), ap.shape[0],
                                                 ap.ctypes.data, ctypes.byref(dep)),
               "dmimo_server_add_deployment")
        return dep.value

    def submit(self, dep: int, user_xyz_host, precoder, points: Points, sigma2: float,
               p_total: float, prec, power, sinr=None) -> int:
        import numpy as np
        u = np.ascontiguousarray(user_xyz_host, dtype=np.float64)
        pc = PRECODERS[precoder] if isinstance(precoder, str) else int(precoder)
        t = ctypes.c_uint64()
        _check(lib().dmimo_server_submit(self._h, int(dep), u.shape[0], u.ctypes.data, pc,
                                         ctypes.byref(points), float(sigma2), float(p_total),
                                         _prec(prec), _ptr(power), _ptr(sinr), ctypes.byref(t)),
               "dmimo_server_submit")
        self._keep[t.value] = (power, sinr, points)
        return t.value

    def set_pa_schedule(self, lambdas, eta_rel, gamma_lin: float):
        """Layer schedule of "pa" queries (host sequences), and their SINR target."""
        import numpy as np
        lam = np.ascontiguousarray(lambdas, dtype=np.float64)
        er = np.ascontiguousarray(eta_rel, dtype=np.float64)
        if lam.shape != er.shape:
            raise ValueError("lambdas and eta_rel need the same length")
        _check(lib().dmimo_server_set_pa_schedule(self._h, lam.size, lam.ctypes.data,
                                                  er.ctypes.data, float(gamma_lin)),
               "dmimo_server_set_pa_schedule")

    def poll(self, ticket: int):
        st, ts, td = _i32(), _f64(), _f64()
        _check(lib().dmimo_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(st),
                                       ctypes.byref(ts), ctypes.byref(td)), "dmimo_server_poll")
        return st.value, ts.value, td.value

    def wait(self, ticket: int, timeout_s: float = 60.0) -> int:
        st = _i32()
        _check(lib().dmimo_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s),
                                       ctypes.byref(st)), "dmimo_server_wait")
        return st.value

    def release(self, ticket: int):
        _check(lib().dmimo_server_release(self._h, ctypes.c_uint64(ticket)), "dmimo_server_release")
        self._keep.pop(ticket, None)

    def cancel(self, ticket: int):
        """Withdraw a query not admitted yet (DmimoError with DMIMO_E_BUSY otherwise)."""
        _check(lib().dmimo_server_cancel(self._h, ctypes.c_uint64(ticket)), "dmimo_server_cancel")

    def set_queue_timeout(self, seconds: float):
        _check(lib().dmimo_server_set_queue_timeout(self._h, float(seconds)),
               "dmimo_server_set_queue_timeout")

    def query_info(self, ticket: int) -> int:
        """The precoder's info word of a finished query (ZF: the failed pivot, or 0)."""
        v = _i32()
        _check(lib().dmimo_server_query_info(self._h, ctypes.c_uint64(ticket), ctypes.byref(v)),
               "dmimo_server_query_info")
        return v.value

    def stats(self) -> dict:
        c, tm, tk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        q, r = _i32(), _i32()
        _check(lib().dmimo_server_stats(self._h, ctypes.byref(c), ctypes.byref(tm), ctypes.byref(tk),
                                        ctypes.byref(q), ctypes.byref(r)), "dmimo_server_stats")
        return {"completed": c.value, "terms": tm.value, "launches": tk.value, "queued": q.value,
                "running": r.value}

    def close(self):
        if self._h:
            _check(lib().dmimo_server_destroy(self._h), "dmimo_server_destroy")
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def version() -> str:
    return lib().dmimo_version().decode()
