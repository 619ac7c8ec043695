"""ctypes binding of libfftenkf.so (include/fftenkf.h): argument marshalling only.

Every step of the analysis runs in the HIP kernels behind the C ABI.  PyTorch
supplies device memory and the current stream.  If the library has not been
built, or the call fails, a RuntimeError is raised; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Union

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfftenkf.so")

OK, EINVAL, EUNSUPPORTED, EDEVICE, ENOMEM = 0, -1, -2, -3, -4
F32, F64 = 0, 1


class Ens(ctypes.Structure):
    """Mirror of struct fftenkf_ens."""

    _fields_ = [
        ("n_members", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("members", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("r_scalar", ctypes.c_double),
    ]


class Mlp(ctypes.Structure):
    """Mirror of struct fftenkf_mlp (eight device float32 pointers)."""

    _fields_ = [(name, ctypes.c_void_p) for name in ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4")]


MLP_SHAPES = {"W1": (26, 64), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (64, 64), "b3": (64,),
              "w4": (64,), "b4": (1,)}

class Filter(ctypes.Structure):
    """Mirror of struct fftenkf_filter."""

    _fields_ = [
        ("ny", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("members", ctypes.c_void_p),
        ("data", ctypes.c_void_p),
        ("R_spec", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("r_scalar", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


_lib: Optional[ctypes.CDLL] = None

EXPORTS = {
    "fftenkf_analyze": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "fftenkf_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fftenkf_analyze_noalloc": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                               ctypes.c_void_p]),
    "fftenkf_noalloc_max_bytes": (ctypes.c_size_t, []),
    "fftenkf_max_members": (ctypes.c_int, [ctypes.c_int]),
    "fftenkf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fftenkf_last_error": (ctypes.c_char_p, []),
    "fftenkf_debug_spectra": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "fftenkf_debug_perturb": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                             ctypes.c_void_p]),
    "fftenkf_debug_fail_next": (None, [ctypes.c_int]),
    "fftenkf_profile_events": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "fftenkf_analyze_learned": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                               ctypes.POINTER(Mlp), ctypes.c_void_p]),
    "fftenkf_analyze_spectrum": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                                ctypes.c_void_p, ctypes.c_void_p]),
    "fftenkf_release_caches": (ctypes.c_int, []),
    "fftenkf_analyze_dst": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                           ctypes.c_void_p]),
    "fftenkf_workspace_bytes_dst": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fftenkf_debug_dst_coeffs": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.c_void_p]),
    "fftenkf_analyze_batch": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Filter), ctypes.c_int,
                                             ctypes.c_void_p]),
    "fftenkf_tile_rows_options": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "fftenkf_set_tile_rows": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fftenkf_tile_rows": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "fftenkf_analyze_multi": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_uint64, ctypes.c_void_p]),
    "fftenkf_workspace_bytes_multi": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                        ctypes.c_int]),
    "fftenkf_max_members_multi": (ctypes.c_int, [ctypes.c_int]),
    "fftenkf_analyze_morph": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_uint64,
                                             ctypes.c_void_p]),
    "fftenkf_workspace_bytes_morph": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                        ctypes.c_int, ctypes.c_int]),
    "fftenkf_max_members_morph": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "fftenkf_debug_fft2": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "fftenkf_debug_learned_spectrum": (ctypes.c_int, [ctypes.POINTER(Ens), ctypes.c_void_p, ctypes.POINTER(Mlp),
                                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}


def lib() -> ctypes.CDLL:
    """Load libfftenkf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1001_1588_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status: int, what: str) -> None:
    if status != OK:
        msg = lib().fftenkf_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed: {lib().fftenkf_strerror(status).decode()} ({status}): {msg}")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}: float32 or float64")


def workspace_bytes(n_members: int, ny: int, nx: int, dtype: torch.dtype) -> int:
    code = F32 if dtype == torch.float32 else F64
    return int(lib().fftenkf_workspace_bytes(n_members, ny, nx, code))


def max_members(dtype: torch.dtype) -> int:
    return int(lib().fftenkf_max_members(F32 if dtype == torch.float32 else F64))


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _make_ens(ens: torch.Tensor, workspace: Optional[torch.Tensor], r_scalar: float) -> tuple:
    if ens.dim() != 3:
        raise ValueError("ens must be [N, ny, nx]")
    if not ens.is_cuda:
        raise ValueError("ens must be a device tensor")
    if not ens.is_contiguous():
        raise ValueError("ens must be contiguous")
    N, ny, nx = ens.shape
    need = workspace_bytes(N, ny, nx, ens.dtype)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=ens.device)
    e = Ens(n_members=N, ny=ny, nx=nx, dtype=_dtype_code(ens), members=ens.data_ptr(),
            workspace=workspace.data_ptr(), workspace_bytes=workspace.numel() * workspace.element_size(),
            stream=torch.cuda.current_stream(ens.device).cuda_stream, r_scalar=float(r_scalar))
    return e, workspace


def _rspec(R_spec: Union[torch.Tensor, float, None]):
    if R_spec is None or isinstance(R_spec, (int, float)):
        return None, float(R_spec or 0.0)
    return R_spec, 0.0


def analyze(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float], seed: int,
            out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One FFT EnKF analysis (eq. (3) with eq. (2)); returns the analysis ensemble.

    R_spec is a [ny, nx//2+1] tensor of R's eigenvalues or a float r (R = r I).
    out may be ens itself (in place).  Enqueued on the current stream."""
    R_t, r = _rspec(R_spec)
    e, ws = _make_ens(ens, workspace, r)
    if out is None:
        out = torch.empty_like(ens)
    st = lib().fftenkf_analyze(ctypes.byref(e), data.data_ptr(), _ptr(R_t), ctypes.c_uint64(seed & (2**64 - 1)),
                               out.data_ptr())
    _check(st, "fftenkf_analyze")
    return out


def analyze_noalloc(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float], seed: int,
                    out: torch.Tensor) -> torch.Tensor:
    """fftenkf_analyze_noalloc: the analysis with the library's static scratch as
    its workspace; `out` must be given (the call allocates nothing)."""
    if ens.dim() != 3 or not ens.is_cuda or not ens.is_contiguous():
        raise ValueError("ens must be a contiguous device tensor [N, ny, nx]")
    N, ny, nx = ens.shape
    R_t, r = _rspec(R_spec)
    e = Ens(n_members=N, ny=ny, nx=nx, dtype=_dtype_code(ens), members=ens.data_ptr(), workspace=None,
            workspace_bytes=0, stream=torch.cuda.current_stream(ens.device).cuda_stream, r_scalar=float(r))
    st = lib().fftenkf_analyze_noalloc(ctypes.byref(e), data.data_ptr(), _ptr(R_t),
                                       ctypes.c_uint64(seed & (2**64 - 1)), out.data_ptr())
    _check(st, "fftenkf_analyze_noalloc")
    return out


def analyze_multi(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float], seed: int,
                  out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Multi-block analysis (eq. (6)): ens [N, M, ny, nx] member-major, data observing block 0."""
    if ens.dim() != 4 or not ens.is_cuda or not ens.is_contiguous():
        raise ValueError("ens must be a contiguous device tensor [N, M, ny, nx]")
    N, M, ny, nx = ens.shape
    R_t, r = _rspec(R_spec)
    code = _dtype_code(ens)
    if workspace is None:
        need = int(lib().fftenkf_workspace_bytes_multi(N, M, ny, nx, code))
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=ens.device)
    e = Ens(n_members=N, ny=ny, nx=nx, dtype=code, members=ens.data_ptr(), workspace=workspace.data_ptr(),
            workspace_bytes=workspace.numel(), stream=torch.cuda.current_stream(ens.device).cuda_stream,
            r_scalar=float(r))
    if out is None:
        out = torch.empty_like(ens)
    st = lib().fftenkf_analyze_multi(ctypes.byref(e), M, data.data_ptr(), _ptr(R_t),
                                     ctypes.c_uint64(seed & (2**64 - 1)), out.data_ptr())
    _check(st, "fftenkf_analyze_multi")
    return out


def analyze_morph(ens: torch.Tensor, data: torch.Tensor, R, seed: int, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The extended-state analysis of the morphing EnKF: ens [N, M, ny, nx]
    member-major, data [K, ny, nx] observing blocks 0 .. K-1; R is a
    [K, ny, nx//2+1] tensor of eigenvalues or a sequence of K floats."""
    if ens.dim() != 4 or not ens.is_cuda or not ens.is_contiguous():
        raise ValueError("ens must be a contiguous device tensor [N, M, ny, nx]")
    if data.dim() != 3 or not data.is_contiguous():
        raise ValueError("data must be a contiguous [K, ny, nx] tensor")
    N, M, ny, nx = ens.shape
    K = int(data.shape[0])
    code = _dtype_code(ens)
    if isinstance(R, torch.Tensor):
        R_t, r_arr = R, None
    else:
        R_t, r_arr = None, (ctypes.c_double * K)(*[float(x) for x in R])
    if workspace is None:
        need = int(lib().fftenkf_workspace_bytes_morph(N, M, K, ny, nx, code))
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=ens.device)
    e = Ens(n_members=N, ny=ny, nx=nx, dtype=code, members=ens.data_ptr(), workspace=workspace.data_ptr(),
            workspace_bytes=workspace.numel(), stream=torch.cuda.current_stream(ens.device).cuda_stream,
            r_scalar=0.0)
    if out is None:
        out = torch.empty_like(ens)
    st = lib().fftenkf_analyze_morph(ctypes.byref(e), M, K, data.data_ptr(), _ptr(R_t), r_arr,
                                     ctypes.c_uint64(seed & (2**64 - 1)), out.data_ptr())
    _check(st, "fftenkf_analyze_morph")
    return out


def _dst_ens(ens: torch.Tensor, workspace: Optional[torch.Tensor], r_scalar: float):
    if ens.dim() != 3 or not ens.is_cuda or not ens.is_contiguous():
        raise ValueError("ens must be a contiguous device tensor [N, ny, nx]")
    N, ny, nx = ens.shape
    code = _dtype_code(ens)
    if workspace is None:
        need = int(lib().fftenkf_workspace_bytes_dst(N, ny, nx, code))
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=ens.device)
    e = Ens(n_members=N, ny=ny, nx=nx, dtype=code, members=ens.data_ptr(), workspace=workspace.data_ptr(),
            workspace_bytes=workspace.numel(), stream=torch.cuda.current_stream(ens.device).cuda_stream,
            r_scalar=float(r_scalar))
    return e, workspace


def analyze_dst(ens: torch.Tensor, data: torch.Tensor, R_dst: Union[torch.Tensor, float], seed: int,
                out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The analysis in the real sine basis: R_dst [ny, nx] (eigenvalues of R in that basis) or a float r."""
    R_t, r = _rspec(R_dst)
    e, ws = _dst_ens(ens, workspace, r)
    if out is None:
        out = torch.empty_like(ens)
    st = lib().fftenkf_analyze_dst(ctypes.byref(e), data.data_ptr(), _ptr(R_t), ctypes.c_uint64(seed & (2**64 - 1)),
                                   out.data_ptr())
    _check(st, "fftenkf_analyze_dst")
    return out


def debug_dst_coeffs(ens: torch.Tensor, data: torch.Tensor) -> torch.Tensor:
    """Orthonormal sine coefficients [N+1, ny, nx] of the members and d."""
    e, ws = _dst_ens(ens, None, 0.0)
    N, ny, nx = ens.shape
    out = torch.empty((N + 1, ny, nx), dtype=ens.dtype, device=ens.device)
    _check(lib().fftenkf_debug_dst_coeffs(ctypes.byref(e), data.data_ptr(), out.data_ptr()), "fftenkf_debug_dst_coeffs")
    return out


def analyze_spectrum(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float], seed: int,
                     lam: torch.Tensor, out: Optional[torch.Tensor] = None,
                     workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Eq. (3) with prescribed covariance eigenvalues lam [ny, nx//2+1] (unitary scale) in place of eq. (2)."""
    R_t, r = _rspec(R_spec)
    e, ws = _make_ens(ens, workspace, r)
    N, ny, nx = ens.shape
    if tuple(lam.shape) != (ny, nx // 2 + 1) or lam.dtype != ens.dtype or not lam.is_contiguous():
        raise ValueError("lam must be a contiguous [ny, nx//2+1] tensor of the ensemble's dtype")
    if out is None:
        out = torch.empty_like(ens)
    st = lib().fftenkf_analyze_spectrum(ctypes.byref(e), data.data_ptr(), _ptr(R_t),
                                        ctypes.c_uint64(seed & (2**64 - 1)), lam.data_ptr(), out.data_ptr())
    _check(st, "fftenkf_analyze_spectrum")
    return out


def debug_spectra(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float],
                  with_spectra: bool = True):
    """(c_hat, gain, spectra) per bin, spectra = unitary half spectra of members then d."""
    R_t, r = _rspec(R_spec)
    e, ws = _make_ens(ens, None, r)
    N, ny, nx = ens.shape
    nh = nx // 2 + 1
    c_hat = torch.empty((ny, nh), dtype=ens.dtype, device=ens.device)
    gain = torch.empty_like(c_hat)
    spec = torch.empty((N + 1, ny, nh, 2), dtype=ens.dtype, device=ens.device) if with_spectra else None
    st = lib().fftenkf_debug_spectra(ctypes.byref(e), data.data_ptr(), _ptr(R_t), c_hat.data_ptr(), gain.data_ptr(),
                                     _ptr(spec))
    _check(st, "fftenkf_debug_spectra")
    return c_hat, gain, spec


def debug_perturb(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float], seed: int):
    """Unitary spectral perturbations e_hat [N, ny, nx//2+1, 2] drawn for `seed`."""
    R_t, r = _rspec(R_spec)
    e, ws = _make_ens(ens, None, r)
    N, ny, nx = ens.shape
    out = torch.empty((N, ny, nx // 2 + 1, 2), dtype=ens.dtype, device=ens.device)
    st = lib().fftenkf_debug_perturb(ctypes.byref(e), data.data_ptr(), _ptr(R_t),
                                     ctypes.c_uint64(seed & (2**64 - 1)), out.data_ptr())
    _check(st, "fftenkf_debug_perturb")
    return out


def mlp_weights(weights: dict, device) -> dict:
    """Device float32 copies of the perceptron's weights (W1 [26, 64] .. b4 [1])."""
    out = {}
    for name, shape in MLP_SHAPES.items():
        t = torch.as_tensor(weights[name], dtype=torch.float32).reshape(shape)
        out[name] = t.to(device).contiguous()
    return out


def _mlp_struct(w: dict) -> Mlp:
    for name, shape in MLP_SHAPES.items():
        t = w[name]
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"mlp weight {name} must be a contiguous float32 device tensor of shape {shape}")
    return Mlp(**{name: w[name].data_ptr() for name in MLP_SHAPES})


def analyze_learned(ens: torch.Tensor, data: torch.Tensor, R_spec: Union[torch.Tensor, float], seed: int,
                    weights: dict, out: Optional[torch.Tensor] = None,
                    workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Eq. (3) with the perceptron's lambda_hat in place of c_hat (float32); weights from mlp_weights."""
    R_t, r = _rspec(R_spec)
    e, ws = _make_ens(ens, workspace, r)
    m = _mlp_struct(weights)
    if out is None:
        out = torch.empty_like(ens)
    st = lib().fftenkf_analyze_learned(ctypes.byref(e), data.data_ptr(), _ptr(R_t),
                                       ctypes.c_uint64(seed & (2**64 - 1)), ctypes.byref(m), out.data_ptr())
    _check(st, "fftenkf_analyze_learned")
    return out


def debug_learned_spectrum(ens: torch.Tensor, data: torch.Tensor, weights: dict):
    """(c_hat, lambda_hat, mu): the sample spectrum, the perceptron's estimate and the mean of c_hat."""
    e, ws = _make_ens(ens, None, 0.0)
    m = _mlp_struct(weights)
    N, ny, nx = ens.shape
    c_hat = torch.empty((ny, nx // 2 + 1), dtype=torch.float32, device=ens.device)
    lam = torch.empty_like(c_hat)
    mu = torch.empty(1, dtype=torch.float32, device=ens.device)
    st = lib().fftenkf_debug_learned_spectrum(ctypes.byref(e), data.data_ptr(), ctypes.byref(m), c_hat.data_ptr(),
                                              lam.data_ptr(), mu.data_ptr())
    _check(st, "fftenkf_debug_learned_spectrum")
    return c_hat, lam, mu


def debug_rfft2(ens: torch.Tensor) -> torch.Tensor:
    """Unitary half spectra [N, ny, nx//2+1, 2] of the fields ens [N, ny, nx] (the library's forward transform)."""
    e, ws = _make_ens(ens, None, 0.0)
    N, ny, nx = ens.shape
    out = torch.empty((N, ny, nx // 2 + 1, 2), dtype=ens.dtype, device=ens.device)
    _check(lib().fftenkf_debug_fft2(ctypes.byref(e), 0, None, out.data_ptr()), "fftenkf_debug_fft2")
    return out


def debug_irfft2(spectra: torch.Tensor, nx: int) -> torch.Tensor:
    """Real fields [N, ny, nx] from unitary half spectra [N, ny, nx//2+1, 2] (the library's inverse transform)."""
    if spectra.dim() != 4 or spectra.shape[-1] != 2 or spectra.shape[2] != nx // 2 + 1 or not spectra.is_contiguous():
        raise ValueError("spectra must be a contiguous [N, ny, nx//2+1, 2] tensor")
    N, ny = spectra.shape[:2]
    out = torch.empty((N, ny, nx), dtype=spectra.dtype, device=spectra.device)
    e, ws = _make_ens(out, None, 0.0)
    _check(lib().fftenkf_debug_fft2(ctypes.byref(e), 1, spectra.data_ptr(), out.data_ptr()), "fftenkf_debug_fft2")
    return out


def tile_rows_options(ny: int, nx: int, dtype: torch.dtype) -> list:
    code = F32 if dtype == torch.float32 else F64
    buf = (ctypes.c_int * 8)()
    n = lib().fftenkf_tile_rows_options(ny, nx, code, buf, 8)
    return [int(buf[i]) for i in range(min(n, 8))]


def set_tile_rows(ny: int, nx: int, dtype: torch.dtype, rows: int) -> None:
    code = F32 if dtype == torch.float32 else F64
    _check(lib().fftenkf_set_tile_rows(ny, nx, code, rows), "fftenkf_set_tile_rows")


def tile_rows(ny: int, nx: int, dtype: torch.dtype) -> int:
    return int(lib().fftenkf_tile_rows(ny, nx, F32 if dtype == torch.float32 else F64))


class Batch:
    """Independent analyses of uneven grids (fftenkf_analyze_batch), with the
    device buffers for them: inputs [N, ny, nx] per filter, one workspace slab
    cut into per-filter pieces, outputs.  `run()` enqueues the whole batch on
    the current stream; `capture()` records it into a graph that `replay()`
    runs again on the same buffers."""

    def __init__(self, ens: list, data: list, R: list, seeds: list, out: Optional[list] = None):
        if not (len(ens) == len(data) == len(R) == len(seeds)):
            raise ValueError("ens, data, R and seeds need one entry per filter")
        self.ens, self.data, self.R, self.seeds = ens, data, R, seeds
        self.N = int(ens[0].shape[0])
        self.dtype = ens[0].dtype
        code = _dtype_code(ens[0])
        self.out = out if out is not None else [torch.empty_like(e) for e in ens]
        sizes = [(workspace_bytes(self.N, e.shape[1], e.shape[2], self.dtype) + 255) // 256 * 256 for e in ens]
        self.workspace = torch.empty(max(sum(sizes), 256), dtype=torch.uint8, device=ens[0].device)
        base, off = self.workspace.data_ptr(), 0
        arr = (Filter * len(ens))()
        for i, e in enumerate(ens):
            if e.dim() != 3 or not e.is_cuda or not e.is_contiguous() or e.dtype != self.dtype or e.shape[0] != self.N:
                raise ValueError(f"filter {i}: ens must be a contiguous [N, ny, nx] device tensor like the others")
            R_t, r = _rspec(R[i])
            arr[i] = Filter(ny=e.shape[1], nx=e.shape[2], members=e.data_ptr(), data=data[i].data_ptr(),
                            R_spec=_ptr(R_t), out=self.out[i].data_ptr(), workspace=base + off,
                            workspace_bytes=sizes[i], r_scalar=float(r), seed=seeds[i] & (2**64 - 1))
            off += sizes[i]
        self._filters = arr
        self._code = code
        self.graph = None

    def run(self) -> list:
        st = lib().fftenkf_analyze_batch(self.N, self._code, self._filters, len(self._filters),
                                         torch.cuda.current_stream(self.ens[0].device).cuda_stream)
        _check(st, "fftenkf_analyze_batch")
        return self.out

    def capture(self) -> None:
        """Record the batch into a HIP graph (after one eager run, which sets up
        the library's tables and kernel attributes outside the capture)."""
        self.run()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(self.graph, stream=s):
                self.run()
        torch.cuda.current_stream().wait_stream(s)

    def replay(self) -> list:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self.out


def debug_fail_next(status: int) -> None:
    lib().fftenkf_debug_fail_next(status)


def profile_events(events) -> None:
    """Record the 4 given hipEvent_t handles around the sweeps of the next analyze."""
    if not events:
        _check(lib().fftenkf_profile_events(None, 0), "fftenkf_profile_events")
        return
    arr = (ctypes.c_void_p * len(events))(*events)
    _check(lib().fftenkf_profile_events(arr, len(events)), "fftenkf_profile_events")
