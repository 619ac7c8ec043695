"""The C-ABI library loads, exports what include/fftenkf.h declares, and rejects
bad arguments before touching the GPU (these run without a device)."""

import ctypes
import os
import re

import pytest

from paper_1001_1588_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftenkf.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(fftenkf_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fftenkf_analyze", "fftenkf_workspace_bytes", "fftenkf_strerror", "fftenkf_last_error",
                 "fftenkf_debug_spectra", "fftenkf_debug_perturb"):
        assert must in names


def test_library_exports_every_declared_symbol(built_lib):
    lib = ctypes.CDLL(built_lib)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTS) == set(declared_functions())


def _ens(**kw):
    d = dict(n_members=4, ny=16, nx=16, dtype=_lib.F32, members=0x100000, workspace=0x800000,
             workspace_bytes=1 << 20, stream=None, r_scalar=0.05)
    d.update(kw)
    return _lib.Ens(**d)


def call(e, data=0x200000, R=None, out=0x300000):
    lib = _lib.lib()
    return lib.fftenkf_analyze(ctypes.byref(e) if e is not None else None, data, R, 1, out)


@pytest.mark.parametrize("kw,status", [
    (dict(dtype=2), _lib.EINVAL),
    (dict(n_members=1), _lib.EINVAL),
    (dict(n_members=0), _lib.EINVAL),
    (dict(ny=12), _lib.EUNSUPPORTED),
    (dict(nx=4), _lib.EUNSUPPORTED),
    (dict(nx=8192), _lib.EUNSUPPORTED),
    (dict(ny=0), _lib.EUNSUPPORTED),
    (dict(n_members=25), _lib.EUNSUPPORTED),
    (dict(n_members=9, dtype=_lib.F64), _lib.EUNSUPPORTED),
    (dict(members=None), _lib.EINVAL),
    (dict(workspace=None), _lib.EINVAL),
    (dict(workspace_bytes=1000), _lib.EINVAL),
    (dict(members=0x100008), _lib.EINVAL),
    (dict(workspace=0x800010), _lib.EINVAL),
], ids=lambda v: str(v))
def test_validation_errors(built_lib, kw, status):
    assert call(_ens(**kw)) == status
    assert _lib.lib().fftenkf_last_error().decode()


def test_null_descriptor_and_buffers(built_lib):
    assert call(None) == _lib.EINVAL
    assert call(_ens(), data=None) == _lib.EINVAL
    assert call(_ens(), out=None) == _lib.EINVAL
    assert call(_ens(), out=0x300004) == _lib.EINVAL                   # misaligned
    assert call(_ens(r_scalar=-1.0)) == _lib.EINVAL                    # negative R without R_spec
    assert call(_ens(r_scalar=float("nan"))) == _lib.EINVAL


def test_partial_overlap_rejected(built_lib):
    field = 16 * 16 * 4
    assert call(_ens(), out=0x100000 + field) == _lib.EINVAL            # out overlaps members, not equal
    assert call(_ens(), data=0x800000 + 256) == _lib.EINVAL              # data inside the workspace
    assert call(_ens(), R=0x200000 + 64) == _lib.EINVAL                  # R_spec overlaps data
    assert call(_ens(workspace=0x100000 + 256)) == _lib.EINVAL          # workspace overlaps members


def _mlp(**kw):
    d = {name: 0x900000 + 0x10000 * i for i, name in enumerate(_lib.MLP_SHAPES)}
    d.update(kw)
    return _lib.Mlp(**d)


def call_learned(e, mlp, data=0x200000, out=0x300000):
    lib = _lib.lib()
    return lib.fftenkf_analyze_learned(ctypes.byref(e), data, None, 1, ctypes.byref(mlp) if mlp is not None else None,
                                       out)


def test_learned_validation(built_lib):
    assert call_learned(_ens(), None) == _lib.EINVAL
    assert call_learned(_ens(dtype=_lib.F64), _mlp()) == _lib.EUNSUPPORTED
    assert call_learned(_ens(), _mlp(W2=None)) == _lib.EINVAL
    assert "W2" in _lib.lib().fftenkf_last_error().decode()
    assert call_learned(_ens(), _mlp(b4=0x900002)) == _lib.EINVAL          # misaligned
    assert call_learned(_ens(n_members=25), _mlp()) == _lib.EUNSUPPORTED
    lib = _lib.lib()
    e = _ens()
    assert lib.fftenkf_debug_learned_spectrum(ctypes.byref(e), 0x200000, None, 0x300000, 0x400000,
                                              0x500000) == _lib.EINVAL
    e64 = _ens(dtype=_lib.F64)
    assert lib.fftenkf_debug_learned_spectrum(ctypes.byref(e64), 0x200000, ctypes.byref(_mlp()), 0x300000,
                                              0x400000, 0x500000) == _lib.EUNSUPPORTED


def test_workspace_formula(built_lib):
    lib = _lib.lib()
    for (N, ny, nx, dt, s) in [(20, 2048, 2048, 0, 4), (5, 64, 64, 1, 8), (2, 8, 8, 0, 4), (24, 4096, 4096, 0, 4)]:
        nh = nx // 2 + 1
        r256 = lambda b: (b + 255) // 256 * 256  # noqa: E731
        # spectra of the N+1 fields (kx < nx/2: the Nyquist column is folded into
        # kx = 0), then c_hat and lambda_hat planes, then one float per unit
        R = min(ny, (16 if nx <= 2048 else 8) if dt == 0 else (8 if nx <= 2048 else 4))
        L = ny // R
        C = min(nx // 2, 256 // (L // min(4, L)))
        units = R * (nx // 2 // C)
        raw = r256(r256(r256((N + 1) * ny * (nx // 2) * 2 * s) + ny * nh * s) + ny * nh * s) + 4 * units
        assert lib.fftenkf_workspace_bytes(N, ny, nx, dt) == r256(raw)
    assert lib.fftenkf_workspace_bytes(1, 8, 8, 0) == 0
    assert lib.fftenkf_workspace_bytes(4, 8, 12, 0) == 0
    assert lib.fftenkf_workspace_bytes(4, 8, 8, 3) == 0
    assert lib.fftenkf_max_members(0) == 24 and lib.fftenkf_max_members(1) == 8


def test_strerror(built_lib):
    lib = _lib.lib()
    assert lib.fftenkf_strerror(0) == b"success"
    assert lib.fftenkf_strerror(-2) == b"unsupported shape"
    assert lib.fftenkf_strerror(7) == b"unknown status"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_profile_events_arguments(built_lib):
    lib = _lib.lib()
    arr = (ctypes.c_void_p * 6)(*([0x1000] * 6))
    assert lib.fftenkf_profile_events(arr, 5) == _lib.EINVAL
    assert lib.fftenkf_profile_events(None, 4) == _lib.EINVAL
    nulls = (ctypes.c_void_p * 6)()
    assert lib.fftenkf_profile_events(nulls, 6) == _lib.EINVAL
    assert lib.fftenkf_profile_events(None, 0) == _lib.OK


def test_release_caches_and_fft2_arguments(built_lib):
    lib = _lib.lib()
    assert lib.fftenkf_release_caches() == _lib.OK
    e = _ens()
    assert lib.fftenkf_debug_fft2(ctypes.byref(e), 2, None, 0x300000) == _lib.EINVAL       # direction
    assert lib.fftenkf_debug_fft2(ctypes.byref(e), 0, None, None) == _lib.EINVAL           # no output
    assert lib.fftenkf_debug_fft2(ctypes.byref(e), 1, None, 0x300000) == _lib.EINVAL       # inverse needs spectra
    assert lib.fftenkf_debug_fft2(ctypes.byref(e), 0, None, 0x300008) == _lib.EINVAL       # misaligned
    assert lib.fftenkf_debug_fft2(ctypes.byref(e), 0, None, 0x100000 + 64) == _lib.EINVAL  # out overlaps members


def test_multi_validation_and_workspace(built_lib):
    lib = _lib.lib()
    e = _ens()
    call_m = lambda ens, M, **kw: lib.fftenkf_analyze_multi(ctypes.byref(ens), M, kw.get("data", 0x200000),  # noqa: E731
                                                            None, 1, kw.get("out", 0x300000))
    assert call_m(e, 0) == _lib.EINVAL
    assert call_m(e, 65) == _lib.EINVAL
    assert call_m(_ens(n_members=13), 2) == _lib.EUNSUPPORTED
    assert call_m(_ens(n_members=5, dtype=_lib.F64), 2) == _lib.EUNSUPPORTED
    assert call_m(_ens(ny=12), 2) == _lib.EUNSUPPORTED
    assert call_m(e, 2, out=0x100000 + 16 * 16 * 4 * 4) == _lib.EINVAL   # out overlaps members (N*M fields)
    assert lib.fftenkf_max_members_multi(0) == 12 and lib.fftenkf_max_members_multi(1) == 4
    # the multi-block workspace is that of an analysis with N * M members
    for (N, M, ny, nx, dt) in [(10, 4, 1024, 1024, 0), (3, 2, 16, 8, 1)]:
        assert lib.fftenkf_workspace_bytes_multi(N, M, ny, nx, dt) == lib.fftenkf_workspace_bytes(N * M, ny, nx, dt)
    assert lib.fftenkf_workspace_bytes_multi(4, 0, 16, 16, 0) == 0


def test_batch_validation_and_tuning(built_lib):
    lib = _lib.lib()
    f = _lib.Filter(ny=16, nx=16, members=0x100000, data=0x200000, R_spec=None, out=0x300000, workspace=0x800000,
                    workspace_bytes=1 << 20, r_scalar=0.01, seed=1)
    arr = (_lib.Filter * 2)(f, f)
    assert lib.fftenkf_analyze_batch(1, 0, arr, 1, None) == _lib.EINVAL         # N < 2
    assert lib.fftenkf_analyze_batch(4, 3, arr, 1, None) == _lib.EINVAL         # dtype
    assert lib.fftenkf_analyze_batch(25, 0, arr, 1, None) == _lib.EUNSUPPORTED
    assert lib.fftenkf_analyze_batch(4, 0, None, 1, None) == _lib.EINVAL
    assert lib.fftenkf_analyze_batch(4, 0, arr, 2, None) == _lib.EINVAL         # two filters write the same out
    assert "overlaps" in lib.fftenkf_last_error().decode()
    bad = _lib.Filter(ny=12, nx=16, members=0x100000, data=0x200000, R_spec=None, out=0x300000, workspace=0x800000,
                      workspace_bytes=1 << 20, r_scalar=0.01, seed=1)
    assert lib.fftenkf_analyze_batch(4, 0, (_lib.Filter * 1)(bad), 1, None) == _lib.EUNSUPPORTED
    assert lib.fftenkf_analyze_batch(4, 0, arr, 0, None) == _lib.OK             # nothing to do
    buf = (ctypes.c_int * 4)()
    assert lib.fftenkf_tile_rows_options(256, 256, 0, buf, 4) == 3 and list(buf[:3]) == [4, 8, 16]
    assert lib.fftenkf_tile_rows_options(8, 64, 0, buf, 4) == 2 and list(buf[:2]) == [4, 8]  # R <= ny
    assert lib.fftenkf_tile_rows_options(4096, 1024, 0, buf, 4) == 2 and list(buf[:2]) == [8, 16]  # ny / R <= 512
    assert lib.fftenkf_tile_rows_options(64, 4096, 0, buf, 4) == 1 and buf[0] == 8
    assert lib.fftenkf_tile_rows(256, 256, 0) == 8 and lib.fftenkf_tile_rows(2048, 2048, 0) == 16
    assert lib.fftenkf_set_tile_rows(256, 256, 0, 16) == _lib.OK and lib.fftenkf_tile_rows(256, 256, 0) == 16
    assert lib.fftenkf_set_tile_rows(256, 256, 0, 0) == _lib.OK and lib.fftenkf_tile_rows(256, 256, 0) == 8
    assert lib.fftenkf_set_tile_rows(256, 256, 0, 32) == _lib.EUNSUPPORTED
    assert lib.fftenkf_set_tile_rows(4096, 1024, 0, 4) == _lib.EUNSUPPORTED      # a 1024-point transform
    assert lib.fftenkf_set_tile_rows(256, 256, 0, 4) == _lib.OK and lib.fftenkf_tile_rows(256, 256, 0) == 4
    assert lib.fftenkf_set_tile_rows(256, 256, 0, 0) == _lib.OK


def test_dst_validation(built_lib):
    lib = _lib.lib()
    e = _ens(workspace_bytes=1 << 30)
    assert lib.fftenkf_analyze_dst(ctypes.byref(e), None, None, 1, 0x300000) == _lib.EINVAL
    assert lib.fftenkf_analyze_dst(ctypes.byref(_ens(workspace_bytes=1000)), 0x200000, None, 1, 0x300000) == _lib.EINVAL
    assert lib.fftenkf_analyze_dst(ctypes.byref(_ens(ny=12)), 0x200000, None, 1, 0x300000) == _lib.EUNSUPPORTED
    e2 = _ens(workspace_bytes=1 << 30, r_scalar=-1.0)
    assert lib.fftenkf_analyze_dst(ctypes.byref(e2), 0x200000, None, 1, 0x300000) == _lib.EINVAL
    # the sine-basis analysis reorders inside sweeps 1 and 3: same workspace
    for (N, ny, nx, dt) in [(20, 2048, 2048, 0), (5, 64, 64, 1)]:
        assert lib.fftenkf_workspace_bytes_dst(N, ny, nx, dt) == lib.fftenkf_workspace_bytes(N, ny, nx, dt) > 0


@pytest.mark.parametrize("r,dtype,status", [
    (float("inf"), _lib.F32, _lib.EINVAL),
    (float("inf"), _lib.F64, _lib.EINVAL),
    (float("-inf"), _lib.F64, _lib.EINVAL),
    (1e39, _lib.F32, _lib.EINVAL),        # finite in double, infinite in float32
], ids=lambda v: str(v))
def test_non_finite_r_scalar_rejected_by_every_entry_point(built_lib, r, dtype, status):
    """R = r I needs r finite in the working precision: an infinite r gives an
    infinite perturbation amplitude where the gain is exactly 0 (0 * inf = NaN)."""
    lib = _lib.lib()
    e = _ens(r_scalar=r, dtype=dtype, n_members=4, workspace_bytes=1 << 30)
    assert call(e) == status
    assert "r_scalar" in lib.fftenkf_last_error().decode()
    assert lib.fftenkf_analyze_multi(ctypes.byref(e), 2, 0x200000, None, 1, 0x300000) == status
    assert lib.fftenkf_analyze_dst(ctypes.byref(e), 0x200000, None, 1, 0x300000) == status
    f = _lib.Filter(ny=16, nx=16, members=0x100000, data=0x200000, R_spec=None, out=0x300000, workspace=0x800000,
                    workspace_bytes=1 << 20, r_scalar=r, seed=1)
    assert lib.fftenkf_analyze_batch(4, dtype, (_lib.Filter * 1)(f), 1, None) == status
    assert "filter 0" in lib.fftenkf_last_error().decode()


def test_large_finite_r_scalar_accepted_by_validation(built_lib):
    """1e39 is finite in float64: validation passes it (the call then fails only
    because these fake pointers are not device memory)."""
    e = _ens(r_scalar=1e39, dtype=_lib.F64, workspace_bytes=1 << 30)
    assert call(e) != _lib.OK
    assert "r_scalar" not in _lib.lib().fftenkf_last_error().decode()


def test_noalloc_entry_point_limits(built_lib):
    """The entry point that allocates nothing: its static scratch is 64 MiB;
    shapes whose workspace exceeds it, and the usual shape errors, are rejected
    before any device call (these pointers are not device memory)."""
    lib = _lib.lib()
    assert lib.fftenkf_noalloc_max_bytes() == 64 << 20
    big = _ens(n_members=20, ny=2048, nx=2048, workspace=None, workspace_bytes=0)
    assert lib.fftenkf_analyze_noalloc(ctypes.byref(big), 0x200000, None, 1, 0x300000) == _lib.EINVAL
    assert "static scratch" in lib.fftenkf_last_error().decode()
    assert lib.fftenkf_analyze_noalloc(None, 0x200000, None, 1, 0x300000) == _lib.EINVAL
    bad = _ens(ny=12, workspace=None, workspace_bytes=0)
    assert lib.fftenkf_analyze_noalloc(ctypes.byref(bad), 0x200000, None, 1, 0x300000) == _lib.EUNSUPPORTED
    # the largest float32 member count that fits on a 1024 x 1024 grid is 13
    assert lib.fftenkf_workspace_bytes(13, 1024, 1024, 0) <= 64 << 20 < lib.fftenkf_workspace_bytes(14, 1024, 1024, 0)
