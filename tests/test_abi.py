"""The C ABI: the built library exports every entry point the header
declares, and host-side argument validation runs (and fails cleanly)
without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2003_06027_amd import cnn as N
from paper_2003_06027_amd import seisgrad as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    syms = set()
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", f)).read()
            syms |= set(re.findall(r"SG_API\s+[\w\s\*]+?\b(\w+)\s*\(", hdr))
    return sorted(syms)


def test_header_declares_the_paper_calls():
    syms = declared_symbols()
    for name in ("init_model", "forward_shots", "adjoint_gradient", "misfit"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(S.EXPORTS) | set(N.EXPORTS)


def test_workspace_bytes_validation_on_host():
    d = S.desc(nx=100, nz=50, npml=10, nt=100)
    n = S.workspace_bytes(d, 4, 100)
    assert n > 0
    # more shots or receivers never need less memory
    assert S.workspace_bytes(d, 8, 100) > n
    assert S.workspace_bytes(d, 4, 200) >= n
    bad = S.desc(nx=0, nz=50)
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(bad, 1, 1)
    assert "bad grid" in str(e.value)
    # physics / dimensions not provided by this build are reported as such
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(S.desc(ndim=4, nx=10, nz=10, ny=10), 1, 1)


def test_size_limits_on_host():
    """The largest grids the kernels' index arithmetic supports are accepted,
    one step beyond is refused with a message (no GPU needed)."""
    # 3-D: a z chunk and its window planes must stay below 4 GiB of byte offsets
    ok = S.desc(ndim=3, nx=3500, ny=3500, nz=64, npml=0, nt=10)
    assert S.workspace_bytes(ok, 1, 1) > 0
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(S.desc(ndim=3, nx=4000, ny=4000, nz=64, npml=0, nt=10), 1, 1)
    assert "planes" in str(e.value)        # workspace_bytes returns 0; the message names the limit
    # 3-D: 12-bit plane field of the receiver sort key
    assert S.workspace_bytes(S.desc(ndim=3, nx=8, ny=8, nz=4095, npml=0, nt=10), 1, 1) > 0
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(S.desc(ndim=3, nx=8, ny=8, nz=4000, npml=48, nt=10), 1, 1)
    assert "padded planes in z" in str(e.value)
    # receivers per shot: 20-bit receiver ids
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(S.desc(nx=100, nz=50, npml=10, nt=10), 1, 1 << 20)
    assert "receivers" in str(e.value)
    assert S.workspace_bytes(S.desc(nx=100, nz=50, npml=10, nt=10), 1, (1 << 20) - 1) > 0
    # elastic: the adjoint passes take the shot as the grid's y index, the
    # forward passes number their cell blocks over all shots with an int
    el = S.desc(physics=S.SG_ELASTIC, nx=100, nz=50, npml=10, nt=10)
    assert S.workspace_bytes(el, 65535, 1) > 0
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(el, 65536, 1)
    assert "too many elastic shots" in str(e.value)
    # 625 x 2500 blocks of 32 x 8 or 313 x 5000 blocks of 64 x 4 per shot: the larger count bounds
    big = S.desc(physics=S.SG_ELASTIC, nx=20000, nz=20000, nt=10)
    assert S.workspace_bytes(big, 1372, 1) > 0
    with pytest.raises(S.SeisError) as e:
        S.workspace_bytes(big, 1373, 1)
    assert "too many elastic shots" in str(e.value)


def test_init_model_rejects_null_arguments_without_gpu():
    d = S.desc(nx=100, nz=50, npml=10, nt=100)
    h = C.c_void_p()
    rc = S.lib().init_model(C.byref(d), None, None, None, 1, 10, 0, None, 0, None, C.byref(h))
    assert rc == S.SG_EINVAL
    assert b"device pointers" in S.lib().last_error()
    rc = S.lib().init_model(None, None, None, None, 1, 10, 0, None, 0, None, C.byref(h))
    assert rc == S.SG_EINVAL


def test_misfit_and_adjoint_reject_bad_arguments_without_gpu():
    assert S.lib().misfit(None, None, None, 10, None, None, None) == S.SG_EINVAL
    assert S.lib().forward_shots(None, None, None, 1, None) == S.SG_EINVAL
    assert S.lib().adjoint_gradient(None, None, None, None, None, None, None, None) == S.SG_EINVAL
    assert S.lib().ricker(10.0, 0.1, 1e-3, 0, None, None) == S.SG_EINVAL


def test_cnn_entry_points_validate_on_host():
    L = N.lib()
    assert L.cnn_workspace_bytes(0, 4, 4) == 0
    assert L.cnn_workspace_bytes(2, 256, 256) > 8 * 2 * 256 * 256 * 64
    assert L.cnn_forward(None, None, 1, 8, 8, None, None, 0, None) == S.SG_EINVAL
    assert L.cnn_forward(None, None, 0, 8, 8, None, None, 0, None) == S.SG_EINVAL
    assert b"positive" in L.last_error()
    assert L.cnn_pack(None, None, 1, None, 1, 5, 5, 4, 1, None, None, None, None) == S.SG_EINVAL
    assert L.cnn_adam(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None) == S.SG_EINVAL
    assert L.cnn_conv3x3(None, 1, 4, 4, None, None, None, None, 0, None, None, None) == S.SG_EINVAL
    # the epilogue's 16-byte accesses: a misaligned output, residual or gate is refused before any launch
    # (the addresses below are never dereferenced)
    for res, gate, y, y32 in ((None, None, 4096 + 2, None), (4096 + 8, None, 4096, None),
                              (None, 4096 + 4, 4096, None), (None, None, 4096, 4096 + 12)):
        assert L.cnn_conv3x3(4096, 1, 4, 4, 4096, None, res, gate, 0, y, y32, None) == S.SG_EINVAL
        assert b"16-byte aligned" in L.last_error()
    assert L.cnn_conv3x3(4096, 1, 1 << 15, 1 << 14, 4096, None, None, None, 0, 4096, None, None) == S.SG_EINVAL
    assert b"too large" in L.last_error()
