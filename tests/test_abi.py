"""The C-ABI library loads, exports every declared entry point, and validates
its arguments on the host (no device work: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plcg.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(plcg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1905_06850_amd import plcg
    lib = ctypes.CDLL(plcg.LIB_PATH)
    names = _declared()
    assert "plcg_solve" in names and "plcg_create" in names and "plcg_poll" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(plcg.SYMBOLS)


def test_version():
    from paper_1905_06850_amd import plcg
    assert plcg.plcg_version() >= 100


def _create(kind=1, nx=8, ny=8, nz=1, method=1, l=2, lmin=0.0, lmax=8.0):
    from paper_1905_06850_amd import plcg
    desc = plcg.plcg_operator_desc(kind, nx, ny, nz)
    cfg = plcg.plcg_config(method, l, lmin, lmax, None, 0, -1, 0)
    h = ctypes.c_void_p()
    st = plcg.plcg_create(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kwargs", [
    dict(kind=7), dict(nx=0), dict(ny=-3), dict(kind=2, nz=0), dict(kind=1, nz=4),
    dict(l=0), dict(l=9), dict(method=5), dict(lmin=1.0, lmax=1.0), dict(lmin=3.0, lmax=2.0),
    dict(nx=65536, ny=65536), dict(kind=3), dict(kind=4),
])
def test_create_rejects_bad_arguments(kwargs):
    from paper_1905_06850_amd import plcg
    st, h = _create(**kwargs)
    assert st == plcg.PLCG_E_INVALID
    assert not h.value
    assert plcg.plcg_last_error()


def test_null_arguments():
    from paper_1905_06850_amd import plcg
    assert plcg.plcg_create(None, None, None) == plcg.PLCG_E_INVALID
    res = plcg.plcg_result()
    assert plcg.plcg_solve(None, 0, 0, 1e-8, 10, None, ctypes.byref(res)) == plcg.PLCG_E_INVALID
    assert plcg.plcg_poll(None, 1, ctypes.byref(res)) == plcg.PLCG_E_INVALID
    assert plcg.plcg_apply(None, 0, 0, None) == plcg.PLCG_E_INVALID
    assert plcg.plcg_copy(0, 0, 10, None) == plcg.PLCG_E_INVALID
    assert plcg.plcg_destroy(None) == plcg.PLCG_OK
    assert plcg.plcg_size(None) == -1


def test_jacobi_flag_needs_a_csr_operator():
    from paper_1905_06850_amd import plcg
    desc = plcg.plcg_operator_desc(1, 8, 8, 1, None, 0, None, None, None, 1)
    cfg = plcg.plcg_config(1, 2, 0.0, 8.0, None, 0, -1, 0)
    h = ctypes.c_void_p()
    assert plcg.plcg_create(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(h)) == \
        plcg.PLCG_E_INVALID
    assert not h.value


def test_resident_support_table():
    """Which systems the one-workgroup kernels take: up to PLCG_RESIDENT_MAX
    unknowns, p(l)-CG spread over 960 threads with the widths that fit the
    registers (stencils: 5 unknowns per thread up to l = 2, 3 at l = 3, 2 at
    l = 4, 1 beyond; CSR narrower), CG over 1024 threads."""
    from paper_1905_06850_amd import plcg
    sup = plcg.resident_supported
    assert plcg.PLCG_RESIDENT_MAX == 4800
    for kind in ("2d5", "3d7", "diag", "csr"):
        assert sup(kind, 1, "plcg", 8) and sup(kind, 960, "plcg", 8)
        assert not sup(kind, 961, "plcg", 8)
        assert sup(kind, 4800, "cg") and not sup(kind, 4801, "cg")
        assert not sup(kind, 0, "cg")
    assert sup("2d5", 4800, "plcg", 2) and not sup("2d5", 4800, "plcg", 3)
    assert sup("2d5", 2880, "plcg", 3) and not sup("2d5", 2881, "plcg", 3)
    assert sup("3d7", 2880, "plcg", 3) and not sup("3d7", 2881, "plcg", 3)
    assert sup("2d5", 1920, "plcg", 4) and not sup("2d5", 1921, "plcg", 4)
    assert sup("csr", 3840, "plcg", 1) and not sup("csr", 3841, "plcg", 1)
    assert not sup("2d5", 961, "plcg", 5) and not sup(9, 10, "cg")
    assert not sup("2d5", 10, "plcg", 0) and not sup("2d5", 10, "plcg", 9)


@pytest.mark.parametrize("nx,ny,method,l,precision", [(61, 80, 1, 1, 0), (64, 64, 1, 3, 0),
                                                      (64, 64, 1, 1, 1), (8, 8, 1, 2, 1)])
def test_create_rejects_resident_where_unavailable(nx, ny, method, l, precision):
    from paper_1905_06850_amd import plcg
    desc = plcg.plcg_operator_desc(1, nx, ny, 1)
    cfg = plcg.plcg_config(method, l, 0.0, 8.0, None, 0, -1, 0, precision, 0.0,
                           plcg.PLCG_LAUNCH_RESIDENT)
    h = ctypes.c_void_p()
    assert plcg.plcg_create(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(h)) == \
        plcg.PLCG_E_INVALID
    assert not h.value
    cfg.launch_mode = 7
    assert plcg.plcg_create(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(h)) == \
        plcg.PLCG_E_INVALID


def test_create_rejects_unknown_x_update():
    from paper_1905_06850_amd import plcg
    desc = plcg.plcg_operator_desc(1, 64, 64, 1)
    assert plcg.X_UPDATES == {"auto": 0, "every": 1, "paired": 2}
    for xu in (-1, 3):
        cfg = plcg.plcg_config(1, 2, 0.0, 8.0, None, 0, -1, 0, 0, 0.0, 0, xu)
        h = ctypes.c_void_p()
        assert plcg.plcg_create(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(h)) == \
            plcg.PLCG_E_INVALID
        assert not h.value


@pytest.mark.parametrize("kind,nx,ny,nz,l,hist", [
    (3, 8, 8, 1, 2, 0), (4, 8, 8, 1, 2, 0),     # diagonal / CSR: need library copies
    (1, 8, 8, 1, 2, 16),                        # history needs a handle
    (1, 8, 8, 1, 9, 0), (1, 0, 8, 1, 2, 0),     # the checks of plcg_create
    (1, 2048, 2048, 1, 1, 0),                   # 6 vectors of 32 MiB: beyond the array
    (2, 256, 256, 256, 3, 0),
])
def test_noalloc_rejects_before_device_work(kind, nx, ny, nz, l, hist):
    """plcg_solve_noalloc refuses what it cannot do before touching the device
    (so this runs without a GPU), with a message; the size limit names the
    bytes the system would need."""
    from paper_1905_06850_amd import plcg
    desc = plcg.plcg_operator_desc(kind, nx, ny, nz)
    cfg = plcg.plcg_config(1, l, 0.0, 8.0, None, 0, -1, hist)
    res = plcg.plcg_result()
    st = plcg.plcg_solve_noalloc(ctypes.byref(desc), ctypes.byref(cfg), 16, 32, 1e-8, 10, None,
                                 ctypes.byref(res))
    assert st == plcg.PLCG_E_INVALID
    msg = plcg.plcg_last_error()
    assert msg
    if nx == 2048 or nz == 256:
        assert b"bytes" in msg and str(plcg.PLCG_NOALLOC_BYTES).encode() in msg
    assert plcg.plcg_solve_noalloc(None, None, 0, 0, 1e-8, 10, None, None) == plcg.PLCG_E_INVALID


@pytest.mark.parametrize("kind,nz,coef,jacobi", [
    (1, 1, (16, None, None), 0),        # cy missing
    (2, 4, (16, 32, None), 0),          # cz missing in 3D
    (1, 1, (None, 32, None), 0),        # cy without cx
    (4, 1, (16, 32, None), 0),          # coefficients on a diagonal operator
    (1, 1, (None, None, None), 1),      # Jacobi scaling of the constant stencil
])
def test_create_rejects_bad_edge_coefficients(kind, nz, coef, jacobi):
    """Descriptor checks of the variable-coefficient stencil made before any
    device access (the addresses are never read)."""
    from paper_1905_06850_amd import plcg
    desc = plcg.plcg_operator_desc(kind, 8, 8, nz, 64 if kind == plcg.PLCG_OP_DIAG else None, 0,
                                   None, None,
                                   None, jacobi, *coef)
    cfg = plcg.plcg_config(1, 2, 0.0, 2.0, None, 0, -1, 0)
    h = ctypes.c_void_p()
    assert plcg.plcg_create(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(h)) == \
        plcg.PLCG_E_INVALID
    assert not h.value
    assert plcg.plcg_last_error()


def test_struct_layouts_match_the_header(tmp_path):
    """Every structure of include/plcg.h has the size and field offsets of its
    ctypes mirror in the binding (a plain C program built with the host
    compiler prints them)."""
    import shutil
    import subprocess
    from paper_1905_06850_amd import plcg
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    exe = tmp_path / "abi_layout"
    src = os.path.join(ROOT, "tests", "c", "abi_layout.c")
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    seen = set()
    for line in out.splitlines():
        parts = line.split()
        cls = getattr(plcg, parts[0])
        seen.add(parts[0])
        if parts[1] == "size":
            assert ctypes.sizeof(cls) == int(parts[2]), line
        else:
            assert getattr(cls, parts[1]).offset == int(parts[2]), line
    assert seen == {"plcg_operator_desc", "plcg_config", "plcg_result", "plcg_batch_config",
                    "plcg_system_desc", "plcg_request", "plcg_request_outcome"}
