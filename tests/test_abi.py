"""The C ABI library: it loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "matprobe.h")
LIB = os.path.join(ROOT, "paper_1101_3615_amd", "libmatprobe.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mp_[a-zA-Z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: python -m paper_1101_3615_amd.build"
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings_without_device():
    lib = ctypes.CDLL(LIB)
    lib.mp_strerror.restype = ctypes.c_char_p
    assert lib.mp_strerror(0) == b"ok"
    assert lib.mp_strerror(-2).startswith(b"out of device memory")
    assert lib.mp_strerror(-99) == b"unknown error"
    # argument validation happens before any device call
    lib.mp_last_error.restype = ctypes.c_char_p
    assert lib.mp_create(None, None, None, None) == -1
    assert b"null" in lib.mp_last_error()


def test_python_binding_imports_without_device():
    import paper_1101_3615_amd as M
    assert callable(M.probe_fit) and callable(M.apply_Hinv)
    from paper_1101_3615_amd._lib import EXPORTS
    assert set(EXPORTS) <= set(declared())


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: without the built library the binding raises before any compute."""
    from paper_1101_3615_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libmatprobe.so"))
    with pytest.raises(RuntimeError, match="is missing"):
        _lib.lib()


def test_create_rejects_grids_past_the_32_bit_offset_limit():
    """mp_create refuses a grid whose padded wavefield slice or FP64 image reaches 1 GiB (the
    sweeps address them with 32-bit buffer offsets) before any device call; the same call with
    a small grid gets past that check (and fails later only for want of a GPU here)."""
    import numpy as np
    from paper_1101_3615_amd import _lib as L
    lib = ctypes.CDLL(LIB)
    lib.mp_last_error.restype = ctypes.c_char_p
    src = np.zeros((1, 3), dtype=np.int32)
    rec = np.array([[1, 0, 0]], dtype=np.int32)
    a = L.Acq(1, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 1,
              rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), 10.0, 0.1, 1e-3, 10)
    o = L.Opts(1, 0, 1, 0, 1e-3, 0)   # MP_F32, MP_SNAP_FULL
    ctx = ctypes.c_void_p()
    big = L.Grid(3, (ctypes.c_int * 3)(640, 640, 640), 10.0, 20)
    assert lib.mp_create(ctypes.byref(big), ctypes.byref(a), ctypes.byref(o), ctypes.byref(ctx)) == -1
    assert b"too large" in lib.mp_last_error()
    small = L.Grid(3, (ctypes.c_int * 3)(64, 64, 64), 10.0, 20)
    lib.mp_create(ctypes.byref(small), ctypes.byref(a), ctypes.byref(o), ctypes.byref(ctx))
    assert b"too large" not in lib.mp_last_error()


def test_basis_descriptor_validation_without_device():
    """mp_basis_create checks the descriptor on the host: the Fourier-angular family
    (Sec. 1.2) needs its tables, a positive TL scale, bounded orders, indices and modes."""
    import numpy as np
    from paper_1101_3615_amd import _lib as L
    lib = ctypes.CDLL(LIB)
    lib.mp_last_error.restype = ctypes.c_char_p
    P = ctypes.POINTER(ctypes.c_int)
    modes = np.array([[0, 0, 0, 0], [1, 0, 2, 1]], np.int32)
    mults = np.array([[0, 0], [3, 2]], np.int32)

    def make(ndim=2, family=1, modes=modes, mults=mults, order=1, L_=0.5):
        d = L.BasisDesc(ndim, len(modes), None, len(mults), None, family, modes.ctypes.data_as(P),
                        mults.ctypes.data_as(P), order, L_)
        h = ctypes.c_void_p()
        rc = lib.mp_basis_create(ctypes.byref(d), ctypes.byref(h))
        if rc == 0:
            lib.mp_basis_destroy(h)
        return rc, lib.mp_last_error()

    assert make()[0] == 0
    assert make(ndim=3)[0] == 0
    assert make(family=7) == (-1, b"unknown basis family")
    assert make(L_=0.0)[1] == b"tl_scale must be positive"
    assert make(order=3)[1] == b"order must be in [-2, 2]"
    assert make(mults=np.array([[17, 0]], np.int32))[1] == b"angular index out of range"
    assert make(ndim=3, mults=np.array([[9, 0]], np.int32))[1] == b"angular index out of range"
    assert make(mults=np.array([[0, 17]], np.int32))[1] == b"rational Chebyshev degree must be in [0, 16]"
    assert make(modes=np.array([[0, 1, 0, 0]], np.int32))[1] == b"2D Fourier modes need m_y = 0"
    assert make(modes=np.array([[0, 0, 0, 2]], np.int32))[1] == b"mode phase must be 0 (cos) or 1 (sin)"


def test_curvelet_descriptor_validation_and_wedges():
    """Host-only calls: the descriptor's checks and the wedge list (same order as the
    oracle's frame)."""
    import ctypes
    import numpy as np
    from oracle import curvelet as C
    from paper_1101_3615_amd import _lib as L
    lib = ctypes.CDLL(LIB)
    lib.mp_curvelet_destroy.restype = None
    h = ctypes.c_void_p()
    bad = [L.CurveletDesc(1, 8, 4, 8, 100, 1e-4), L.CurveletDesc(3, 5, 4, 8, 100, 1e-4),
           L.CurveletDesc(3, 8, 0, 8, 100, 1e-4), L.CurveletDesc(3, 8, 4, 0, 100, 1e-4),
           L.CurveletDesc(3, 8, 4, 8, 0, 1e-4), L.CurveletDesc(3, 8, 4, 8, 100, 0.0)]
    for d in bad:
        assert lib.mp_curvelet_create(ctypes.byref(d), ctypes.byref(h)) == L.MP_EINVAL
    d = L.CurveletDesc(4, 8, 4, 8, 100, 1e-4)
    assert lib.mp_curvelet_create(ctypes.byref(d), ctypes.byref(h)) == L.MP_OK
    n = ctypes.c_int()
    assert lib.mp_curvelet_wedges(h, ctypes.byref(n), None) == L.MP_OK
    lst = np.zeros(3 * n.value, dtype=np.int32)
    assert lib.mp_curvelet_wedges(h, ctypes.byref(n), lst.ctypes.data_as(ctypes.POINTER(ctypes.c_int))) == L.MP_OK
    assert [tuple(lst[3 * w:3 * w + 3]) for w in range(n.value)] == C.wedges(4, 8)
    lib.mp_curvelet_destroy(h)


def test_header_is_plain_c_and_links(tmp_path):
    """include/matprobe.h compiles as C99 and a C program links against the library and
    calls its host-only entry points (no GPU needed): the boundary needs no C++ or torch."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler")
    names = declared()
    src = tmp_path / "probe.c"
    refs = "\n".join(f"  (void *)&{n}," for n in names)
    src.write_text(f"""#include <stdio.h>
#include <string.h>
#include "matprobe.h"
static void *const every_entry_point[] = {{
{refs}
}};
int main(void) {{
  mp_curvelet_desc d = {{4, 8, 4, 16, 100, 1e-4}};
  mp_curvelets *cv = NULL;
  int n = 0;
  if (mp_curvelet_create(&d, &cv) != MP_OK) return 1;
  if (mp_curvelet_wedges(cv, &n, NULL) != MP_OK) return 2;
  mp_curvelet_destroy(cv);
  if (mp_create(NULL, NULL, NULL, NULL) != MP_EINVAL) return 3;
  printf("%d %s %u\\n", n, mp_strerror(MP_ESTATE), (unsigned)(sizeof every_entry_point / sizeof every_entry_point[0]));
  return 0;
}}
""")
    exe = tmp_path / "probe"
    libdir = os.path.dirname(LIB)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                        "-L", libdir, "-lmatprobe", "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
    n, rest = r.stdout.split(" ", 1)
    assert int(n) == 1 + 8 + 8 + 16
    assert rest.startswith("no background set")
    assert int(rest.split()[-1]) == len(names)
