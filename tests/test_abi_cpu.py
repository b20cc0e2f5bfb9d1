"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid configurations before touching HIP."""
import ctypes
import os
import re

import pytest

from paper_2502_20610_amd import fdtd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "fdtd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fdtd.load_library()
    declared = _header_functions()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(fdtd.EXPORTS)


def test_config_struct_matches_header_layout():
    # uint32 + 3 int32 + 2 double + 3 int32 + 3 int32 + pointer, natural alignment
    assert ctypes.sizeof(fdtd.Config) == 64


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and field offsets of the two ABI structs, as a C compiler lays
    them out from include/fdtd.h, equal the binding's ctypes layouts."""
    import subprocess
    fields = {"fdtd_config": [f[0] for f in fdtd.Config._fields_],
              "fdtd_adjoint_spec": [f[0] for f in fdtd.AdjointSpec._fields_]}
    src = ['#include <stddef.h>', '#include <stdio.h>', '#include "fdtd.h"', "int main(void) {"]
    for st, names in fields.items():
        src.append('printf("%%s size %%zu\\n", "%s", sizeof(%s));' % (st, st))
        for n in names:
            src.append('printf("%%s %%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (st, n, st, n))
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st, cls in (("fdtd_config", fdtd.Config), ("fdtd_adjoint_spec", fdtd.AdjointSpec)):
        assert got[(st, "size")] == ctypes.sizeof(cls)
        for n in fields[st]:
            assert got[(st, n)] == getattr(cls, n).offset, (st, n)


def test_adjoint_rejects_bad_arguments_without_gpu():
    lib = fdtd.load_library()
    spec = fdtd.AdjointSpec()
    spec.struct_size = ctypes.sizeof(fdtd.AdjointSpec)
    g = (ctypes.c_float * 8)()
    # a NULL context is rejected before anything else
    assert lib.fdtd_adjoint(None, ctypes.byref(spec), g, fdtd.HOST) == fdtd.FDTD_EINVAL


def _cfg(**kw):
    c = fdtd.Config()
    c.struct_size = ctypes.sizeof(fdtd.Config)
    c.nx, c.ny, c.nz = kw.get("shape", (8, 8, 8))
    c.dt, c.dx = kw.get("dt", 0.5), kw.get("dx", 1.0)
    for a, b in enumerate(kw.get("bc", (0, 0, 0))):
        c.bc[a] = b
    c.scheme = kw.get("scheme", 0)
    c.storage = kw.get("storage", 0)
    c.device = kw.get("device", 0)
    c.stream = None
    return c


@pytest.mark.parametrize("kw,code", [
    (dict(shape=(0, 8, 8)), fdtd.FDTD_EINVAL),
    (dict(shape=(8, -1, 8)), fdtd.FDTD_EINVAL),
    (dict(shape=(1024, 1024, 1025)), fdtd.FDTD_EINVAL),
    (dict(dt=0.58), fdtd.FDTD_EINVAL),          # dt*sqrt(3) >= dx
    (dict(dt=0.0), fdtd.FDTD_EINVAL),
    (dict(dx=-1.0), fdtd.FDTD_EINVAL),
    (dict(dt=float("nan")), fdtd.FDTD_EINVAL),
    (dict(bc=(0, 2, 0)), fdtd.FDTD_EINVAL),
    (dict(scheme=7), fdtd.FDTD_EINVAL),
    (dict(scheme=3), fdtd.FDTD_EINVAL),
    (dict(storage=5), fdtd.FDTD_EINVAL),
    (dict(device=-1), fdtd.FDTD_EINVAL),
])
def test_create_rejects_invalid_config_without_gpu(kw, code):
    lib = fdtd.load_library()
    h = ctypes.c_void_p(123)
    cfg = _cfg(**kw)
    rc = lib.fdtd_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == code
    assert h.value is None
    msg = lib.fdtd_last_error(None).decode()
    assert msg and msg != "no error"


def test_struct_size_mismatch_and_null_args():
    lib = fdtd.load_library()
    h = ctypes.c_void_p()
    cfg = _cfg()
    cfg.struct_size = 12
    assert lib.fdtd_create(ctypes.byref(cfg), ctypes.byref(h)) == fdtd.FDTD_EINVAL
    assert lib.fdtd_create(None, ctypes.byref(h)) == fdtd.FDTD_EINVAL
    assert lib.fdtd_create(ctypes.byref(_cfg()), None) == fdtd.FDTD_EINVAL


def test_null_context_calls_are_safe():
    lib = fdtd.load_library()
    assert lib.fdtd_destroy(None) == fdtd.FDTD_OK
    assert lib.fdtd_current_step(None) == -1
    assert lib.fdtd_step(None, 1) == fdtd.FDTD_EINVAL
    assert lib.fdtd_synchronize(None) == fdtd.FDTD_EINVAL
    assert lib.fdtd_set_option(None, 0, 0) == fdtd.FDTD_EINVAL
    assert lib.fdtd_adjoint(None, None, None, 0) == fdtd.FDTD_EINVAL
    assert lib.fdtd_set_field_scale(None, (ctypes.c_int32 * 6)()) == fdtd.FDTD_EINVAL
    assert lib.fdtd_step_batch(None, 1, 1) == fdtd.FDTD_EINVAL
    assert lib.fdtd_set_lossy_materials(None, *([None] * 6), 0) == fdtd.FDTD_EINVAL
    assert lib.fdtd_invariants(None, (ctypes.c_double * 7)(), None, None, 0) == fdtd.FDTD_EINVAL
    assert isinstance(lib.fdtd_last_error(None), bytes)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fdtd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fdtd, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        fdtd.load_library()
