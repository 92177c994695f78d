"""Host-only checks of the C ABI: the built library loads and exports every
entry point include/hfe.h declares; grid validation and workspace sizing run
without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfe.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hfe_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_2207_10657_amd import hfe
    if not os.path.exists(hfe.LIB_PATH):
        pytest.skip("libhfe.so not built")
    return hfe, hfe.load_library()


def test_every_declared_symbol_is_exported():
    hfe, lib = _lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares exactly these
    assert sorted(hfe.EXPORTS) == names


def test_workspace_sizing_and_grid_validation():
    hfe, lib = _lib()
    assert hfe.workspace_bytes((64, 64, 64), "q1") > 64 ** 3 * 8 * 3 * 11
    assert hfe.workspace_bytes((32, 32), "p1pair") > 0
    # unsupported: odd nx, lengths outside the FFT set, plane too large for LDS
    assert hfe.workspace_bytes((8, 8, 7), "q1") == 0
    assert hfe.workspace_bytes((8, 8, 10), "q1") == 0
    assert hfe.workspace_bytes((8, 256, 256), "q1") == 0
    # element / dimension mismatch
    g = hfe._grid((8, 8), "q1")
    assert lib.hfe_workspace_bytes(ctypes.byref(g)) == 0


def test_create_rejects_bad_arguments_without_gpu():
    hfe, lib = _lib()
    g = hfe._grid((8, 8, 8), "q1")
    out = ctypes.c_void_p()
    # null workspace / misaligned workspace are rejected before any device call
    assert lib.hfe_create(ctypes.byref(g), None, 1 << 30, None, ctypes.byref(out)) == -1
    assert lib.hfe_create(ctypes.byref(g), ctypes.c_void_p(8), 1 << 30, None, ctypes.byref(out)) == -1
    # too small a workspace
    assert lib.hfe_create(ctypes.byref(g), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == -2
    assert lib.hfe_last_error(None) == b"null context"


def test_binding_constants_match_the_header():
    """The binding's material kinds are the header's (parsed from
    include/hfe.h)."""
    hfe, _ = _lib()
    text = open(os.path.join(os.path.dirname(__file__), "..", "include", "hfe.h")).read()
    consts = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(HFE_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    for name in ("HFE_ELASTIC", "HFE_DAMAGE_ENERGY_NORM", "HFE_DAMAGE_TENSILE"):
        assert getattr(hfe, name) == consts[name], name


def test_header_is_plain_c(tmp_path):
    """include/hfe.h compiles as strict C99 with every warning enabled (no
    C++ or HIP types in the boundary)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    src = tmp_path / "use_header.c"
    src.write_text('#include "hfe.h"\nint main(void) {\n  hfe_material m;\n'
                   '  m.kind = HFE_DAMAGE_TENSILE;\n  return m.kind == HFE_DAMAGE_TENSILE ? 0 : 1;\n}\n')
    out = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc,
                          str(src), "-o", str(tmp_path / "use_header")],
                         capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert subprocess.run([str(tmp_path / "use_header")]).returncode == 0


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the header's size and field
    offsets (compiled with the system C compiler)."""
    import shutil
    import subprocess
    hfe, _ = _lib()
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    pairs = [("hfe_solver_params", hfe._Params), ("hfe_solve_report", hfe._Report),
             ("hfe_newton_record", hfe._Record), ("hfe_material", hfe._Material),
             ("hfe_grid", hfe._Grid), ("hfe_tuning", hfe._Tuning),
             ("hfe_lbfgs_params", hfe._LbfgsParams), ("hfe_lbfgs_report", hfe._LbfgsReport)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hfe.h"', 'int main(void) {']
    expect = []
    for cname, ct in pairs:
        lines.append('  printf("%%zu\\n", sizeof(%s));' % cname)
        expect.append(ctypes.sizeof(ct))
        for f, _ in ct._fields_:
            lines.append('  printf("%%zu\\n", offsetof(%s, %s));' % (cname, f))
            expect.append(getattr(ct, f).offset)
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    out = subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)],
                         capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == expect
