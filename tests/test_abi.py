"""The C-ABI library loads and exports every entry point include/pe.h
declares; host-side argument checks fail cleanly (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pe.h")
LIB = os.path.join(ROOT, "paper_2401_04865_amd", "libpe.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pe_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("pe_create", "pe_set_system", "pe_solve_polarization", "pe_forces_torques",
              "pe_apply_potential", "pe_destroy", "pe_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_header():
    from paper_2401_04865_amd import binding
    names = set(declared()) - {"pe_last_error"}
    assert names <= set(binding.SIGNATURES), names - set(binding.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_errors_before_any_launch():
    from paper_2401_04865_amd import binding as B
    lib = B.lib()
    h = ctypes.c_void_p()
    p = B.make_params([10, 10, 10], [16, 16, 15])          # odd mesh[2]
    assert lib.pe_create(ctypes.byref(p), None, ctypes.byref(h)) == B.PE_ERR_ARG
    assert b"even" in lib.pe_last_error(None)
    p = B.make_params([10, 10, 10], [14, 16, 16], P=8)      # 14 = 2*7: factor 7 unsupported
    assert lib.pe_create(ctypes.byref(p), None, ctypes.byref(h)) == B.PE_ERR_ARG
    p = B.make_params([10, 10, 10], [16, 16, 16], P=20)
    assert lib.pe_create(ctypes.byref(p), None, ctypes.byref(h)) == B.PE_ERR_ARG
    p = B.make_params([-1, 10, 10], [16, 16, 16])
    assert lib.pe_create(ctypes.byref(p), None, ctypes.byref(h)) == B.PE_ERR_ARG


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the structs have the C sizes and offsets (checked by
    compiling the header with gcc)."""
    import shutil
    import subprocess
    from paper_2401_04865_amd import binding as B
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = {"pe_params": [f for f, _ in B.pe_params._fields_],
              "pe_solve_info": [f for f, _ in B.pe_solve_info._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(c), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for st, cls in (("pe_params", B.pe_params), ("pe_solve_info", B.pe_solve_info)):
        assert int(out[st]) == ctypes.sizeof(cls)
        for f in fields[st]:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_library_allocates_no_device_memory():
    """Every device buffer comes from the caller's workspace: no source of
    the library calls a device allocator."""
    import glob
    srcs = glob.glob(os.path.join(ROOT, "paper_2401_04865_amd", "csrc", "*.hip")) + \
        glob.glob(os.path.join(ROOT, "paper_2401_04865_amd", "csrc", "*.hpp"))
    assert srcs
    pat = re.compile(r"\b(hipMalloc|hipMallocAsync|hipMallocManaged|hipMallocPitch|hipMalloc3D|hipExtMallocWithFlags|"
                     r"hipMallocFromPoolAsync|hipFree|hipFreeAsync)\s*\(")
    for f in srcs:
        text = re.sub(r"//[^\n]*", "", open(f).read())
        assert not pat.search(text), f
