"""The C-ABI library loads and exports every entry point include/mfs.h
declares, and rejects bad arguments on the host before touching a GPU
(CPU only: no kernel is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfs.h")
LIB = os.path.join(ROOT, "paper_2409_04215_amd", "libmfs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmfs.so is not built (run paper_2409_04215_amd/build.py)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mfs_p2p_stokes", "mfs_p2p_laplace", "mfs_precond_apply", "mfs_matvec", "mfs_gmres_solve",
                 "mfs_p2p_stokes_backward", "mfs_p2p_laplace_backward", "mfs_gmres_solve_backward"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_argument_errors(lib):
    lib.mfs_last_error.restype = ctypes.c_char_p
    i64 = ctypes.c_int64
    p = ctypes.POINTER(ctypes.c_int64)
    # n_sys < 1
    st = lib.mfs_p2p_stokes(i64(0), None, None, None, None, None, None, None, ctypes.c_double(1.0), 1, 1, None)
    assert st == -1 and b"n_sys" in lib.mfs_last_error()
    # non-monotone system pointers
    sp = (ctypes.c_int64 * 3)(0, 2, 1)
    bp = (ctypes.c_int64 * 3)(0, 1, 2)
    st = lib.mfs_p2p_laplace(i64(2), sp, bp, bp, None, None, None, None, 1, 1, None)
    assert st == -1
    # NULL plan everywhere
    assert lib.mfs_plan_create(None, None, None) == -1
    assert lib.mfs_matvec(None, None, None, 1, None) == -1
    assert lib.mfs_gmres_solve(None, None, None, ctypes.c_double(1e-5), 10, 1, 0, None, None, None) == -1
    assert lib.mfs_plan_destroy(None) == 0


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback: with libmfs.so missing, the first call raises."""
    from paper_2409_04215_amd import mfs
    monkeypatch.setattr(mfs, "LIB_PATH", str(tmp_path / "missing_libmfs.so"))
    monkeypatch.setattr(mfs, "_lib", None)
    with pytest.raises(ImportError):
        mfs.lib()
    with pytest.raises(ImportError):
        mfs.version()


def test_plan_descriptor_layout_matches_the_header():
    """The ctypes descriptor lists the C struct's fields in order (the binding
    passes it by pointer)."""
    from paper_2409_04215_amd import mfs
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} mfs_plan_desc;", text, flags=re.S).group(1)
    c_fields = re.findall(r"\*?\s*([a-z_0-9]+);", body)
    assert [f[0] for f in mfs.PlanDesc._fields_] == c_fields


def test_header_is_plain_c_and_the_layout_matches_the_binding(tmp_path):
    """A C99 program includes mfs.h, links libmfs.so and calls it (no GPU call):
    the header is plain C, and the byte offsets of mfs_plan_desc agree with the
    ctypes descriptor the Python binding passes."""
    import shutil
    import subprocess
    from paper_2409_04215_amd import mfs
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f[0] for f in mfs.PlanDesc._fields_]
    src = tmp_path / "abi.c"
    src.write_text(
        "#include <stddef.h>\n#include <stdio.h>\n#include \"mfs.h\"\n"
        "int main(void) {\n"
        "  printf(\"%s\\n\", mfs_version());\n"
        f"  printf(\"%zu\\n\", sizeof(mfs_plan_desc));\n"
        + "".join(f"  printf(\"%zu\\n\", offsetof(mfs_plan_desc, {f}));\n" for f in fields)
        + "  return mfs_plan_destroy(NULL);\n}\n")
    exe = tmp_path / "abi"
    inc = os.path.join(ROOT, "include")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe),
                        LIB, f"-Wl,-rpath,{os.path.dirname(LIB)}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "gfx950" in r.stdout.splitlines()[0]
    nums = [int(x) for x in r.stdout.splitlines()[1:]]
    assert nums[0] == ctypes.sizeof(mfs.PlanDesc)
    assert nums[1:] == [getattr(mfs.PlanDesc, f).offset for f in fields]
