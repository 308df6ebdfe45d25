"""The C-ABI library loads without a GPU and exports every function that
include/stag.h declares; argument checks that precede any device work behave
as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stag.h")
LIB = os.path.join(ROOT, "paper_1710_09178_amd", "libstag.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stag_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1710_09178_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (stag_\w+)", out))
    assert set(names) <= exported


def test_create_rejects_bad_dims_before_touching_the_gpu(lib):
    lib.stag_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    for dims in [(4, 4, 4, 3), (4, 0, 4, 4), (1, 4, 4, 4)]:
        arr = (ctypes.c_int * 4)(*dims)
        assert lib.stag_create(ctypes.byref(h), arr, None) == -1
        assert b"even" in lib.stag_last_error(None)
    assert lib.stag_create(None, (ctypes.c_int * 4)(4, 4, 4, 4), None) == -1


def test_null_handle_calls_are_rejected(lib):
    assert lib.stag_dslash(None, None, None, 1) == -1
    assert lib.stag_destroy(None) == 0
    assert lib.stag_field_bytes(None, 0) == 0


def _prototypes():
    """name -> list of parameter declarations, parsed from include/stag.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    protos = {}
    for m in re.finditer(r"\b(?:stag_status|const char\*|size_t|int)\s+(stag_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", text):
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        protos[m.group(1)] = params
    return protos


def test_binding_signatures_match_the_header():
    """Every ctypes signature of the Python binding has the header's arity and
    puts pointers exactly where the C prototype has pointers (an argument-order
    mistake here would hand an integer to C as an address)."""
    import ctypes as C

    from paper_1710_09178_amd import stag
    lib = stag.load_library()
    protos = _prototypes()
    scalar = (C.c_int, C.c_uint32, C.c_uint64, C.c_double, C.c_size_t, C.c_long)
    checked = 0
    for name, params in protos.items():
        fn = getattr(lib, name)
        if fn.argtypes is None:
            continue
        assert len(fn.argtypes) == len(params), name
        for decl, at in zip(params, fn.argtypes):
            is_ptr = "*" in decl or "[" in decl or decl.split()[0] in ("stag_handle", "stag_batch_handle",
                                                                       "stag_surrogate_handle")
            if is_ptr:
                assert at is C.c_void_p or issubclass(at, C._Pointer) or at is C.c_char_p, (name, decl, at)
            else:
                assert at in scalar, (name, decl, at)
        checked += 1
    assert checked >= 25


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built library every entry raises."""
    from paper_1710_09178_amd import stag as S
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", os.path.join(ROOT, "paper_1710_09178_amd", "no_such_libstag.so"))
    with pytest.raises(RuntimeError):
        S.load_library()
    with pytest.raises(RuntimeError):
        S.Lattice((4, 4, 4, 4))


def test_product_package_does_not_use_the_oracle():
    """The HIP path and the oracle share nothing: no module of the package
    imports or names the oracle."""
    pkg = os.path.join(ROOT, "paper_1710_09178_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_binding_structs_match_the_header_layout(tmp_path):
    """Size and field offsets of every struct the binding mirrors, compiled
    from include/stag.h by the host C compiler, against the ctypes
    structures (a field added to one side only would shift every later one)."""
    import shutil

    from paper_1710_09178_amd import stag
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"stag_rational": stag.CRational, "stag_solve_info": stag.CSolveInfo,
             "stag_mixed_opts": stag.CMixedOpts, "stag_hmc_params": stag.CHMCParams,
             "stag_traj_info": stag.CTrajInfo, "stag_chain_policy": stag.CChainPolicy,
             "stag_batch_opts": stag.CBatchOpts, "stag_batch_info": stag.CBatchInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "stag.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
