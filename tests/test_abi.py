"""The C-ABI library: it loads without a GPU, exports every function the
headers declare, and the Python binding's structures follow the header's
field order (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")


def _headers():
    return [os.path.join(INC, f) for f in sorted(os.listdir(INC)) if f.endswith(".h")]


def _declared_functions():
    names = set()
    for h in _headers():
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(ps_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def _struct_fields(name):
    src = open(os.path.join(INC, "ps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    end = re.search(r"\}\s*" + name + ";", src)
    assert end, name
    start = src.rfind("typedef struct {", 0, end.start())
    body = src[start + len("typedef struct {"):end.start()]
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"\[\w+\]", "", decl)
        for part in decl.split(","):
            fields.append(re.findall(r"\w+", part)[-1])
    return fields


@pytest.fixture(scope="module")
def lib():
    from paper_2606_26785_amd import build
    path = build.OUT
    if not os.path.exists(path):
        pytest.skip("libps.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(path)


def test_headers_declare_the_boundary():
    names = _declared_functions()
    for need in ("ps_create", "ps_grid", "ps_eval", "ps_destroy", "ps_grid_destroy", "ps_default_params",
                 "ps_strerror", "ps_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_structs_follow_header():
    import paper_2606_26785_amd as P
    for cname, cls in (("ps_params", P.ps_params), ("ps_stats", P.ps_stats), ("ps_matrix_desc", P.ps_matrix_desc)):
        assert [f[0] for f in cls._fields_] == _struct_fields(cname), cname


def test_default_params_without_gpu(lib):
    import paper_2606_26785_amd as P
    p = P.default_params()
    assert p.r == 8 and p.k_max == 32 and p.eta > 0 and p.lipschitz == 1


def test_binding_struct_layout_matches_the_c_compiler(tmp_path):
    """Field offsets and struct sizes of the binding's ctypes structures equal
    what a C compiler lays out from include/ps.h (catches a field of the wrong
    width, which the field order alone would not)."""
    import subprocess
    import paper_2606_26785_amd as P
    structs = (("ps_params", P.ps_params), ("ps_stats", P.ps_stats), ("ps_matrix_desc", P.ps_matrix_desc))
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ps.h"', "int main(void) {"]
    for cname, _ in structs:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in _struct_fields(cname):
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", INC, str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, cls in structs:
        assert ctypes.sizeof(cls) == got[(cname, "size")], cname
        for f in _struct_fields(cname):
            assert getattr(cls, f).offset == got[(cname, f)], (cname, f)


def _kind_c(param):
    param = param.strip()
    if "*" in param:
        return "ptr"
    if re.search(r"\bdouble\b", param):
        return "f64"
    if re.search(r"\bint64_t\b", param):
        return "i64"
    if re.search(r"\b(int32_t|int|ps_status|ps_kind)\b", param):
        return "i32"
    raise AssertionError("unclassified parameter: " + param)


def _kind_ctypes(t):
    if t in (ctypes.c_void_p, ctypes.c_char_p) or (isinstance(t, type) and issubclass(t, ctypes._Pointer)):
        return "ptr"
    if t is ctypes.c_double:
        return "f64"
    if t is ctypes.c_int64:
        return "i64"
    if t in (ctypes.c_int32, ctypes.c_int):
        return "i32"
    raise AssertionError("unclassified ctypes type: %r" % (t,))


def test_binding_signatures_follow_the_headers(lib):
    """Every function the binding declares has the parameter kinds and widths
    of its prototype in include/*.h."""
    import paper_2606_26785_amd as P
    lib_b = P.load()
    protos = {}
    for h in _headers():
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"\b(ps_\w+)\s*\(([^)]*)\)\s*;", src):
            params = [p for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
            protos[m.group(1)] = [_kind_c(p) for p in params]
    checked = 0
    for name, kinds in protos.items():
        fn = getattr(lib_b, name)
        if fn.argtypes is None:
            continue
        assert [_kind_ctypes(t) for t in fn.argtypes] == kinds, name
        checked += 1
    assert checked >= 15
