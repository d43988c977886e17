"""CPU checks of the boundary: the library builds, loads and exports every entry point
declared in include/ensf.h; the binding's structs match the header's."""
import ctypes
import os
import re

import pytest

from paper_2407_12168_amd import ensf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ensf.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_entry_points():
    names = set()
    for h in HEADERS:
        names |= set(re.findall(r"^\s*(?:ensf_status|void|const char\*|int64_t)\s+(ensf_\w+)\s*\(",
                                open(h).read(), flags=re.M))
    return sorted(names)


def test_headers_declare_the_binding_names():
    from paper_2407_12168_amd import sqg, surrogate
    from paper_2407_12168_amd import vit
    assert declared_entry_points() == sorted(ensf.EXPORTS + surrogate.EXPORTS + sqg.EXPORTS +
                                             vit.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ensf.LIB_PATH):
        pytest.skip("libensf.so not built")
    return ctypes.CDLL(ensf.LIB_PATH)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_entry_points():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults(lib):
    L = ensf._lib()
    assert L.ensf_status_string(0) == b"ok"
    assert L.ensf_status_string(1) == b"invalid argument"
    o = ensf.ensf_default_options()
    assert o.precision == 0 and o.obs_op == 0 and o.eps_alpha == 0.05 and o.use_graph == 1


def test_create_rejects_null_out_pointer(lib):
    L = ensf._lib()
    assert L.ensf_create(None, None) == ensf.ENSF_EINVAL
    assert L.ensf_destroy(None) == ensf.ENSF_OK


def test_struct_layout_matches_header(tmp_path):
    # compile the header with the host C compiler and compare sizes and field offsets
    src = tmp_path / "layout.c"
    fields = {"ensf_options": [f[0] for f in ensf.ensf_options._fields_],
              "ensf_problem": [f[0] for f in ensf.ensf_problem._fields_]}
    body = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void){']
    for st, names in fields.items():
        body.append(f'printf("%zu\\n", sizeof({st}));')
        body += [f'printf("%zu\\n", offsetof({st}, {n}));' for n in names]
    body.append("return 0;}")
    src.write_text("\n".join(body))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for st in (ensf.ensf_options, ensf.ensf_problem):
        want.append(ctypes.sizeof(st))
        want += [getattr(st, n).offset for n, _ in st._fields_]
    assert got == want
