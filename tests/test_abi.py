"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/rbf.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rbf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2502_12878_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2502_12878_amd import build
        build.build()
    return _abi.lib()


def test_header_declares_the_paper_verbs():
    names = _declared()
    for verb in ("rbf_build_nodes", "rbf_build_stencils", "rbf_compute_weights", "rbf_iterate"):
        assert verb in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2502_12878_amd import _abi
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, f"{name} has no Python binding"


def test_status_strings(lib):
    assert lib.rbf_status_string(0) == b"ok"
    assert lib.rbf_status_string(3) == b"singular local system"
    assert lib.rbf_status_string(99) == b"unknown status"
    assert lib.rbf_version().startswith(b"rbf-mi355x")


def test_null_handle_rejected(lib):
    assert lib.rbf_build_nodes(None, 2, 10, 0.3, 0, None, None) == 1
    assert lib.rbf_set_nodes(None, 2, 10, None, None) == 1
    assert lib.rbf_build_stencils(None, 12, None) == 1
    assert lib.rbf_compute_weights(None, 2, None, 0) == 1
    assert lib.rbf_iterate(None, None, None, None, None) == 1
    assert lib.rbf_destroy(None) == 1
    assert lib.rbf_last_error(None) == b"null handle"


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = C.c_void_p()
    assert lib.rbf_create(C.byref(h), 0, None, None) == 1
    assert not h.value


_CTYPES = {"double": C.c_double, "int64_t": C.c_int64, "int32_t": C.c_int32, "const double *": C.c_void_p}


def test_iter_struct_layout_matches_header():
    """Field order and types of the ABI structs as the header declares them
    (comma-separated declarators included)."""
    from paper_2502_12878_amd import _abi
    text = open(HEADER).read()
    for cls, cname in ((_abi.rbf_iter_params, "rbf_iter_params"), (_abi.rbf_iter_report, "rbf_iter_report"),
                       (_abi.rbf_operator_info, "rbf_operator_info")):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", text).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            m = re.match(r"((?:const\s+)?\w+\s*\*?)\s*(.*)", decl)
            ctype = m.group(1).replace(" *", " *").strip()
            for name in m.group(2).split(","):
                name = name.strip().lstrip("*")
                if "*" in m.group(1):
                    ctype = "const double *"
                fields.append((name, ctype))
        assert [f for f, _ in cls._fields_] == [f for f, _ in fields], cname
        for (f, t), (_, ct) in zip(cls._fields_, fields):
            assert C.sizeof(t) == C.sizeof(_CTYPES[ct]), (cname, f)


def test_package_import_does_not_need_a_gpu():
    import paper_2502_12878_amd as pkg
    assert hasattr(pkg, "Problem") and hasattr(pkg, "SolveK")


def test_shipped_tuning_file_is_valid():
    """The tuned shapes shipped for MI355X: JSON, one entry per operator key,
    every value within the candidate sets the autotuner draws from."""
    import json
    path = os.path.join(ROOT, "paper_2502_12878_amd", "tuned_gfx950.json")
    if not os.path.exists(path):
        pytest.skip("no shipped tuning file")
    d = json.load(open(path))
    assert d
    # the library's cache writer rewrites the file line by line: each entry
    # (key and whole value list) must sit on one line
    body = [l for l in open(path).read().splitlines() if l.strip() not in ("{", "}", "")]
    assert len(body) == len(d)
    assert all(l.strip().startswith('"') and l.rstrip(",").endswith("]") for l in body)
    for key, v in d.items():
        kind = key.split("|")[0]
        assert kind in ("sweep", "sweep32", "sweepT", "weights"), key
        if kind == "weights":
            assert v[0] in (8, 16)
            continue
        assert len(v) in (6, 7, 8), key
        assert v[0] in (2, 4, 8) and v[1] in (4, 8, 16, 32), key
        assert all(x in (0, 1) for x in v[2:]), key
        assert "gfx950" in key
