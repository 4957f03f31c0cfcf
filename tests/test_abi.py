"""The C-ABI library loads and exports every function include/crk.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "crk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(crk_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_passes():
    names = _declared()
    for n in ("crk_build_cells", "crk_moments", "crk_corrections", "crk_derivatives"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2202_02840_amd as crk
    path = crk.library_path()
    assert os.path.exists(path), "build libcrk.so first"
    lib = ctypes.CDLL(path)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(crk._lib.EXPORTS) == set(_declared())


def test_version_and_defaults_without_gpu():
    import paper_2202_02840_amd as crk
    assert "gfx950" in crk.version()
    p = crk.Params.default(268.0)
    assert abs(p.nh - 4.0) < 1e-3 and p.Cl == 2.0 and p.Cq == 1.0 and p.eps == 0.1
    assert abs(p.eta_crit * p.nh - 1.0) < 1e-15 and abs(p.eta_fold * p.nh - 0.2) < 1e-15


def test_no_gpu_fails_loudly():
    import torch
    import paper_2202_02840_amd as crk
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        crk.Context(0)


def _prototypes():
    """name -> number of parameters of each function include/crk.h declares."""
    src = open(os.path.join(ROOT, "include", "crk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for name, args in re.findall(r"\b(crk_[a-z_]+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S):
        args = args.strip()
        out[name] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_the_header():
    """The ctypes binding passes as many arguments as each prototype takes."""
    import paper_2202_02840_amd as crk
    L = crk._lib.lib()
    protos = _prototypes()
    assert set(protos) == set(_declared())
    for name, nargs in protos.items():
        assert len(getattr(L, name).argtypes) == nargs, name
