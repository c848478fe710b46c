"""CPU checks of the C-ABI library: it loads, exports every function that
include/borth.h declares, and its host-only entry points behave without a GPU.
No compute calls are made here."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "borth.h"
LIB = ROOT / "paper_1806_01036_amd" / "libborth.so"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(borth_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not LIB.exists():
        from paper_1806_01036_amd import build
        build.build(force=False)
    return ctypes.CDLL(str(LIB))


def test_header_declares_the_path():
    names = declared_functions()
    for required in ["borth_gram", "borth_factor", "borth_update", "borth_orthonormalize",
                     "borth_batch_orthonormalize", "borth_autotune", "borth_create",
                     "borth_destroy"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_export():
    from paper_1806_01036_amd import _lib
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_host_only_entry_points(lib):
    lib.borth_status_string.restype = ctypes.c_char_p
    assert lib.borth_status_string(0) == b"ok"
    assert b"breakdown" in lib.borth_status_string(4)
    assert lib.borth_status_string(99) == b"unknown status"
    from paper_1806_01036_amd import _lib
    o = _lib.borth_opts()
    lib.borth_default_opts(ctypes.byref(o))
    assert (o.gram, o.fact, o.passes, o.sched, o.flags) == (1, 0, 2, 0, 0)
    assert o.shift < 0
    # null context is rejected before anything touches a device
    assert lib.borth_destroy(None) == 1
    assert lib.borth_orthonormalize(None, 10, 2, 0, None, 2, None, 0, 0, None, 2, None, None,
                                    None, None) == 1


def test_no_oracle_in_product():
    """The product path neither imports nor links the oracle."""
    pkg = ROOT / "paper_1806_01036_amd"
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.hip")) + list(pkg.rglob("*.cpp")) \
            + list(pkg.rglob("*.hpp")):
        text = f.read_text()
        assert "import oracle" not in text and "from oracle" not in text, f
        assert "liboracle" not in text and "oracle.c" not in text, f


def test_struct_layouts_match_binding(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout (gcc)."""
    import shutil
    import subprocess
    from paper_1806_01036_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"borth_opts": _lib.borth_opts, "borth_info": _lib.borth_info,
               "borth_block": _lib.borth_block, "borth_iter_info": _lib.borth_iter_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "borth.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{ROOT / 'include'}", str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(out[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)


def test_binding_rejects_host_and_malformed_tensors():
    """The binding's tensor checks run before any pointer reaches the
    library (which cannot check device memory): host tensors, wrong ranks
    and non-tensors are refused on the CPU already."""
    import types
    import torch
    import paper_1806_01036_amd as borth
    ctx = types.SimpleNamespace(device=0)
    for bad in (torch.zeros((10, 3), dtype=torch.float64), torch.zeros(10, dtype=torch.float64),
                [[1.0, 2.0]], None):
        with pytest.raises(borth.ArgumentError):
            borth._mat(bad, "X", ctx)
    err = borth.ArgumentError("x")
    assert isinstance(err, ValueError) and isinstance(err, borth.BorthError)
    assert err.status == borth.ERR_ARG
