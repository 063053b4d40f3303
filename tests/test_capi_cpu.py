"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/crk.h declares, and argument errors are
caught on the host before any device work."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_2510_03557_amd import binding

ROOT = Path(__file__).resolve().parents[1]


def header_functions():
    text = (ROOT / "include" / "crk.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_header_declares_the_six_operations():
    names = header_functions()
    for op in ("build_tree", "build_interaction_lists", "crk_density",
               "crk_coefficients", "crk_hydro_forces", "shortrange_gravity",
               "crk_integrate"):
        assert op in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.EXPORTS) <= set(header_functions())


def test_null_context_is_rejected_on_host(lib):
    assert lib.crk_density(None, None, None, None, None) == binding.CRK_EINVAL
    assert "context" in binding.last_error()
    assert lib.build_interaction_lists(None, None) == binding.CRK_EINVAL
    assert lib.crk_sync(None, None) == binding.CRK_EINVAL
    assert lib.crk_graph_launch(None) == binding.CRK_EINVAL


def test_bad_precision_is_rejected_on_host(lib):
    h = ctypes.c_void_p()
    assert lib.crk_ctx_create(ctypes.byref(h), 7, None, None) == binding.CRK_EINVAL
    assert lib.crk_ctx_create(None, 1, None, None) == binding.CRK_EINVAL


def test_context_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    st = lib.crk_ctx_create(ctypes.byref(h), binding.CRK_FP32, None, None)
    assert st == binding.CRK_EDEVICE
    assert not h.value


def test_missing_library_fails_loudly(tmp_path):
    """The binding refuses to run without the built HIP library (there is
    no fallback path)."""
    with pytest.raises(ImportError):
        binding.load(tmp_path / "libcrk.so")


def test_package_never_touches_the_oracle():
    """The library, its binding and the step driver share no code with the
    oracle: no import, include or link of anything under oracle/."""
    pkg = ROOT / "paper_2510_03557_amd"
    offenders = []
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.hip")) + \
            list(pkg.rglob("*.h")) + list((ROOT / "include").rglob("*.h")):
        text = f.read_text()
        if re.search(r"^\s*(import|from)\s+oracle\b", text, re.M) or \
                "crk_oracle" in text or "libcrk_oracle" in text:
            offenders.append(str(f.relative_to(ROOT)))
    assert not offenders, offenders


def test_binding_rejects_mismatched_tensors():
    """The binding hands raw addresses to the library, so it checks every
    tensor first: dtype, contiguity, length, then that it lives on the
    device.  Each mismatch raises CRK_EINVAL before any library call."""
    import torch
    ok = torch.zeros(8, dtype=torch.float32)
    cases = [
        (torch.zeros(8, dtype=torch.float64), torch.float32, 8, "dtype"),
        (torch.zeros(8, dtype=torch.int64), torch.int32, 8, "dtype"),
        (torch.zeros(4, 4, dtype=torch.float32).t(), torch.float32, 8,
         "contiguous"),
        (torch.zeros(7, dtype=torch.float32), torch.float32, 8, "elements"),
        (ok, torch.float32, 8, "device"),  # host tensor
    ]
    for t, dtype, n, what in cases:
        with pytest.raises(binding.CrkError) as e:
            binding.check_tensor(t, dtype, n, "arg")
        assert e.value.status == binding.CRK_EINVAL
        assert what in str(e.value), (what, str(e.value))
    binding.check_tensor(None, torch.float32, 8, "arg")  # NULL passes


def test_context_checks_plane_triples_before_the_library():
    """Three-plane arguments (accelerations, positions) are checked plane by
    plane; the check needs no device (it fails on the host tensor)."""
    import torch
    ctx = binding.Context.__new__(binding.Context)  # no device context
    ctx.dtype = torch.float32
    planes = [torch.zeros(5, dtype=torch.float32) for _ in range(3)]
    with pytest.raises(binding.CrkError) as e:
        ctx._p3(planes[:2], 5, "a")
    assert "three planes" in str(e.value)
    with pytest.raises(binding.CrkError) as e:
        ctx._p3([planes[0], None, planes[2]], 5, "a")
    assert "null plane" in str(e.value)
    with pytest.raises(binding.CrkError) as e:
        ctx._p3(planes, 6, "a")
    assert "elements" in str(e.value)
    with pytest.raises(binding.CrkError) as e:
        ctx._p3(planes, 5, "a")
    assert "device" in str(e.value)
    assert ctx._p3(None, 5, "a") is None


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built against include/crk.h prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = [binding.crk_params, binding.crk_boxes, binding.crk_tuning,
               binding.crk_tree_info]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "crk.h"',
             "int main(void) {"]
    for cls in structs:
        n = cls.__name__
        lines.append(f'    printf("{n} %zu\\n", sizeof({n}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{n}.{f} %zu\\n", offsetof({n}, {f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", str(ROOT / "include"), str(src),
                    "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cls in structs:
        n = cls.__name__
        assert int(got[n]) == ctypes.sizeof(cls), n
        for f, _ in cls._fields_:
            assert int(got[f"{n}.{f}"]) == getattr(cls, f).offset, (n, f)
