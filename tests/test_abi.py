"""The C-ABI library loads and exports every symbol include/mgp.h declares;
the Python binding agrees with the header; host-side validation and planning
work without a GPU (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2605_30082_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgp.h")


def header_text():
    with open(HEADER) as f:
        return f.read()


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", header_text(), flags=re.S)
    names = re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert sorted(L.SIGNATURES) == names


def test_enum_values_match_header():
    text = header_text()
    for name in ("MG_OK", "MG_EINVAL", "MG_ENOMEM", "MG_EHIP", "MG_ENOCONV", "MG_ENONFINITE",
                 "MG_BC_NEUMANN", "MG_PREC_FP64", "MG_PREC_MIXED", "MG_FLAG_ZERO_GUESS",
                 "MG_FLAG_TIMING", "MG_FLAG_FCG", "MG_FLAG_LEVEL_LAUNCHES", "MG_K_SWEEP", "MG_K_RESTRICT", "MG_K_PROLONG", "MG_K_OUTER",
                 "MG_K_NORM", "MG_K_SWEEP2", "MG_K_SWEEP2R", "MG_K_COUNT"):
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m, name
        assert int(m.group(1)) == getattr(L, name), name
    for name in ("MG_HIST_MAX", "MG_MAX_LEVELS"):
        m = re.search(rf"#define\s+{name}\s+(\d+)", text)
        assert int(m.group(1)) == getattr(L, name)


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mgp.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(mg_opts), sizeof(mg_stats),"
        " offsetof(mg_stats, rel_res), offsetof(mg_stats, hist), offsetof(mg_stats, kernel_ms),"
        " offsetof(mg_stats, kernel_launches), offsetof(mg_stats, kernel_bytes)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals == [ctypes.sizeof(L.MgOpts), ctypes.sizeof(L.MgStats), L.MgStats.rel_res.offset,
                    L.MgStats.hist.offset, L.MgStats.kernel_ms.offset, L.MgStats.kernel_launches.offset,
                    L.MgStats.kernel_bytes.offset]


@pytest.mark.parametrize("dims,cm,expect", [
    ((512, 512, 512), 4, 8), ((32, 32, 32), 4, 4), ((48, 48, 48), 4, 5), ((64, 64, 16), 4, 5),
    ((4, 4, 4), 4, 1), ((7, 8, 8), 4, 0), ((64, 64, 8), 4, 0), ((0, 4, 4), 4, 0), ((16, 16, 16), 2, 4),
    ((16, 16, 16), 1, 5),
])
def test_plan_levels_matches_oracle_rule(dims, cm, expect):
    import oracle
    lib = L.load()
    got = lib.mg_plan_levels(L.dims_arg(dims), cm)
    assert got == expect
    assert oracle.num_levels(dims, cm) == expect


def test_setup_rejects_bad_arguments_before_any_device_work():
    lib = L.load()
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    opts = L.MgOpts(2, 2, 100, 4, L.MG_PREC_FP64, 0)
    st = lib.mg_setup(ctypes.byref(ctx), fake, fake, fake, L.dims_arg((7, 8, 8)), 1 / 8, L.MG_BC_NEUMANN,
                      ctypes.byref(opts), None)
    assert st == L.MG_EINVAL and not ctx.value
    assert "cannot be coarsened" in L.last_error(None)
    st = lib.mg_setup(ctypes.byref(ctx), fake, fake, fake, L.dims_arg((8, 8, 8)), 1 / 8, 5,
                      ctypes.byref(opts), None)
    assert st == L.MG_EINVAL and "MG_BC_NEUMANN" in L.last_error(None)
    st = lib.mg_setup(ctypes.byref(ctx), None, fake, fake, L.dims_arg((8, 8, 8)), 1 / 8, 0,
                      ctypes.byref(opts), None)
    assert st == L.MG_EINVAL
    st = lib.mg_setup(ctypes.byref(ctx), fake, fake, fake, L.dims_arg((8, 8, 8)), -1.0, 0,
                      ctypes.byref(opts), None)
    assert st == L.MG_EINVAL
    for bad in (L.MgOpts(2, 2, 0, 4, 0, 0), L.MgOpts(0, 0, 10, 4, 0, 0), L.MgOpts(2, 2, 10, 5, 0, 0),
                L.MgOpts(2, 2, 10, 4, 7, 0), L.MgOpts(2, 2, 10, 4, 0, 64), L.MgOpts(2, 2, 300, 4, 0, 0)):
        st = lib.mg_setup(ctypes.byref(ctx), fake, fake, fake, L.dims_arg((8, 8, 8)), 1 / 8, 0,
                          ctypes.byref(bad), None)
        assert st == L.MG_EINVAL and L.last_error(None) == "invalid options"
    assert lib.mg_last_error(None) is not None


def test_density_setup_rejects_bad_arguments_before_any_device_work():
    lib = L.load()
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    opts = L.MgOpts(2, 2, 100, 4, L.MG_PREC_MIXED, 0)
    st = lib.mg_setup_density(ctypes.byref(ctx), None, L.dims_arg((8, 8, 8)), 1 / 8, 0, ctypes.byref(opts), None)
    assert st == L.MG_EINVAL and not ctx.value and L.last_error(None) == "NULL argument"
    st = lib.mg_setup_density(ctypes.byref(ctx), fake, L.dims_arg((7, 8, 8)), 1 / 8, 0, ctypes.byref(opts), None)
    assert st == L.MG_EINVAL and "cannot be coarsened" in L.last_error(None)
    st = lib.mg_setup_density(ctypes.byref(ctx), fake, L.dims_arg((8, 8, 8)), 1 / 8, 3, ctypes.byref(opts), None)
    assert st == L.MG_EINVAL and "MG_BC_NEUMANN" in L.last_error(None)
    assert lib.mg_update_density(None, fake) == L.MG_EINVAL
    assert lib.mg_set_timing_classes(None, 1) == L.MG_EINVAL
    assert lib.mg_density_from_vof(fake, fake, L.dims_arg((4, 0, 4)), 1.0, 1.0, 1.0, fake, None) == L.MG_EINVAL
    assert lib.mg_density_from_vof(fake, fake, L.dims_arg((4, 4, 4)), 1.0, -1.0, 1.0, fake, None) == L.MG_EINVAL
    assert lib.mg_density_from_vof(fake, None, L.dims_arg((4, 4, 4)), 1.0, 1.0, 1.0, fake, None) == L.MG_EINVAL
    assert lib.mg_faces_from_density(fake, L.dims_arg((4, 4, 0)), fake, fake, fake, None) == L.MG_EINVAL
    assert lib.mg_faces_from_density(None, L.dims_arg((4, 4, 4)), fake, fake, fake, None) == L.MG_EINVAL
    assert lib.mg_density_grad(fake, L.dims_arg((0, 4, 4)), fake, fake, fake, fake, None) == L.MG_EINVAL
    assert lib.mg_density_grad(fake, L.dims_arg((4, 4, 4)), fake, None, fake, fake, None) == L.MG_EINVAL


def test_context_free_calls_validate_arguments():
    lib = L.load()
    fake = ctypes.c_void_p(0x1000)
    assert lib.mg_faces_from_vof(fake, fake, L.dims_arg((0, 4, 4)), 1.0, 1.0, 1.0, fake, fake, fake,
                                 None) == L.MG_EINVAL
    assert lib.mg_faces_from_vof(fake, fake, L.dims_arg((4, 4, 4)), -1.0, 1.0, 1.0, fake, fake, fake,
                                 None) == L.MG_EINVAL
    assert lib.mg_divergence(fake, fake, None, L.dims_arg((4, 4, 4)), 0.25, 1.0, fake, None) == L.MG_EINVAL
    assert lib.mg_divergence(fake, fake, fake, L.dims_arg((4, 4, 4)), 0.0, 1.0, fake, None) == L.MG_EINVAL
    assert lib.mg_solve(None, fake, fake, 1e-10, None) == L.MG_EINVAL
    assert lib.mg_last_error(None) is not None
    lib.mg_destroy(None)


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle, and the library loader fails loudly."""
    pkg = os.path.join(ROOT, "paper_2605_30082_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "mg_oracle" not in text and "liboracle" not in text, f
    src = open(os.path.join(pkg, "_lib.py")).read()
    assert "raise ImportError" in src
