"""The C-ABI library loads on the CPU host and exports every function that
include/refeig.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "refeig.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|char\s*\*|const char\s*\*)\s*\*?\s*(\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    path = os.path.join(ROOT, "paper_2602_19090_amd", "librefeig.so")
    if not os.path.exists(path):
        from paper_2602_19090_amd import build
        build.build()
    from paper_2602_19090_amd import binding   # loads torch's HIP runtime first
    return binding._lib


def test_header_declares_expected_functions():
    names = _declared()
    for f in ("refine_eigvecs", "refeig_workspace_bytes", "refeig_default_opts", "refeig_strerror",
              "refeig_split_cols", "refeig_slice_gemm", "refine_eigvecs_herm",
              "refeig_herm_workspace_bytes", "refeig_slice_gemm_fp8", "refeig_digits_to_e4m3",
              "refeig_server_create", "refeig_server_submit", "refeig_server_wait",
              "refeig_server_destroy"):
        assert f in names, names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_host_only_entry_points(lib):
    """Entry points that touch no device memory work on a host without a GPU."""
    from paper_2602_19090_amd import binding as rb
    o = rb.default_opts()
    assert o.max_iter == 8 and o.delta_safety == 8.0 and o.mode == rb.REFEIG_OZAKI_INT8
    assert rb.strerror(rb.REFEIG_E_GAP).startswith("two eigenvalue")
    b = rb.workspace_bytes(8192)
    assert 8e9 < b < 24e9   # n = 8192: planes, slots, and A residues at up to 4 digit levels
    with pytest.raises(ValueError):
        rb.workspace_bytes(0)
    hb = rb.herm_workspace_bytes(4096)
    assert 4e9 < hb < 12e9
    with pytest.raises(ValueError):
        rb.herm_workspace_bytes(4097)


def test_mfma_probe_rejects_bad_arguments_without_a_gpu():
    """refeig_mfma_ceiling checks its arguments before any HIP call."""
    import ctypes
    from paper_2602_19090_amd import binding as rb
    out = [ctypes.c_double() for _ in range(3)]
    for variant, seconds in ((3, 0.1), (-1, 0.1), (0, 0.0), (0, 11.0)):
        st = rb._lib.refeig_mfma_ceiling(variant, seconds, None, *[ctypes.byref(o) for o in out])
        assert st == rb.REFEIG_E_ARG, (variant, seconds, st)
    assert rb._lib.refeig_mfma_ceiling(0, 0.1, None, None, None, None) == rb.REFEIG_E_ARG


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a C program that gcc builds."""
    import subprocess
    import tempfile
    lines = [f'printf("%zu\\n", sizeof({struct}));']
    lines += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src = ("#include <stdio.h>\n#include <stddef.h>\n#include \"refeig.h\"\nint main(void) {\n"
           + "\n".join(lines) + "\nreturn 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("cname,pyname", [("refeig_opts", "Opts"), ("refeig_report", "Report")])
def test_binding_struct_layout_matches_header(lib, cname, pyname):
    """Every ctypes field sits at the offset the C compiler gives it in the header."""
    from paper_2602_19090_amd import binding as rb
    py = getattr(rb, pyname)
    fields = [f for f, _ in py._fields_]
    size, offs = _c_layout(cname, fields)
    assert ctypes.sizeof(py) == size
    for f, off in zip(fields, offs):
        assert getattr(py, f).offset == off, f


def test_binding_lists_every_declared_symbol():
    """binding.EXPORTED names exactly the functions the header declares."""
    from paper_2602_19090_amd import binding as rb
    assert sorted(rb.EXPORTED) == _declared()


def test_graph_batch_rejects_bad_options_without_a_gpu():
    """refeig_batch_workspace_bytes is host-only: it refuses options the captured batch cannot
    run (no fixed iteration count, host planning, a padded order above 4096)."""
    from paper_2602_19090_amd import binding as rb
    with pytest.raises(ValueError):
        rb.batch_workspace_bytes([64, 100], rb.default_opts())
    with pytest.raises(ValueError):
        rb.batch_workspace_bytes([64, 100], rb.default_opts(fixed_iters=2, plan=1))
    with pytest.raises(ValueError):
        rb.batch_workspace_bytes([64, 4200], rb.default_opts(fixed_iters=2))
    assert rb.batch_workspace_bytes([64, 100], rb.default_opts(fixed_iters=2)) > 0
