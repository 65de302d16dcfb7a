"""The C-ABI library loads and exports every entry point the header declares; host-side
validation and sizing (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2207_04252_amd import rossbi, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rossbi_mi355x.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:rb_status|const char\s*\*|void)\s+\*?\s*(rb_\w+)\s*\(", text, flags=re.M)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rossbi.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    return rossbi.load()


def test_header_declares_entry_points():
    names = declared_functions()
    assert set(names) == set(rossbi.EXPORTS), names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout():
    # rb_config: 8 int32 + 6 + 1 + 3 + 3 + 4 + 6 + 12 doubles, 2 int32, 9 doubles, 2 int32,
    # 4 doubles, 2 int32, 4 doubles, 2 int32
    assert ctypes.sizeof(rossbi.rb_config) == (8 * 4 + (6 + 1 + 3 + 3 + 4 + 6 + 12) * 8 + 2 * 4
                                               + 9 * 8 + 2 * 4 + 4 * 8 + 2 * 4 + 4 * 8 + 2 * 4)
    assert ctypes.sizeof(rossbi.rb_diag) == (8 + 8 + 4 + 4 + 8 + 8 + 8 + 4 + 4 + 5 * 8 + 5 * 8 + 8 + 8
                                             + 8 * 8 + 8)


def test_struct_layout_matches_c_compiler(tmp_path):
    """The header compiled by the host C compiler gives the binding's sizes and offsets."""
    import os
    import subprocess
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    fields = [f[0] for f in rossbi.rb_config._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", offsetof(rb_config, {f}));\n' for f in fields)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"rossbi_mi355x.h\"\n"
                   "int main(void) {\n" + body +
                   '  printf("%zu\\n%zu\\n", sizeof(rb_config), sizeof(rb_diag));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", inc, "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(rossbi.rb_config, f).offset for f in fields]
    assert got[:-2] == want
    assert got[-2:] == [ctypes.sizeof(rossbi.rb_config), ctypes.sizeof(rossbi.rb_diag)]


@pytest.mark.parametrize("name", list(synth.CONFIGS))
def test_query_sizes(lib, name):
    cfg = synth.CONFIGS[name]
    c = rossbi.to_config(cfg)
    b = rossbi.rb_buffers()
    assert lib.rb_query_sizes(ctypes.byref(c), ctypes.byref(b)) == rossbi.RB_OK
    assert b.state_bytes == cfg.n_fields * cfg.n_cells * 8
    assert b.stage_bytes == b.state_bytes
    # tables are two-dimensional (axisymmetric): small next to the state
    assert 0 < b.work_bytes < max(64 << 20, b.state_bytes // 4)


@pytest.mark.parametrize("mut", [
    dict(nr=2), dict(nth=2), dict(nz=2), dict(gamma=1.0), dict(cfl=0.0), dict(r_in=-1.0),
    dict(stokes=(0.1,) * 5, eps_dust=(0.01,) * 5, hd_over_h=(0.3,) * 5),
    dict(stokes=(-0.1,), eps_dust=(0.01,), hd_over_h=(0.3,)),
])
def test_query_sizes_rejects_bad_config(lib, mut):
    cfg = synth.C2_DISC.with_(**mut)
    c = rossbi.to_config(cfg) if cfg.n_dust <= 4 else None
    if c is None:
        c = rossbi.to_config(cfg.with_(stokes=(), eps_dust=(), hd_over_h=()))
        c.n_dust = 5
    b = rossbi.rb_buffers()
    assert lib.rb_query_sizes(ctypes.byref(c), ctypes.byref(b)) == rossbi.RB_EINVAL


def test_null_arguments_rejected(lib):
    assert lib.rb_query_sizes(None, None) == rossbi.RB_EINVAL
    assert lib.rb_step(None, 1, None, None) == rossbi.RB_EINVAL
    assert lib.rb_get_fields(None, None, 0) == rossbi.RB_EINVAL
    assert lib.rb_last_error(None) == b"null context"


def test_fp32_form_needs_a_disc_background(lib):
    """The FP32-perturbation form stores deviations from a stationary flow: the Sod
    annulus (no stationary flow) and gamma other than 7/5 are refused; drag_exact takes
    0 or 1 only."""
    b = rossbi.rb_buffers()
    sod = rossbi.to_config(synth.C1_SOD, precision=rossbi.RB_FP32_PERT)
    assert lib.rb_query_sizes(ctypes.byref(sod), ctypes.byref(b)) == rossbi.RB_EINVAL
    g53 = rossbi.to_config(synth.C2_DISC.with_(gamma=5.0 / 3.0), precision=rossbi.RB_FP32_PERT)
    assert lib.rb_query_sizes(ctypes.byref(g53), ctypes.byref(b)) == rossbi.RB_EINVAL
    ok = rossbi.to_config(synth.C2_DISC, precision=rossbi.RB_FP32_PERT)
    assert lib.rb_query_sizes(ctypes.byref(ok), ctypes.byref(b)) == rossbi.RB_OK
    bad = rossbi.to_config(synth.C3_BIFLUID)
    bad.drag_exact = 2
    assert lib.rb_query_sizes(ctypes.byref(bad), ctypes.byref(b)) == rossbi.RB_EINVAL
