"""CPU-side checks of the C-ABI: the library loads and exports every symbol
declared in include/vd.h; host-only entry points behave without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "vd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vd_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2509_07175_amd as vd
    if not os.path.exists(vd.LIB_PATH):
        pytest.fail("libvd.so is not built (python -m paper_2509_07175_amd.build)")
    lib = C.CDLL(vd.LIB_PATH)
    names = _declared()
    assert "vd_clip_cells" in names and "vd_cell_moments_backward" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(vd.exported_symbols())


def test_host_only_entry_points():
    import paper_2509_07175_amd as vd
    lib = vd.load()
    o = vd.Options.default()
    assert o.sites_per_cell == 2.0 and o.improved_search == 0 and o.use_straddle_edges == 0
    assert lib.vd_status_string(4) == b"VD_ERR_CAPACITY"
    assert lib.vd_status_string(6) == b"VD_ERR_NOT_READY"
    assert lib.vd_domain_info(None, None) == 1
    assert lib.vd_domain_adjacency(None, None, None) == 1
    # argument checks happen before any device work
    h = C.c_void_p()
    assert lib.vd_build_grid(None, 10, None, 0.0, 0.0, None, C.byref(h)) == 1
    assert b"n < 1" in lib.vd_last_error() or b"NULL" in lib.vd_last_error()
    assert lib.vd_clip_cells(None, None, None, None, C.byref(h)) == 1


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2509_07175_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "vd_oracle" not in txt, f


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: --gpus 2 exits with status 2 and a
    message, before any device work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets that a C
    compiler gives the structs of include/vd.h."""
    import shutil
    import subprocess
    import paper_2509_07175_amd as vd
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"vd_options": vd.Options, "vd_cells_info_t": vd._Info, "vd_cells_view_t": vd._View,
               "vd_domain_info_t": vd._DomainInfo, "vd_batch": vd._Batch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(py, fname).offset, f"{cname}.{fname}"
