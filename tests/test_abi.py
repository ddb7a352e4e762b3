"""The C-ABI library loads and exports every entry point its header declares;
host-side argument checks return status codes without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ugp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ugp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2406_09733_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2406_09733_amd import build
        build.build()
    return P.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["ugp_create", "ugp_destroy", "ugp_build_bvh", "ugp_transmittance", "ugp_sample_collision",
              "ugp_saturation", "ugp_emitter_query", "ugp_render", "ugp_sync", "ugp_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for n in _declared():
        assert hasattr(L, n), n


def test_binding_names_match_header():
    import paper_2406_09733_amd as P
    assert sorted(P.EXPORTS) == _declared()


def test_status_strings(L):
    for code in range(7):
        s = L.ugp_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0


def test_host_side_argument_checks(L):
    # none of these reach the device
    assert L.ugp_create(0, None, None) == 1
    assert L.ugp_build_bvh(None, None, C.c_float(0.01)) == 1
    assert L.ugp_refit_bvh(None, None) == 1
    assert L.ugp_transmittance(None, 1, None, None, None, None) == 1
    assert L.ugp_sample_collision(None, 1, None, None, None, None, None) == 1
    assert L.ugp_render(None, None, None, None, None) == 1
    assert L.ugp_sync(None) == 1
    assert L.ugp_destroy(None) == 1
    assert L.ugp_set_path_pool(None, C.c_int64(0)) == 1
    assert L.ugp_set_tail_paths(None, C.c_int64(0)) == 1
    assert L.ugp_accum_cdf_backward(None, None, C.c_int64(1), None, None, None, None) == 1
    assert L.ugp_rf_render_backward(None, None, C.c_int64(1), None, None, None, None) == 1


def test_create_without_gpu_reports_device_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert L.ugp_create(0, None, C.byref(h)) == 3


def test_binding_structs_match_the_header_layout(tmp_path):
    # every struct the binding passes by pointer has the header's field names,
    # offsets and size (a C program built against include/ugp.h prints them)
    import shutil
    import subprocess
    import paper_2406_09733_amd as P
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"ugp_scene": P._Scene, "ugp_camera": P._Camera, "ugp_render_params": P._Params,
               "ugp_render_stats": P._Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ugp.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU and says so for any other count
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
