"""Pins of the oracle's counter-based generator (Philox, SC'11)."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox4x32_known_answers(orc):
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_philox4x64_matches_numpy(orc):
    # numpy's Philox bit generator is the 4x64-10 member of the same family;
    # it increments the counter before the first block.  Agreement pins the
    # round structure (S-box, permutation, key schedule) shared by both widths.
    for key in ([0, 0], [123, 456], [2**64 - 1, 7]):
        g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=[0, 0, 0, 0])
        ref = [g.random_raw() for _ in range(8)]
        got = list(orc.philox4x64_10([1, 0, 0, 0], key)) + list(orc.philox4x64_10([2, 0, 0, 0], key))
        assert [int(x) for x in got] == [int(x) for x in ref]


def test_philox_uniform_statistics(orc):
    # top-24-bit uniforms of successive counters: mean 1/2, variance 1/12
    u = []
    for i in range(4000):
        x = orc.philox4x32_10([i, 7, 3, 0], [11, 0])
        u.extend((x >> 8) / 2.0 ** 24)
    u = np.array(u)
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.01


def test_philox_batch_equals_single_calls(orc):
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2 ** 32, (257, 4), dtype=np.uint64).astype(np.uint32)
    got = orc.philox4x32_10(c, [5, 9])
    for i in (0, 1, 100, 256):
        assert got[i].tolist() == orc.philox4x32_10(c[i], [5, 9]).tolist()


def test_oracle_binding_structs_match_its_header(tmp_path):
    # the oracle's camera and render parameters as the binding lays them out
    # equal the C header's (a C program built against oracle/ugp_oracle.h)
    import ctypes as C
    import shutil
    import subprocess
    import oracle as O
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"orc_camera": O._Camera, "orc_render_params": O._Params}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ugp_oracle.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(root, "oracle"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
