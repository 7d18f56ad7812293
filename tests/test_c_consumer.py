"""CPU: a plain C99 program built against include/hexval.h and libhexval.so.
The header compiles as strict C, the struct layouts the C compiler sees are
the ones the ctypes binding declares, and argument errors come back as
status codes without a GPU."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1706_01613_amd import hexval as hx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1706_01613_amd")

STRUCTS = {
    "hexval_mesh_t": ["points", "n_points", "connectivity", "n"],
    "hexval_stats_t": ["n_elements", "n_subdivided", "n_nodes", "n_exact", "n_recheck", "n_rounds",
                       "max_level", "timing", "ms_first_pass", "ms_recheck", "ms_subdivision",
                       "ms_total", "block_threads", "n_exact_host", "grid_blocks", "walk_layers",
                       "reserved", "walk_stride"],
    "hexval_opts_t": ["precision", "max_depth", "validate_indices", "block_threads",
                      "queue_capacity", "grid_blocks", "stream", "stats", "walk_layers", "reserved"],
    "hexval_request_t": ["mesh", "host_points", "host_conn", "verdicts", "min_coeffs"],
}


def _program():
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hexval.h"', "int main(void) {"]
    for name, fields in STRUCTS.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'    printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += [
        "    hexval_opts_t o;",
        "    hexval_opts_default(&o);",
        '    printf("default %d %d %d\\n", o.precision, o.max_depth, o.validate_indices);',
        '    printf("null_points %d\\n", hexval_check(NULL, NULL, 5, NULL, NULL));',
        '    printf("negative_n %d\\n", hexval_check(NULL, NULL, -1, NULL, NULL));',
        '    printf("empty %d\\n", hexval_check(NULL, NULL, 0, NULL, NULL));',
        "    return 0;",
        "}",
    ]
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def c_output(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(PKG, "libhexval.so")):
        pytest.fail("libhexval.so is not built")
    d = tmp_path_factory.mktemp("c_consumer")
    src, exe = d / "consumer.c", d / "consumer"
    src.write_text(_program())
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", PKG, "-lhexval",
                    f"-Wl,-rpath,{PKG}"], check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, check=True)
    out = {}
    for line in r.stdout.splitlines():
        if line.startswith("default "):
            out["default"] = line[len("default "):]
            continue
        *key, value = line.split()
        out[" ".join(key)] = value
    return out


def test_struct_layouts_match_the_binding(c_output):
    for name, fields in STRUCTS.items():
        cls = getattr(hx, name)
        assert int(c_output[f"{name} size"]) == ctypes.sizeof(cls), name
        for f in fields:
            assert int(c_output[f"{name} {f}"]) == getattr(cls, f).offset, (name, f)
        assert [f for f, _ in cls._fields_] == fields, name


def test_defaults_and_argument_errors_without_gpu(c_output):
    assert c_output["default"] == f"{hx.FP64} 6 0"
    assert int(c_output["null_points"]) == hx.E_ARG
    assert int(c_output["negative_n"]) == hx.E_ARG
    assert int(c_output["empty"]) == hx.OK
