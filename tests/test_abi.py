"""The C-ABI library loads and exports every entry point include/bm.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2512_14193_amd import binding, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "bm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|void|const char \*)\s*(bm_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        build.build(verbose=False)
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == names


def test_strerror_without_device():
    lib = binding.lib()
    assert lib.bm_strerror(0) == b"ok"
    assert lib.bm_strerror(-1) == b"invalid argument"
    assert b"singular" in lib.bm_strerror(3)


def test_problem_bytes_without_device():
    # host arithmetic only: the sum of bm_create's allocations
    b = {n: binding.problem_bytes(n) for n in (512, 1024, 2048, 4096)}
    for n, v in b.items():
        # blocks and U33 (80 N^2 bytes), O(N) vectors, the exchange buffers (34 MB),
        # the split-K partials of the solve (at most 1024 x 256 rows x 32 columns)
        # and those of the Schur complement beside the LU (16 slices of N x 64)
        assert 80 * n * n < v < 80 * n * n + (4096 + 16 * 64 * 16) * n + 200 * 2 ** 20, (n, v)
    # the Schur partials only where the segmented product is available (N <= 4096)
    assert binding.problem_bytes(4098) - binding.problem_bytes(4096) < 80 * (4098 ** 2 - 4096 ** 2) + 2 ** 20
    assert binding.problem_bytes(512, "ordinary") < b[512]
    lib = binding.lib()
    out = ctypes.c_int64(0)
    for n in (7, 9, 0, 65538):
        assert lib.bm_problem_bytes(n, 0, ctypes.byref(out)) == binding.BM_E_ARG
    assert lib.bm_strerror(binding.BM_E_BUDGET).startswith(b"request exceeds")
    assert lib.bm_strerror(binding.BM_E_CANCELED) == b"request canceled"


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the C layout (sizes and field
    offsets from a C program compiled against include/bm.h)."""
    import subprocess
    structs = {"bm_geometry": binding.BMGeometry, "bm_params": binding.BMParams,
               "bm_server_config": binding.BMServerConfig, "bm_request": binding.BMRequest,
               "bm_request_result": binding.BMRequestResult, "bm_server_counters": binding.BMServerCounters,
               "bm_fds_config": binding.BMFdsConfig}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        cname, f, v = line.split()
        got[(cname, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
