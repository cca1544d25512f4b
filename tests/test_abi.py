"""The C-ABI library loads and exports every entry point include/ising.h
declares; host-only calls work without a GPU."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ising.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("ising_create_csr", "ising_create_dense", "ising_solve", "ising_energy",
                 "ising_default_params", "ising_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2509_01928_amd as L
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [name for name in declared_symbols() if not hasattr(lib, name)]
    assert not missing, missing


def test_host_only_calls():
    import paper_2509_01928_amd as L
    assert L.ising_version().count(".") == 2
    assert L.ising_status_string(L.ISING_OK) == "ok"
    assert "symmetric" in L.ising_status_string(3)
    assert L.ising_status_string(99) == "unknown status"
    # argument errors are reported before any device work
    out = ctypes.c_void_p()
    st = L.lib.ising_create_csr(0, 0, None, None, None, L.ISING_F32, None, 0, None,
                                ctypes.byref(out))
    assert st == L.ISING_E_INVALID_ARG and out.value is None
    assert "n=0" in L.ising_last_error()
    st = L.lib.ising_solve(None, None, 1, 1, None, None, None, None, None)
    assert st == L.ISING_E_INVALID_ARG
    L.ising_destroy(None)


def test_struct_layouts_match_header(tmp_path):
    """The binding's structures have the sizes and field offsets the C
    header gives them (compiled with the host C compiler)."""
    import subprocess
    import paper_2509_01928_amd as L
    fields = {"ising_params": ["alpha", "beta", "eps", "algo", "q", "x_dtype", "reserved"],
              "ising_stats": ["iters_done", "converged", "nonfinite", "H_last", "r_last"],
              "ising_info": ["n", "n_iter", "nnz", "is_dense", "has_field", "integer_J", "val_dtype",
                             "row_len", "geometry"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ising.h"', "int main(void) {"]
    for t, fs in fields.items():
        lines.append(f'  printf("{t} %zu\\n", sizeof({t}));')
        for f in fs:
            lines.append(f'  printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c11", "-I", include, str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for t, fs in fields.items():
        cls = getattr(L, t)
        assert ctypes.sizeof(cls) == int(got[t]), t
        for f in fs:
            assert getattr(cls, f).offset == int(got[f"{t}.{f}"]), (t, f)
