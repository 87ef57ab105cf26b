"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and rejects invalid arguments on the host before any
HIP call."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gabm.h")


@pytest.fixture(scope="module")
def L():
    from paper_2207_09714_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2207_09714_amd import build

        build.build()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:gabm_status|const char \*)\s*(gabm_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gabm_graph_build", "gabm_graph_info", "gabm_graph_destroy", "gabm_er_daily",
                     "gabm_transmit_fwd", "gabm_sample_infect", "gabm_progress_stages", "gabm_transmit_bwd",
                     "gabm_param_grad_reduce", "gabm_day_fwd", "gabm_day_bwd", "gabm_sim_workspace_size"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(L.EXPORTS)
    assert lib.gabm_version().decode().startswith("gabm")


def test_graph_build_rejects_bad_arguments_on_host(L):
    lib = L.lib()
    h = C.c_void_p()
    assert lib.gabm_graph_build(None, None, C.byref(h)) == L.EINVAL
    assert b"NULL" in lib.gabm_last_error()
    offs = np.array([0, 10], np.int32)
    age = np.zeros(10, np.uint8)  # never dereferenced: validation fails first
    d = L.GraphDesc()
    d.n_agents, d.n_pops, d.pop_offsets, d.age, d.n_age, d.n_edges = 0, 1, offs.ctypes.data, age.ctypes.data, 8, 0
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    d.n_agents = 10
    d.n_age = 0
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    d.n_age = 17
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    d.n_age = 8
    bad = np.array([0, 9], np.int32)
    d.pop_offsets = bad.ctypes.data
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    assert b"pop_offsets" in lib.gabm_last_error()
    nonmono = np.array([0, 5, 5, 10], np.int32)
    d.pop_offsets, d.n_pops = nonmono.ctypes.data, 3
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    d.pop_offsets, d.n_pops = offs.ctypes.data, 1
    d.n_edges = 5  # src/dst NULL
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    d.n_edges = 0
    d.er_mean_deg = float("nan")
    assert lib.gabm_graph_build(C.byref(d), None, C.byref(h)) == L.EINVAL
    assert h.value is None


def test_other_entry_points_reject_null_handles(L):
    lib = L.lib()
    p = L.Params()
    r = L.Rng()
    s = L.GraphStats()
    assert lib.gabm_graph_info(None, C.byref(s)) == L.EINVAL
    assert lib.gabm_transmit_fwd(None, None, 0, C.byref(p), 0, C.byref(r), 0, None, None, None) == L.EINVAL
    assert lib.gabm_sample_infect(None, None, C.byref(p), C.byref(r), 0, None, None, None, None) == L.EINVAL
    assert lib.gabm_transmit_bwd(None, None, C.byref(r), 0, None, None) == L.EINVAL
    assert lib.gabm_sim_forward(None, C.byref(p), C.byref(r), None, 0, None, None) == L.EINVAL
    assert lib.gabm_sim_backward(None, C.byref(p), C.byref(r), None, None, None, None) == L.EINVAL
    assert lib.gabm_sim_destroy(None) == L.OK
    assert lib.gabm_graph_destroy(None) == L.OK


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2207_09714_amd import _lib

    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_binding_structs_match_the_header(L, tmp_path):
    """Every struct the binding passes across the ABI has the size and field
    offsets the C header gives it (the header compiled by the host C compiler)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"gabm_graph_desc": L.GraphDesc, "gabm_graph_stats": L.GraphStats, "gabm_params": L.Params,
               "gabm_rng": L.Rng, "gabm_run_desc": L.RunDesc, "gabm_kernel_times": L.KernelTimes,
               "gabm_fwd_out": L.FwdOut, "gabm_grads": L.Grads}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gabm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            cname, key, val = line.split()
            got[(cname, key)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
