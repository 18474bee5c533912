"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/spcg.h declares, and its host-side sketch randomness equals the
oracle's bit for bit (Sec. 2.1 SRHT signs/permutation, Sec. 2.2 nested sets).
No compute call touches a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.sketch import hat_slot_rows, input_perm, sign_vector, slot_rows

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spcg.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(spcg_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2607_25272_amd as spcg
    return spcg.load()


def test_header_declares_the_boundary_entry_points():
    names = _declared_functions()
    for required in ("spcg_sketch", "spcg_precond_build", "spcg_pcg_stage", "spcg_solve"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(lib._name)
    missing = [n for n in _declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2607_25272_amd import _lib
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(_declared_functions()) <= bound


def test_version_string(lib):
    assert b"gfx950" in lib.spcg_version()


@pytest.mark.parametrize("seed,L,m,r", [(1, 15, 12800, 300), (20261203, 11, 1024, 96),
                                        (7, 3, 6, 5), (2**63 + 5, 20, 4096, 64)])
def test_host_tables_equal_oracle(seed, L, m, r):
    import paper_2607_25272_amd as spcg
    t = spcg.spcg_sketch_tables_host(seed, L, m, r)
    assert np.array_equal(t["slot_rows"], slot_rows(seed, L, m))
    assert np.array_equal(t["hat_rows"], hat_slot_rows(seed, L, r))
    assert np.array_equal(t["input_perm"], input_perm(seed, L))
    bits = np.unpackbits(t["sign_bits"], bitorder="little")[: 1 << L]
    assert np.array_equal(1.0 - 2.0 * bits, sign_vector(seed, L))


def test_host_tables_reject_bad_sizes(lib):
    import paper_2607_25272_amd as spcg
    with pytest.raises(spcg.SpcgError):
        spcg.spcg_sketch_tables_host(1, 4, 17, 1)
    assert lib.spcg_sketch_tables_host(1, 0, 1, 1, None, None, None, None) == spcg.SPCG_E_INVALID_ARG


def test_null_arguments_are_rejected_without_a_device(lib):
    import paper_2607_25272_amd as spcg
    from paper_2607_25272_amd import _lib
    assert lib.spcg_ctx_create(0, None, None) == spcg.SPCG_E_INVALID_ARG
    assert lib.spcg_ctx_destroy(None) == spcg.SPCG_E_INVALID_ARG
    assert lib.spcg_sketch_get_info(None, None) == spcg.SPCG_E_INVALID_ARG
    o = _lib.SolveOpts()
    lib.spcg_solve_opts_default(ctypes.byref(o))
    assert (o.a, o.T, o.sketch.seed, o.sketch.growth) == (3, 100, 1, 2)
    assert abs(o.tol - 5e-7) < 1e-20


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler
    gives the header's structs."""
    import subprocess

    from paper_2607_25272_amd import _lib
    structs = {"spcg_mat": _lib.SpcgMat, "spcg_sketch_opts": _lib.SketchOpts,
               "spcg_sketch_info": _lib.SketchInfo, "spcg_precond_opts": _lib.PrecondOpts,
               "spcg_stage_opts": _lib.StageOpts, "spcg_stage_stats": _lib.StageStats,
               "spcg_solve_opts": _lib.SolveOpts, "spcg_solve_stats": _lib.SolveStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spcg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_schedule_constants_match_the_oracle():
    from oracle import mlp
    from paper_2607_25272_amd import _lib
    assert (_lib.SPCG_MLP_F, _lib.SPCG_MLP_H, _lib.SPCG_MLP_O) == (mlp.F, mlp.H, mlp.O)
    assert _lib.SPCG_MLP_PARAMS == mlp.n_params()
    assert _lib.SPCG_MLP_S_SCALE == mlp.S_SCALE and _lib.SPCG_MLP_LAMBDA == mlp.LAMBDA
