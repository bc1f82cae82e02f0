"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every entry point include/dsmc.h declares, the ctypes structs match the C
layout, and the product package never reaches into the oracle."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsmc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dsmc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2602_21244_amd import _lib
    path = _lib.LIB_PATH
    if not os.path.exists(path):
        from paper_2602_21244_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.dsmc_version().startswith(b"dsmc-gfx950")


def test_declared_names_have_bindings():
    from paper_2602_21244_amd import _lib
    missing = [n for n in _declared() if n not in _lib.SIGNATURES]
    assert not missing, missing


def test_struct_layout_matches_header():
    from paper_2602_21244_amd import _lib as L
    structs = {"dsmc_vec3": L.Vec3, "dsmc_rng": L.Rng, "dsmc_status": L.Status,
               "dsmc_pairs": L.Pairs, "dsmc_xs": L.Xs, "dsmc_potential": L.Potential,
               "dsmc_quad": L.Quad, "dsmc_mlp": L.Mlp, "dsmc_anet": L.Anet,
               "dsmc_chi_table": L.ChiTable, "dsmc_domain": L.Domain,
               "dsmc_match_schedule": L.MatchSchedule}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write("\n".join(lines))
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-o", exe, c])
        out = subprocess.check_output([exe], text=True)
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_host_argument_errors(lib):
    from paper_2602_21244_amd import _lib as L
    # null pointers and bad sizes are rejected on the host without a GPU call
    assert lib.dsmc_sort_cells(10, 0, None, L.F64, L.Vec3(), L.Vec3(), None, None, None, 0,
                               None, None) == L.DSMC_E_ARG
    assert b"n_cells" in lib.dsmc_last_error()
    assert lib.dsmc_moment_match(4, None, L.F64, L.Vec3(), None, 0, None, None, None) == L.DSMC_E_ARG
    assert lib.dsmc_set_block_threshold(0) == L.DSMC_E_ARG
    assert lib.dsmc_set_block_threshold(40) == L.DSMC_OK
    assert lib.dsmc_get_block_threshold() == 40
    assert lib.dsmc_select_pairs_ntc_ws(100, 1000) > 4 * 100
    # angle network / table: null structs and bad shapes
    assert lib.dsmc_anet_forward(None, 10, None, None, None, 0, None) == L.DSMC_E_ARG
    a = L.Anet()
    a.n_layers = 2
    a.dims[0], a.dims[1], a.dims[2] = 3, 8, 1     # dims[0] must be 2
    assert lib.dsmc_anet_ws(C.byref(a), 10) == 0
    assert lib.dsmc_huber_loss(0, None, None, None, None, None) == L.DSMC_E_ARG
    assert lib.dsmc_apply_pairs_match(4, None, L.F64, L.Vec3(), L.Pairs(), 0, None, L.MM_APPLY,
                                      None, 0, None, None) == L.DSMC_E_ARG
    d = L.Domain()
    d.nx, d.ny, d.Lx, d.Ly, d.m = 4, 4, 1.0, 1.0, 1.0
    d.kind[0], d.kind[1], d.kind[2], d.kind[3] = 0, 1, 2, 2       # periodic side without partner
    for q in range(4):
        d.T_w[q] = 300.0
    assert lib.dsmc_move(10, L.F64, L.Vec3(), L.Vec3(), C.byref(d), 1.0, L.Rng(), None, None,
                         None) == L.DSMC_E_ARG
    assert b"periodic" in lib.dsmc_last_error()
    assert lib.dsmc_gather(5, L.F64, None, L.Vec3(), L.Vec3(), None) == L.DSMC_E_ARG
    assert lib.dsmc_sample(0, None, L.F64, L.Vec3(), None, None) == L.DSMC_E_ARG
    assert lib.dsmc_sample_fields(3, None, 1.0, 1.0, 1.0, None, None) == L.DSMC_E_ARG
    t = L.ChiTable(1, 4, 0.0, 1.0, None)
    assert lib.dsmc_collide_table(C.byref(t), 4, L.F64, L.Vec3(), L.Pairs(), L.Rng(), 1.0, 0,
                                  None, 0, None) == L.DSMC_E_ARG


def test_product_package_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2602_21244_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "dsmc_oracle" not in src, f
