"""The C-ABI library builds, loads and exports every declared entry point (no GPU).

Only host-side calls that never touch a device are made here.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flexiwalk.h")
LIB = os.path.join(ROOT, "paper_2512_00705_amd", "libflexiwalk.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fw_[a-z_0-9]+)\s*\(", text)))


if not os.path.exists(LIB):  # a fresh checkout: build once (hipcc cross-compiles without a GPU)
    subprocess.check_call([sys.executable, os.path.join(ROOT, "paper_2512_00705_amd", "_build.py")])


@pytest.fixture(scope="module")
def lib():
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_exported(lib):
    names = _declared()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(fw_[a-z_0-9]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert getattr(lib, n) is not None


def test_binding_names_match_header():
    import paper_2512_00705_amd as fw
    assert sorted(fw.EXPORTED) == _declared()
    for n in fw.EXPORTED:
        assert callable(getattr(fw, n))


def test_host_only_argument_checks():
    import paper_2512_00705_amd as fw
    with pytest.raises(fw.FlexiWalkError) as e:
        fw.fw_logic_node2vec(0.0, 1.0)
    assert e.value.code == fw.FW_E_INVALID and "p and q" in fw.fw_last_error()
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_logic_node2vec(1.0, float("inf"))
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_logic_metapath([])
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_logic_metapath(list(range(65)))
    lg = fw.fw_logic_metapath([0, 1, 2, 3, 4])
    assert lg.kind == fw.FW_METAPATH and lg.schema_len == 5 and list(lg.schema[:5]) == [0, 1, 2, 3, 4]
    lg = fw.fw_logic_node2vec(2.0, 0.5, True)
    assert (lg.kind, lg.weighted, lg.p, lg.q) == (fw.FW_NODE2VEC, 1, 2.0, 0.5)
    pl = fw.fw_plan_default()
    assert (pl.rho, pl.d_lo, pl.rjs_cap, pl.lanes, pl.bound, pl.proposal) == (8.0, 0, 1024, 64, 0, 0)
    assert (pl.hub_deg, pl.hub_lanes, pl.rvs_share) == (0, 64, 0)
    with pytest.raises(fw.FlexiWalkError):
        fw.fw_graph_create(-1, 0, None, None)


def test_struct_layouts_match_header():
    """ctypes mirrors of the C structs have the sizes and field offsets the C compiler
    gives them."""
    import paper_2512_00705_amd as fw
    fields = [("fw_plan", f) for f, _ in fw.fw_plan._fields_] + [("fw_query", f) for f, _ in fw.fw_query._fields_]
    offs = "".join(f'printf("%zu\\n", offsetof({s}, {f}));' for s, f in fields)
    src = ("#include <stdio.h>\n#include <stddef.h>\n#include \"flexiwalk.h\"\nint main(void){printf(\"%zu %zu %zu\\n\","
           "sizeof(fw_csr), sizeof(fw_logic), sizeof(fw_plan));printf(\"%zu\\n\", sizeof(fw_query));" + offs +
           "return 0;}\n")
    d = os.path.join(ROOT, "_build")
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "sizes.c")
    exe = os.path.join(d, "sizes")
    open(c, "w").write(src)
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
    sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(fw.fw_csr), ctypes.sizeof(fw.fw_logic), ctypes.sizeof(fw.fw_plan),
            ctypes.sizeof(fw.fw_query)]
    want += [getattr(fw.fw_plan if s == "fw_plan" else fw.fw_query, f).offset for s, f in fields]
    assert sizes == want
