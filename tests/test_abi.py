"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/eis.h declares, and its pure host arithmetic is right.  No compute
call is made here (there is no GPU in this environment)."""
import ctypes
import os
import re

import pytest

import paper_2507_06579_amd as eis
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "eis.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(eis_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_is_built_and_loads():
    assert os.path.exists(eis.lib_path()), "run __graft_entry__.build() first"
    eis.lib()


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(eis.lib_path())
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(eis.EXPORTED_SYMBOLS)


def test_abi_version_and_strings():
    assert eis.eis_abi_version() == eis.ABI_VERSION == 8
    for st in eis.Status:
        assert eis.eis_strerror(int(st))
    assert eis.eis_strerror(12345) == "unknown status"


@pytest.mark.parametrize("a,b", [(0, 0), (5, 5), (6, 5), (5, 6), (6, 13), (6, 14), (0, 10**6 + 1),
                                 (10**9, 10**9 + 10**7), (10**11 - 10**8, 10**11),
                                 (123456789, 123456790), (10**12 - 7, 10**12)])
def test_candidate_lattice_matches_oracle(a, b):
    assert eis.eis_num_candidates(a, b) == oracle.num_candidates(a, b)
    assert eis.eis_first_candidate(a) == oracle.first_candidate(a)


def test_create_without_gpu_fails_loudly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(eis.EisError) as ei:
        eis.Context()
    assert ei.value.status == eis.Status.EDEVICE


def test_no_oracle_in_product_sources():
    pkg = os.path.join(ROOT, "paper_2507_06579_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    src = f.read()
                assert "import oracle" not in src and "liboracle" not in src, fn
                assert "orc_" not in src, fn
