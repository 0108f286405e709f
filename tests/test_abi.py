"""The C-ABI library loads on the CPU and exports every entry point that
include/homotif.h declares; host-only queries agree with the oracle."""
import os
import re

import pytest

from oracle.classes import table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "homotif.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("count_exact", "hm_graph_create", "hm_graph_destroy", "hm_num_classes"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2209_10241_amd as hm
    lib = hm.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared entry point
    from paper_2209_10241_amd.binding import SIGNATURES
    assert sorted(SIGNATURES) == _declared()


@pytest.mark.parametrize("k", [3, 4])
def test_host_class_table_matches_oracle(k):
    import paper_2209_10241_amd as hm
    t = table(k)
    assert hm.hm_num_classes(k) == t.n_classes
    for c in range(t.n_classes):
        assert hm.hm_class_info(k, c) == (t.canon_masks[c], t.maxcard[c], t.countmax[c])
    for p in range(1 << t.n_bits):
        assert hm.hm_pattern_class(k, p) == t.class_of[p]


def test_host_errors():
    import paper_2209_10241_amd as hm
    with pytest.raises(hm.HMError) as e:
        hm.hm_num_classes(5)
    assert e.value.code == -2
    with pytest.raises(hm.HMError):
        hm.hm_class_info(4, 171)
    with pytest.raises(hm.HMError):
        hm.hm_pattern_class(4, 2048)
