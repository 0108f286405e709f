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
    for need in ("count_exact", "count_baseline", "hm_graph_create", "hm_graph_destroy", "hm_num_classes"):
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


def test_null_arguments_are_refused_before_the_device():
    # argument checks run on the host and return before any HIP call
    import ctypes
    import paper_2209_10241_amd as hm
    lib = hm.lib()
    buf = (ctypes.c_uint64 * 256)()
    assert lib.count_baseline(None, 4, buf, buf, None) == hm.binding.HM_EINVAL
    assert lib.count_baseline(None, 4, None, None, None) == hm.binding.HM_EINVAL
    assert lib.count_exact(None, 4, buf, None) == hm.binding.HM_EINVAL
    # count_exact_many: counts, workers and order are checked before any HIP call
    E, U = hm.binding.HM_EINVAL, hm.binding.HM_EUNSUPPORTED
    assert lib.count_exact_many(-1, None, None, None, None, None, 1, 4, None, 3, None) == E
    assert lib.count_exact_many(2, None, None, None, None, None, 1, 4, None, 0, None) == E
    assert lib.count_exact_many(2, None, None, None, None, None, 1, 4, None, 17, None) == E
    assert lib.count_exact_many(2, None, None, None, None, None, 1, 5, None, 3, None) == U
    assert lib.count_exact_many(2, None, None, None, None, None, 1, 4, None, 3, None) == E
    assert "NULL" in hm.lib().hm_last_error().decode()
    assert lib.count_exact_many(0, None, None, None, None, None, 1, 4, None, 3, None) == hm.binding.HM_OK


def test_options_host_logic():
    """Options are process-wide host settings: values in range are kept, values
    out of range and unknown options are refused (no GPU call)."""
    import paper_2209_10241_amd as hm
    cases = [(hm.HM_OPT_BITSET_MAX_NODES, 8192, [-1, 8193]),
             (hm.HM_OPT_SAMPLE_CHUNK_SCALE, 1, [0, 1025]),
             (hm.HM_OPT_ONE_PASS_MAX_EDGES, 1 << 20, [-1, (1 << 20) + 1]),
             (hm.HM_OPT_HUB_MIN_DEGREE, 256, [-1, 1 << 32]),
             (hm.HM_OPT_DEDUP_TAG_BITS, 32, [-2, 33])]
    for opt, default, bad in cases:
        assert hm.hm_get_option(opt) == default
        for b in bad:
            with pytest.raises(hm.HMError):
                hm.hm_set_option(opt, b)
        assert hm.hm_get_option(opt) == default
        hm.hm_set_option(opt, default - 1 if default > 1 else default + 1)
        assert hm.hm_get_option(opt) == (default - 1 if default > 1 else default + 1)
        hm.hm_set_option(opt, default)
    with pytest.raises(hm.HMError):
        hm.hm_set_option(99, 1)


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_sample_sizes_rule():
    """Stratum sample sizes (Section 5; the 1:3:2 split of the appendix's
    parameter search), host only: proportional is ceil(f |E_j|); the paper's
    split gives every non-empty stratum at least one draw and an empty one none."""
    import math
    import paper_2209_10241_amd as hm
    n = (1000, 400, 37)
    got = hm.hm_sample_sizes_for(4, n, 0.013)
    assert got == {2: math.ceil(0.013 * 1000), 3: math.ceil(0.013 * 400), 4: math.ceil(0.013 * 37)}
    assert hm.hm_sample_sizes_for(3, n, 0.5) == {2: 500, 3: 200, 4: 0}
    # S = ceil(0.1 * 1437) = 144 -> 24 / 72 / 48
    assert hm.hm_sample_sizes_for(4, n, 0.1, hm.HM_ALLOC_PAPER) == {2: 24, 3: 72, 4: 48}
    # S = ceil(0.001 * 1437) = 2 < 6: floor(S/6) would leave the pairs undrawn
    small = hm.hm_sample_sizes_for(4, n, 0.001, hm.HM_ALLOC_PAPER)
    assert small == {2: 1, 3: 1, 4: 1}
    assert hm.hm_sample_sizes_for(4, (0, 400, 37), 0.001, hm.HM_ALLOC_PAPER)[2] == 0
    for bad in (0.0, 1.5, float("nan")):
        with pytest.raises(hm.HMError):
            hm.hm_sample_sizes_for(4, n, bad)
    with pytest.raises(hm.HMError):
        hm.hm_sample_sizes_for(4, n, 0.1, 7)
    with pytest.raises(hm.HMError) as e:
        hm.hm_sample_sizes_for(5, n, 0.1)
    assert e.value.code == -2
