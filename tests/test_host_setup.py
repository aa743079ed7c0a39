"""Host-side logic of libnls, checked on the CPU (no device is touched):
exported symbols, overlap maps and owners against the oracle (bit-exact),
band widths, GDSW interface components, and error paths."""
import ctypes

import numpy as np
import pytest

import synth
import paper_2410_24138_amd.nls as nls
from oracle import P1Problem, Schwarz
from tests._lib import ensure_built


@pytest.fixture(scope="module")
def lib():
    return ensure_built()


def test_exports_every_declared_symbol(lib):
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(nls.HERE), "include", "nls.h")).read()
    declared = set(re.findall(r"\b(nls_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(nls.SYMBOLS)
    for s in declared:
        assert hasattr(lib, s), s


CASES = [
    dict(n=12, boxes=3, overlap=1),
    dict(n=13, boxes=3, overlap=2, uneven=True),
    dict(n=16, boxes=4, overlap=2),
    dict(n=9, boxes=1, overlap=1),
]


@pytest.mark.parametrize("kw", CASES)
def test_partition_maps_match_oracle(lib, kw):
    case = synth.small_case(**kw)
    S = Schwarz(P1Problem(case), "one_level")
    m = nls.inspect_partition(case)
    for i, s in enumerate(S.subs):
        V = m["v"][m["off_v"][i]:m["off_v"][i + 1]]
        G = m["g"][m["off_g"][i]:m["off_g"][i + 1]]
        np.testing.assert_array_equal(V, s["V"])
        np.testing.assert_array_equal(G, s["Gam"])
        # band widths of the structural pattern of J_ii (node pairs of the
        # patch elements, both in V_i)
        lc = s["lconn"]
        r = np.repeat(lc, 3, axis=1).ravel()
        c = np.tile(lc, (1, 3)).ravel()
        keep = (r < len(V)) & (c < len(V))
        assert m["kl"][i] == max(0, (r[keep] - c[keep]).max())
        assert m["ku"][i] == max(0, (c[keep] - r[keep]).max())
    # the owner's copy of every node is the node itself, in the owner's V
    own = m["own_pos"]
    np.testing.assert_array_equal(m["v"][own], np.arange(len(case["xy"])))
    owner = np.searchsorted(m["off_v"], own, side="right") - 1
    np.testing.assert_array_equal(owner, S.owner)


@pytest.mark.parametrize("kw", [dict(n=12, boxes=3, overlap=1),
                                dict(n=16, boxes=4, overlap=1),
                                dict(n=13, boxes=3, overlap=2, uneven=True)])
def test_coarse_components_match_oracle(lib, kw):
    case = synth.small_case(two_level=True, **kw)
    S = Schwarz(P1Problem(case), "additive")
    comps = nls.inspect_coarse(case)
    assert len(comps) == S.n0
    for a, (b, _) in zip(comps, S.components):
        np.testing.assert_array_equal(a, b)


def test_config2_component_count(lib):
    case = synth.config2()
    comps = nls.inspect_coarse(case)
    assert len(comps) == 15 * 15 + 2 * 16 * 15


def test_partition_errors(lib):
    case = synth.small_case(n=8, boxes=2, overlap=1)
    bad = dict(case)
    bad["overlap"] = 0
    with pytest.raises(nls.NLSError) as e:
        nls.inspect_partition(bad)
    assert e.value.code == nls.NLS_EPARTITION
    bad = dict(case)
    bad["n_sub"] = 5  # subdomain 4 is empty
    with pytest.raises(nls.NLSError) as e:
        nls.inspect_partition(bad)
    assert e.value.code == nls.NLS_EPARTITION
    bad = dict(case)
    part = case["elem_part"].copy()
    part[0] = 9
    bad["elem_part"] = part
    with pytest.raises(nls.NLSError) as e:
        nls.inspect_partition(bad)
    assert e.value.code == nls.NLS_EINVAL


def test_default_options_and_strerror(lib):
    o = nls.default_options()
    assert o.outer_rtol == 1e-8 and o.gmres_restart == 50 and o.inner_maxit == 30
    assert lib.nls_strerror(nls.NLS_ELIMIT) == b"size exceeds a kernel limit"
    assert lib.nls_create(None, None) == nls.NLS_EINVAL
