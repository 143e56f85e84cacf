"""The C-ABI library loads and exports every entry point its headers declare
(no compute calls: this runs without a GPU)."""

import os
import re

import numpy as np
import pytest

from paper_1607_00315_amd import sic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(sic_[A-Za-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_is_built():
    assert os.path.exists(sic.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    L = sic.lib()
    declared = _declared()
    assert len(declared) >= 20
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_the_headers():
    assert _declared() == set(sic.SIGNATURES)


def test_error_strings_without_device():
    assert sic.strerror(sic.SIC_EINVAL) == "invalid argument"
    assert sic.strerror(sic.SIC_ENOCONV).startswith("not converged")
    assert sic.strerror(12345) == "unknown error"


def test_host_hierarchy_matches_oracle():
    """The level-set ranking is host logic in the library (no device work)."""
    from oracle import steps
    rng = np.random.default_rng(9)
    n = 5000
    supp = np.unique(rng.integers(0, n * n, 800))
    free = np.unique(np.concatenate([rng.integers(0, n * n, 20000), supp[:300]]))
    g = np.round(rng.random(free.size), 3)      # many ties
    r1, s1 = sic.hierarchy(n, supp, free, g)
    r2, s2 = steps.hierarchy(supp, free, g)
    assert np.array_equal(r1, r2)
    assert [int(x) for x in s1] == [int(x) for x in s2]
