"""The oracle still reproduces the stored digests of its outputs on the seeded
benchmark inputs (tests/golden/oracle_digests.json, written by
tests/golden/make_golden.py from the oracle alone).  A failure means the
oracle's arithmetic changed: such a change must name the passage or reading
that justifies it, and regenerate the digests."""
from __future__ import annotations

import json
import os

import pytest

from tests.golden import make_golden as mg

STORED = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_digests.json")))


@pytest.mark.parametrize("name", [n for n, _, _ in mg.cases()])
def test_oracle_reproduces_stored_digest(name):
    fn = {n: f for n, _, f in mg.cases()}[name]
    a = fn()
    assert list(a.shape) == STORED[name]["shape"] and str(a.dtype) == STORED[name]["dtype"]
    assert mg.digest(a) == STORED[name]["sha256"]
