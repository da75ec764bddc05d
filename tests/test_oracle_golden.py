"""The oracle's tiny-configuration outputs still match the digest written by
tests/golden/make_golden.py (which calls only the oracle)."""
import json
import os

import numpy as np
import pytest

from tests.golden.make_golden import summarise

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tiny_oracle.json")))


@pytest.mark.parametrize("ev", GOLD["events"], ids=lambda e: f"seed{e['seed']}")
def test_oracle_matches_golden(ev):
    got = summarise(ev["seed"])
    for k, v in ev.items():
        if isinstance(v, float):
            assert abs(got[k] - v) <= 1e-9 * max(1.0, abs(v)), k
        else:
            assert got[k] == v, k
