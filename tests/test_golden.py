"""The oracle reproduces its stored outputs (tests/golden/, written by
tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import numpy as np
import pytest

from tests.golden.make_golden import CASES, make

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(HERE, name + ".json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_reproduces_golden(oracle_lib, name):
    doc = load(name)
    batch, consts = make(doc["inputs"])
    rc, out, summ = oracle_lib.fit_batch(batch, consts)
    assert rc == 0
    for k, v in doc["results"].items():
        want = np.array(v, dtype=np.uint64 if k == "chi2" else np.int64)
        got = out[k].astype(np.uint64 if k == "chi2" else np.int64).reshape(want.shape)
        assert np.array_equal(got, want), k
    assert {k: int(v) for k, v in summ.items()} == doc["summary"]
