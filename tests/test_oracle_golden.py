"""Regression guard on the oracle: its small_l64 result must keep matching
tests/golden/small_l64_oracle.json (written by tests/golden/make_golden.py,
which calls only the oracle). A change to the oracle's arithmetic shows up here
and must be justified by the passage of the paper it follows."""
import json
import os

from tests.golden.make_golden import small_l64_summary

HERE = os.path.dirname(os.path.abspath(__file__))


def test_small_l64_golden():
    stored = json.load(open(os.path.join(HERE, "golden", "small_l64_oracle.json")))
    assert small_l64_summary() == stored
