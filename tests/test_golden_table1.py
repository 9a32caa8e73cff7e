"""The FIRE parameter defaults used everywhere equal the paper's Table 1."""
import json
import os

from paper_1908_02038_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_defaults.json")


def test_input_defaults_match_table1():
    ref = json.load(open(GOLDEN))
    p = inputs.fire_params(1.0)
    for k, v in ref.items():
        if not k.startswith("_"):
            assert p[k] == v, k
