"""The generated inputs behind the stored oracle results have not moved:
SHA-256 of the benchmark, nine-heavy-atom, large-molecule and serving
batches (prefixes) and of water, against tests/golden/molgen_sha.json
(written by tests/golden/make_molgen_sha.py)."""
import importlib.util
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _maker():
    spec = importlib.util.spec_from_file_location("make_molgen_sha", os.path.join(HERE, "golden", "make_molgen_sha.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_generated_inputs_match_pins():
    mk = _maker()
    with open(os.path.join(HERE, "golden", "molgen_sha.json")) as f:
        pins = json.load(f)
    assert set(pins) == set(mk.SETS)
    for name, make in mk.SETS.items():
        assert mk.digest(make()) == pins[name], name
