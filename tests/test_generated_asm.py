"""The committed inline-assembly include files are exactly what their
generators produce (a generator edited without regenerating, or an include
edited by hand, fails here)."""
import importlib.util
import os

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2602_05179_amd",
                    "csrc")


@pytest.mark.parametrize("gen,inc", [
    ("gen_window_asm.py", "window_min_asm.inc"),
    ("gen_argmin_asm.py", "window_argmin_asm.inc"),
    ("gen_multiring_asm.py", "window_min_multi_asm.inc"),
])
def test_include_matches_generator(gen, inc, monkeypatch):
    monkeypatch.syspath_prepend(CSRC)  # generators import each other
    spec = importlib.util.spec_from_file_location(gen[:-3], os.path.join(CSRC, gen))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(CSRC, inc)) as fh:
        committed = fh.read()
    assert mod.render() == committed, "%s is stale: run python %s" % (inc, gen)
