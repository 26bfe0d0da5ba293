import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1809_01029_amd import synth  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def mech_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("mechs")


_CACHE = {}


def workload_file(name, directory):
    """Write (once per session) the description of a named synthetic workload."""
    key = (name, str(directory))
    if key not in _CACHE:
        m = synth.workload_mechanism(name)
        path = os.path.join(str(directory), f"{name}.pjm")
        synth.write_mechanism(m, path)
        _CACHE[key] = (m, path)
    return _CACHE[key]


def tiny_file(seed, directory, ns=7, nr=10, **kw):
    key = ("tiny", seed, ns, nr, tuple(sorted(kw.items())), str(directory))
    if key not in _CACHE:
        m = synth.make_mechanism(ns, nr, seed, mix=TINY_MIX, zipf=0.5, **kw)
        path = os.path.join(str(directory), f"tiny_{seed}_{ns}_{nr}_{len(_CACHE)}.pjm")
        synth.write_mechanism(m, path)
        _CACHE[key] = (m, path)
    return _CACHE[key]


# Tiny random mechanisms for the oracle pins: every reaction type, some
# irreversible reactions; these seeds give a drawable 7-species/10-reaction
# mechanism with and without bath-gas participation.
TINY_MIX = synth.MixSpec(third_body=0.1, falloff=0.2, irreversible=0.2)
TINY_SEEDS = (3, 6, 8, 11, 13)


# Tiny random mechanisms with every reaction type the library supports (SRI
# falloff, chemically activated, P-Log and Chebyshev besides the default mix);
# these seeds give a drawable 12-species/24-reaction mechanism with and
# without bath-gas participation.
TYPES_MIX = synth.MixSpec(third_body=0.1, falloff=0.1, irreversible=0.1, sri=0.1, chem_act=0.15,
                          plog=0.15, cheb=0.1)
TYPES_SEEDS = (3, 5, 6, 13, 14)


def types_file(seed, directory, bath=False):
    key = ("types", seed, bath, str(directory))
    if key not in _CACHE:
        kw = dict(bath_reactions=1, bath_efficiency=True) if bath else {}
        m = synth.make_mechanism(12, 24, seed, mix=TYPES_MIX, zipf=0.5, **kw)
        path = os.path.join(str(directory), f"types_{seed}_{int(bath)}.pjm")
        synth.write_mechanism(m, path)
        _CACHE[key] = (m, path)
    return _CACHE[key]
