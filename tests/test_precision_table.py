"""The precision statement at the benchmark shapes (CPU).

tests/golden/precision_mirror_vs_fp64.json is written by
tests/golden/make_precision_table.py, which calls only the oracle: for the
L = 8 and L = 16 Gaussian workloads (32 samples, 2000 sweeps, measurements
every 10 sweeps over the second half) it holds, per observable of eqs. 3-6 and
per temperature slot, the value with binary32 fields and acceptance (the
engine's arithmetic, bit-identical to the oracle's mirror mode) and with
binary64 fields, libm exp and 53-bit uniforms, and the paired jackknife z of
their difference.  Binary32 must not bias any result: every |z| stays below
4.5 and the rms z near one.  The L = 8 case is recomputed here and must
reproduce the stored table exactly.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "golden", "precision_mirror_vs_fp64.json")
SCRIPT = os.path.join(HERE, "golden", "make_precision_table.py")


def load_script():
    spec = importlib.util.spec_from_file_location("make_precision_table", SCRIPT)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def table():
    with open(TABLE) as f:
        return json.load(f)


def test_table_covers_the_script_cases():
    mod = load_script()
    got = [c["case"] for c in table()["cases"]]
    assert got == mod.CASES


@pytest.mark.parametrize("config", ["L8_gauss", "L16_gauss"])
def test_binary32_does_not_bias_any_observable(config):
    case = next(c for c in table()["cases"] if c["case"]["config"] == config)
    zs = []
    for name, o in case["observables"].items():
        z = np.array(o["z"], dtype=np.float64)
        z = z[np.isfinite(z)]
        assert np.all(np.abs(z) < 4.5), (config, name, z)
        zs.extend(np.abs(z).tolist())
    zs = np.array(zs)
    assert len(zs) >= 100
    assert np.sqrt((zs ** 2).mean()) < 2.0
    s = case["summary"]
    assert s["comparisons"] == len(zs) and abs(s["max_abs_z"] - zs.max()) < 1e-12


def test_L8_case_reproduces_the_table():
    mod = load_script()
    stored = next(c for c in table()["cases"] if c["case"]["config"] == "L8_gauss")
    fresh = mod.run_case(stored["case"], threads=os.cpu_count() or 1)
    for name, o in stored["observables"].items():
        for key in ("mirror", "binary64", "err"):
            a = np.array(o[key], dtype=np.float64)
            b = np.array(fresh["observables"][name][key], dtype=np.float64)
            assert np.array_equal(a, b, equal_nan=True), (name, key)
