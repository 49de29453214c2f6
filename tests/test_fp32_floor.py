"""Evidence for the FP32 parity tolerance of the 48^3 workload (config 1).

The workload's Gaussian current leaves a permanent charge dipole in air.
Rounding in the strong fields near the source deposits small spurious
charges whose static fields reach the far probes, where the true field is
weak.  An FP32-storage run of the same recurrence (tests/fp32_emulation.py)
shows the size of that floor per probe; the GPU parity test holds each
probe to the larger of 1e-5 and a multiple of it."""
import numpy as np

from paper_2207_06908_amd import scenarios as S
from tests.fp32_emulation import run_fp32
from tests.parity import probe_errors


def test_emulation_in_fp64_is_the_oracle(oracle_mod):
    """Stored and rounded in float64, the emulated recurrence reproduces the
    oracle's probes (1e-12): the FP32 run below differs from the oracle only
    by its storage precision."""
    sc = S.config1(n_steps=120)
    ref = oracle_mod.run_scenario(sc, S.apply)
    got = run_fp32(sc, oracle_mod, dtype=np.float64)
    errs = probe_errors(got, ref)
    assert max(errs.values()) <= 1e-12, errs


def test_fp32_storage_floor_of_config1(oracle_mod):
    """FP32 storage alone leaves several probes of config 1 above 1e-5 of
    their own norm (all of them in air, in the dipole's static field), and
    none above 2e-4."""
    sc = S.config1()
    ref = oracle_mod.run_scenario(sc, S.apply)
    got = run_fp32(sc, oracle_mod)
    errs = probe_errors(got, ref)
    print("FP32-storage floor per probe:", {k: f"{v:.2e}" for k, v in errs.items()})
    above = [k for k, v in errs.items() if v > 1e-5]
    assert len(above) >= 2, errs
    for (name, _kind, _ax, _i, _j, k, _n) in sc.probes:
        if name in above:
            assert k >= 16          # in air, above the soil layers
    assert max(errs.values()) <= 2e-4
