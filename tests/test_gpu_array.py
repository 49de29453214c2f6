"""The apparent-resistivity array of the paper's second example (three
four-pole Debye soil layers, eight thin wires, a Heidler current source,
0.5 m CPML): GPU against the FP64 oracle over the first 6000 steps (the
source starts near step 1940), and a long GPU run that must stay finite and
bounded."""
import numpy as np
import pytest

from paper_2207_06908_amd import scenarios as S
from tests.parity import assert_probes_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_06908_amd import fdtd
    fdtd.lib()
    return fdtd


def test_array_probes_against_oracle(fd, oracle_mod):
    sc = S.config_array(n_steps=6000)
    print("array 6000 steps", flush=True)
    ref = oracle_mod.run_scenario(sc, S.apply)
    got = fd.run_scenario(sc, S.apply, precision=32)
    assert max(float(np.abs(v).max()) for v in ref.values()) > 0
    assert_probes_close(got, ref, 1e-5)


def test_array_long_run_stays_bounded(fd):
    """200,000 steps (19 us of the 400 us run): the probes stay finite, and
    the source-current probe follows the Heidler current's scale."""
    n = 200_000
    sc = S.config_array(n_steps=n)
    print("array long run", flush=True)
    g = fd.Grid.from_params(sc.params(), precision=32)
    ids = S.apply(sc, g)
    for _ in range(10):
        g.step(n // 10)
    cur, volt = g.probe(ids[0]), g.probe(ids[1])
    assert np.isfinite(cur).all() and np.isfinite(volt).all()
    src = sc.sources[0][4]
    assert 0.5 * np.abs(src).max() <= np.abs(cur).max() <= 2.0 * np.abs(src).max()
    # no late-time growth: the second half stays below twice the first half's peak
    assert np.abs(volt[n // 2:]).max() <= 2.0 * np.abs(volt[:n // 2]).max()
    assert np.abs(cur[n // 2:]).max() <= 2.0 * np.abs(cur[:n // 2]).max()
