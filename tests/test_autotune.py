"""Autotuner: cache handling and candidate validity on the host; on the GPU,
a tuned grid and a tuned batch give bitwise the results of the defaults."""
import json

import numpy as np
import pytest

from paper_2207_06908_amd import autotune as T
from paper_2207_06908_amd import fdtd
from paper_2207_06908_amd import scenarios as S


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert T.load_cache(p) == {}
    T.store("a", {"variant": 2}, p)
    T.store("b", {"variant": 3}, p)
    assert T.load_cache(p) == {"a": {"variant": 2}, "b": {"variant": 3}}
    with open(p, "w") as f:
        f.write("not json")
    assert T.load_cache(p) == {}


def test_keys_name_device_shape_and_precision():
    k = T.grid_key({"nx": 512, "ny": 512, "nz": 384, "npml": 10}, 32, device="MI355X")
    assert k == "MI355X|grid|512x512x384|npml10|fp32"
    kb = T.batch_key([(32, 40, 50), (96, 96, 96)], 8, device="MI355X")
    assert kb.startswith("MI355X|batch|2|") and kb.endswith("|npml8|fp32")


def test_every_grid_candidate_is_accepted_by_the_library():
    g = fdtd.Grid(nx=12, ny=10, nz=9, dx=0.5, max_steps=4)
    for cand in T.GRID_CANDIDATES:
        g.set_kernel(*cand)          # host-side validation only


def test_cached_choice_is_returned_without_measuring(tmp_path):
    p = str(tmp_path / "tune.json")
    T.store("k", {"variant": 1, "tile_y": 0, "tile_z": 0, "ms_per_step": 1.0}, p)

    def never(_n):
        raise AssertionError("should not build a grid")

    assert T.tune_grid(never, "k", path=p)["variant"] == 1


@pytest.mark.gpu
def test_tuned_grid_and_batch_match_defaults(tmp_path):
    p = str(tmp_path / "tune.json")
    sc = S.config2(nx=70, ny=66, nz=60, dx=0.5, npml=8, wire_cells=10, n_steps=40, e_probe_offsets=(5, 10))

    def make(n):
        s2 = S.config2(nx=70, ny=66, nz=60, dx=0.5, npml=8, wire_cells=10, n_steps=n, e_probe_offsets=(5, 10))
        g = fdtd.Grid.from_params(s2.params(), precision=32)
        S.apply(s2, g)
        return g

    key = T.grid_key(sc.params())
    choice = T.tune_grid(make, key, path=p, steps=6, warmup=2)
    assert (choice["variant"], choice["tile_y"], choice["tile_z"]) in T.GRID_CANDIDATES
    assert json.load(open(p))[key] == choice
    ref = fdtd.run_scenario(sc, S.apply, precision=32)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    ids = S.apply(sc, g)
    T.apply_grid(g, choice)
    g.step(sc.n_steps)
    for pr, i in zip(sc.probes, ids):
        assert np.array_equal(g.probe(i), ref[pr[0]])

    scs = S.config3(n_grids=6, n_steps=30)

    def make_b(n):
        grids = []
        for s in S.config3(n_grids=6, n_steps=n):
            gg = fdtd.Grid.from_params(s.params(), precision=32)
            S.apply(s, gg)
            grids.append(gg)
        return fdtd.Batch(grids)

    kb = T.batch_key([(s.nx, s.ny, s.nz) for s in scs], 8)
    cb = T.tune_batch(make_b, kb, path=p, steps=4, warmup=2)
    assert (cb["tile_x"], cb["tile_y"], cb["tile_z"], int(cb["persistent"])) in T.BATCH_CANDIDATES
    a = fdtd.run_batch(scs, S.apply)
    b = fdtd.run_batch(scs, S.apply, tile=(cb["tile_x"], cb["tile_y"], cb["tile_z"]), persistent=cb["persistent"])
    for x, y in zip(a, b):
        for name in x:
            assert np.array_equal(x[name], y[name])
