"""Tile searches that resume: with a measurement file set
(ofl_set_tune_cache), a repeated search takes every gene's time from the file
and measures nothing, a longer search measures only the genes it has not
measured before, and the tile found still reproduces the oracle."""

import sys

import numpy as np
import pytest

import oracle
import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA, TOL_GOSA_F32, TOL_P_F32, p_rel_err, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, skipped there
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="needs a GPU")]


def say(*args):
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def lines(path):
    with open(path) as f:
        rows = [ln.split() for ln in f if ln.strip()]
    keys = [(r[2], r[3]) for r in rows]
    assert len(keys) == len(set(keys)), "a gene was measured twice under one key"
    return rows


@pytest.fixture
def cache(tmp_path):
    path = str(tmp_path / "tune.txt")
    ofl.ofl_set_tune_cache(path)
    yield path
    ofl.ofl_set_tune_cache(None)


def test_grid_search_resumes_from_its_measurements(cache):
    a = synth.make_problem(70, 29, 23, seed=40)
    g = ofl.Grid(a)
    # the search seeds its population with the grid's current tile: every
    # search below starts from the same one, so they are the same search
    start = ofl.ofl_get_tile(g.handle)
    ga = dict(population=5, generations=2, probe_iters=2, repeats=1, seed=7)
    say("grid tune, first search")
    r1 = ofl.ofl_grid_tune(g.handle, ofl.ga_params(**ga))
    n1 = len(lines(cache))
    assert r1.from_cache == 0 and n1 == r1.evaluated
    say("grid tune, same search again")
    ofl.ofl_set_tile(g.handle, start)
    r2 = ofl.ofl_grid_tune(g.handle, ofl.ga_params(**ga))
    assert r2.evaluated == r1.evaluated and r2.from_cache == r2.evaluated
    assert len(lines(cache)) == n1
    assert r2.best.as_dict() == r1.best.as_dict() and r2.best_ms == r1.best_ms
    say("grid tune, two more generations")
    ofl.ofl_set_tile(g.handle, start)
    r3 = ofl.ofl_grid_tune(g.handle, ofl.ga_params(**dict(ga, generations=4)))
    assert r3.from_cache >= r1.evaluated  # the first generations replay from the file
    assert len(lines(cache)) == n1 + (r3.evaluated - r3.from_cache)
    assert r3.best_ms <= r1.best_ms
    # the tile the search leaves on the grid reproduces the oracle
    gosa = ofl.ofl_jacobi_run(g.handle, 4, OMEGA)
    p_ref, g_ref = oracle.jacobi(a, 4, float(OMEGA))
    assert p_rel_err(g.p, p_ref) <= TOL_P_F32 and rel_err(gosa, g_ref) <= TOL_GOSA_F32
    # another grid shape is another key: nothing is reused
    h = ofl.Grid(synth.make_problem(40, 21, 19, seed=41))
    r4 = ofl.ofl_grid_tune(h.handle, ofl.ga_params(**ga))
    assert r4.from_cache == 0
    g.close()
    h.close()


def test_batch_search_resumes_from_its_measurements(cache):
    grids = [ofl.Grid(synth.make_problem(*s, seed=sum(s)), row_align=4) for s in ((45, 20, 17), (70, 13, 11))]
    b = ofl.ofl_batch_create([g.handle for g in grids])
    start = ofl.ofl_batch_get_tile(b)
    ga = dict(population=4, generations=2, probe_iters=2, repeats=1, seed=9)
    r1 = ofl.ofl_batch_tune(b, ofl.ga_params(**ga))
    n1 = len(lines(cache))
    ofl.ofl_batch_set_tile(b, start)
    r2 = ofl.ofl_batch_tune(b, ofl.ga_params(**ga))
    assert r1.from_cache == 0 and n1 == r1.evaluated
    assert r2.from_cache == r2.evaluated == r1.evaluated and len(lines(cache)) == n1
    assert r2.best.as_dict() == r1.best.as_dict()
    ofl.ofl_batch_destroy(b)
    for g in grids:
        g.close()


def test_unwritable_cache_fails_before_measuring(tmp_path):
    ofl.ofl_set_tune_cache(str(tmp_path / "no" / "such" / "dir" / "tune.txt"))
    try:
        g = ofl.Grid(synth.make_problem(40, 12, 10))
        with pytest.raises(ofl.OflError) as e:
            ofl.ofl_grid_tune(g.handle, ofl.ga_params(population=2, generations=1, probe_iters=1, repeats=1))
        assert e.value.code == ofl.OFL_EINVAL and "tune cache" in ofl.ofl_last_error()
        g.close()
    finally:
        ofl.ofl_set_tune_cache(None)


def _seed_time(path, gene):
    times = [float(r[4]) for r in lines(path) if int(r[3], 16) == gene]
    assert len(times) == 1, times
    return times[0]


def test_searches_measure_the_tile_they_start_from(cache):
    """The population starts with the current tile's gene: it must decode back
    to a buildable tile and be measured (a finite time in the file). The default
    FP32 grid tile (4 points per lane, 4 rows, 2-plane chunks, NT loads and
    stores, early coefficient loads, at most 3 work-groups per CU) is gene
    0x239a; the default batch
    tile (each grid's own width, 1 row, 2-plane chunks, NT loads and stores,
    bit 14 set) is gene 0x4192."""
    g = ofl.Grid(synth.make_problem(200, 21, 19, seed=42))
    assert ofl.ofl_get_tile(g.handle).as_dict() == dict(vec=4, rows=4, kchunk=2, flags=7, occupancy=3)
    ofl.ofl_grid_tune(g.handle, ofl.ga_params(population=2, generations=1, probe_iters=2, repeats=1))
    assert np.isfinite(_seed_time(cache, 0x239A))
    h = ofl.Grid(synth.make_problem(45, 20, 17, seed=43), row_align=4)
    b = ofl.ofl_batch_create([h.handle])
    assert ofl.ofl_batch_get_tile(b).as_dict() == dict(vec=0, rows=1, kchunk=2, flags=3, occupancy=0)
    ofl.ofl_batch_tune(b, ofl.ga_params(population=2, generations=1, probe_iters=2, repeats=1))
    assert np.isfinite(_seed_time(cache, 0x4192))
    ofl.ofl_batch_destroy(b)
    g.close()
    h.close()
