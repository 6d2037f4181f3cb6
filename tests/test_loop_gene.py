"""Host-side checks of the per-loop gene (Sec. 4.2.2: one gene bit per loop
statement that passes the offload screen): the loop table, gene decoding,
region settings and argument checks. No GPU is touched."""

import numpy as np
import pytest

import paper_2011_03602_amd as ofl
import synth
from helpers import OMEGA


def _grid(I=9, J=7, K=6):
    return ofl.Grid(synth.make_problem(I, J, K))


def test_loop_table_lists_the_program_loops_in_order():
    g = _grid(9, 7, 6)
    t = ofl.ofl_loop_table(g.handle)
    assert len(t) == ofl.OFL_NLOOPS
    assert t[0] == (-1, -1, 0, 0)  # the iteration loop fails the screen: trip n reads what trip n-1 wrote
    extents = {ofl.OFL_LEVEL_K: 4, ofl.OFL_LEVEL_J: 5, ofl.OFL_LEVEL_I: 7}
    for n in range(3):
        for lev in range(3):
            assert t[1 + 3 * n + lev] == (n, lev, extents[lev], 1)
    g.close()


def _decode(gene):
    """The decoding rule restated: bits follow the screened loops (S k,j,i, R k,j,i,
    C k,j,i); a nest is on the GPU if any of its bits is set, its region opening at
    the outermost set one."""
    mask, levels = 0, [0, 0, 0]
    for n in range(3):
        for lev in range(3):
            if (gene >> (3 * n + lev)) & 1:
                mask |= 1 << n
                levels[n] = lev
                break
    return mask, levels


def test_every_loop_gene_decodes_to_its_regions():
    g = _grid()
    for gene in range(1 << 9):
        for mode in (ofl.OFL_XFER_HOISTED, ofl.OFL_XFER_PER_ITER):
            ofl.ofl_set_loop_gene(g.handle, gene, mode)
            mask, levels, m = ofl.ofl_get_regions(g.handle)
            want_mask, want_levels = _decode(gene)
            assert (mask, m) == (want_mask, mode), gene
            for n in range(3):
                if (mask >> n) & 1:
                    assert levels[n] == want_levels[n], (gene, n)
    g.close()


def test_bits_inside_an_offloaded_loop_change_nothing():
    g = _grid()
    ofl.ofl_set_loop_gene(g.handle, 0b001_001_001)
    base = ofl.ofl_get_regions(g.handle)
    assert base == (7, [0, 0, 0], ofl.OFL_XFER_HOISTED)
    ofl.ofl_set_loop_gene(g.handle, 0b111_111_111)
    assert ofl.ofl_get_regions(g.handle) == base
    ofl.ofl_set_loop_gene(g.handle, 0b100_010_110)  # S at j, R at j, C at i
    assert ofl.ofl_get_regions(g.handle) == (7, [1, 1, 2], ofl.OFL_XFER_HOISTED)
    g.close()


def test_region_settings_and_argument_checks():
    g = _grid()
    h = g.handle
    ofl.ofl_set_regions(h, 5, [2, 1, 1], ofl.OFL_XFER_PER_ITER)
    assert ofl.ofl_get_regions(h) == (5, [2, 1, 1], ofl.OFL_XFER_PER_ITER)
    ofl.ofl_set_offload_mask(h, 7)  # whole-nest regions again
    assert ofl.ofl_get_regions(h) == (7, [0, 0, 0], ofl.OFL_XFER_HOISTED)
    for bad in (lambda: ofl.ofl_set_loop_gene(h, 1 << 9), lambda: ofl.ofl_set_loop_gene(h, 1, 3),
                lambda: ofl.ofl_set_regions(h, 8, [0, 0, 0]), lambda: ofl.ofl_set_regions(h, 7, [0, 3, 0]),
                lambda: ofl.ofl_set_regions(h, 7, [-1, 0, 0]), lambda: ofl.ofl_set_regions(h, 7, [0, 0, 0], 2),
                lambda: ofl.ofl_grid_search_loops(h, 2, OMEGA, xfer_mode=5),
                lambda: ofl.ofl_grid_search_loops(h, 0, OMEGA),
                lambda: ofl.ofl_grid_search_loops(h, 2, OMEGA, time_limit_ms=float("nan"))):
        with pytest.raises(ofl.OflError) as e:
            bad()
        assert e.value.code == ofl.OFL_EINVAL
    g.close()


def test_cpu_gene_runs_and_levels_of_cpu_nests_are_ignored():
    a = synth.make_problem(11, 8, 7)
    g1, g2 = ofl.Grid(a), ofl.Grid(a)
    ofl.ofl_set_loop_gene(g1.handle, 0)
    ofl.ofl_set_regions(g2.handle, 0, [2, 2, 1])
    r1 = ofl.ofl_jacobi_run(g1.handle, 3, OMEGA)
    r2 = ofl.ofl_jacobi_run(g2.handle, 3, OMEGA)
    assert np.array_equal(g1.p, g2.p) and r1 == r2
    s = ofl.ofl_get_stats(g2.handle)
    assert list(s.gpu_regions) == [0, 0, 0] and list(s.cpu_nests) == [3, 3, 3]
    g1.close()
    g2.close()
