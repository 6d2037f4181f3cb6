"""The GA of the paper's search loop (Sec. 4.2.2) through ofl_ga_search, on
synthetic fitness landscapes: runs on the host only."""

import math

import pytest

import paper_2011_03602_amd as ofl


def _landscape(target, bits):
    calls = []

    def evaluate(gene):
        calls.append(gene)
        return 1.0 + bin((gene ^ target) & ((1 << bits) - 1)).count("1")
    return evaluate, calls


def test_finds_the_optimum_of_a_smooth_landscape():
    evaluate, calls = _landscape(0b1011001101, 10)
    r = ofl.ofl_ga_search(10, evaluate, ofl.ga_params(population=16, generations=20, seed=7, mutation=0.08))
    assert r.best_gene == 0b1011001101 and r.best_time == 1.0
    assert r.evaluated == len(calls) == len(set(calls))  # every distinct gene measured once


def test_deterministic_under_a_seed():
    ga = ofl.ga_params(population=8, generations=6, seed=11)
    e1, c1 = _landscape(0x5A, 8)
    e2, c2 = _landscape(0x5A, 8)
    r1 = ofl.ofl_ga_search(8, e1, ga)
    r2 = ofl.ofl_ga_search(8, e2, ga)
    assert c1 == c2 and r1.best_gene == r2.best_gene and r1.best_time == r2.best_time
    e3, c3 = _landscape(0x5A, 8)
    ofl.ofl_ga_search(8, e3, ofl.ga_params(population=8, generations=6, seed=12))
    assert c3 != c1


def test_best_is_the_minimum_over_measured_genes():
    seen = {}

    def evaluate(gene):
        t = 1.0 + ((gene * 2654435761) % 1000) / 10.0
        seen[gene] = t
        return t
    r = ofl.ofl_ga_search(9, evaluate, ofl.ga_params(population=10, generations=8, seed=3, elite=2))
    assert r.best_time == min(seen.values())
    assert seen[r.best_gene] == r.best_time


def test_wrong_and_unbuildable_genes_score_zero():
    # genes with bit 0 set give wrong results (+inf, the paper's infinite time),
    # genes with bit 1 set cannot be built (NaN, the paper's dropped loops)
    bad = {"wrong": 0, "nobuild": 0}

    def evaluate(gene):
        if gene & 1:
            bad["wrong"] += 1
            return math.inf
        if gene & 2:
            bad["nobuild"] += 1
            return math.nan
        return 1.0 + gene / 64.0
    r = ofl.ofl_ga_search(6, evaluate, ofl.ga_params(population=12, generations=8, seed=5))
    assert r.best_gene & 3 == 0 and math.isfinite(r.best_time)
    assert r.rejected == bad["wrong"] + bad["nobuild"] > 0


def test_seed_gene_is_measured_and_kept_by_elitism():
    evaluate, calls = _landscape(0x33, 8)
    r = ofl.ofl_ga_search(8, evaluate, ofl.ga_params(population=4, generations=1, seed=1), seed_gene=0x33)
    assert 0x33 in calls and r.best_gene == 0x33


def test_all_wrong_gives_infinite_time():
    r = ofl.ofl_ga_search(4, lambda g: math.inf, ofl.ga_params(population=4, generations=3, seed=2))
    assert math.isinf(r.best_time) and r.rejected == r.evaluated


@pytest.mark.parametrize("bits,ga", [(0, None), (31, None), (4, ofl.ga_params(population=1)),
                                     (4, ofl.ga_params(mutation=1.5)), (4, ofl.ga_params(elite=99))])
def test_bad_arguments(bits, ga):
    with pytest.raises(ofl.OflError) as e:
        ofl.ofl_ga_search(bits, lambda g: 1.0, ga)
    assert e.value.code == ofl.OFL_EINVAL
