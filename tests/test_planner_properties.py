"""Properties of the transfer planner (Sec. 4.2.2 rules) on random programs:
every plan ofl_plan_nests returns is replayed on a model of the two memories
and must keep each nest's inputs valid on its side, copy only from a valid
copy, never re-send an array the device already holds in the hoisted
placement, and leave what the program reads after the loop valid on the
host."""

import pytest

import paper_2011_03602_amd as ofl

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402


@st.composite
def programs(draw):
    narrays = draw(st.integers(1, 8))
    nnests = draw(st.integers(1, 4))
    full = (1 << narrays) - 1
    nests = []
    for _ in range(nnests):
        reads = draw(st.integers(0, full))
        writes = draw(st.integers(0, full))
        partial = draw(st.integers(0, full)) & writes
        nests.append((reads, writes, partial))
    live = draw(st.integers(0, full))
    mask = draw(st.integers(0, (1 << nnests) - 1))
    mode = draw(st.sampled_from([ofl.OFL_XFER_PER_ITER, ofl.OFL_XFER_HOISTED]))
    iters = draw(st.integers(1, 3))
    return narrays, nests, live, mask, mode, iters


def bits(x, n):
    return [a for a in range(n) if (x >> a) & 1]


@settings(max_examples=300, deadline=None)
@given(programs())
def test_replayed_plans_keep_every_rule(prog):
    narrays, nests, live, mask, mode, iters = prog
    xs, hv_end, dv_end = ofl.ofl_plan_nests(nests, narrays, live, mask, mode, iters, True)
    host, dev = [1] * narrays, [0] * narrays
    pos = 0

    def apply(x):
        _, _, _, a, d = x
        if d == 0:
            assert host[a], "upload from a stale host copy"
            if mode == ofl.OFL_XFER_HOISTED:
                assert not dev[a], "hoisted placement re-sent an array the device holds"
            dev[a] = 1
        else:
            assert dev[a], "download from a stale device copy"
            host[a] = 1

    for it in range(iters):
        for n, (reads, writes, partial) in enumerate(nests):
            gpu = (mask >> n) & 1
            before = []
            while pos < len(xs) and xs[pos][:3] == (it, n, 0):
                before.append(xs[pos])
                apply(xs[pos])
                pos += 1
            need = bits(reads | partial, narrays)
            side = dev if gpu else host
            assert all(side[a] for a in need), (it, n, "input not valid on the nest's side")
            if gpu and mode == ofl.OFL_XFER_PER_ITER:
                # every input the host held is sent, each time
                sent = {x[3] for x in before}
                assert {a for a in need} <= sent | {a for a in need if not host[a]}
            for a in bits(writes, narrays):
                if gpu:
                    dev[a], host[a] = 1, 0
                else:
                    host[a], dev[a] = 1, 0
            while pos < len(xs) and xs[pos][:3] == (it, n, 1):
                assert gpu and mode == ofl.OFL_XFER_PER_ITER and (writes >> xs[pos][3]) & 1
                apply(xs[pos])
                pos += 1
            if gpu and mode == ofl.OFL_XFER_PER_ITER:
                assert all(host[a] for a in bits(writes, narrays)), "per-iteration GPU write not copied back"
    while pos < len(xs):
        assert xs[pos][0] == iters and xs[pos][1] == -1
        apply(xs[pos])
        pos += 1
    assert all(host[a] for a in bits(live, narrays)), "an array read after the loop is stale on the host"
    assert [int(x) for x in hv_end] == host and [int(x) for x in dv_end] == dev


def test_library_program_is_one_such_table():
    nests, live = ofl.ofl_program_vars()
    for mask in range(8):
        for mode in (0, 1):
            a, _, _ = ofl.ofl_plan(mask, mode, 3, True)
            b, _, _ = ofl.ofl_plan_nests(nests, 14, live, mask, mode, 3, True)
            assert a == b
