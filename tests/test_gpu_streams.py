"""Sweeps with the independent message updates on several streams (forked
from and joined into the handle's stream, direct launches and captured
graphs), and expectations with the bonds on several streams, give
bit-identical messages, distances and rho_ij to every launch on one
stream."""
import numpy as np
import pytest

from synth import inputs as syn

from gpu_cases import problem, set_random_messages, oracle_for

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")


def _sweeps(kind, ts, streams, graph, sweeps=3, **kw):
    P, desc = problem(kind, **kw)
    g = pn.PepsNet(desc, ts)
    g.use_streams(streams)
    g.use_graph(graph)
    O = oracle_for(P, ts, kw["chi"], kw.get("trunc", 0), kw.get("q", 2), kw.get("p", 8),
                   kw.get("seed", 0))
    set_random_messages(g, O, P, 21)
    errs = [g.blockbp_sweep(1, 0.0)[1] for _ in range(sweeps)]
    rho, ss, e = g.blockbp_expect()
    return errs, g.get_messages(), (np.array(rho), np.array(ss), e)


@pytest.mark.parametrize("case", [
    ("infinite", syn.simple_update_cell(3, seed=2, steps=5), dict(N=3, D=3, chi=16, trunc=1, seed=7)),
    ("finite", syn.finite_patch_tensors(4, 4, 2, seed=1), dict(Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=4)),
])
def test_streams_bit_identical(case):
    kind, ts, kw = case
    print(f"case {kind} {kw}", flush=True)
    e1, m1, x1 = _sweeps(kind, ts, 1, False, **kw)
    for streams, graph in ((4, False), (2, True), (4, True)):
        e, m, x = _sweeps(kind, ts, streams, graph, **kw)
        print(f"  streams {streams} graph {graph}: {e} E {x[2]}", flush=True)
        assert e == e1
        assert np.array_equal(x[0], x1[0]) and np.array_equal(x[1], x1[1]) and x[2] == x1[2]
        for a, b in zip(m1, m):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_two_host_threads_share_the_extra_streams():
    """Two handles swept at the same time from two host threads (each forking
    its lane groups onto the device's shared extra streams, one capturing its
    graph) give the same results as one after the other."""
    import threading

    ts = syn.simple_update_cell(3, seed=2, steps=5)
    kw = dict(N=3, D=3, chi=16, trunc=1, seed=7)

    def make(graph):
        P, desc = problem("infinite", **kw)
        g = pn.PepsNet(desc, ts)
        g.use_graph(graph)
        O = oracle_for(P, ts, kw["chi"], 1, 2, 8, 7)
        set_random_messages(g, O, P, 23)
        return g

    def run(g, out, k):
        out[k] = ([g.blockbp_sweep(1, 0.0)[1] for _ in range(3)], g.get_messages())

    ref = {}
    for k, graph in enumerate((True, False)):
        g = make(graph)
        run(g, ref, k)
        g.close()
    hs = [make(True), make(False)]
    got = {}
    th = [threading.Thread(target=run, args=(hs[k], got, k)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for k in range(2):
        assert got[k][0] == ref[k][0]
        for a, b in zip(ref[k][1], got[k][1]):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        hs[k].close()
