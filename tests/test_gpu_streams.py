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
