"""Batched sweeps (pepsnet_batch_*): independent blocks of different N, D and
chi advanced in one merged launch sequence give bit-identical messages and
convergence distances to sweeping each handle on its own, with and without
graph replay; and the batch stays on the oracle's trajectory."""
import numpy as np
import pytest

from synth import inputs as syn

from gpu_cases import message_diff, oracle_for, problem

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")

CASES = [
    ("finite", dict(Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=4), lambda: syn.finite_patch_tensors(4, 4, 2, seed=1)),
    ("infinite", dict(N=2, D=2, chi=8), lambda: syn.random_unit_cell(2, seed=3)),
    ("infinite", dict(N=3, D=3, chi=16, trunc=1, q=1, p=4, seed=9), lambda: syn.random_unit_cell(3, seed=4)),
    ("infinite", dict(N=2, D=3, chi=8, prec=1), lambda: syn.random_unit_cell(3, seed=5)),
]


def _make():
    nets, probs = [], []
    for kind, kw, gen in CASES:
        P, desc = problem(kind, **kw)
        ts = gen()
        nets.append(pn.PepsNet(desc, ts))
        probs.append((P, ts, kw))
    return nets, probs


@pytest.mark.parametrize("graph", [False, True])
def test_batch_bit_identical_to_single(graph):
    single, _ = _make()
    batched, probs = _make()
    b = pn.Batch(batched)
    b.use_graph(graph)
    for it in range(3):
        errs_b, ms = b.sweep(1)
        errs_s = []
        for g in single:
            _, e, _ = g.blockbp_sweep(1, 0.0)
            errs_s.append(e)
        print(f"sweep {it}: batch {errs_b.tolist()} single {errs_s} ({ms:.2f} ms)", flush=True)
        assert np.array_equal(errs_b, np.array(errs_s))
    for gs, gb in zip(single, batched):
        ms_, mb_ = gs.get_messages(), gb.get_messages()
        for A, B in zip(ms_, mb_):
            for x, y in zip(A, B):
                assert np.array_equal(x, y)
    gf, nl = b.stats()
    assert gf > 0 and nl > 0
    b.close()


def test_batch_follows_oracle_and_rejects_separate_sweeps():
    nets, probs = _make()
    b = pn.Batch(nets)
    b.sweep(2)
    P, ts, kw = probs[1]
    O = oracle_for(P, ts, kw["chi"], kw.get("trunc", 0), kw.get("q", 2), kw.get("p", 8), kw.get("seed", 0))
    O.sweep()
    O.sweep()
    assert message_diff(nets[1], O, P) < 1e-10
    nets[0].blockbp_sweep(1, 0.0)
    with pytest.raises(pn.PepsnetError):
        b.sweep(1)
    b.close()
