"""GPU parity of the learning step (Eq. blockBP:kagome:numerics:learning_step1,
alpha = 1 - damping) and of Hermitised messages (Sec. "'Hermitize' MPSs"):
the HIP sweep through the C ABI against the oracle's BlockBP with the same
options, from seeded random (non-Hermitian) messages, sweep by sweep.
Tolerance 1e-10 on the convergence distance and on the messages (FP64; the
two sides differ only in rounding order).  chi is small enough that every
MPS sum (bonds up to 2 chi) is cut back to chi, so the compression runs."""
import numpy as np
import pytest

from oracle import bubble as bb
from oracle.dense import message_operator
from synth import inputs as syn

from gpu_cases import message_diff, oracle_for, problem, set_random_messages, slot_keys

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")


def _run(kind, ts, sweeps, randmsg, **kw):
    P, desc = problem(kind, **kw)
    g = pn.PepsNet(desc, ts)
    O = oracle_for(P, ts, kw["chi"], kw.get("trunc", 0), kw.get("q", 2), kw.get("p", 8),
                   kw.get("seed", 0), kw.get("chi_env"), kw.get("hermitize", False),
                   kw.get("damping", 0.0))
    set_random_messages(g, O, P, randmsg)
    print(f"case {kind} {kw} seed {randmsg}", flush=True)
    for it in range(sweeps):
        bb.DEGENERATE.clear()
        done, err, _ = g.blockbp_sweep(1, 0.0)
        eo = O.sweep()
        assert done == 1
        print(f"  sweep {it}: gpu {err:.15g} oracle {eo:.15g}", flush=True)
        if not bb.DEGENERATE:
            assert abs(err - eo) < 1e-10 * max(1.0, eo)
            assert message_diff(g, O, P) < 1e-10
    return P, g, O


def test_hex_damping_fp64():
    ts = syn.random_unit_cell(2, seed=3)
    _run("infinite", ts, 4, 11, N=2, D=2, chi=8, damping=0.3)


def test_hex_hermitize_fp64():
    ts = syn.random_unit_cell(2, seed=3)
    P, g, O = _run("infinite", ts, 3, 12, N=2, D=2, chi=8, hermitize=True)
    # every stored message, read as an operator on its ket and bra legs, is
    # Hermitian
    got = g.get_messages()
    for m, k in enumerate(slot_keys(P)):
        X = message_operator(bb.mps_dense(got[m]), 2)
        assert np.abs(X - X.conj().T).max() < 1e-10 * np.abs(X).max()


def test_hex_both_t2_fp64():
    """Both options with the randomized split inside the update; the sums
    are still compressed by exact SVDs."""
    ts = syn.random_unit_cell(2, seed=4)
    _run("infinite", ts, 3, 13, N=2, D=2, chi=8, trunc=1, q=1, p=4, seed=7, hermitize=True,
         damping=0.5)


def test_finite_both_fp64():
    """Open patch: messages of different lengths and caps, some slots below
    their caps after the update."""
    ts = syn.finite_patch_tensors(4, 4, 2, seed=1)
    _run("finite", ts, 3, 14, Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=4, hermitize=True,
         damping=0.25)



def test_streams_and_graph_bit_identical_with_both_options():
    """Lane groups on separate streams and graph replay leave the sweep with
    the stability options bit-identical to one stream, direct launches."""
    ts = syn.random_unit_cell(2, seed=5)
    out = []
    for streams, graph in ((1, False), (4, False), (4, True)):
        P, desc = problem("infinite", N=2, D=2, chi=8, hermitize=True, damping=0.4)
        g = pn.PepsNet(desc, ts)
        g.use_streams(streams)
        g.use_graph(graph)
        O = oracle_for(P, ts, 8, 0, 2, 8, 0, None, True, 0.4)
        set_random_messages(g, O, P, 17)
        errs = [g.blockbp_sweep(1, 0.0)[1] for _ in range(3)]
        out.append((errs, g.get_messages()))
        g.close()
    for errs, msgs in out[1:]:
        assert errs == out[0][0]
        for a, b in zip(out[0][1], msgs):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
