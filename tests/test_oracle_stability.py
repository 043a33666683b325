"""Pins of the learning step (Eq. blockBP:kagome:numerics:learning_step1) and
of Hermitised messages (Sec. "'Hermitize' MPSs") in the oracle: the MPS sum
against the dense sum, the Hermitian conjugate against the dense operator,
a Hermitised message read as an operator is Hermitian, the learned message
is proportional to alpha new + (1 - alpha) old when nothing is truncated,
and a fixed point of the plain map stays one of the damped map."""
import numpy as np

from oracle import bubble as bb
from oracle import geometry as geo
from oracle.blockbp import BlockBP
from oracle.dense import message_operator
from synth import inputs as syn


def _rand_mps(rng, shapes):
    return [rng.standard_normal(s) + 1j * rng.standard_normal(s) for s in shapes]


def test_mps_sum_is_the_dense_sum():
    rng = np.random.default_rng(1)
    A = _rand_mps(rng, [(1, 4, 3), (3, 4, 5), (5, 4, 1)])
    B = _rand_mps(rng, [(1, 4, 2), (2, 4, 4), (4, 4, 1)])
    S = bb.mps_sum(A, B, 0.3 - 0.2j, 1.7)
    ref = (0.3 - 0.2j) * bb.mps_dense(A) + 1.7 * bb.mps_dense(B)
    assert np.abs(bb.mps_dense(S) - ref).max() < 1e-13
    C = bb.compressed_sum(A, B, 0.3 - 0.2j, 1.7, 64)     # no truncation
    d = bb.mps_dense(C)
    assert abs(np.linalg.norm(d) - 1) < 1e-13
    ov = np.vdot(d, ref) / np.linalg.norm(ref)
    assert abs(abs(ov) - 1) < 1e-12                      # proportional


def test_hermitian_conjugate_and_hermitised_message():
    rng = np.random.default_rng(2)
    D = 2
    A = _rand_mps(rng, [(1, D * D, 3), (3, D * D, 4), (4, D * D, 1)])
    X = message_operator(bb.mps_dense(A), D)
    Xd = message_operator(bb.mps_dense(bb.hermitian_conjugate(A, [D, D, D])), D)
    assert np.abs(Xd - X.conj().T).max() < 1e-13
    H = bb.compressed_sum(A, bb.hermitian_conjugate(A, [D, D, D]), 0.5, 0.5, 64)
    Y = message_operator(bb.mps_dense(H), D)
    assert np.abs(Y - Y.conj().T).max() < 1e-13
    ref = 0.5 * (X + X.conj().T)
    ov = np.vdot(Y, ref) / (np.linalg.norm(Y) * np.linalg.norm(ref))
    assert abs(abs(ov) - 1) < 1e-12


def _random_start(O, seed):
    keys = sorted(O.msgs)
    shapes = [[x.shape for x in O.msgs[k]] for k in keys]
    for k, A in zip(keys, syn.random_messages(shapes, seed)):
        O.msgs[k] = [np.array(a) for a in A]


def test_learning_step_mixes_old_and_new():
    """chi large enough that no bond is cut: the damped update is the plain
    update's message mixed with the old one, alpha new + (1 - alpha) old, up
    to the unit norm and real positive trace."""
    H = geo.HexProblem(2)
    ts = syn.random_unit_cell(2, seed=5)
    plain = BlockBP(H, ts, chi=64, chi_env=0)
    damped = BlockBP(H, ts, chi=64, chi_env=0, damping=0.3)
    _random_start(plain, 9)
    _random_start(damped, 9)
    key = H.msg_keys[0]
    sk = plain._store_key(key)
    new = bb.mps_dense(plain.update(key))
    old = bb.mps_dense(plain.msgs[sk])
    gotA = damped.update(key)
    got = bb.mps_dense(gotA)
    ref = 0.7 * new + 0.3 * old
    ov = np.vdot(got, ref) / (np.linalg.norm(got) * np.linalg.norm(ref))
    assert abs(abs(ov) - 1) < 1e-12     # the same ray
    legs = damped._recv_legs(sk)
    tr = bb.trace(gotA, [damped._dim(s, l) for (s, l) in legs])
    assert tr.real > 0 and abs(tr.imag) < 1e-12 * abs(tr)   # unit norm, real positive trace
    assert abs(np.linalg.norm(got) - 1) < 1e-12


def test_fixed_point_is_kept_by_the_damped_map():
    H = geo.HexProblem(2)
    ts = syn.simple_update_cell(2, seed=2, steps=5)
    O = BlockBP(H, ts, chi=16, chi_env=16)
    O.run(tol=1e-12, max_sweeps=60)
    D = BlockBP(H, ts, chi=16, chi_env=16, damping=0.4)
    D.msgs = {k: [a.copy() for a in v] for k, v in O.msgs.items()}
    assert D.sweep() < 1e-10
