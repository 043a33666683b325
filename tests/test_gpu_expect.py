"""GPU parity of the expectation boundary and of the exact contraction mode,
through the C ABI: caller-chosen bonds and operators, rho_ij entry by entry,
the chain state messaging itself (transfer-matrix reference), the exact
in-block contraction (chi_env = 0) against the dense exact BlockBP, runs to
convergence, and checkpoint / resume.  Tolerance 1e-10 (FP64)."""
import numpy as np
import pytest

from oracle import bubble as bb
from oracle import geometry as geo
from oracle.dense import SX, SY, SZ, DenseBlockBP, H_SS, expect_op, ss_from_rho
from synth import inputs as syn

from gpu_cases import message_diff, oracle_for, oracle_rhos, problem, unit
from test_oracle_rho_pins import chain_bond_refs, chain_cell_dir

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")

I2 = np.eye(2)
SP = np.array([[0, 1], [0, 0]], complex)
OPS = [H_SS, np.kron(0.5 * SZ, I2), np.kron(SX, SZ), np.kron(SP, SP.T), np.kron(SY, SX)]


def _unit(r):
    return r / np.trace(r)


def test_expect_bond_subset_and_operators():
    """A bond subset in a caller's order and five operators (three of them
    not symmetric under i <-> j, one not Hermitian) against the oracle's
    rho; the subset's values equal the full table's bit for bit (the same
    kernels run for the same bonds)."""
    ts = syn.random_unit_cell(2, seed=3)
    P, desc = problem("infinite", N=2, D=2, chi=8)
    g = pn.PepsNet(desc, ts)
    O = oracle_for(P, ts, 8, 0, 2, 8, 0)
    for _ in range(4):
        g.blockbp_sweep(1, 0.0)
        O.sweep()
    bonds = g.bonds()
    ids = [4, 0, 3]
    rho_s, vals, e = g.blockbp_expect(bond_ids=ids, ops=OPS)
    assert e is None and vals.shape == (3, len(OPS))
    rho_all, vals_all, e_all = g.blockbp_expect(ops=OPS)
    ref = oracle_rhos(O, bonds)
    for k, b in enumerate(ids):
        assert np.array_equal(rho_s[k], rho_all[b]) and np.array_equal(vals[k], vals_all[b])
        assert np.abs(_unit(rho_s[k]) - unit(ref[b])).max() < 1e-10
        for q, op in enumerate(OPS):
            assert abs(vals[k, q] - expect_op(ref[b], op)) < 1e-10, (b, q)
    # the default call reports <S.S> per bond and the energy per site
    _, ss, e = g.blockbp_expect()
    assert np.allclose(ss, vals_all[:, 0].real, atol=1e-14, rtol=0)
    assert abs(e - sum(ss) / 3) < 1e-14
    with pytest.raises(pn.PepsnetError):
        g.blockbp_expect(bond_ids=[0, 0])
    with pytest.raises(pn.PepsnetError):
        g.blockbp_expect(bond_ids=[len(bonds)])


@pytest.mark.parametrize("direction", [0, 60, 120])
def test_chain_state_against_transfer_matrix(direction):
    """Decoupled chains messaging themselves through the hexagonal block:
    the converged rho_ij of the six unique bonds equal the infinite chain's
    exact reduced density matrices."""
    H = geo.HexProblem(2)
    ts, A, B, phi = chain_cell_dir(2, seed=40 + direction, direction=direction)
    _, desc = problem("infinite", N=2, D=2, chi=4)
    g = pn.PepsNet(desc, ts)
    done, err, _ = g.blockbp_sweep(60, 1e-12)
    assert err <= 1e-12
    rho, _, _ = g.blockbp_expect()
    refs = chain_bond_refs(H, direction, A, B, phi)
    assert [tuple(b) for b in g.bonds()] == [tuple(b) for b in H.central_bonds()]
    for b, ref in enumerate(refs):
        assert np.abs(_unit(rho[b]) - ref).max() < 1e-10, b


def test_exact_mode_cfg1_anchor():
    """4x4-cell patch, 2x2-cell blocks, D=2, chi=4, exact in-block
    contraction (chi_env = 0): messages are exact at chi=4, so the GPU must
    follow the dense exact BlockBP sweep by sweep and converge to 1e-10
    within 30 sweeps, with the dense rho_ij at the fixed point."""
    ts = syn.finite_patch_tensors(4, 4, 2, seed=1)
    P, desc = problem("finite", Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=4, chi_env=0)
    g = pn.PepsNet(desc, ts)
    Bd = DenseBlockBP(P, ts)
    keys = list(P.msg_keys)
    for it in range(3):
        _, err, _ = g.blockbp_sweep(1, 0.0)
        ed = Bd.sweep()
        assert abs(err - ed) < 1e-10
        got = g.get_messages()
        for m, k in enumerate(keys):
            assert np.linalg.norm(bb.mps_dense(got[m]) - Bd.msgs[k]) < 1e-10
    done, err, _ = g.blockbp_sweep(27, 1e-10)
    Bd.run(tol=1e-10, max_sweeps=27)
    assert err <= 1e-10
    rho, ss, _ = g.blockbp_expect()
    for b, (i, j) in enumerate(g.bonds()):
        ref = _unit(Bd.rho(i, j))
        assert np.abs(_unit(rho[b]) - ref).max() < 1e-10
        assert abs(ss[b] - ss_from_rho(ref)) < 1e-10


def test_exact_mode_compresses_like_the_oracle():
    """4x4-cell patch, 2x2-cell blocks, D=2, chi=2 with exact in-block
    contraction: the exact three-leg messages need bond 4 and are compressed
    to 2 by exact truncated SVDs, as the oracle does; three sweeps from
    identity."""
    ts = syn.finite_patch_tensors(4, 4, 2, seed=6)
    P, desc = problem("finite", Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=2, chi_env=0)
    g = pn.PepsNet(desc, ts)
    O = oracle_for(P, ts, 2, 0, 2, 8, 0, chi_env=0)
    bb.DEGENERATE.clear()
    for _ in range(3):
        _, err, _ = g.blockbp_sweep(1, 0.0)
        eo = O.sweep()
        assert abs(err - eo) < 1e-10
    assert not bb.DEGENERATE
    assert message_diff(g, O, P) < 1e-10


def test_checkpoint_resume_bit_identical():
    """10 sweeps, messages saved, a new handle restored from them and swept
    10 more times, equals 20 sweeps on one handle bit for bit."""
    ts = syn.simple_update_cell(3, seed=2)
    _, desc = problem("infinite", N=2, D=3, chi=16)
    a = pn.PepsNet(desc, ts)
    a.blockbp_sweep(10, 0.0)
    saved = a.get_messages()
    _, ea, _ = a.blockbp_sweep(10, 0.0)
    b = pn.PepsNet(desc, ts)
    b.set_messages(saved)
    _, eb, _ = b.blockbp_sweep(10, 0.0)
    assert ea == eb
    for x, y in zip(a.get_messages(), b.get_messages()):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    assert np.array_equal(a.blockbp_expect()[1], b.blockbp_expect()[1])


def test_converged_cfg1_truncated_against_oracle():
    """The 4x4-cell patch with truncated boundary chains (chi_env = chi = 4)
    run to 1e-10 on both sides: converged <S.S> and rho_ij per bond."""
    ts = syn.finite_patch_tensors(4, 4, 2, seed=1)
    P, desc = problem("finite", Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=4)
    g = pn.PepsNet(desc, ts)
    O = oracle_for(P, ts, 4, 0, 2, 8, 0)
    done, err, _ = g.blockbp_sweep(30, 1e-10)
    so, eo = O.run(tol=1e-10, max_sweeps=30)
    print(f"sweeps gpu {done} oracle {so}, err {err:.3e} {eo:.3e}")
    assert err <= 1e-10 and eo <= 1e-10 and done == so
    rho, ss, _ = g.blockbp_expect()
    ref = oracle_rhos(O, g.bonds())
    n_skip = 0
    for b, r in enumerate(ref):
        if r is None:
            n_skip += 1
            continue
        assert np.abs(_unit(rho[b]) - unit(r)).max() < 1e-10
        assert abs(ss[b] - ss_from_rho(r)) < 1e-10
    assert n_skip <= 1


def test_converged_cfg2_energy_against_oracle():
    """Hexagonal block N=3, D=3, chi=16, simple-update tensors, T1: run to
    1e-10 on both sides; energy per site and every bond's rho_ij."""
    ts = syn.simple_update_cell(3, seed=2, steps=20, dtau=0.05)
    P, desc = problem("infinite", N=3, D=3, chi=16)
    g = pn.PepsNet(desc, ts)
    O = oracle_for(P, ts, 16, 0, 2, 8, 0)
    done, err, _ = g.blockbp_sweep(40, 1e-10)
    so, eo = O.run(tol=1e-10, max_sweeps=40)
    print(f"sweeps gpu {done} oracle {so}, err {err:.3e} {eo:.3e}")
    assert err <= 1e-10 and eo <= 1e-10
    rho, ss, e = g.blockbp_expect()
    ref = oracle_rhos(O, g.bonds())
    assert all(r is not None for r in ref)
    for b, r in enumerate(ref):
        assert np.abs(_unit(rho[b]) - unit(r)).max() < 1e-10
    e_ref = sum(ss_from_rho(r) for r in ref) / 3
    print(f"E/site gpu {e:.15f} oracle {e_ref:.15f}")
    assert abs(e - e_ref) < 1e-10
