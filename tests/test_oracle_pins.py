"""Pins of the oracle against facts fixed by the thesis and by mathematics.

Each test names the passage or the fact it checks.  Everything here runs on
the CPU in a few seconds."""
import os

import numpy as np
import pytest

from oracle import bubble as bb
from oracle import geometry as geo
from oracle import rng
from oracle.blockbp import BlockBP
from oracle.dense import (DenseBlockBP, PlainBP, contract, double_layer,
                          message_operator, rho_statevector, ss_from_rho,
                          statevector, H_SS, SX, SY, SZ)
from synth import inputs as syn

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(x) for x in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    assert [rng.output(1234567, n) for n in range(5)] == vals


def test_sign_sketch_is_balanced_and_reproducible():
    key = rng.stream_key(7, [1, 2, 3, 4, 5])
    A = rng.sign_matrix(key, 64, 16)
    B = rng.sign_matrix(key, 64, 16)
    assert np.array_equal(A, B)
    assert np.allclose(np.abs(A), 1.0)
    assert abs(np.mean(A.real)) < 0.15 and abs(np.mean(A.imag)) < 0.15
    assert not np.array_equal(A, rng.sign_matrix(rng.stream_key(7, [1, 2, 3, 4, 6]), 64, 16))


# ------------------------------------------------------ P3: exact contraction
@pytest.mark.parametrize("Lx,Ly", [(2, 2), (3, 2)])
def test_single_block_equals_statevector(Lx, Ly):
    """A single block covering the whole open patch has no messages; both the
    dense contraction and the boundary chain (no truncation) must reproduce
    the statevector's bond energies."""
    F = geo.FiniteProblem(Lx, Ly, Lx, Ly)
    ts = syn.finite_patch_tensors(Lx, Ly, 2, seed=11)
    psi = statevector(F.net, ts)
    Bd = DenseBlockBP(F, ts)
    Bb = BlockBP(F, ts, chi=4, chi_env=0)
    for n, ((i, _), (j, _)) in enumerate(F.net.bonds()):
        ref = ss_from_rho(rho_statevector(psi, i, j))
        assert abs(ss_from_rho(Bd.rho(i, j)) - ref) < 1e-12
        if n % 3 == 0:
            assert abs(ss_from_rho(Bb.rho(i, j, n)) - ref) < 1e-12


# ----------------------------------------------------------- P4: tree graphs
def _tree_net(edges, n):
    net = geo.Network()
    deg = [0] * n
    for (a, la, b, lb) in edges:
        deg[a] = max(deg[a], la + 1)
        deg[b] = max(deg[b], lb + 1)
    for s in range(n):
        net.sites.append({"cell": (s, 0), "kind": "T", "xy": (4 * s, 0),
                          "tensor": s, "dirs": [0] * deg[s]})
    for (a, la, b, lb) in edges:
        net.link[(a, la)] = (b, lb)
        net.link[(b, lb)] = (a, la)
    return net


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_bp_exact_on_trees(seed):
    """BP is exact on loop-free networks (Sec. "Introduction to
    Belief-Propagation")."""
    n = 11
    edges, ts = syn.tree_peps(n, 2, seed)
    net = _tree_net(edges, n)
    psi = statevector(net, ts)
    bp = PlainBP(net, ts)
    sweeps, err = bp.run(tol=1e-13, max_sweeps=200)
    assert err < 1e-12
    for (a, la, b, lb) in edges:
        assert abs(ss_from_rho(bp.rho(a, b)) - ss_from_rho(rho_statevector(psi, a, b))) < 1e-11


def test_blockbp_exact_on_chain_of_blocks():
    """Column blocks of a 3x2-cell patch form a chain of blocks (a tree), so
    BlockBP with exact messages is exact; the boundary chain with bond 4
    reproduces it (each inter-column message has three legs)."""
    F = geo.FiniteProblem(3, 2, block_of_cell=lambda c: c[0])
    assert len(F.blocks) == 3 and len(F.msg_keys) == 4
    ts = syn.finite_patch_tensors(3, 2, 2, seed=5)
    psi = statevector(F.net, ts)
    Bd = DenseBlockBP(F, ts)
    Bb = BlockBP(F, ts, chi=4, chi_env=0)
    for _ in range(4):
        Bd.sweep()
        Bb.sweep()
    for n, ((i, _), (j, _)) in enumerate(F.net.bonds()):
        ref = ss_from_rho(rho_statevector(psi, i, j))
        assert abs(ss_from_rho(Bd.rho(i, j)) - ref) < 1e-11
        assert abs(ss_from_rho(Bb.rho(i, j, n)) - ref) < 1e-11


# ---------------------------------------------- P1: exact-mode BlockBP (cfg1)
def test_cfg1_dense_equals_boundary_chain():
    """Finite 4x4-cell patch, 2x2-cell blocks, D=2, chi=4: messages are exact
    at chi=4 (three-leg messages of leg dimension 4, one-leg vectors), so the
    dense exact BlockBP and the boundary chain without in-block truncation
    must agree at every sweep, and converge to 1e-10 within 30 sweeps."""
    F = geo.FiniteProblem(4, 4, 2, 2)
    ts = syn.finite_patch_tensors(4, 4, 2, seed=1)
    Bd = DenseBlockBP(F, ts)
    Bb = BlockBP(F, ts, chi=4, chi_env=0)
    for it in range(3):
        e1, e2 = Bd.sweep(), Bb.sweep()
        assert abs(e1 - e2) < 1e-12
        for k in Bd.msgs:
            assert np.linalg.norm(bb.mps_dense(Bb.msgs[k]) - Bd.msgs[k]) < 1e-12
    sweeps, err = Bd.run(tol=1e-10, max_sweeps=30)
    assert err <= 1e-10 and sweeps < 30


# ------------------------------------------------- P6: product states (closed form)
def test_product_state_finite_closed_form():
    """For a product state <S_i.S_j> = <S_i>.<S_j>."""
    Lx, Ly = 4, 2
    F = geo.FiniteProblem(Lx, Ly, 2, 2)
    ts, phis = syn.product_state_patch(Lx, Ly, 2, seed=9)
    Bb = BlockBP(F, ts, chi=2, chi_env=2)
    Bb.run(tol=1e-12, max_sweeps=6)

    def svec(phi):
        return 0.5 * np.real([phi.conj() @ S @ phi for S in (SX, SY, SZ)])

    for n, ((i, _), (j, _)) in enumerate(F.net.bonds()):
        want = svec(phis[F.net.sites[i]["tensor"]]) @ svec(phis[F.net.sites[j]["tensor"]])
        assert abs(ss_from_rho(Bb.rho(i, j, n)) - want) < 1e-12


@pytest.mark.parametrize("trunc", ["T1", "T2"])
def test_q0_120_state_energy(trunc):
    """In-plane 120-degree product state: every bond is (1/4) cos 120 = -1/8,
    energy per site (1/3) * 6 * (-1/8) = -1/4 on the infinite lattice."""
    H = geo.HexProblem(2)
    ts = syn.q0_120_state_cell(2, seed=4)
    Bb = BlockBP(H, ts, chi=4, chi_env=4, trunc=trunc, q=1, p=2, seed=3)
    Bb.run(tol=1e-12, max_sweeps=4)
    es = Bb.bond_energies(H.central_bonds())
    assert np.allclose(es, -0.125, atol=1e-12)
    assert abs(sum(es) / 3 + 0.25) < 1e-12


def test_singlet_state_energy():
    """Singlet on every DL-DR bond, U polarised: -3/4 on DL-DR, 0 on the
    other five unique bonds, energy per site -1/4."""
    H = geo.HexProblem(2)
    ts = syn.singlet_cell(2)
    Bb = BlockBP(H, ts, chi=4, chi_env=4)
    Bb.run(tol=1e-12, max_sweeps=4)
    es = Bb.bond_energies(H.central_bonds())
    assert np.allclose(es, [0, 0, -0.75, 0, 0, 0], atol=1e-12)
    Bd = DenseBlockBP(H, ts)
    Bd.run(tol=1e-12, max_sweeps=4)
    ed = [ss_from_rho(Bd.rho(i, j)) for i, j in H.central_bonds()]
    assert np.allclose(ed, [0, 0, -0.75, 0, 0, 0], atol=1e-12)


# -------------------------------------------------- P8/P9: gauge and scale
def test_gauge_covariance_of_fixed_point():
    """An invertible gauge G / G^{-1} on an inter-block bond leaves the state,
    hence the BlockBP fixed point's local expectations, unchanged."""
    F = geo.FiniteProblem(4, 2, 2, 2)
    ts = syn.finite_patch_tensors(4, 2, 2, seed=21)
    (s1, l1), (s2, l2) = next(b for b in F.net.bonds()
                              if F.block_of[b[0][0]] != F.block_of[b[1][0]])
    G = syn.cgauss(np.random.default_rng(3), (2, 2)) + 2 * np.eye(2)
    g = [t.copy() for t in ts]
    g[s1] = np.moveaxis(np.tensordot(np.moveaxis(g[s1], 1 + l1, -1), G, axes=1), -1, 1 + l1)
    g[s2] = np.moveaxis(np.tensordot(np.moveaxis(g[s2], 1 + l2, -1),
                                     np.linalg.inv(G).T, axes=1), -1, 1 + l2)
    A = DenseBlockBP(F, ts)
    B = DenseBlockBP(F, g)
    A.run(tol=1e-13, max_sweeps=60)
    B.run(tol=1e-13, max_sweeps=60)
    for (i, _), (j, _) in F.net.bonds():
        assert abs(ss_from_rho(A.rho(i, j)) - ss_from_rho(B.rho(i, j))) < 1e-10


def test_scale_invariance():
    """t_s -> c t_s leaves every normalised message and expectation unchanged."""
    H = geo.HexProblem(2)
    ts = syn.random_unit_cell(2, seed=8)
    A = BlockBP(H, ts, chi=4, chi_env=4)
    B = BlockBP(H, [3.7 * ts[0], 0.01 * ts[1], 250.0 * ts[2]], chi=4, chi_env=4)
    for _ in range(3):
        A.sweep()
        B.sweep()
    for k in A.msgs:
        assert bb.diff_norm(A.msgs[k], B.msgs[k]) < 1e-12
    (i, j) = H.central_bonds()[0]
    assert abs(ss_from_rho(A.rho(i, j)) - ss_from_rho(B.rho(i, j))) < 1e-12


# ----------------------------------------------------- P10: message invariants
def _dense_to_mps(M):
    """Exact MPS (sites [l, P, r], boundary bonds 1) of a dense message by
    successive QR factorisations, with no truncation."""
    legs = M.shape
    sites, X, l = [], M.reshape(1, -1), 1
    for P in legs[:-1]:
        Q, X = np.linalg.qr(X.reshape(l * P, -1))
        sites.append(Q.reshape(l, P, Q.shape[1]))
        l = Q.shape[1]
    sites.append(X.reshape(l, legs[-1], 1))
    return sites


def test_exact_messages_are_hermitian_psd_unit_norm():
    """Exact-mode messages are unit-norm Hermitian positive semi-definite
    operators (ket legs rows, bra legs columns), as the PSD start of
    Sec. "Introduction to Belief-Propagation" is preserved by the update."""
    H = geo.HexProblem(2)
    ts = syn.random_unit_cell(2, seed=12)
    Bd = DenseBlockBP(H, ts)
    Bb = BlockBP(H, ts, chi=16, chi_env=0)
    Bd.sweep()
    Bb.sweep()
    for k, A in Bb.msgs.items():
        assert np.linalg.norm(bb.mps_dense(A) - Bd.msgs[k]) < 1e-12
    for _ in range(2):
        Bd.sweep()
    for M in Bd.msgs.values():
        X = message_operator(M, 2)
        assert abs(np.linalg.norm(M) - 1) < 1e-14
        assert np.linalg.norm(X - X.conj().T) < 1e-13
        ev = np.linalg.eigvalsh(0.5 * (X + X.conj().T))
        assert ev.min() >= -1e-12 * ev.max()


def test_fixed_point_residual():
    """P2: the exact dense update and the exact boundary-chain update share
    their fixed point: at the dense map's converged messages, written as
    exact MPS, one chain sweep leaves every message unchanged."""
    H = geo.HexProblem(2)
    ts = syn.simple_update_cell(2, seed=2, steps=5)
    Bd = DenseBlockBP(H, ts)
    err = np.inf
    for _ in range(60):
        err = Bd.sweep()
        if err < 1e-12:
            break
    assert err < 1e-12
    Bb = BlockBP(H, ts, chi=16, chi_env=0)
    Bb.msgs = {k: _dense_to_mps(Bd.msgs[k]) for k in Bb.msgs}
    assert Bb.sweep() < 1e-10


# ----------------------------------------------------- P11: truncation semantics
def test_t1_eckart_young():
    rs = np.random.default_rng(0)
    M = syn.cgauss(rs, (30, 24)) @ np.diag(0.7 ** np.arange(24)) @ syn.cgauss(rs, (24, 24))
    L, R = bb.truncated_split(M, 6, "T1")
    S = np.linalg.svd(M, compute_uv=False)
    assert abs(np.linalg.norm(M - L @ R) ** 2 - np.sum(S[6:] ** 2)) < 1e-12 * np.sum(S ** 2)
    assert np.linalg.norm(L.conj().T @ L - np.eye(6)) < 1e-13


def test_t2_limits():
    """T2 equals T1 when the sketch spans the whole range, and converges to
    T1 with power iterations on a decaying spectrum."""
    rs = np.random.default_rng(1)
    U, _ = np.linalg.qr(syn.cgauss(rs, (60, 60)))
    V, _ = np.linalg.qr(syn.cgauss(rs, (50, 50)))
    M = U[:, :50] @ np.diag(0.5 ** np.arange(50)) @ V.conj().T
    key = rng.stream_key(5, [1, 1, 1, 1, 1])
    L1, R1 = bb.truncated_split(M, 8, "T1")
    L2, R2 = bb.truncated_split(M, 8, "T2", q=0, p=60, key=key)
    assert np.linalg.norm(L1 @ R1 - L2 @ R2) < 1e-12
    L3, R3 = bb.truncated_split(M, 8, "T2", q=4, p=8, key=key)
    assert np.linalg.norm(L1 @ R1 - L3 @ R3) < 1e-10


# ------------------------------------------------- P12: rotation covariance
def _rot_site(net):
    from fractions import Fraction as Fr
    site_at = {st["xy"]: s for s, st in enumerate(net.sites)}

    def rot(s):
        # +120 degrees about the centre (1, 1/3) of the up-triangle at cell 0
        X, Y = net.sites[s]["xy"]
        u, v = Fr(X) - 1, Fr(Y) - Fr(1, 3)
        return site_at[(int(1 - (u + 3 * v) / 2), int(Fr(1, 3) + (u - v) / 2))]
    return rot


def test_rotation_covariance():
    """Rotating the infinite problem by 120 degrees (U -> DL -> DR, faces
    f -> f+2; the hexagonal block keeps the lattice's rotation symmetry,
    Sec. "Comparison") maps the message of face f onto the message of face
    f+2 -- to rounding also with truncated boundary chains, whose sweep
    orders rotate with the block -- and the expectation on a bond onto the
    expectation on the rotated bond."""
    H = geo.HexProblem(2)
    ts = syn.random_unit_cell(2, seed=31)
    tr = syn.rotate_cell_120(ts)
    A = BlockBP(H, ts, chi=6, chi_env=6)
    B = BlockBP(H, tr, chi=6, chi_env=6)
    for _ in range(3):
        A.sweep()
        B.sweep()
    for f in range(6):
        assert bb.diff_norm(A.msgs[f], B.msgs[(f + 2) % 6]) < 1e-11
    rot = _rot_site(H.net)
    Ad, Bd = DenseBlockBP(H, ts), DenseBlockBP(H, tr)
    for _ in range(4):
        Ad.sweep()
        Bd.sweep()
    for i, j in H.central_bonds():
        assert abs(ss_from_rho(Ad.rho(i, j)) - ss_from_rho(Bd.rho(rot(i), rot(j)))) < 1e-12
