"""Pins of the oracle's two-site density matrices rho_ij element by element,
and of the infinite block's self-messaging (Alg. BlockBP_singleBlock: the
message computed toward one face replaces the message on the opposite face),
against references that share nothing with the BlockBP code.

* Exact contraction (P3): on patches a single block covers, and on a chain
  of blocks (a tree of blocks, so BlockBP is exact), rho_ij / Tr rho_ij must
  equal the statevector's reduced density matrix entry by entry -- an i/j
  transposition, a dropped conjugate or a wrong carried-pair order fails.
* Observables that are not symmetric under i <-> j (<S^z_i>, <X_i Z_j>)
  from rho_ij match the statevector.
* P5, a chain messaging itself: a unit cell whose network splits into
  decoupled infinite chains (``synth.chain_cell``).  The exact environment of
  an infinite chain is the dominant eigenvector of its transfer matrix
  (``numpy.linalg.eig``), so every rho_ij of the six unique bonds is known
  in closed form; the block's fixed point must reproduce it.  A message put
  on the wrong face or leg, or the two chain directions swapped, gives a
  different fixed point.  Chains along the three lattice directions cross
  different face pairs.
"""
import numpy as np
import pytest

from oracle import bubble as bb
from oracle import geometry as geo
from oracle.blockbp import BlockBP
from oracle.dense import (DenseBlockBP, SX, SY, SZ, expect_op, rho_statevector,
                          statevector)
from synth import inputs as syn

I2 = np.eye(2)


def _unit(r):
    return r / np.trace(r)


def _op_on_state(psi, ops):
    """<psi| prod_k O_k |psi> / <psi|psi> with O_k acting on axis k."""
    phi = psi
    for ax, O in ops.items():
        phi = np.moveaxis(np.tensordot(O, phi, axes=([1], [ax])), 0, ax)
    return complex(np.vdot(psi, phi) / np.vdot(psi, psi))


@pytest.mark.parametrize("Lx,Ly", [(2, 2), (3, 2)])
def test_rho_elementwise_single_block(Lx, Ly):
    F = geo.FiniteProblem(Lx, Ly, Lx, Ly)
    ts = syn.finite_patch_tensors(Lx, Ly, 2, seed=11)
    psi = statevector(F.net, ts)
    Bd = DenseBlockBP(F, ts)
    Bb = BlockBP(F, ts, chi=4, chi_env=0)
    for n, ((i, _), (j, _)) in enumerate(F.net.bonds()):
        ref = _unit(rho_statevector(psi, i, j))
        assert np.abs(_unit(Bd.rho(i, j)) - ref).max() < 1e-12
        if n % 2 == 0:
            assert np.abs(_unit(Bb.rho(i, j, n)) - ref).max() < 1e-12


def test_rho_elementwise_chain_of_blocks():
    """Column blocks of a 3x2-cell patch (a chain of blocks): every bond,
    inter-block ones included, entry by entry."""
    F = geo.FiniteProblem(3, 2, block_of_cell=lambda c: c[0])
    ts = syn.finite_patch_tensors(3, 2, 2, seed=5)
    psi = statevector(F.net, ts)
    Bb = BlockBP(F, ts, chi=4, chi_env=0)
    for _ in range(4):
        Bb.sweep()
    n_inter = 0
    for n, ((i, _), (j, _)) in enumerate(F.net.bonds()):
        ref = _unit(rho_statevector(psi, i, j))
        assert np.abs(_unit(Bb.rho(i, j, n)) - ref).max() < 1e-11
        n_inter += F.block_of[i] != F.block_of[j]
    assert n_inter >= 6


def test_asymmetric_observables():
    """<S^z_i> and <X_i Z_j> from rho_ij against the statevector; the
    statevector values of <X_i Z_j> and <Z_i X_j> differ, so reading rho with
    i and j exchanged fails."""
    F = geo.FiniteProblem(2, 2, 2, 2)
    ts = syn.finite_patch_tensors(2, 2, 2, seed=17)
    psi = statevector(F.net, ts)
    Bb = BlockBP(F, ts, chi=4, chi_env=0)
    n_disc = 0
    for n, ((i, _), (j, _)) in enumerate(F.net.bonds()):
        rho = Bb.rho(i, j, n)
        sz_i = expect_op(rho, np.kron(0.5 * SZ, I2))
        sz_j = expect_op(rho, np.kron(I2, 0.5 * SZ))
        xz = expect_op(rho, np.kron(SX, SZ))
        zx = expect_op(rho, np.kron(SZ, SX))
        assert abs(sz_i - _op_on_state(psi, {i: 0.5 * SZ})) < 1e-12
        assert abs(sz_j - _op_on_state(psi, {j: 0.5 * SZ})) < 1e-12
        ref_xz = _op_on_state(psi, {i: SX, j: SZ})
        assert abs(xz - ref_xz) < 1e-12
        assert abs(zx - _op_on_state(psi, {i: SZ, j: SX})) < 1e-12
        n_disc += abs(ref_xz - _op_on_state(psi, {i: SZ, j: SX})) > 1e-3
        # a non-Hermitian operator: <S^+_i S^-_j> is complex
        sp = np.array([[0, 1], [0, 0]], complex)
        assert abs(expect_op(rho, np.kron(sp, sp.T)) -
                   _op_on_state(psi, {i: sp, j: sp.T})) < 1e-12
    assert n_disc >= len(F.net.bonds()) // 2


# ------------------------------------------------ P5: chains messaging themselves
# chain members per direction: kind -> (back slot, forward slot), first kind
# of the two-site chain unit first; the third kind is a product site
CHAIN_DIRS = {
    0: {"DL": (2, 0), "DR": (2, 0), "_order": ("DL", "DR"), "_product": "U"},
    60: {"DL": (3, 1), "U": (2, 0), "_order": ("DL", "U"), "_product": "DR"},
    120: {"DR": (3, 1), "U": (3, 1), "_order": ("DR", "U"), "_product": "DL"},
}


def chain_cell_dir(D, seed, direction):
    """``synth.chain_cell`` (horizontal chains) placed on the slots of the
    chains along ``direction`` degrees."""
    (_, A, B, phi) = syn.chain_cell(D, seed)
    rng = np.random.default_rng(seed + 1000)
    spec = CHAIN_DIRS[direction]
    first, second = spec["_order"]
    mats = {first: A, second: B}
    ts = {}
    for kind in ("U", "DL", "DR"):
        if kind == spec["_product"]:
            vs = [syn.cgauss(rng, (D,)) for _ in range(4)]
            ts[kind] = np.einsum("p,a,b,c,e->pabce", phi, *vs)
            continue
        back, fwd = spec[kind]
        X = mats[kind]
        others = [l for l in range(4) if l not in (back, fwd)]
        vs = {l: syn.cgauss(rng, (D,)) for l in others}
        # t[p, slots] = X[p, back, fwd] * v[other slots]
        t = np.einsum("pbf,x,y->pbfxy", X, vs[others[0]], vs[others[1]])
        perm = [0] + [1 + [back, fwd, others[0], others[1]].index(l) for l in range(4)]
        ts[kind] = np.transpose(t, perm)
    return [ts["U"], ts["DL"], ts["DR"]], A, B, phi


def chain_reference(A, B):
    """Exact reduced density matrices of the infinite chain ... A B A B ...
    (A[p, back, fwd]): transfer matrices E_X[(b b'), (f f')] =
    sum_p X[p, b, f] conj(X[p, b', f']), fixed points of E_A E_B from
    numpy.linalg.eig.  Returns rho of (A, B) in the same unit, (B, A) across
    the unit boundary, and the single-site rho of A and of B."""
    D = A.shape[1]

    def E(X, O=None):
        O = I2 if O is None else O
        # sum_{p, p'} X[p] O[p', p] conj(X[p'])
        return np.einsum("pbf,qp,qcg->bcfg", X, O, X.conj()).reshape(D * D, D * D)

    def site(X):   # [p, p', (b b'), (f f')]
        return np.einsum("pbf,qcg->pqbcfg", X, X.conj()).reshape(2, 2, D * D, D * D)

    T = E(A) @ E(B)
    w, V = np.linalg.eig(T)
    r = V[:, np.argmax(np.abs(w))]
    w2, V2 = np.linalg.eig(T.T)
    l = V2[:, np.argmax(np.abs(w2))]
    sA, sB = site(A), site(B)
    # (A, B) inside a unit: l | A | B | r
    rab = np.einsum("x,pqxy,styz,z->psqt", l, sA, sB, r).reshape(4, 4)
    # (B, A) across the boundary: l E_A | B | A | E_B r
    lA, rB = l @ E(A), E(B) @ r
    rba = np.einsum("x,pqxy,styz,z->psqt", lA, sB, sA, rB).reshape(4, 4)
    ra = np.einsum("x,pqxy,y->pq", l, sA, E(B) @ r)
    rb = np.einsum("x,pqxy,y->pq", lA, sB, r)
    return _unit(rab), _unit(rba), _unit(ra), _unit(rb)


def _swap(rho):
    return rho.reshape(2, 2, 2, 2).transpose(1, 0, 3, 2).reshape(4, 4)


def chain_bond_refs(H, direction, A, B, phi):
    """Reference rho_ij for each unique bond (i, j) of the central cell."""
    spec = CHAIN_DIRS[direction]
    first, second = spec["_order"]
    rab, rba, ra, rb = chain_reference(A, B)
    single = {first: ra, second: rb}
    pp = _unit(np.outer(phi, phi.conj()))
    net = H.net
    out = []
    for i, j in H.central_bonds():
        ki, kj = net.sites[i]["kind"], net.sites[j]["kind"]
        li = next(l for l in range(4) if isinstance(net.link.get((i, l)), tuple)
                  and net.link[(i, l)][0] == j)
        if ki == spec["_product"]:
            out.append(np.kron(pp, single[kj]))
            continue
        if kj == spec["_product"]:
            out.append(np.kron(single[ki], pp))
            continue
        back, fwd = spec[ki]
        i_first = li == fwd
        kf = ki if i_first else kj
        rho = rab if kf == first else rba
        out.append(rho if i_first else _swap(rho))
    return out


@pytest.mark.parametrize("direction", [0, 60, 120])
@pytest.mark.parametrize("N", [2, 3])
def test_p5_chain_messaging_itself(direction, N):
    H = geo.HexProblem(N)
    ts, A, B, phi = chain_cell_dir(2, seed=40 + direction, direction=direction)
    Bb = BlockBP(H, ts, chi=4, chi_env=4)
    sweeps, err = Bb.run(tol=1e-12, max_sweeps=60)
    assert err <= 1e-12
    refs = chain_bond_refs(H, direction, A, B, phi)
    for n, ((i, j), ref) in enumerate(zip(H.central_bonds(), refs)):
        got = _unit(Bb.rho(i, j, n))
        assert np.abs(got - ref).max() < 1e-10, (n, i, j)
    # the chain bonds are genuinely correlated, so the pin is not vacuous
    rab = chain_reference(A, B)[0]
    assert np.abs(rab - np.kron(chain_reference(A, B)[2], chain_reference(A, B)[3])).max() > 1e-3
