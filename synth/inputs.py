"""Seeded site tensors for kagome PEPS problems.

Layout of every ket tensor: ``t[p, l0, l1, l2, l3]`` (complex128, C order),
p the physical index (d = 2) and l0..l3 the virtual legs ordered by bond
angle counter-clockwise from +x.  Legs that leave a finite patch have
dimension 1.

Leg angles per site kind (multiples of 60 degrees):
  DL: 0, 60, 180, 240     DR: 0, 120, 180, 300     U: 60, 120, 240, 300
and the six bonds of the three-site unit cell (used by the simple-update
generator) are, as (site kind, slot) pairs:
  b0 U-DL  (U,2)-(DL,1)   b1 U-DR  (U,3)-(DR,1)   b2 DL-DR (DL,0)-(DR,2)
  b3 DR-DL' (DR,0)-(DL,2) b4 U-DL' (U,0)-(DL,3)   b5 U-DR' (U,1)-(DR,3)
"""
from __future__ import annotations

import numpy as np

KINDS = ("U", "DL", "DR")
BOND_SLOTS = [(("U", 2), ("DL", 1)), (("U", 3), ("DR", 1)), (("DL", 0), ("DR", 2)),
              (("DR", 0), ("DL", 2)), (("U", 0), ("DL", 3)), (("U", 1), ("DR", 3))]
# unit-cell bond carried by each (kind, slot)
SLOT_BOND = {}
for _b, (_x, _y) in enumerate(BOND_SLOTS):
    SLOT_BOND[_x] = _b
    SLOT_BOND[_y] = _b


def cgauss(rng, shape):
    """i.i.d. complex Gaussian, real and imaginary parts N(0, 1/2)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def random_unit_cell(D, seed, d=2, normalize=True):
    """Three unique ket tensors (U, DL, DR) with i.i.d. complex Gaussian entries."""
    rng = np.random.default_rng(seed)
    ts = []
    for _ in KINDS:
        t = cgauss(rng, (d, D, D, D, D))
        if normalize:
            t /= np.linalg.norm(t)
        ts.append(t)
    return ts


def finite_patch_tensors(Lx, Ly, D, seed, d=2):
    """Ket tensors of an open Lx x Ly-cell patch, site order: cell (i, j)
    row-major (j outer), within a cell U, DL, DR.  Off-patch legs get
    dimension 1."""
    cells = [(i, j) for j in range(Ly) for i in range(Lx)]
    off = {"DL": [(0, 0), (0, 0), (-1, 0), (0, -1)],
           "DR": [(1, 0), (0, 0), (0, 0), (1, -1)],
           "U": [(0, 1), (-1, 1), (0, 0), (0, 0)]}
    rng = np.random.default_rng(seed)
    out = []
    for (i, j) in cells:
        for k in KINDS:
            dims = []
            for (di, dj) in off[k]:
                ii, jj = i + di, j + dj
                dims.append(D if (0 <= ii < Lx and 0 <= jj < Ly) else 1)
            out.append(cgauss(rng, (d, *dims)))
    return out


def product_state_cell(D, phis, seed):
    """Product state: t = phi[p] * v0[l0] v1[l1] v2[l2] v3[l3] with random
    rank-1 virtual vectors.  ``phis`` = three spinors (U, DL, DR)."""
    rng = np.random.default_rng(seed)
    ts = []
    for phi in phis:
        vs = [cgauss(rng, (D,)) for _ in range(4)]
        t = np.einsum("p,a,b,c,e->pabce", np.asarray(phi, complex), *vs)
        ts.append(t / np.linalg.norm(t))
    return ts


def spinor(theta, phi):
    """Spin-1/2 coherent state pointing along (theta, phi)."""
    return np.array([np.cos(theta / 2), np.exp(1j * phi) * np.sin(theta / 2)])


def q0_120_state_cell(D, seed):
    """In-plane 120-degree product state (U, DL, DR at 0, 120, 240 degrees)."""
    phis = [spinor(np.pi / 2, a) for a in (0.0, 2 * np.pi / 3, 4 * np.pi / 3)]
    return product_state_cell(D, phis, seed)


def singlet_cell(D):
    """DL-DR singlet in every cell, U polarised up, all other legs pinned to
    virtual index 0.  Needs D >= 2."""
    if D < 2:
        raise ValueError("D >= 2 needed")
    tU = np.zeros((2, D, D, D, D), complex)
    tU[0, 0, 0, 0, 0] = 1.0
    tDL = np.zeros((2, D, D, D, D), complex)
    tDR = np.zeros((2, D, D, D, D), complex)
    for a in range(2):
        tDL[a, a, 0, 0, 0] = 1.0          # DL slot 0 faces DR of the same cell
    eps = np.array([[0.0, 1.0], [-1.0, 0.0]]) / np.sqrt(2.0)
    for a in range(2):
        for p in range(2):
            tDR[p, 0, 0, a, 0] = eps[a, p]  # DR slot 2 faces DL of the same cell
    return [tU, tDL, tDR]


# ------------------------------------------------------- simple update inputs
def heisenberg_gate(tau):
    """exp(-tau * S.S) on two spin-1/2, from the singlet projector."""
    s = np.array([0.0, 1.0, -1.0, 0.0]) / np.sqrt(2.0)
    Ps = np.outer(s, s)
    Pt = np.eye(4) - Ps
    return np.exp(-tau / 4.0) * Pt + np.exp(3.0 * tau / 4.0) * Ps


def simple_update_cell(D, seed, steps=20, dtau=0.05, d=2):
    """Three-site kagome unit cell from ``steps`` second-order Trotter steps of
    imaginary time (Heisenberg J = 1) with the simple update, started from
    seeded random complex tensors.  Used only to make inputs that look like
    an imaginary-time-evolved state."""
    rng = np.random.default_rng(seed)
    t = {k: cgauss(rng, (d, D, D, D, D)) for k in KINDS}
    lam = [np.ones(D) for _ in range(6)]
    order = list(range(6)) + list(range(5, -1, -1))
    for _ in range(steps):
        for b in order:
            (ka, la), (kb, lb) = BOND_SLOTS[b]
            A = _absorb(t[ka], ka, lam, skip=la)
            B = _absorb(t[kb], kb, lam, skip=lb)
            A = np.moveaxis(A, 1 + la, -1)          # [p, others..., k]
            B = np.moveaxis(B, 1 + lb, -1)
            A = A * lam[b]
            g = heisenberg_gate(dtau / 2).reshape(d, d, d, d)
            th = _gate_pair(g, A, B)
            sa = A.shape[:-1]
            sb = B.shape[:-1]
            M = th.reshape(int(np.prod(sa)), int(np.prod(sb)))
            U, S, Vh = np.linalg.svd(M, full_matrices=False)
            U, S, Vh = U[:, :D], S[:D], Vh[:D]
            lam[b] = S / np.linalg.norm(S)
            Anew = U.reshape(*sa, D)
            Bnew = Vh.T.reshape(*sb, D)
            Anew = np.moveaxis(Anew, -1, 1 + la)
            Bnew = np.moveaxis(Bnew, -1, 1 + lb)
            t[ka] = _absorb(Anew, ka, lam, skip=la, power=-1)
            t[kb] = _absorb(Bnew, kb, lam, skip=lb, power=-1)
    out = []
    for k in KINDS:
        x = t[k]
        for l in range(4):
            x = _leg_scale(x, l, np.sqrt(lam[SLOT_BOND[(k, l)]]))
        out.append(x / np.linalg.norm(x))
    return out


def _gate_pair(g, A, B):
    # A: [p, a1, a2, a3, k], B: [q, b1, b2, b3, k] -> th[p', a.., q', b..]
    AB = np.tensordot(A, B, axes=([A.ndim - 1], [B.ndim - 1]))  # [p, a.., q, b..]
    na = A.ndim - 2
    AB = np.moveaxis(AB, 1 + na, 1)                              # [p, q, a.., b..]
    th = np.tensordot(g, AB, axes=([2, 3], [0, 1]))              # [p', q', a.., b..]
    th = np.moveaxis(th, 1, 1 + na)                              # [p', a.., q', b..]
    return th


def _leg_scale(x, l, v):
    shape = [1] * x.ndim
    shape[1 + l] = v.size
    return x * v.reshape(shape)


def _absorb(x, kind, lam, skip, power=1):
    for l in range(4):
        if l == skip:
            continue
        v = lam[SLOT_BOND[(kind, l)]]
        if power < 0:
            v = 1.0 / np.maximum(v, 1e-12)
        x = _leg_scale(x, l, v)
    return x


def product_state_patch(Lx, Ly, D, seed, d=2):
    """Product-state ket tensors on an open patch (same site order as
    ``finite_patch_tensors``): t = phi[p] * v0[l0] ... with random spinors phi
    and random virtual vectors.  Returns (tensors, spinors)."""
    rng = np.random.default_rng(seed)
    shapes = [t.shape for t in finite_patch_tensors(Lx, Ly, D, seed=0, d=d)]
    ts, phis = [], []
    for sh in shapes:
        phi = cgauss(rng, (d,))
        phi /= np.linalg.norm(phi)
        vs = [cgauss(rng, (n,)) for n in sh[1:]]
        t = np.einsum("p,a,b,c,e->pabce", phi, *vs)
        ts.append(t)
        phis.append(phi)
    return ts, phis


def chain_cell(D, seed, d=2):
    """Unit cell whose network splits into decoupled horizontal chains.
    DL and DR carry a random MPS tensor on their horizontal legs (slot 2 to
    the left, slot 0 to the right) and a fixed random vector on each of their
    two other legs; U is a product of a random spinor and four random
    vectors.  Every bond leaving the horizontal chains then contracts two
    fixed vectors to a scalar, so the infinite lattice is a stack of
    identical infinite chains ... DL DR DL DR ... times scalars.  Returns
    (tensors [U, DL, DR], A, B, phi) with A[p, left, right] the DL chain
    tensor, B the DR one and phi the U spinor."""
    rng = np.random.default_rng(seed)
    A = cgauss(rng, (d, D, D))
    B = cgauss(rng, (d, D, D))
    phi = cgauss(rng, (d,))
    phi /= np.linalg.norm(phi)
    vU = [cgauss(rng, (D,)) for _ in range(4)]
    w = [cgauss(rng, (D,)) for _ in range(2)]
    u = [cgauss(rng, (D,)) for _ in range(2)]
    tU = np.einsum("p,a,b,c,e->pabce", phi, *vU)
    # t[p, l0 (right), l1, l2 (left), l3]
    tDL = np.einsum("plr,b,e->prble", A, w[0], w[1])
    tDR = np.einsum("plr,b,e->prble", B, u[0], u[1])
    return [tU, tDL, tDR], A, B, phi


def rotate_cell_120(ts):
    """Unit cell of the lattice rotated by 120 degrees about the centre of an
    up-triangle: U -> DL -> DR -> U, every bond direction advancing by two
    60-degree steps (leg slots permuted accordingly)."""
    tU, tDL, tDR = ts
    new_DL = np.transpose(tU, (0, 3, 4, 1, 2))
    new_DR = np.transpose(tDL, (0, 4, 1, 2, 3))
    new_U = np.transpose(tDR, (0, 4, 1, 2, 3))
    return [new_U, new_DL, new_DR]


def tree_peps(n_sites, D, seed, d=2, max_degree=4):
    """Random tree-shaped PEPS: returns (edges, tensors) where edges are
    (s1, slot1, s2, slot2) and each site tensor is t[p, slots...]."""
    rng = np.random.default_rng(seed)
    deg = [0] * n_sites
    edges = []
    for s in range(1, n_sites):
        cand = [x for x in range(s) if deg[x] < max_degree]
        par = int(rng.choice(cand))
        edges.append((par, deg[par], s, deg[s]))
        deg[par] += 1
        deg[s] += 1
    ts = [cgauss(rng, (d,) + (D,) * deg[s]) for s in range(n_sites)]
    return edges, ts


def random_messages(shapes, seed):
    """Seeded generic messages for a handle's static message shapes: for each
    message a list of (l, P, r) site shapes; every site i.i.d. complex
    Gaussian.  Used as a non-degenerate starting point."""
    rng = np.random.default_rng(seed)
    out = []
    for sites in shapes:
        A = [cgauss(rng, sh) for sh in sites]
        nrm = 1.0
        for x in A:
            nrm *= np.linalg.norm(x)
        A[0] = A[0] / max(nrm, 1e-300)
        out.append(A)
    return out
