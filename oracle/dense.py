"""Exact (dense) references: statevector, double-layer contraction, plain BP
and exact-mode BlockBP.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Double-layer ("braket") tensor: each ket tensor is contracted with its
  complex conjugate over the physical leg, every virtual leg of dimension D
  becoming a double leg of dimension D^2 (Sec. "PGM-TN Duality").  Fused
  index I = ket * D + bra.
* Plain BP message update m_{a->b} = Tr(T_a prod_{c in N_a \\ b} m_{c->a})
  (Eq. BP:DefiningEquation) with the Frobenius convergence distance of
  Eq. bp:convergenceCriterium; BP is exact on trees (Sec. "Introduction to
  Belief-Propagation").
* Exact-mode BlockBP: M_{a->b} = contract(B_a prod_{c != b} M_{c->a})
  (Eq. blockBP:DefiningEquation) with every message kept as a dense tensor
  over its face legs, normalised to unit norm and real positive trace.
* Heisenberg bond energy <S_i.S_j> with S = sigma/2 (Eq. res:afm-h:hamiltonian).

The contraction helper sums every repeated label; the pairwise order only
changes rounding, never the value.
"""
from __future__ import annotations

import numpy as np

SX = np.array([[0, 1], [1, 0]], complex)
SY = np.array([[0, -1j], [1j, 0]], complex)
SZ = np.array([[1, 0], [0, -1]], complex)
H_SS = 0.25 * (np.kron(SX, SX) + np.kron(SY, SY) + np.kron(SZ, SZ))


def contract(tensors, labels, out):
    """Sum over every label not in ``out``; result axes ordered as ``out``."""
    T = [np.asarray(t) for t in tensors]
    L = [list(l) for l in labels]
    for t, l in zip(T, L):
        if t.ndim != len(l):
            raise ValueError("label count mismatch")
    dims = {}
    for t, l in zip(T, L):
        for x, n in zip(l, t.shape):
            if dims.setdefault(x, n) != n:
                raise ValueError(f"dimension mismatch on label {x}")
    while len(T) > 1:
        best = None
        for i in range(len(T)):
            si = set(L[i])
            for j in range(i + 1, len(T)):
                sh = si & set(L[j])
                if not sh:
                    continue
                keep = [x for x in L[i] + L[j] if x not in sh]
                size = int(np.prod([dims[x] for x in keep])) if keep else 1
                if best is None or size < best[0]:
                    best = (size, i, j, sh)
        if best is None:
            i, j, sh = 0, 1, set()
        else:
            _, i, j, sh = best
        sh = sorted(sh, key=str)
        ai = [L[i].index(x) for x in sh]
        aj = [L[j].index(x) for x in sh]
        R = np.tensordot(T[i], T[j], axes=(ai, aj))
        LR = [x for x in L[i] if x not in sh] + [x for x in L[j] if x not in sh]
        for k in sorted((i, j), reverse=True):
            del T[k]
            del L[k]
        T.append(R)
        L.append(LR)
    R, LR = T[0], L[0]
    if sorted(map(str, LR)) != sorted(map(str, out)):
        raise ValueError("open labels do not match the requested output")
    return np.transpose(R, [LR.index(x) for x in out])


def double_layer(t, open_phys=False):
    """T[I0, I1, ...] = sum_p t[p, k...] conj(t[p, b...]), I = k*D + b.
    With ``open_phys`` the physical pair is kept as a trailing (p, p') axis
    pair fused to p*d + p'."""
    t = np.asarray(t)
    n = t.ndim - 1
    d = t.shape[0]
    ket = list(range(1, n + 1))
    bra = list(range(n + 1, 2 * n + 1))
    if open_phys:
        R = np.einsum(t, [0] + ket, t.conj(), [2 * n + 1] + bra,
                      [x for pair in zip(ket, bra) for x in pair] + [0, 2 * n + 1])
        return R.reshape(*[s * s for s in t.shape[1:]], d * d)
    R = np.einsum(t, [0] + ket, t.conj(), [0] + bra,
                  [x for pair in zip(ket, bra) for x in pair])
    return R.reshape(*[s * s for s in t.shape[1:]])


def bond_label(net, s, l):
    o = net.link[(s, l)]
    if isinstance(o, tuple) and len(o) == 2 and o[0] != "face":
        a, b = sorted([(s, l), o])
        return ("b", a, b)
    return ("e", s, l)


def ss_from_rho(rho):
    """<S_i . S_j> = Re Tr(rho h) / Re Tr(rho), rho indexed [(pi pj), (pi' pj')]."""
    return float(np.real(np.trace(rho @ H_SS)) / np.real(np.trace(rho)))


def expect_op(rho, op):
    """<O> = Tr(rho O) / Tr(rho) for a two-site operator O given as a
    d^2 x d^2 matrix in the (p_i p_j) basis (rows bra, columns ket:
    O[(p_i' p_j'), (p_i p_j)] = <p_i' p_j'| O |p_i p_j>), rho indexed
    [(p_i p_j), (p_i' p_j')].  Complex for a non-Hermitian O."""
    return complex(np.trace(rho @ op) / np.trace(rho))


def _unit_hermitian(rho):
    """rho / Tr rho, Hermitian part (a contracted rho carries rounding in
    its anti-Hermitian part)."""
    r = rho / np.trace(rho)
    return 0.5 * (r + r.conj().T)


def _psd_sqrt(X):
    """Principal square root of a Hermitian positive semi-definite matrix
    from its eigendecomposition; eigenvalues below zero (rounding) count as
    zero."""
    w, V = np.linalg.eigh(X)
    return (V * np.sqrt(np.clip(w, 0.0, None))) @ V.conj().T


def partial_transpose_b(rho, d=2):
    """rho^{T_B} of a two-site matrix indexed [(p_i p_j), (p_i' p_j')]:
    the second site's indices exchanged."""
    return rho.reshape(d, d, d, d).transpose(0, 3, 2, 1).reshape(d * d, d * d)


def negativity(rho, d=2):
    """Eq. res:negativity: (||rho^{T_B}||_1 - 1) / 2 for rho normalised to
    unit trace, the trace norm being the sum of the absolute eigenvalues of
    the (Hermitian) partial transpose."""
    w = np.linalg.eigvalsh(partial_transpose_b(_unit_hermitian(rho), d))
    return float((np.sum(np.abs(w)) - 1.0) / 2.0)


def fidelity(rho, sigma):
    """Eq. metrics:fidelity: (Tr sqrt(sqrt(rho) sigma sqrt(rho)))^2 for rho
    and sigma normalised to unit trace."""
    r, s = _unit_hermitian(rho), _unit_hermitian(sigma)
    sr = _psd_sqrt(r)
    M = sr @ s @ sr
    w = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
    return float(np.sum(np.sqrt(np.clip(w, 0.0, None))) ** 2)


def rho_from_carry(R, order, i, j, d=2):
    """R over the carried pairs listed in ``order`` (fused p*d + p' each) ->
    rho[(p_i p_j), (p_i' p_j')]."""
    R = np.asarray(R).reshape([d] * (2 * len(order)))
    ai, aj = order.index(i), order.index(j)
    R = np.transpose(R, [2 * ai, 2 * aj, 2 * ai + 1, 2 * aj + 1])
    return R.reshape(d * d, d * d)


# ------------------------------------------------------------- statevector
def statevector(net, tensors, sites=None):
    """psi[p_s for s in sites] of the PEPS restricted to ``sites`` (legs
    leaving the set must have dimension 1)."""
    sites = list(range(len(net.sites))) if sites is None else list(sites)
    inside = set(sites)
    T, L = [], []
    for s in sites:
        t = np.asarray(tensors[net.sites[s]["tensor"]])
        lab = [("p", s)]
        sl = [slice(None)]
        for l in range(net.nslots(s)):
            o = net.link[(s, l)]
            if isinstance(o, tuple) and len(o) == 2 and o[0] != "face" and o[0] in inside:
                lab.append(bond_label(net, s, l))
                sl.append(slice(None))
            else:
                if t.shape[1 + l] != 1:
                    raise ValueError("statevector needs dimension-1 legs at the boundary")
                sl.append(0)
        T.append(t[tuple(sl)])
        L.append(lab)
    return contract(T, L, [("p", s) for s in sites])


def rho_statevector(psi, i, j):
    """Two-site density matrix of sites at axes i, j of psi."""
    n = psi.ndim
    rest = [k for k in range(n) if k not in (i, j)]
    R = np.tensordot(psi, psi.conj(), axes=(rest, rest))   # [pi, pj, pi', pj']
    if i > j:
        R = np.transpose(R, [1, 0, 3, 2])
    d = psi.shape[i]
    return R.reshape(d * d, d * d)


# ---------------------------------------------------------------- plain BP
def identity_vec(D):
    return np.eye(D).reshape(D * D) / np.sqrt(D)


class PlainBP:
    """Plain BP on the double-layer network of ``net``: one message per
    directed internal bond, a D^2 vector (a D x D matrix), initialised to the
    normalised identity (PSD, Sec. "Introduction to Belief-Propagation")."""

    def __init__(self, net, tensors):
        self.net = net
        self.tensors = [np.asarray(t) for t in tensors]
        self.m = {}
        for (s, l), o in net.link.items():
            if isinstance(o, tuple) and len(o) == 2 and o[0] != "face":
                D = self.tensors[net.sites[s]["tensor"]].shape[1 + l]
                self.m[(s, l)] = identity_vec(D)     # message from s through slot l

    def _incoming(self, s, l):
        o = self.net.link[(s, l)]
        if o is None:
            return np.ones(1)
        return self.m[o]                              # message from the other end

    def update(self, s, l):
        t = self.tensors[self.net.sites[s]["tensor"]]
        T = double_layer(t)
        ops, labs = [T], [list(range(T.ndim))]
        for k in range(T.ndim):
            if k != l:
                ops.append(self._incoming(s, k))
                labs.append([k])
        v = contract(ops, labs, [l])
        return v / np.linalg.norm(v)

    def sweep(self):
        new = {key: self.update(*key) for key in self.m}
        err = max(np.linalg.norm(new[k] - self.m[k]) for k in self.m)
        self.m = new
        return err

    def run(self, tol=1e-12, max_sweeps=500):
        for it in range(max_sweeps):
            err = self.sweep()
            if err <= tol:
                return it + 1, err
        return max_sweeps, err

    def rho(self, i, j):
        """rho_ij from T_i, T_j (physical legs open) and all other incoming
        messages."""
        li = next(l for l in range(self.net.nslots(i))
                  if isinstance(self.net.link[(i, l)], tuple)
                  and self.net.link[(i, l)][0] == j)
        lj = self.net.link[(i, li)][1]
        ops, labs = [], []
        for s, lx in ((i, li), (j, lj)):
            t = self.tensors[self.net.sites[s]["tensor"]]
            T = double_layer(t, open_phys=True)
            lab = [("bond", i, li) if k == lx else (s, k) for k in range(T.ndim - 1)] + [("p", s)]
            ops.append(T)
            labs.append(lab)
            for k in range(T.ndim - 1):
                if k != lx:
                    ops.append(self._incoming(s, k))
                    labs.append([(s, k)])
        R = contract(ops, labs, [("p", i), ("p", j)])
        return rho_from_carry(R, [i, j], i, j)


# --------------------------------------------------------- exact-mode BlockBP
class DenseBlockBP:
    """BlockBP with every message a dense tensor (exact contraction of the
    block with its incoming messages).  Works for ``FiniteProblem`` and
    ``HexProblem``; Jacobi updates (all messages from the previous sweep)."""

    def __init__(self, prob, tensors, init="identity", seed=0):
        self.prob = prob
        self.tensors = [np.asarray(t) for t in tensors]
        self.msgs = {}
        for key in prob.msg_keys:
            legs = self._stored_legs(key)
            self.msgs[key] = self._init_msg(legs, init, seed)

    def _dim(self, s, l):
        return self.tensors[self.prob.net.sites[s]["tensor"]].shape[1 + l]

    def _stored_legs(self, key):
        """(s, l) legs of the receiving block, in storage order."""
        P = self.prob
        if P.kind == "finite":
            a, b = key
            return P.faces[b][P.face_index(b, ("block", a))]["legs"]
        return P.faces[0][key]["legs"]

    def _init_msg(self, legs, init, seed):
        vs = []
        for (s, l) in legs:
            vs.append(identity_vec(self._dim(s, l)))
        M = vs[0]
        for v in vs[1:]:
            M = np.multiply.outer(M, v)
        return M / np.linalg.norm(M)

    def _incoming(self, b, face):
        P = self.prob
        key = P.incoming_key(b, face)
        legs = P.faces[b][face]["legs"]
        if key is None:
            return np.ones([1] * len(legs)), legs
        return self.msgs[key], legs

    def _region_ops(self, region_blocks, open_sites=(), skip_faces=()):
        P = self.prob
        ops, labs = [], []
        for b in region_blocks:
            for s in P.blocks[b]:
                t = self.tensors[P.net.sites[s]["tensor"]]
                T = double_layer(t, open_phys=s in open_sites)
                lab = [bond_label(P.net, s, l) for l in range(P.net.nslots(s))]
                if s in open_sites:
                    lab.append(("p", s))
                ops.append(T)
                labs.append(lab)
            for n, f in enumerate(P.faces[b]):
                if (b, n) in skip_faces:
                    continue
                if f["key"][0] == "block" and f["key"][1] in region_blocks:
                    continue
                M, legs = self._incoming(b, n)
                ops.append(M)
                labs.append([bond_label(P.net, s, l) for (s, l) in legs])
        return ops, labs

    def update(self, key):
        P = self.prob
        a, fa, recv = P.update_target(key)
        ops, labs = self._region_ops([a], skip_faces=[(a, fa)])
        out = [bond_label(P.net, s, l) for (s, l) in recv]
        M = contract(ops, labs, out)
        return fix_phase(M / np.linalg.norm(M))

    def sweep(self):
        new = {k: self.update(k) for k in self.prob.msg_keys}
        err = max(np.linalg.norm(new[k] - self.msgs[k]) for k in new)
        if self.prob.kind == "infinite":
            new = {self.prob.store_key(k): v for k, v in new.items()}
            err = max(np.linalg.norm(new[k] - self.msgs[k]) for k in new)
        self.msgs = new
        return err

    def run(self, tol=1e-10, max_sweeps=30):
        err = np.inf
        for it in range(max_sweeps):
            err = self.sweep()
            if err <= tol:
                return it + 1, err
        return max_sweeps, err

    def rho(self, i, j):
        P = self.prob
        region = sorted({P.block_of[i], P.block_of[j]})
        ops, labs = self._region_ops(region, open_sites=(i, j))
        R = contract(ops, labs, [("p", i), ("p", j)])
        return rho_from_carry(R, [i, j], i, j)


def dense_trace(M):
    """Trace of a dense message read as an operator (sum of its ket = bra
    entries)."""
    X = M
    for ax in range(M.ndim):
        D = int(round(np.sqrt(X.shape[0])))
        X = X.reshape(D, D, *X.shape[1:])
        X = np.trace(X, axis1=0, axis2=1) if X.ndim > 2 else np.trace(X)
    return complex(X)


def fix_phase(M):
    """Unit phase that makes the message's trace real positive."""
    tr = dense_trace(M)
    return M * (np.conj(tr) / abs(tr)) if abs(tr) > 0 else M


def message_operator(M, D):
    """Dense message over k legs (fused ket*D+bra) as a D^k x D^k matrix with
    ket legs as rows and bra legs as columns."""
    k = M.ndim
    X = M.reshape([D, D] * k)
    X = np.transpose(X, list(range(0, 2 * k, 2)) + list(range(1, 2 * k, 2)))
    return X.reshape(D ** k, D ** k)
