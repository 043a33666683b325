"""Boundary-MPS ("bubblecon") contraction of a block, oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. "The boundary-MPS method": a bubble, kept as an MPS with one
leg per tensor, swallows the network tensor by tensor; when the number of
legs crossing the bubble exceeds what the MPS holds, a tensor is split in two
by SVD and the new bond is truncated to at most chi.  Supporting readings:

* Canonical form (Sec. "Canonical MPS"): before each split the orthogonality
  centre is moved onto the sites being swallowed with QR (to the right) or LQ
  (to the left) steps, so the truncation of the split is the locally optimal
  one.  Reduced factorisations: a factor of an m x n matrix keeps min(m, n).
* Mantissa-exponent numbers (Sec. "Mantissa and Exponent"): after every
  swallow the centre tensor is divided by its Frobenius norm and log10 of the
  norm is accumulated in ``logscale``.
* A chain site is a tensor A[l, P, r]; its leg P fuses (ket, bra, carried...)
  row-major, with ket/bra of dimension D_leg each (double leg, I = k*D + b)
  and each carried factor d*d (physical pair p*d + p' of an open site).
* Canonical gauge: QR factors carry a real non-negative R diagonal and the
  left factor of every split has, in each column, its largest-modulus entry
  real positive.  No represented tensor changes; the gauge makes every bond
  basis unique, which the randomized sketch (applied on a bond index) needs.
* Truncation keeps exactly min(chi, rank) values -- with rank = min(rows,
  cols) -- and no relative cutoff.  Splits whose kept and dropped singular
  values are degenerate are recorded in ``DEGENERATE`` (ambiguous cut).  ``trunc="T1"``: full SVD.
  ``trunc="T2"``: randomized range finder with q power iterations and p
  oversampling (Halko, Martinsson & Tropp 2011, Alg. 4.4) followed by an exact
  SVD of the projected matrix; the sketch comes from ``oracle.rng``.  T2 falls
  back to T1 when chi + p >= min(rows, cols).
"""
from __future__ import annotations

import numpy as np

from . import rng as _rng


class Chain:
    def __init__(self, sites, legs, carries, center=0):
        self.A = list(sites)           # [l, P, r]
        self.legs = list(legs)         # leg ids
        self.legdim = []               # ket (= bra) dimension of each leg
        self.carries = [list(c) for c in carries]
        self.center = center
        self.logscale = 0.0

    def __len__(self):
        return len(self.A)


# Splits whose kept and discarded singular values are degenerate to within
# DEGENERATE_TOL * sigma_1 (the truncation is then ambiguous); tests read and
# reset this list to exclude such results from parity checks.
DEGENERATE = []
DEGENERATE_TOL = 1e-8
# Splits whose kept singular values contain a degenerate non-zero pair: the
# new bond's basis is then a free rotation, which a later randomized sketch
# (applied on that bond) sees; T2 results after such a split are not unique.
GAUGE_AMBIGUOUS = []


def _record(S, keep, rows, cols):
    if len(S) == 0 or S[0] == 0:
        return
    if keep < len(S) and S[keep - 1] - S[keep] < DEGENERATE_TOL * S[0] \
            and S[keep - 1] > DEGENERATE_TOL * S[0]:
        DEGENERATE.append((rows, cols, keep))
    kept = S[:keep]
    big = kept > DEGENERATE_TOL * S[0]
    gaps = kept[:-1][big[1:]] - kept[1:][big[1:]]
    if np.any(gaps < DEGENERATE_TOL * S[0]):
        GAUGE_AMBIGUOUS.append((rows, cols, keep))


def _qr(M):
    Q, R = np.linalg.qr(M, mode="reduced")
    return Q, R


def qr_pos(M):
    """Reduced QR with the diagonal of R real and non-negative: a unique
    factorisation for full column rank (canonical gauge of the new bond)."""
    Q, R = np.linalg.qr(M, mode="reduced")
    d = np.diag(R)
    ph = np.ones(len(d), complex)
    nz = np.abs(d) > 0
    ph[nz] = d[nz] / np.abs(d[nz])
    return Q * ph[None, :], R * ph.conj()[:, None]


def fix_columns(L, R):
    """Canonical gauge of a split bond: each column of L gets its entry of
    largest modulus (first one on ties) real and positive; R's rows follow."""
    L = L.copy()
    R = R.copy()
    for j in range(L.shape[1]):
        i = int(np.argmax(L[:, j].real ** 2 + L[:, j].imag ** 2))
        a = abs(L[i, j])
        if a > 0:
            ph = L[i, j] / a
            L[:, j] *= np.conj(ph)
            R[j, :] *= ph
    return L, R


def move_right(ch, j):
    """Left-canonicalise site j and push the remainder into site j+1."""
    A = ch.A[j]
    l, P, r = A.shape
    Q, R = qr_pos(A.reshape(l * P, r))
    ch.A[j] = Q.reshape(l, P, Q.shape[1])
    ch.A[j + 1] = np.tensordot(R, ch.A[j + 1], axes=([1], [0]))


def move_left(ch, j):
    """Right-canonicalise site j and push the remainder into site j-1."""
    A = ch.A[j]
    l, P, r = A.shape
    # A = L Q with Q having orthonormal rows: QR of A^H
    Q, R = qr_pos(A.reshape(l, P * r).conj().T)
    k = Q.shape[1]
    ch.A[j] = Q.conj().T.reshape(k, P, r)
    ch.A[j - 1] = np.tensordot(ch.A[j - 1], R.conj().T, axes=([2], [0]))


def move_center(ch, lo, hi):
    while ch.center < lo:
        move_right(ch, ch.center)
        ch.center += 1
    while ch.center > hi:
        move_left(ch, ch.center)
        ch.center -= 1


def truncated_split(M, chi, trunc="T1", q=2, p=8, key=None):
    """M (rows x cols) -> (left, right) with left having orthonormal columns,
    left @ right the rank-keep truncation, keep = min(chi, rows, cols)
    (chi <= 0: no truncation)."""
    rows, cols = M.shape
    full = min(rows, cols)
    keep = full if chi <= 0 else min(chi, full)
    if trunc == "T1" or chi <= 0 or chi + p >= full:
        U, S, Vh = np.linalg.svd(M, full_matrices=False)
        _record(S, keep, rows, cols)
        return fix_columns(U[:, :keep], S[:keep, None] * Vh[:keep])
    k = chi + p
    Om = _rng.sign_matrix(key, cols, k)
    Y = M @ Om
    for _ in range(q):
        Q, _ = _qr(Y)
        Z = M.conj().T @ Q
        Q2, _ = _qr(Z)
        Y = M @ Q2
    Q, _ = _qr(Y)
    B = Q.conj().T @ M
    Ub, S, Vh = np.linalg.svd(B, full_matrices=False)
    _record(S, keep, rows, cols)
    return fix_columns(Q @ Ub[:, :keep], S[:keep, None] * Vh[:keep])


# largest intermediate (elements) numpy may form inside one swallow's sum
EINSUM_MAX_ELEMS = 1 << 27


def _unfuse_dims(ch, j):
    D = ch.legdim[j]
    return [D, D] + [4] * len(ch.carries[j])


def swallow(ch, step, t, chi, trunc="T1", q=2, p=8, keyfn=None, d=2):
    """Swallow one site (ket tensor t[p, slot0..]) into the chain.

    ``step`` comes from ``geometry.sweep_schedule``: the site's in-legs are
    chain positions pos..pos+r-1 (slots ``in_slots``), its out-legs
    ``out_slots`` replace them.  The double layer is applied as ket then bra
    (same value as contracting with the double-layer tensor).  Carried
    physical pairs of the swallowed chain sites, followed by the site's own
    pair when it is open, ride on the first out-leg."""
    pos, ins, outs = step["pos"], step["in_slots"], step["out_slots"]
    r, s = len(ins), len(outs)
    move_center(ch, pos, pos + r - 1)
    a, b = ch.A[pos].shape[0], ch.A[pos + r - 1].shape[2]
    # unfuse every leg into (ket, bra, carries...); consecutive run sites
    # share their bond label
    labels = [0]
    nxt = [1]

    def new():
        nxt[0] += 1
        return nxt[0]

    ket_lab, bra_lab, carry_labs, carry_ids = {}, {}, [], []
    run, run_labels = [], []
    left = 0
    for j in range(r):
        A = ch.A[pos + j]
        dims = _unfuse_dims(ch, pos + j)
        kl, bl = new(), new()
        ket_lab[ins[j]], bra_lab[ins[j]] = kl, bl
        cl = [new() for _ in ch.carries[pos + j]]
        carry_labs += cl
        carry_ids += ch.carries[pos + j]
        right = 1 if j == r - 1 else new()
        run.append(A.reshape([A.shape[0]] + dims + [A.shape[2]]))
        run_labels.append([left] + [kl, bl] + cl + [right])
        labels += [kl, bl] + cl
        left = right
    labels.append(1)
    nslot = t.ndim - 1
    pl = new()
    ket_t = [pl] + [ket_lab.get(l) for l in range(nslot)]
    bra_t = [pl] + [bra_lab.get(l) for l in range(nslot)]
    out_k, out_b = {}, {}
    for l in outs:
        out_k[l], out_b[l] = new(), new()
        ket_t[1 + l] = out_k[l]
        bra_t[1 + l] = out_b[l]
    if step["open"]:
        bra_t[0] = new()
        own = [pl, bra_t[0]]
        carry_ids = carry_ids + [step["site"]]
    else:
        own = []
    # carried factors sit right after the first out-leg's (ket, bra) pair
    if s == 0:
        out_labels = [0] + carry_labs + own + [1]
    else:
        out_labels = [0, out_k[outs[0]], out_b[outs[0]]] + carry_labs + own
        for l in outs[1:]:
            out_labels += [out_k[l], out_b[l]]
        out_labels += [1]
    # the sum over every repeated label of (run sites, t, conj t); numpy
    # picks the order of the pairwise sums (the value does not depend on it),
    # with intermediates capped at EINSUM_MAX_ELEMS so that no step holds the
    # merged run (a D^(2r) chi^2 tensor) where that is large
    ops = []
    for A, lab in zip(run, run_labels):
        ops += [A, lab]
    R = np.einsum(*ops, t, ket_t, t.conj(), bra_t, out_labels,
                  optimize=("greedy", EINSUM_MAX_ELEMS))
    Qtot = int(np.prod([4] * len(carry_ids))) if carry_ids else 1
    out_dims = [t.shape[1 + l] for l in outs]
    if s == 0:
        R = R.reshape(a, Qtot, b)
        if step["absorb"] == "right":
            N = ch.A[pos + r]
            X = np.tensordot(R, N, axes=([2], [0]))            # [a, Q, P, c]
            X = np.transpose(X, (0, 2, 1, 3))
            X = X.reshape(a, N.shape[1] * Qtot, N.shape[2])
            tgt = pos + r
        else:
            N = ch.A[pos - 1]
            X = np.tensordot(N, R, axes=([2], [0]))            # [c, P, Q, b]
            X = X.reshape(N.shape[0], N.shape[1] * Qtot, b)
            tgt = pos - 1
        ch.A[tgt] = X
        ch.carries[tgt] = ch.carries[tgt] + carry_ids
        nrm = np.linalg.norm(X)
        ch.A[tgt] = X / nrm
        ch.logscale += np.log10(nrm)
        del ch.A[pos:pos + r], ch.legs[pos:pos + r]
        del ch.legdim[pos:pos + r], ch.carries[pos:pos + r]
        ch.center = tgt if tgt < pos else tgt - r
        return
    phys = [od * od for od in out_dims]
    phys[0] *= Qtot
    R = R.reshape([a] + phys + [b])
    new_sites = []
    left = a
    rest = R
    for m in range(s - 1):
        rows = left * phys[m]
        cols = int(np.prod(phys[m + 1:])) * b
        key = keyfn(m) if keyfn is not None else None
        L, Rt = truncated_split(rest.reshape(rows, cols), chi, trunc, q, p, key)
        k = L.shape[1]
        new_sites.append(L.reshape(left, phys[m], k))
        rest = Rt.reshape([k] + phys[m + 1:] + [b])
        left = k
    last = rest.reshape(left, phys[-1], b)
    nrm = np.linalg.norm(last)
    new_sites.append(last / nrm)
    ch.logscale += np.log10(nrm)
    ch.A[pos:pos + r] = new_sites
    ch.legs[pos:pos + r] = step["out_ids"]
    ch.legdim[pos:pos + r] = out_dims
    ch.carries[pos:pos + r] = [carry_ids] + [[] for _ in range(s - 1)]
    ch.center = pos + s - 1


def right_canonical(ch):
    """Centre to site 0 with every other site right-canonical, unit norm.
    Returns log10 of the removed norm."""
    move_center(ch, len(ch) - 1, len(ch) - 1)
    move_center(ch, 0, 0)
    nrm = np.linalg.norm(ch.A[0])
    ch.A[0] = ch.A[0] / nrm
    return np.log10(nrm)


def compress(A, chi):
    """Right-canonical MPS ``A`` (centre at 0) truncated left to right to
    bond chi with full SVDs, returned right-canonical with unit norm."""
    ch = Chain(A, [None] * len(A), [[] for _ in A], center=0)
    for j in range(len(A) - 1):
        l, P, r = ch.A[j].shape
        L, R = truncated_split(ch.A[j].reshape(l * P, r), chi, "T1")
        ch.A[j] = L.reshape(l, P, L.shape[1])
        ch.A[j + 1] = np.tensordot(R, ch.A[j + 1], axes=([1], [0]))
    ch.center = len(A) - 1
    right_canonical(ch)
    return ch.A


def schmidt_spectra(A):
    """Singular values of every cut of an open MPS (gauge-invariant): a
    left-to-right QR sweep gives X_j with left part = Q X_j, a right-to-left
    sweep of QR factorisations of the transposed sites gives Y_j with right
    part = Y_j Q', and the cut's values are those of X_j Y_j."""
    n = len(A)
    X = [None] * n
    R = np.ones((1, 1), complex)
    for j in range(n - 1):
        M = np.tensordot(R, A[j], axes=([1], [0]))
        l, P, r = M.shape
        _, R = qr_pos(M.reshape(l * P, r))
        X[j] = R
    out = [None] * (n - 1)
    L = np.ones((1, 1), complex)
    for j in range(n - 1, 0, -1):
        M = np.tensordot(A[j], L, axes=([2], [0]))
        l, P, r = M.shape
        _, Rt = qr_pos(M.reshape(l, P * r).T)
        L = Rt.T
        out[j - 1] = np.linalg.svd(X[j - 1] @ L, compute_uv=False)
    return out


def trace(A, dims):
    """Trace of an MPS message read as an operator (ket legs rows, bra legs
    columns): contract each site's leg with vec(I_D)."""
    v = np.ones(1, complex)
    for x, D in zip(A, dims):
        idx = [k * D + k for k in range(D)]
        v = v @ x[:, idx, :].sum(axis=1)
    return complex(v.reshape(-1)[0])


def fix_phase(A, dims):
    """Multiply a message by the unit phase that makes its trace real and
    positive (in place on site 0)."""
    tr = trace(A, dims)
    if abs(tr) > 0:
        A[0] = A[0] * (np.conj(tr) / abs(tr))
    return A


def reverse(A):
    return [x.transpose(2, 1, 0) for x in A[::-1]]


def mps_dense(A):
    """Dense tensor of an open MPS (for checks on small messages)."""
    X = A[0]
    for B in A[1:]:
        X = np.tensordot(X, B, axes=([X.ndim - 1], [0]))
    return X.reshape(X.shape[1:-1])


def mps_sum(A, B, a=1.0, b=1.0):
    """a A + b B for two open MPS on the same legs, as the MPS whose bond
    spaces are the direct sums of theirs (first site [a A_0, b B_0] along its
    right bond, inner sites block-diagonal, last site stacked along its left
    bond; Schollwoeck 2011)."""
    n = len(A)
    if n == 1:
        return [a * A[0] + b * B[0]]
    out = []
    for j in range(n):
        x, y = A[j], B[j]
        lx, P, rx = x.shape
        ly, _, ry = y.shape
        if j == 0:
            z = np.zeros((1, P, rx + ry), complex)
            z[:, :, :rx] = a * x
            z[:, :, rx:] = b * y
        elif j == n - 1:
            z = np.zeros((lx + ly, P, 1), complex)
            z[:lx] = x
            z[lx:] = y
        else:
            z = np.zeros((lx + ly, P, rx + ry), complex)
            z[:lx, :, :rx] = x
            z[lx:, :, rx:] = y
        out.append(z)
    return out


def compressed_sum(A, B, a, b, chi):
    """a A + b B brought to right-canonical form with unit norm and
    truncated to bond chi by exact SVDs (``compress``)."""
    S = mps_sum(A, B, a, b)
    ch = Chain(S, [None] * len(S), [[] for _ in S], center=0)
    right_canonical(ch)
    if max(x.shape[2] for x in ch.A) > chi:
        return compress(ch.A, chi)
    return ch.A


def hermitian_conjugate(A, dims):
    """A^dagger of a message read as an operator: every site's double leg
    (ket, bra), of dimension D^2 with D = dims[j], has its two indices
    exchanged, and every tensor is conjugated."""
    out = []
    for x, D in zip(A, dims):
        l, P, r = x.shape
        out.append(x.reshape(l, D, D, r).transpose(0, 2, 1, 3).conj().reshape(l, P, r))
    return out


def diff_norm(A, B):
    """||A - B||_F of two MPS on the same legs, from the direct-sum MPS and a
    left-to-right QR sweep (accurate to rounding of ||A||, ||B||)."""
    n = len(A)
    if n == 1:
        return float(np.linalg.norm(A[0] - B[0]))
    R = np.ones((1, 1))
    for j in range(n):
        a, b = A[j], B[j]
        if j == 0:
            X = np.concatenate([a, -b], axis=2)
        elif j == n - 1:
            X = np.concatenate([a, b], axis=0)
        else:
            la, P, ra = a.shape
            lb, _, rb = b.shape
            X = np.zeros((la + lb, P, ra + rb), complex)
            X[:la, :, :ra] = a
            X[la:, :, ra:] = b
        M = np.tensordot(R, X, axes=([1], [0]))
        l, P, r = M.shape
        if j == n - 1:
            return float(np.linalg.norm(M))
        Q, R = _qr(M.reshape(l * P, r))
    raise AssertionError


def overlap_with_carries(chain_A, chain_carries, msg_A):
    """sum over legs of chain (sites with carried factors) times message MPS
    (same legs, same order).  Returns (vector over the carried factors in
    chain order, list of carried ids)."""
    L = np.ones((1, 1, 1))                              # [c, d, Qacc]
    ids = []
    for A, car, M in zip(chain_A, chain_carries, msg_A):
        l, PQ, r = A.shape
        Q = 4 ** len(car)
        P = PQ // Q
        A4 = A.reshape(l, P, Q, r)
        # L[c, d, X] A4[c, I, q, e] M[d, I, f] -> [e, f, X, q]
        T = np.einsum("cdx,ciqe,dif->efxq", L, A4, M)
        L = T.reshape(T.shape[0], T.shape[1], -1)
        ids += car
    return L.reshape(-1), ids
