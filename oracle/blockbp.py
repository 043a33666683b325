"""BlockBP with MPS messages and boundary-MPS block contraction (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Message update: M_{a->b} = contract(B_a prod_{c != b} M_{c->a})
  (Eq. blockBP:DefiningEquation), the contraction done by the boundary chain
  of ``oracle.bubble`` following ``geometry.sweep_schedule``.
* Infinite lattice: one block messaging itself; the message computed toward
  face f replaces the message on the opposite face (Alg. BlockBP_singleBlock).
* Jacobi schedule: every message of sweep i+1 is computed from the messages
  of sweep i, as the algorithm builds Messages^{(i+1)} from Messages^{(i)}.
* Initial messages: normalised identity vec(I_D)/sqrt(D) on every leg (a
  positive semi-definite start, Sec. "Introduction to Belief-Propagation").
* Messages are stored right-canonical with unit norm, legs in the receiving
  face's counter-clockwise order, every bond zero-padded to the static
  dimension min(chi, product of double-leg dimensions on either side) (the
  represented tensor is unchanged; fixed shapes also fix the T2 sketch
  layout), and with real positive trace as operators
  (ket legs rows, bra legs columns).  The update fixes a message only up to a
  complex phase; a positive semi-definite message has positive trace, and
  without this convention a round-off phase is multiplied by the number of
  incoming messages at every sweep of the infinite block.
* Convergence distance: Frobenius norm of the difference of the unit-norm
  messages (Eq. bp:convergenceCriterium), maximum over all messages, from the
  direct-sum MPS.
* Local expectation <S_i.S_j> = Re Tr(rho h)/Re Tr(rho) with h = S.S,
  S = sigma/2 (Eq. res:afm-h:hamiltonian).  rho_ij is contracted by one sweep
  of the block holding both sites (both sites open, their physical pairs
  carried on out-legs) toward a chosen face, closed with the incoming message
  on that face.  For a bond between blocks a and b the sweep of a toward b
  (site i open) produces a carried message that then feeds b's sweep (site j
  open).  Energy per site = (1/3) sum over the six unique bonds of the unit
  cell (each site has four bonds, each bond two sites).

Parity: pinned by the tests in tests/test_oracle_*.py (statevector, exact
dense BlockBP, trees, closed-form product and singlet states, invariants).
T2 truncation beyond its T1 limit is parity-unpinned (tested only against
itself on the GPU and against T1 as a report).
"""
from __future__ import annotations

import numpy as np

from . import bubble as bb
from . import geometry as geo
from . import rng as _rng
from .dense import identity_vec, rho_from_carry, ss_from_rho

PURPOSE_MSG = 1
PURPOSE_EXPECT = 2


class BlockBP:
    def __init__(self, prob, tensors, chi, chi_env=None, trunc="T1", q=2, p=8, seed=0,
                 damping=0.0, hermitize=False):
        self.prob = prob
        self.tensors = [np.asarray(t, complex) for t in tensors]
        self.chi = chi
        self.chi_env = chi if chi_env is None else chi_env
        self.trunc, self.q, self.p, self.seed = trunc, q, p, seed
        # Sec. "Additions for numerical stability": learning step with
        # alpha = 1 - damping, and Hermitised messages (both off by default)
        self.damping, self.hermitize = float(damping), bool(hermitize)
        self.sweeps_done = 0
        self.sched = {}
        self.msgs = {}
        for key in prob.msg_keys:
            skey = self._store_key(key)
            legs = self._recv_legs(skey)
            ident = [identity_vec(self._dim(s, l)).reshape(1, -1, 1) for (s, l) in legs]
            self.msgs[skey] = self._pad_to_caps(ident, legs)

    # ---------------------------------------------------------- bookkeeping
    def _dim(self, s, l):
        return self.tensors[self.prob.net.sites[s]["tensor"]].shape[1 + l]

    def _store_key(self, key):
        return self.prob.store_key(key) if self.prob.kind == "infinite" else key

    def _recv_legs(self, skey):
        P = self.prob
        if P.kind == "infinite":
            return P.faces[0][skey]["legs"]
        a, b = skey
        return P.faces[b][P.face_index(b, ("block", a))]["legs"]

    def _caps(self, legs):
        """Static bond dimensions of a message on ``legs``: bond j is
        min(chi, prod of double-leg dims left of it, prod right of it)."""
        pd = [self._dim(s, l) ** 2 for (s, l) in legs]
        caps = [1]
        for j in range(1, len(pd)):
            caps.append(min(self.chi, int(np.prod(pd[:j])), int(np.prod(pd[j:]))))
        caps.append(1)
        return caps

    def _pad_to_caps(self, A, legs):
        """Zero-pad every bond of a message to its static dimension (the
        represented tensor is unchanged)."""
        caps = self._caps(legs)
        out = []
        for j, x in enumerate(A):
            l, P, r = x.shape
            if l > caps[j] or r > caps[j + 1]:
                raise ValueError("message bond above its static dimension")
            y = np.zeros((caps[j], P, caps[j + 1]), complex)
            y[:l, :, :r] = x
            out.append(y)
        return out

    def _incoming(self, b, face):
        P = self.prob
        key = P.incoming_key(b, face)
        legs = P.faces[b][face]["legs"]
        if key is None:
            return [np.ones((1, 1, 1), complex) for _ in legs]
        return self.msgs[key]

    def schedule(self, b, face, open_sites=()):
        k = (b, face, tuple(sorted(open_sites)))
        if k not in self.sched:
            P = self.prob
            self.sched[k] = geo.sweep_schedule(P.net, P.blocks[b], P.faces[b], face,
                                               open_sites)
        return self.sched[k]

    def msg_index(self, key):
        return self.prob.msg_keys.index(key)

    # ------------------------------------------------------------ one sweep
    def initial_chain(self, b, face, override=None):
        """Incoming messages of every face but ``face``, counter-clockwise
        starting after it.  ``override`` maps a face index to replacement
        (sites, carries) for that face."""
        P = self.prob
        F = P.faces[b]
        nf = len(F)
        A, legs, dims, carries = [], [], [], []
        for k in range(1, nf):
            f = (face + k) % nf
            if override is not None and f in override:
                sites, car = override[f]
            else:
                sites = self._incoming(b, f)
                car = [[] for _ in sites]
            for (s, l), x, c in zip(F[f]["legs"], sites, car):
                A.append(np.array(x, complex))
                legs.append(("in", s, l))
                dims.append(self._dim(s, l))
                carries.append(list(c))
        ch = bb.Chain(A, legs, carries, center=0)
        ch.legdim = dims
        return ch

    def run_sweep(self, b, face, open_sites=(), override=None, tags=(0, 0, 0), last_tag=0):
        """Sketch keys of T2 splits: SplitMix64 stream keys over the tags
        (purpose, index, sub-sweep, step, split, last_tag)."""
        steps, final = self.schedule(b, face, open_sites)
        ch = self.initial_chain(b, face, override)
        P = self.prob
        for n, st in enumerate(steps):
            t = self.tensors[P.net.sites[st["site"]]["tensor"]]

            def keyfn(m, n=n):
                return _rng.stream_key(self.seed, list(tags) + [n, m, last_tag])

            bb.swallow(ch, st, t, self.chi_env, self.trunc, self.q, self.p, keyfn)
        return ch, final

    def update(self, key):
        """New message for ``key`` (unit norm, right-canonical, storage order)."""
        P = self.prob
        a, fa, recv = P.update_target(key)
        # sketch keys are the same at every sweep, so the truncated update is
        # one fixed map whose fixed point BlockBP can reach
        tags = (PURPOSE_MSG, self.msg_index(key), 0)
        ch, final = self.run_sweep(a, fa, tags=tags, last_tag=0)
        if final == list(recv):
            A = ch.A
        elif final == list(recv)[::-1]:
            A = bb.reverse(ch.A)
            ch.center = len(A) - 1 - ch.center
        else:
            raise ValueError("final chain does not match the receiving face")
        out = bb.Chain(A, [None] * len(A), [[] for _ in A], center=ch.center)
        bb.right_canonical(out)
        A = out.A
        if max(x.shape[2] for x in A) > self.chi:
            A = bb.compress(A, self.chi)
        legs = self._recv_legs(self._store_key(key))
        dims = [self._dim(s, l) for (s, l) in legs]
        if self.hermitize or self.damping > 0.0:
            # both act on the finished message: unit norm, trace real positive
            A = bb.fix_phase(A, dims)
        if self.hermitize:   # Sec. "'Hermitize' MPSs": (A + A^dagger) / 2
            A = bb.compressed_sum(A, bb.hermitian_conjugate(A, dims), 0.5, 0.5, self.chi)
        if self.damping > 0.0:
            # Eq. blockBP:kagome:numerics:learning_step1 with alpha = 1 - damping:
            # the replacing message is alpha new + (1 - alpha) old
            old = self.msgs[self._store_key(key)]
            A = bb.compressed_sum(A, old, 1.0 - self.damping, self.damping, self.chi)
        A = self._pad_to_caps(A, legs)
        # unit norm alone leaves the message's global phase free; round-off
        # in it is amplified by the sweep, so fix the trace real positive
        return bb.fix_phase(A, [self._dim(s, l) for (s, l) in legs])

    def sweep(self):
        new = {}
        for key in self.prob.msg_keys:
            new[self._store_key(key)] = self.update(key)
        err = max(bb.diff_norm(new[k], self.msgs[k]) for k in new)
        self.msgs = new
        self.sweeps_done += 1
        return err

    def run(self, tol=1e-10, max_sweeps=30):
        err = np.inf
        for it in range(max_sweeps):
            err = self.sweep()
            if err <= tol:
                return it + 1, err
        return max_sweeps, err

    # ---------------------------------------------------------- expectation
    def _close(self, b, face, ch, final):
        """Contract a finished sweep of block b toward ``face`` with the
        incoming message on that face."""
        P = self.prob
        msg = self._incoming(b, face)
        legs = P.faces[b][face]["legs"]
        if list(final) == list(legs):
            pass
        elif list(final) == list(legs)[::-1]:
            msg = bb.reverse(msg)
        else:
            raise ValueError("final chain does not match the closing face")
        return bb.overlap_with_carries(ch.A, ch.carries, msg)

    def expect_face(self, b):
        """Face closed by the expectation sweep of block b: the first face
        (counter-clockwise from the bottom) carrying a real message, else the
        first face."""
        F = self.prob.faces[b]
        for n, f in enumerate(F):
            if f["key"][0] != "outside":
                return n
        return 0

    def rho(self, i, j, bond_index=0):
        P = self.prob
        a, b = P.block_of[i], P.block_of[j]
        if a == b:
            f = self.expect_face(a)
            ch, final = self.run_sweep(a, f, open_sites=(i, j),
                                       tags=(PURPOSE_EXPECT, bond_index, 0))
            R, ids = self._close(a, f, ch, final)
            return rho_from_carry(R, ids, i, j)
        # block a toward b with i open: a carried message into b
        fa = P.face_index(a, ("block", b))
        fb = P.face_index(b, ("block", a))
        ch, final = self.run_sweep(a, fa, open_sites=(i,),
                                   tags=(PURPOSE_EXPECT, bond_index, 0))
        recv = [P.net.link[sl] for sl in P.faces[b][fb]["legs"]]
        A, car = ch.A, ch.carries
        if final == recv[::-1]:
            A, car = bb.reverse(A), car[::-1]
        elif final != recv:
            raise ValueError("carried message does not match the receiving face")
        cm = bb.Chain(A, [None] * len(A), car, center=len(A) - 1 - ch.center
                      if final == recv[::-1] else ch.center)
        bb.right_canonical(cm)
        A = cm.A
        fe = [n for n in range(len(P.faces[b])) if n != fb]
        fe = next((n for n in fe if P.faces[b][n]["key"][0] != "outside"), fe[0])
        ch2, final2 = self.run_sweep(b, fe, open_sites=(j,), override={fb: (A, car)},
                                     tags=(PURPOSE_EXPECT, bond_index, 1))
        R, ids = self._close(b, fe, ch2, final2)
        return rho_from_carry(R, ids, i, j)

    def bond_energies(self, bonds):
        return [ss_from_rho(self.rho(i, j, n)) for n, (i, j) in enumerate(bonds)]

    def energy_per_site(self):
        """Infinite kagome: (1/3) sum over the six unique bonds."""
        bonds = self.prob.central_bonds()
        return sum(self.bond_energies(bonds)) / 3.0


def dense_message(A):
    return bb.mps_dense(A)
