"""Shared helpers for the GPU parity tests: run the same seeded problem on
the HIP library and on the oracle and compare element by element."""
import numpy as np

from oracle import bubble as bb
from oracle import geometry as geo
from oracle.blockbp import BlockBP
from oracle.dense import ss_from_rho
from synth import inputs as syn

import paper_2603_13304_amd as pn


def problem(kind, **kw):
    if kind == "finite":
        P = geo.FiniteProblem(kw["Lx"], kw["Ly"], kw["bLx"], kw["bLy"])
        desc = pn.binding.make_desc(pn.BBP_KAGOME_OPEN, D=kw["D"], chi=kw["chi"], Lx=kw["Lx"],
                                    Ly=kw["Ly"], bLx=kw["bLx"], bLy=kw["bLy"],
                                    precision=kw.get("prec", 0), trunc=kw.get("trunc", 0),
                                    q=kw.get("q", 2), p=kw.get("p", 8), seed=kw.get("seed", 0),
                                    chi_env=kw.get("chi_env"), swallow_order=kw.get("order", 0),
                                    hermitize=kw.get("hermitize", False),
                                    damping=kw.get("damping", 0.0))
    else:
        P = geo.HexProblem(kw["N"])
        desc = pn.binding.make_desc(pn.BBP_KAGOME_INF_HEX, D=kw["D"], chi=kw["chi"], hex_N=kw["N"],
                                    precision=kw.get("prec", 0), trunc=kw.get("trunc", 0),
                                    q=kw.get("q", 2), p=kw.get("p", 8), seed=kw.get("seed", 0),
                                    chi_env=kw.get("chi_env"), swallow_order=kw.get("order", 0),
                                    hermitize=kw.get("hermitize", False),
                                    damping=kw.get("damping", 0.0))
    return P, desc


def oracle_for(P, ts, chi, trunc, q, p, seed, chi_env=None, hermitize=False, damping=0.0):
    return BlockBP(P, ts, chi=chi, chi_env=chi if chi_env is None else chi_env,
                   trunc="T2" if trunc else "T1", q=q, p=p, seed=seed,
                   hermitize=hermitize, damping=damping)


def slot_keys(P):
    return list(range(6)) if P.kind == "infinite" else list(P.msg_keys)


def set_random_messages(g, O, P, seed):
    keys = slot_keys(P)
    shapes = [[x.shape for x in O.msgs[k]] for k in keys]
    assert shapes == [g.message_shapes(m) for m in range(len(keys))]
    msgs = syn.random_messages(shapes, seed)
    for k, A in zip(keys, msgs):
        O.msgs[k] = [a.copy() for a in A]
    g.set_messages(msgs)


def message_diff(g, O, P):
    got = g.get_messages()
    return max(bb.diff_norm(O.msgs[k], got[m]) for m, k in enumerate(slot_keys(P)))


def oracle_bond_energies(O, bonds):
    """Per-bond <S.S> from the oracle, with None where a truncation in the
    bond's contraction was ambiguous (degenerate singular values at the cut)."""
    return [None if r is None else ss_from_rho(r) for r in oracle_rhos(O, bonds)]


def oracle_rhos(O, bonds):
    """Per-bond rho_ij from the oracle (not normalised: <S.S> is
    Re Tr(rho h) / Re Tr(rho), which differs from the value of rho / Tr rho
    when a non-Hermitian start makes the trace complex), None where a
    truncation in the bond's contraction was ambiguous."""
    out = []
    for n, (i, j) in enumerate(bonds):
        bb.DEGENERATE.clear()
        r = O.rho(i, j, n)
        out.append(None if bb.DEGENERATE else r)
    return out


def unit(r):
    return r / np.trace(r)
