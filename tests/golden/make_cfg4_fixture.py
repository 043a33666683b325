"""Writes cfg4_one_sweep.json: one BlockBP sweep and the expectation on the
infinite kagome lattice at N=4 (111-site hexagonal block), D=6, chi=64, from
the FP64 oracle only (nothing here touches the HIP library).

Inputs (all seeded, shared with the GPU test through ``synth``): site
tensors from 20 second-order simple-update steps (dtau = 0.05, J = 1,
seed 2); messages from ``synth.random_messages`` (seed 41) in the static
message shapes; randomized truncation (Halko, Martinsson & Tropp 2011,
Alg. 4.4) with q = 2, p = 8 and sketch seed 7.

Stored: per message its Frobenius distance to the start (the sweep's
convergence distance) and the Schmidt values of every cut of the new
message (gauge-invariant, ``bubble.schmidt_spectra``); per unique bond
rho_ij (not normalised), <S_i . S_j> and the degenerate cuts met in its
contraction; the energy per site.  Run from the
repository root: python tests/golden/make_cfg4_fixture.py  (about 30 minutes
of CPU).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bubble as bb  # noqa: E402
from oracle import geometry as geo  # noqa: E402
from oracle.blockbp import BlockBP  # noqa: E402
from oracle.dense import ss_from_rho  # noqa: E402
from synth import inputs as syn  # noqa: E402

CFG = {"N": 4, "D": 6, "chi": 64, "trunc": "T2", "q": 2, "p": 8, "sketch_seed": 7,
       "su_seed": 2, "su_steps": 20, "dtau": 0.05, "message_seed": 41}


def main():
    t0 = time.time()
    ts = syn.simple_update_cell(CFG["D"], seed=CFG["su_seed"], steps=CFG["su_steps"],
                                dtau=CFG["dtau"])
    P = geo.HexProblem(CFG["N"])
    O = BlockBP(P, ts, chi=CFG["chi"], chi_env=CFG["chi"], trunc=CFG["trunc"], q=CFG["q"],
                p=CFG["p"], seed=CFG["sketch_seed"])
    keys = list(range(6))
    shapes = [[x.shape for x in O.msgs[k]] for k in keys]
    msgs = syn.random_messages(shapes, CFG["message_seed"])
    for k, A in zip(keys, msgs):
        O.msgs[k] = [a.copy() for a in A]
    start = {k: [a.copy() for a in O.msgs[k]] for k in keys}
    bb.DEGENERATE.clear()
    bb.GAUGE_AMBIGUOUS.clear()
    O.sweep()
    print(f"sweep done {time.time() - t0:.0f} s", flush=True)
    out = dict(CFG)
    out["shapes"] = shapes
    out["degenerate_in_sweep"] = len(bb.DEGENERATE)
    out["gauge_ambiguous_in_sweep"] = len(bb.GAUGE_AMBIGUOUS)
    out["distance"] = [bb.diff_norm(O.msgs[k], start[k]) for k in keys]
    out["schmidt"] = [[s.tolist() for s in bb.schmidt_spectra(O.msgs[k])] for k in keys]
    rhos, ss, degen = [], [], []
    for n, (i, j) in enumerate(P.central_bonds()):
        bb.DEGENERATE.clear()
        r = O.rho(i, j, n)
        degen.append([list(x) for x in bb.DEGENERATE])
        rhos.append([[z.real, z.imag] for z in r.reshape(-1)])
        ss.append(ss_from_rho(r))
        print(f"bond {n} done {time.time() - t0:.0f} s: {ss[-1]:.15f} degenerate cuts {degen[-1]}",
              flush=True)
    # per bond: the (rows, cols, kept) of every split whose kept and dropped
    # singular values are degenerate (the truncation is then not unique)
    out["degenerate_in_expect"] = degen
    out["bonds"] = [list(b) for b in P.central_bonds()]
    out["rho"] = rhos
    out["ss"] = ss
    out["energy_per_site"] = sum(ss) / 3.0
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_one_sweep.json"),
              "w") as f:
        json.dump(out, f)
    print(f"written; E/site {out['energy_per_site']:.15f}", flush=True)


if __name__ == "__main__":
    main()
