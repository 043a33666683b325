"""Serving loop (bbp_server_*): requests on resident states that arrive while
others run are admitted as in-flight slots and HBM budget free up, overlap on
the device, and give the same results as the same requests run alone
(bit-identical: the same kernels on the same inputs)."""
import numpy as np
import pytest

from synth import inputs as syn

from gpu_cases import oracle_for, oracle_rhos, problem

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")

STATES = [
    ("infinite", dict(N=2, D=2, chi=8), lambda s: syn.random_unit_cell(2, seed=s)),
    ("infinite", dict(N=3, D=3, chi=16, prec=1), lambda s: syn.random_unit_cell(3, seed=s)),
    ("finite", dict(Lx=4, Ly=4, bLx=2, bLy=2, D=2, chi=4), lambda s: syn.finite_patch_tensors(4, 4, 2, seed=s)),
    ("infinite", dict(N=2, D=3, chi=8, trunc=1, q=1, p=4, seed=3), lambda s: syn.random_unit_cell(3, seed=s)),
]


def _states(release):
    nets, tens = [], []
    for k, (kind, kw, gen) in enumerate(STATES):
        _, desc = problem(kind, **kw)
        ts = gen(10 + k)
        g = pn.PepsNet(desc, ts)
        if release:
            g.release_workspace()
        nets.append(g)
        tens.append(ts)
    return nets, tens


def _ite_step(ts, k):
    """A perturbed copy of the site tensors, standing in for one imaginary-time
    step (the messages of the previous step are kept: a warm start)."""
    rng = np.random.default_rng(100 + k)
    return [t + 1e-3 * (rng.standard_normal(t.shape) + 1j * rng.standard_normal(t.shape)) for t in ts]


def _run_alone(nets, tens):
    out = []
    srv = pn.Server(1 << 40, 1)
    for k, (g, ts) in enumerate(zip(nets, tens)):
        r1 = srv.poll(srv.submit(g, None, tol=1e-9, max_sweeps=6))
        r2 = srv.poll(srv.submit(g, _ite_step(ts, k), tol=1e-9, max_sweeps=6))
        out.append((r1, r2))
    srv.close()
    return out


def _same(a, b):
    assert a["rc"] == b["rc"] and a["sweeps"] == b["sweeps"]
    assert a["energy"] == b["energy"] and a["err"] == b["err"]
    assert np.array_equal(a["ss"], b["ss"])


def test_server_mix_equals_alone():
    nets_a, tens = _states(release=True)
    alone = _run_alone(nets_a, tens)
    nets_m, _ = _states(release=True)
    srv = pn.Server(1 << 40, 4)
    # all first requests arrive together; the ITE-step requests arrive while
    # the first ones are still running
    t1 = [srv.submit(g, None, tol=1e-9, max_sweeps=6) for g in nets_m]
    t2 = [srv.submit(g, _ite_step(ts, k), tol=1e-9, max_sweeps=6)
          for k, (g, ts) in enumerate(zip(nets_m, tens))]
    mix = [(srv.poll(a), srv.poll(b)) for a, b in zip(t1, t2)]
    st = srv.stats()
    srv.close()
    print("stats", st, flush=True)
    assert st["peak_inflight"] >= 2          # requests overlapped on the device
    for (a1, a2), (m1, m2) in zip(alone, mix):
        _same(a1, m1)
        _same(a2, m2)
        assert m2["sweeps"] <= m1["sweeps"] or m2["err"] <= 1e-9   # warm start


def test_server_hbm_budget_limits_admission():
    nets, tens = _states(release=True)
    ws = [g.memory()[1] for g in nets]
    budget = max(ws)                          # room for one workspace at a time
    srv = pn.Server(budget, 4)
    tickets = [srv.submit(g, None, tol=1e-9, max_sweeps=2) for g in nets]
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= budget
    assert st["completed"] == len(nets)
    assert all(r["sweeps"] == 2 or r["err"] <= 1e-9 for r in res)
    with pytest.raises(pn.PepsnetError):
        small = pn.Server(min(ws) // 2, 1)
        try:
            small.submit(nets[0], None)
        finally:
            small.close()


def test_server_poll_pending_then_done():
    nets, _ = _states(release=False)
    srv = pn.Server(1 << 40, 2)
    t = srv.submit(nets[1], None, tol=0.0, max_sweeps=8)
    first = srv.poll(t, wait=False)
    done = srv.poll(t, wait=True)
    srv.close()
    assert done["sweeps"] == 8 and done["rc"] == pn.binding.BBP_NOT_CONVERGED
    assert first is None or first["sweeps"] == 8
    assert nets[1].memory()[1] > 0
    nets[1].blockbp_sweep(1, 0.0)           # the state's own workspace was kept


def test_server_slots_reused_and_requests_overlap():
    """Workspace slots are allocated while the pool grows and then reused: a
    second round of requests on the same states allocates nothing (each
    state gets back the slot it held, with its resolved descriptors), and
    the device-side windows of requests in flight together intersect."""
    nets, _ = _states(release=True)
    srv = pn.Server(1 << 40, 4)
    warm = [srv.poll(t) for t in [srv.submit(g, None, tol=0.0, max_sweeps=3) for g in nets]]
    n_alloc = srv.stats()["slot_allocations"]
    res = [srv.poll(t) for t in [srv.submit(g, None, tol=0.0, max_sweeps=3) for g in nets]]
    st = srv.stats()
    srv.close()
    print("stats", st, "windows", [r["gpu_window_ms"] for r in res], flush=True)
    assert 1 <= n_alloc <= len(nets)
    assert st["slot_allocations"] == n_alloc
    assert all(r["sweeps"] == 3 for r in warm + res)
    wins = [r["gpu_window_ms"] for r in res]
    assert all(np.isfinite(w).all() and w[1] > w[0] for w in wins)
    pairs = [(i, j) for i in range(len(wins)) for j in range(i + 1, len(wins))
             if max(wins[i][0], wins[j][0]) < min(wins[i][1], wins[j][1])]
    assert pairs, wins
    for g in nets:                            # states left with their workspace released
        assert g.memory()[1] > 0
        with pytest.raises(pn.PepsnetError):
            g.blockbp_sweep(1, 0.0)


def test_server_request_matches_oracle():
    """A served request on a fresh state (identity messages) with new site
    tensors, swept to 1e-10, gives the energy per site and every bond's
    <S.S> of the FP64 oracle run to 1e-10 on the same tensors."""
    from oracle.dense import ss_from_rho
    P, desc = problem("infinite", N=2, D=2, chi=8)
    ts0 = syn.simple_update_cell(2, seed=4, steps=20, dtau=0.05)
    ts = _ite_step(ts0, 7)
    g = pn.PepsNet(desc, ts0)
    g.release_workspace()
    srv = pn.Server(1 << 40, 2)
    r = srv.poll(srv.submit(g, ts, tol=1e-10, max_sweeps=40))
    srv.close()
    O = oracle_for(P, ts, 8, 0, 2, 8, 0)
    so, eo = O.run(tol=1e-10, max_sweeps=40)
    print(f"served: {r['sweeps']} sweeps, err {r['err']:.2e}; oracle {so} sweeps, err {eo:.2e}")
    assert r["rc"] == pn.binding.BBP_OK and r["err"] <= 1e-10 and eo <= 1e-10
    g.acquire_workspace()
    ref = oracle_rhos(O, g.bonds())
    assert all(x is not None for x in ref)
    ss_ref = np.array([ss_from_rho(x) for x in ref])
    e_ref = ss_ref.sum() / 3
    print(f"E/site served {r['energy']:.15f} oracle {e_ref:.15f}")
    assert abs(r["energy"] - e_ref) < 1e-10
    assert np.abs(r["ss"] - ss_ref).max() < 1e-10
    g.close()
