"""blockbp_sweep_noalloc, the sweep that allocates nothing (its workspace and
descriptors live in the library's fixed device array), against blockbp_sweep
on identical handles: two calls in a row, the second on a smaller problem
than the first, so the second runs over what the first left in the array."""
import numpy as np
import pytest

from synth import inputs as syn

from gpu_cases import problem

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")

# (hex face length N, bond dimension D, chi, truncation); the second is smaller
CALLS = [dict(N=3, D=3, chi=16, trunc=0), dict(N=2, D=2, chi=8, trunc=1, q=1, p=4, seed=3)]
TOL = 1e-10   # FP64 parity bar; the two paths run the same kernels


def _flat(msgs):
    return np.concatenate([a.reshape(-1) for m in msgs for a in m])


def _pair(kw, seed):
    _, desc = problem("infinite", **kw)
    ts = syn.random_unit_cell(kw["D"], seed=seed)
    return pn.PepsNet(desc, ts), pn.PepsNet(desc, ts)


def test_noalloc_sweep_matches_blockbp_sweep():
    sizes = []
    for k, kw in enumerate(CALLS):
        ref, na = _pair(kw, seed=20 + k)
        sizes.append(na.memory()[1])
        na.release_workspace()                 # the no-allocation path needs none
        print("case", kw, "workspace bytes", sizes[-1], flush=True)
        r = ref.blockbp_sweep(3, 0.0)
        n = na.blockbp_sweep_noalloc(3, 0.0)
        assert n[0] == r[0] == 3 and n[2] == r[2]
        a, b = _flat(ref.get_messages()), _flat(na.get_messages())
        diff = float(np.max(np.abs(a - b)))
        print("  max |dmsg|", diff, "bit-identical", bool(np.array_equal(a, b)),
              "distances", r[1], n[1], flush=True)
        assert diff <= TOL
        assert abs(n[1] - r[1]) <= TOL
        # a second call continues from the new messages like blockbp_sweep
        r2, n2 = ref.blockbp_sweep(1, 0.0), na.blockbp_sweep_noalloc(1, 0.0)
        assert abs(n2[1] - r2[1]) <= TOL
        assert float(np.max(np.abs(_flat(ref.get_messages()) - _flat(na.get_messages())))) <= TOL
        na.acquire_workspace()
        rho_r, ss_r, e_r = ref.blockbp_expect()
        rho_n, ss_n, e_n = na.blockbp_expect()
        assert abs(e_n - e_r) <= TOL and np.max(np.abs(np.asarray(ss_n) - np.asarray(ss_r))) <= TOL
        ref.close()
        na.close()
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_a_workspace_over_the_limit():
    _, desc = problem("infinite", N=3, D=4, chi=32, trunc=1, q=1, p=8, seed=1)
    g = pn.PepsNet(desc, syn.random_unit_cell(4, seed=3))
    assert g.memory()[1] > pn.binding.NOALLOC_MAX_BYTES
    with pytest.raises(pn.PepsnetError) as e:
        g.blockbp_sweep_noalloc(1, 0.0)
    assert e.value.code == pn.binding.BBP_ENOMEM
    g.blockbp_sweep(1, 0.0)                    # the handle is unaffected
    g.close()


def test_noalloc_with_learning_step_and_hermitised_messages():
    """The no-allocation sweep runs the same plan as blockbp_sweep when the
    stability options add MPS sums to every update (hermitize, damping)."""
    kw = dict(N=2, D=2, chi=8, trunc=0, hermitize=True, damping=0.3)
    ref, na = _pair(kw, seed=31)
    na.release_workspace()
    r = ref.blockbp_sweep(3, 0.0)
    n = na.blockbp_sweep_noalloc(3, 0.0)
    print("distances", r[1], n[1], flush=True)
    assert n[0] == r[0] == 3
    assert abs(n[1] - r[1]) <= TOL
    assert float(np.max(np.abs(_flat(ref.get_messages()) - _flat(na.get_messages())))) <= TOL
    ref.close()
    na.close()
