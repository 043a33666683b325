"""pepsnet_autotune: the fastest k_gemm tile shape per GEMM shape of the
sweep plans, timed on the device and cached in a text file.  A tile shape
never changes the order of any output element's sum, so a tuned handle's
sweeps are bit-identical to an untuned one's; a second handle reading the
cache times nothing and makes the same choices."""
import numpy as np
import pytest

from synth import inputs as syn

from gpu_cases import problem

pytestmark = pytest.mark.gpu

pn = pytest.importorskip("paper_2603_13304_amd")

CASES = [
    dict(N=3, D=3, chi=16, prec=1),                          # FP32 contraction, exact truncation
    dict(N=2, D=3, chi=64, trunc=1, q=1, p=8, seed=3),       # FP64, randomized truncation
]


def _flat(msgs):
    return np.concatenate([a.reshape(-1) for m in msgs for a in m])


@pytest.mark.parametrize("kw", CASES)
def test_autotune_bit_identical_and_cached(kw, tmp_path):
    cache = tmp_path / "tiles.txt"
    _, desc = problem("infinite", **kw)
    ts = syn.simple_update_cell(kw["D"], seed=2, steps=20, dtau=0.05)
    ref, tuned = pn.PepsNet(desc, ts), pn.PepsNet(desc, ts)
    n_timed, n_shapes = tuned.autotune(str(cache))
    print(kw, "shapes timed", n_timed, "tuned", n_shapes, flush=True)
    assert n_timed == n_shapes > 0 and cache.exists()
    lines = [l for l in cache.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == n_shapes
    for g in (ref, tuned):
        g.use_graph(True)
    r, t = ref.blockbp_sweep(3, 0.0), tuned.blockbp_sweep(3, 0.0)
    assert r[1] == t[1]
    assert np.array_equal(_flat(ref.get_messages()), _flat(tuned.get_messages()))
    _, ss_r, e_r = ref.blockbp_expect()
    _, ss_t, e_t = tuned.blockbp_expect()
    assert e_r == e_t and np.array_equal(ss_r, ss_t)
    again = pn.PepsNet(desc, ts)
    assert again.autotune(str(cache)) == (0, n_shapes)
    for g in (ref, tuned, again):
        g.close()
