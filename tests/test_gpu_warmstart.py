"""The learned warm start against the plain solve on held-out load days of
the 617-bus grid: a small network trained on about a hundred of the solver's own
solutions must reach the plain solve's 1 % target in fewer steps than the
plain solve needs from the flat start."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_06650_amd import warmstart
    return warmstart


def test_learned_start_reaches_the_target_sooner(ws_mod):
    from paper_2310_06650_amd import synth
    case = synth.config_case("c2")
    X, Y = ws_mod.generate(case, list(range(10000, 10096)), 8000)
    ws = ws_mod.WarmStart(case, X, Y, width=512, depth=3)
    losses = ws.train(800)
    assert losses[-1] < 0.1 * losses[0]
    rows = ws_mod.compare(case, ws, [20000, 20001], n_warm=8000)
    for r in rows:
        print(r)
        assert r["plain_steps"] > 0 and r["warm_steps"] > 0
        assert r["warm_steps"] < r["plain_steps"]
