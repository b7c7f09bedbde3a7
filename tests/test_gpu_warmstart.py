"""The learned warm start saves steps (reduced size of the 256^2 pipeline).

256 seeded 128^2 cases are advanced to equilibrium by the batched solver,
a four-level U-Net (16..128 channels) is trained on them on the GPU, and 32
unseen cases run cold (Eq. 16) and warm (the network's prediction made
mass-exact) side by side.  The warm runs must reach the cold runs' final
angle within 0.5 degrees sooner (median ratio >= 1.5), with few fallbacks
and the cold mass to FP32 rounding.
"""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_warm_start_reaches_equilibrium_sooner():
    from paper_2202_06516_amd import warmstart as WS
    from paper_2202_06516_amd import workloads as WL
    kw = dict(side=128, rs=(12.0, 32.0), r0=(18.0, 24.0))
    train = WL.warmstart_cases(256, WL.WARM_SEEDS["train"], **kw)
    test = WL.warmstart_cases(32, WL.WARM_SEEDS["test"], **kw)
    rep = WS.run(train, [], test, gen_steps=20000, horizon=20000, epochs=40, levels=4, base=16,
                 log=lambda s: None)
    s = rep["warm_start"]
    print({k: v for k, v in rep.items() if k != "cases"})
    assert rep["train_data"]["dropped"] <= 8
    assert rep["training"]["last"]["train"] < 0.05 * rep["training"]["first"]["train"]
    assert s["max_rel_mass_error"] <= 1e-6
    assert s["evaluated"] >= 24
    assert s["fallbacks"] <= s["evaluated"] // 4
    assert s["median_ratio"] >= 1.5, s
