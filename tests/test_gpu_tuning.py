"""The launch-configuration autotuner.  Block order and collide load
schedule give bitwise the same state; the potential kernel forms (LDS
tiles of either shape with two or four sub-iterations per launch, single
launches) agree to rounding.  lbm_ehd_tune leaves
the handle's state and step count as they were, keeps a graph working, and
the Python cache applies a stored choice without timing."""
import json

import pytest

torch = pytest.importorskip("torch")
from paper_2608_05787_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def batch(sub):
    cases = [inputs.parity_case(n, m, seed=n, sub=sub) for n, m in ((70, 40), (33, 17), (128, 96))]
    return [c[0] for c in cases], [c[1] for c in cases]


def pops(sim, n_inst):
    return [sim.populations(fam, inst=i).clone() for i in range(n_inst) for fam in "fglh"]


ROUNDING = {"fp32": 1e-5, "fp16s": 1e-2, "fp64": 1e-12}


# fp32 K = 3: one single launch and one pair; K = 5: single + a four-iteration
# launch on tall tiles (pairs otherwise); K = 6: a four-iteration launch and a
# tall pair; fp16s K = 4: one four-iteration launch
@pytest.mark.parametrize("prec,sub", [("fp32", (3, 3, 0.0)), ("fp32", (5, 5, 0.0)), ("fp32", (6, 6, 0.0)),
                                      ("fp64", (4, 4, 0.0)), ("fp16s", (2, 2, 0.0)), ("fp16s", (4, 4, 0.0))])
def test_every_configuration_gives_the_same_state(prec, sub):
    print("case tuning configs", prec, sub, flush=True)
    cfgs, inits = batch(sub)
    ref = {}
    for config in range(16):
        sim = binding.Sim(cfgs, inits, precision=prec)
        sim.set_tuning(config)
        assert sim.get_tuning() == config
        sim.step(7)
        got = pops(sim, 3)
        # the potential form: single launches, or pairs on one of the two tile
        # shapes
        if config & binding.TUNE_SINGLE_POTENTIAL:
            form = "single"
        elif config & binding.TUNE_TALL_TILES:
            form = "tall"
        else:
            form = "pairs"
        if form not in ref:
            ref[form] = got
        else:
            assert all(torch.equal(a, b) for a, b in zip(got, ref[form])), config
    for form in ref:
        for a, b in zip(ref[form], ref["pairs"]):
            err = float(torch.linalg.norm(a - b)) / max(float(torch.linalg.norm(b)), 1e-300)
            assert err <= ROUNDING[prec], (form, err)


def test_d3q15_orders_give_the_same_state():
    print("case tuning d3q15", flush=True)
    p, init = inputs.parity_case3d(12, 10, 8, seed=3)
    out = []
    for config in (0, binding.TUNE_LINEAR_ORDER, binding.TUNE_COLLIDE_PER_FAMILY, 5):
        sim = binding.Sim(p, init, precision="fp32")
        sim.set_tuning(config)
        sim.step(5)
        out.append(pops(sim, 1))
    for other in out[1:]:
        assert all(torch.equal(a, b) for a, b in zip(other, out[0]))


def test_tune_restores_state_and_keeps_graph():
    """After tune() the handle (with a captured graph) continues exactly like
    a handle that never tuned, set to the same configuration."""
    print("case tune restore", flush=True)
    cfgs, inits = batch((4, 4, 0.0))
    stream = torch.cuda.Stream()
    a = binding.Sim(cfgs, inits, precision="fp32", stream=stream)
    b = binding.Sim(cfgs, inits, precision="fp32", stream=stream)
    a.step(3)
    b.step(3)
    a.graph(4)
    before = pops(a, 3)
    res = a.autotune(steps=6)
    assert not res["cached"] and res["config"] in range(16)
    # every configuration is timed except tall tiles with single launches
    timed = [c for c in range(16) if res["ms_per_step"][c] > 0]
    assert timed == [c for c in range(16) if not (c & 8 and c & 2)], res
    assert a.get_tuning() == res["config"]
    assert all(torch.equal(x, y) for x, y in zip(pops(a, 3), before))
    b.set_tuning(res["config"])  # the potential forms agree to rounding only
    a.step(9)
    b.step(9)
    assert all(torch.equal(x, y) for x, y in zip(pops(a, 3), pops(b, 3)))


def test_autotune_cache(tmp_path):
    print("case tune cache", flush=True)
    p, init = inputs.parity_case(64, 48, seed=2, sub=(2, 2, 0.0))
    cache = str(tmp_path / "tune.json")
    s1 = binding.Sim(p, init, precision="fp32")
    r1 = s1.autotune(steps=4, cache=cache)
    assert not r1["cached"]
    table = json.load(open(cache))
    assert s1.tuning_key() in table
    s2 = binding.Sim(p, init, precision="fp32")
    r2 = s2.autotune(steps=4, cache=cache)
    assert r2["cached"] and r2["config"] == r1["config"] and s2.get_tuning() == r1["config"]
    # adaptive sub-iterations: the single-launch and tile-shape bits are not
    # timed; FP64: the load-schedule bit is not either
    q = dict(p, sub_min=1, sub_max=6, sub_tol=1e-6)
    r3 = binding.Sim(q, init, precision="fp32").autotune(steps=4)
    assert [c for c in range(16) if r3["ms_per_step"][c] > 0] == [0, 1, 4, 5] and r3["config"] in (0, 1, 4, 5)
    r4 = binding.Sim(p, init, precision="fp64").autotune(steps=4)
    assert [c for c in range(16) if r4["ms_per_step"][c] > 0] == [0, 1, 2, 3, 8, 9]
