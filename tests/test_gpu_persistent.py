"""The grid-resident batch step (lbm_ehd_step_persistent): one cooperative
launch runs whole steps of every instance, with a grid-wide barrier between
the stages.  Its arithmetic is that of the separate launches, so after n
steps its state equals, bitwise, that of lbm_ehd_step in a tall-tile launch
configuration; the checks cover uneven instances (walls and periodic), FP32
and FP16S storage, one and two four-sub-iteration passes per step, an odd
step count, more steps than one launch takes (256), mixing with ordinary
steps, instances smaller than one potential tile, the cases it refuses,
and a barrier wait that runs out (forced from the host with a bound of one
poll)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2608_05787_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def batch(K, sizes=((70, 40, True), (33, 17, False), (128, 96, True))):
    cases = [inputs.parity_case(nx, ny, seed=nx, walls=w, sub=(K, K, 0.0)) for nx, ny, w in sizes]
    return [c[0] for c in cases], [c[1] for c in cases]


def state(sim, n_inst):
    return [sim.populations(fam, inst=i).clone() for i in range(n_inst) for fam in "fglh"]


def assert_same(a, b, n_inst):
    for x, y in zip(state(a, n_inst), state(b, n_inst)):
        assert torch.equal(x, y)
    for i in range(n_inst):
        da, db = a.diagnostics(i), b.diagnostics(i)
        for k in da:  # equal, or nan on both sides (a contour with no crossing)
            assert da[k] == db[k] or (np.isnan(da[k]) and np.isnan(db[k])), (i, k, da[k], db[k])
    assert a.scalars() == b.scalars()


@pytest.mark.parametrize("prec,K,config,steps", [("fp32", 4, 12, 7), ("fp32", 4, 8, 7), ("fp32", 8, 13, 5),
                                                 ("fp16s", 4, 12, 7)])
def test_persistent_equals_step_bitwise(prec, K, config, steps):
    print("case persistent", prec, K, config, steps, flush=True)
    cfgs, inits = batch(K)
    a = binding.Sim(cfgs, inits, precision=prec)
    a.set_tuning(config)
    a.step(steps)
    b = binding.Sim(cfgs, inits, precision=prec)
    b.set_tuning(config)
    b.step_persistent(steps)
    assert_same(a, b, 3)


def test_persistent_with_instances_smaller_than_a_tile():
    """Instances of 2 x 2 to 5 x 3 nodes (walls and periodic) beside a larger
    one: every stage's tables hold blocks and tiles that are mostly outside
    the grid, and the tall tile's ring wraps several times.  Two instances
    run the restoring flux of the order-parameter sum."""
    print("case persistent tiny", flush=True)
    cfgs, inits = batch(4, sizes=((2, 2, False), (3, 2, True), (5, 3, False), (2, 7, True), (70, 40, True)))
    cfgs[2]["sum_relax"] = cfgs[4]["sum_relax"] = 1
    a = binding.Sim(cfgs, inits, precision="fp32")
    a.set_tuning(12)
    a.step(6)
    b = binding.Sim(cfgs, inits, precision="fp32")
    b.set_tuning(12)
    b.step_persistent(6)
    assert_same(a, b, 5)


def test_persistent_over_several_launches_and_mixed_with_steps():
    """300 steps (two launches) on two small instances, then ordinary steps
    and one more persistent block: the same state as ordinary steps all
    along."""
    print("case persistent long", flush=True)
    cfgs, inits = batch(4, sizes=((24, 20, True), (40, 16, False)))
    a = binding.Sim(cfgs, inits, precision="fp32")
    a.set_tuning(12)
    b = binding.Sim(cfgs, inits, precision="fp32")
    b.set_tuning(12)
    a.step(300)
    b.step_persistent(300)
    assert_same(a, b, 2)
    a.step(9)
    b.step(3)
    b.step_persistent(5)
    b.step(1)
    assert_same(a, b, 2)


def test_persistent_limits():
    """Refused, before any launch: D3Q15, FP64, K not a multiple of 4,
    residual-controlled sub-iterations, the two-ion charge model."""
    print("case persistent limits", flush=True)
    cfgs, inits = batch(2, sizes=((24, 20, True),))
    refused = [binding.Sim(cfgs, inits, precision="fp32"),
               binding.Sim([dict(cfgs[0], sub_min=6, sub_max=6)], inits, precision="fp32"),
               binding.Sim([dict(cfgs[0], sub_min=4, sub_max=4)], inits, precision="fp64"),
               binding.Sim([dict(cfgs[0], sub_min=1, sub_max=8, sub_tol=1e-6)], inits, precision="fp32")]
    p3, i3 = inputs.parity_case3d(12, 10, 8, seed=3)
    refused.append(binding.Sim(dict(p3, sub_min=4, sub_max=4), i3, precision="fp32"))
    pn, i_n, _ = inputs.np_eof_channel()
    refused.append(binding.Sim(dict(pn, sub_min=4, sub_max=4), i_n, precision="fp32"))
    for sim in refused:
        before = state(sim, 1)
        with pytest.raises(binding.LbmEhdError):
            sim.step_persistent(2)
        assert all(torch.equal(x, y) for x, y in zip(state(sim, 1), before))
        assert sim.scalars()["steps"] == 0
    ok = binding.Sim([dict(cfgs[0], sub_min=4, sub_max=4)], inits, precision="fp32")
    ok.step_persistent(0)
    assert ok.scalars()["steps"] == 0
    assert np.isfinite(ok.diagnostics()["max_sum_dev"])


def test_barrier_wait_that_runs_out_ends_the_launch():
    """The failure path, forced from the host: with one poll per barrier wait
    the first block to wait gives up before the others arrive, every block
    leaves the launch, and the call reports it (the state is undefined).
    The device is usable afterwards: fresh handles step as before."""
    print("case persistent barrier bound", flush=True)
    cfgs, inits = batch(4, sizes=((128, 96, True), (70, 40, False)))
    a = binding.Sim(cfgs, inits, precision="fp32")
    a.set_tuning(12)
    a.set_persistent_polls(1)
    with pytest.raises(binding.LbmEhdError):
        a.step_persistent(4)
    del a
    torch.cuda.synchronize()
    b = binding.Sim(cfgs, inits, precision="fp32")
    b.set_tuning(12)
    b.step_persistent(4)
    c = binding.Sim(cfgs, inits, precision="fp32")
    c.set_tuning(12)
    c.step(4)
    assert_same(b, c, 2)


def test_stage_times_account_for_the_step():
    """The per-stage clock sums of a timed persistent call: positive, and
    together the call's time per step (host wall clock, which also holds
    the launches' set-up)."""
    import time
    print("case persistent stage times", flush=True)
    cfgs, inits = batch(4)
    sim = binding.Sim(cfgs, inits, precision="fp32")
    sim.set_tuning(12)
    sim.step_persistent(20)
    with pytest.raises(binding.LbmEhdError):
        sim.persistent_stage_times()  # no timed persistent steps yet
    sim.set_persistent_timing(True)
    sim.step_persistent(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step_persistent(200)
    wall_us = (time.perf_counter() - t0) * 1e6 / 200
    st = sim.persistent_stage_times()
    print("stage us per step", st, "wall us per step", wall_us, flush=True)
    assert all(v > 0 for v in st.values())
    assert 0.5 * wall_us < sum(st.values()) <= 1.1 * wall_us
