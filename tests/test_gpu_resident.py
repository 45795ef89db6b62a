"""GPU parity of the resident multi-step path: 1D dense FP64 plans with one
stored block, whose lem_step runs every step of a call in one launch (states
in LDS, stored-block rows in registers), against the CPU oracle's LEM steps
(section 3, update (5)), plus its limits and failure latch."""
import numpy as np
import pytest

import lem_inputs as L
from oracle import lem as olem
from oracle import operator as op
from oracle import partition as P
from oracle.metrics import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1505_02248_amd as lem  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def run(plan, x0, steps):
    xin = dev(x0)
    xout = torch.empty_like(xin)
    plan.step(xin, xout, steps)
    torch.cuda.synchronize()
    return xout.cpu().numpy()


def oracle(p, core, h, x0, steps, dtg=None):
    boxes = P.uniform_boxes(1, p.n, core, h)
    return olem.run(op.sparse(op.from_problem(p)), boxes, 1, p.n, x0, steps, dtg=dtg)


def members(p, ns, seed):
    # scaled and shifted copies of the workload's state
    rng = np.random.default_rng(seed)
    u = p.states[:, 0]
    return np.stack([a * u + 0.1 * np.roll(u, 7 * k)
                     for k, a in enumerate(rng.uniform(0.5, 1.5, size=ns))], axis=1)


def test_c0_workload_100_steps_in_one_launch():
    # 1024 points, 16 cores of 64, decay-bound buffer (25 points)
    p = L.workload_1d()
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", core=64, halo=0,
                    halo_min=4, halo_max=64)
    q = plan.query()
    assert q["resident_steps"] == 1
    h = q["halo_max"]
    got = run(plan, p.states, 100)
    assert rel_l2(got, oracle(p, 64, h, p.states, 100)) <= 1e-12
    assert plan.query()["device_status"] == 0


@pytest.mark.parametrize("ns", [3, 37])
def test_ragged_cores_and_member_groups(ns):
    # 40-point cores (not a multiple of 16), 25 blocks: 2 members per
    # workgroup, the last group partial at 37 members
    p = L.workload_1d(n=1000)
    x0 = members(p, ns, ns)
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", core=40, halo=10,
                    n_states=ns)
    assert plan.query()["resident_steps"] == 1
    got = run(plan, x0, 7)
    assert rel_l2(got, oracle(p, 40, 10, x0, 7)) <= 1e-12


def test_forced_steps():
    p = L.workload_1d(n=256)
    rng = np.random.default_rng(5)
    g = (np.cos(2 * np.pi * 3 * np.arange(p.n) / p.n + rng.uniform(0, 6)) + 0.5)[:, None]
    o = lem.Operator.from_problem(p)
    plan = lem.Plan(lem.Operator(o.ndim, o.n, o.dx, o.vel, o.nu, o.nu_field, forcing=g), p.dt,
                    method="dense", core=64, halo=16)
    assert plan.query()["resident_steps"] == 1
    got = run(plan, p.states, 20)
    want = oracle(p, 64, 16, p.states[:, 0], 20, dtg=p.dt * g[:, 0])
    assert rel_l2(got[:, 0], want) <= 1e-12


def test_one_call_equals_repeated_single_steps():
    p = L.workload_1d()
    x0 = members(p, 5, 2)
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", core=64, halo=20,
                    n_states=5)
    a = run(plan, x0, 9)
    b = x0
    for _ in range(9):
        b = run(plan, b, 1)
    assert np.array_equal(a, b)


def test_nonfinite_state_is_latched():
    p = L.workload_1d()
    x0 = p.states.copy()
    x0[17] = np.nan
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", core=64, halo=20)
    assert plan.query()["resident_steps"] == 1
    run(plan, x0, 4)
    assert plan.query()["device_status"] == 8


def test_plans_that_do_not_fit_keep_the_per_step_launches():
    # 2D, FP32, 128-point cores with a 4-point buffer (box 136 > 128), and a
    # grid whose two states exceed LDS
    p2 = L.workload_2d_ensemble(n=64, n_states=4)
    assert lem.Plan(lem.Operator.from_problem(p2), p2.dt, method="dense", core=16, halo=4,
                    n_states=4).query()["resident_steps"] == 0
    p = L.workload_1d()
    o = lem.Operator.from_problem(p)
    assert lem.Plan(o, p.dt, method="dense", precision="fp32", core=64,
                    halo=16).query()["resident_steps"] == 0
    assert lem.Plan(o, p.dt, method="dense", core=128, halo=4).query()["resident_steps"] == 0
    pb = L.workload_1d(n=16384, cfl=1.0)
    plan = lem.Plan(lem.Operator.from_problem(pb), pb.dt, method="dense", core=64, halo=16)
    assert plan.query()["resident_steps"] == 0
    got = run(plan, pb.states, 2)
    assert rel_l2(got, oracle(pb, 64, 16, pb.states, 2)) <= 1e-12
