"""GPU parity of the dense apply in every launch shape and at the largest
configured workload, against the CPU FP64 oracle (plain LEM definition with
exact local exponentials, sections 3 and 4).

* 256^2 x 64 states, 16^2 cores: each of the eight FP64/FP32 tile shapes at
  the configured buffer (h = 4) and at the decay-bound buffer the benchmark
  uses (h = 14); FP64 within 1e-12, FP32 within 1e-5 (relative l2).
* 512^2 x 128 states, 32^2 cores at h = 8 (configured) and h = 15 (decay
  bound, the benchmarked case), with the launch shape the autotuner picks as
  the benchmark does: FP64 within 1e-12, FP32 and split bf16 (six products)
  within 1e-6; every split-bf16 shape (the 128-state one included) at h = 15.
* Small ensembles (3 states) in FP32 (the eight-lane kernel)."""
import numpy as np
import pytest

import lem_inputs as L
from oracle import lem as olem
from oracle import operator as op
from oracle import partition as P
from oracle.metrics import rel_l2
from oracle_cache import one_step as oracle_one_step
from oracle_cache import problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1505_02248_amd as lem  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def run(plan, x0, steps=1):
    xin = dev(x0)
    xout = torch.empty_like(xin)
    plan.step(xin, xout, steps)
    torch.cuda.synchronize()
    return xout.cpu().numpy()


def c1_problem():
    return problem("c1")  # 256^2, 64 states


def c3_problem():
    return problem("c3")  # 512^2, 128 states


def check_boxes(plan, n, core, h):
    boxes = plan.maps()[0]
    want = np.array([[b.ox, b.oy, b.cx, b.cy, b.h] for b in P.uniform_boxes(2, n, core, h)],
                    dtype=np.int32)
    assert np.array_equal(boxes, want)


@pytest.mark.parametrize("tile", range(8))
@pytest.mark.parametrize("h", [4, 14])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_c1_every_tile_shape(prec, tol, h, tile):
    p = c1_problem()
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", precision=prec,
                    core=16, halo=h, n_states=64, tile=tile)
    assert plan.query()["tile_config"] == tile
    check_boxes(plan, p.n, 16, h)
    got = run(plan, p.states)
    assert rel_l2(got, oracle_one_step("c1", 16, h)) <= tol
    assert plan.query()["device_status"] == 0


def test_tile_that_does_not_fit_is_refused():
    # 40-point 1D cores pad to 64 rows: 64-row waves fit, and the split-bf16
    # shapes only exist as 0 and 1
    p = L.workload_1d(n=1000)
    o = lem.Operator.from_problem(p)
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, p.dt, method="dense", precision="bf16x3", core=40, halo=10, n_states=64,
                 tile=5)
    assert e.value.status == 6
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, p.dt, method="dense", core=40, halo=10, n_states=64, tile=8)
    assert e.value.status == 1
    # 128 states per workgroup at 64 states
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, p.dt, method="dense", precision="bf16x2", core=40, halo=10, n_states=64,
                 tile=4)
    assert e.value.status == 6


@pytest.mark.parametrize("h", [8, 15])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16x3", 1e-6)])
def test_c3_full_size(prec, tol, h):
    p = c3_problem()
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", precision=prec,
                    core=32, halo=h, n_states=128, autotune=True)
    check_boxes(plan, p.n, 32, h)
    got = run(plan, p.states)
    err = rel_l2(got, oracle_one_step("c3", 32, h))
    print(f"c3 h={h} {prec} tile={plan.query()['tile_config']}: rel l2 {err:.2e}")
    assert err <= tol
    assert plan.query()["device_status"] == 0


@pytest.mark.parametrize("tile", range(5))
def test_c3_every_split_bf16_shape(tile):
    # rows per wave 32 / 64, four / eight waves per workgroup, 64 states per
    # workgroup (0-3) or 128 (4), six products
    p = c3_problem()
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", precision="bf16x3",
                    core=32, halo=15, n_states=128, tile=tile)
    assert plan.query()["tile_config"] == tile
    got = run(plan, p.states)
    assert rel_l2(got, oracle_one_step("c3", 32, 15)) <= 1e-6


@pytest.mark.parametrize("tile", range(4))
def test_c1_every_split_bf16_shape_three_products(tile):
    # (the 128-state shape needs n_states % 128 == 0: refused at 64 states,
    # test_tile_that_does_not_fit_is_refused)
    p = c1_problem()
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", precision="bf16x2",
                    core=16, halo=14, n_states=64, tile=tile)
    got = run(plan, p.states)
    assert rel_l2(got, oracle_one_step("c1", 16, 14)) <= 2e-5


def test_fp32_small_ensemble():
    # 3 states: the eight-lane FP32 kernel on 40-point cores with 10-point buffers
    n, ns = 1000, 3
    p = L.workload_1d(n=n)
    x0 = np.repeat(p.states, ns, axis=1) * (1.0 + np.arange(ns))[None, :]
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", precision="fp32",
                    core=40, halo=10, n_states=ns)
    got = run(plan, x0, 3)
    boxes = P.uniform_boxes(1, n, 40, 10)
    want = olem.run(op.sparse(op.from_problem(p)), boxes, 1, n, x0, 3)
    assert rel_l2(got, want) <= 1e-5
