"""Device-side failure paths on the GPU: non-finite values latch the plan's
status word (Krylov, dense in every precision, whole-grid and single-box
global methods), the one-call global action reports them, and a plan whose
Krylov dimension and sub-step limits cannot meet the tolerance is refused.
Every case is an ordinary kernel exit: the NaN travels through the
arithmetic and is caught where the result is written."""
import numpy as np
import pytest

import lem_inputs as L

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1505_02248_amd as lem  # noqa: E402

NONFINITE, NOT_CONVERGED = 8, 4


def poisoned(x, at=(5, 0)):
    y = np.array(x, dtype=np.float64, copy=True)
    y[at] = np.nan
    return y


def step_status(plan, x0, steps=1):
    xin = torch.from_numpy(np.ascontiguousarray(x0)).to("cuda")
    xout = torch.empty_like(xin)
    plan.step(xin, xout, steps)
    torch.cuda.synchronize()
    return plan.query()["device_status"]


def test_krylov_nonfinite_latched():
    p = L.workload_1d()
    o = lem.Operator.from_problem(p)
    plan = lem.Plan(o, p.dt, method="krylov", core=64, halo=16, krylov_tol=1e-12)
    assert step_status(plan, p.states) == 0
    bad = lem.Plan(o, p.dt, method="krylov", core=64, halo=16, krylov_tol=1e-12)
    assert step_status(bad, poisoned(p.states), 2) == NONFINITE


@pytest.mark.parametrize("prec,ns", [("fp64", 64), ("fp32", 64), ("bf16x3", 64), ("bf16x2", 64),
                                     ("fp64", 3), ("fp32", 3)])
def test_dense_nonfinite_latched(prec, ns):
    p = L.workload_2d_ensemble(n=64, n_states=ns)
    o = lem.Operator.from_problem(p)
    kw = dict(method="dense", precision=prec, core=16, halo=4, n_states=ns)
    assert step_status(lem.Plan(o, p.dt, **kw), p.states) == 0
    assert step_status(lem.Plan(o, p.dt, **kw), poisoned(p.states, (700, ns - 1))) == NONFINITE


@pytest.mark.parametrize("n", [32, 128])  # one periodic box / whole-grid kernels
def test_global_nonfinite_latched(n):
    p = L.workload_2d_ensemble(n=n, n_states=2)
    o = lem.Operator.from_problem(p)
    plan = lem.Plan(o, p.dt, method="global", n_states=2, krylov_tol=1e-12)
    assert step_status(plan, p.states) == 0
    plan = lem.Plan(o, p.dt, method="global", n_states=2, krylov_tol=1e-12)
    assert step_status(plan, poisoned(p.states)) == NONFINITE


def test_global_expmv_reports_nonfinite():
    p = L.workload_2d_ensemble(n=128, n_states=2)
    x = torch.from_numpy(poisoned(p.states)).to("cuda")
    y = torch.empty_like(x)
    with pytest.raises(lem.LemError) as e:
        lem.global_expmv(lem.Operator.from_problem(p), p.dt, x, y, n_states=2, tol=1e-12)
    assert e.value.status == NONFINITE


@pytest.mark.parametrize("method", ["krylov", "global"])
def test_unreachable_tolerance_is_not_converged(method):
    # m <= 2 with a single sub-step cannot reach 1e-15 on this operator
    p = L.workload_2d_ensemble(n=64, n_states=1)
    kw = dict(core=16, halo=4) if method == "krylov" else {}
    with pytest.raises(lem.LemError) as e:
        lem.Plan(lem.Operator.from_problem(p), p.dt * 8, method=method, krylov_m_max=2,
                 max_substeps=1, krylov_tol=1e-15, **kw)
    assert e.value.status == NOT_CONVERGED
