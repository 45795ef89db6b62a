"""Oracle results shared by several GPU test modules within one pytest process
(the 512^2 x 128-state LEM steps take tens of seconds on the CPU)."""
import functools

import lem_inputs as L
from oracle import lem as olem
from oracle import operator as op
from oracle import partition as P


@functools.lru_cache(maxsize=None)
def problem(which):
    return L.workload_2d_ensemble() if which == "c1" else L.workload_2d_mixed()


@functools.lru_cache(maxsize=None)
def one_step(which, core, h):
    """The oracle's LEM step (exact local exponentials, uniform cores) of the
    256^2 x 64 ("c1") or 512^2 x 128 ("c3") workload."""
    p = problem(which)
    boxes = P.uniform_boxes(2, p.n, core, h)
    return olem.run(op.sparse(op.from_problem(p)), boxes, 2, p.n, p.states, 1)
