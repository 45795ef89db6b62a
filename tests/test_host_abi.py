"""Host-side tests of the C-ABI library (no GPU needed): the shared library
loads and exports every function include/lem.h declares, and dry-run plans
(partition, buffer widths, index maps -- all host logic) agree with the
oracle bit for bit."""
import ctypes

import numpy as np
import pytest

import lem_inputs as L
import paper_1505_02248_amd as lem
from oracle import halo as H
from oracle import operator as op
from oracle import partition as P


def test_library_exports_every_declared_symbol():
    lib = lem.load()
    names = lem.declared_functions()
    assert {"lem_plan", "lem_step", "lem_global_expmv", "lem_plan_destroy"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def _oracle_maps(boxes, ndim, n):
    bx = [P.Box(*map(int, b)) for b in boxes]
    P.check_tiling(bx, ndim, n)
    G, _, S, _ = P.all_maps(bx, ndim, n)
    return G, S


@pytest.mark.parametrize("ndim,n,c,h", [(1, 1024, 64, 16), (1, 1024, 64, 20), (2, 256, 16, 4),
                                        (2, 512, 32, 8), (2, 64, 16, 7)])
def test_dry_plan_maps_bit_exact(ndim, n, c, h):
    o = lem.Operator(ndim, n, 1.0 / n, (1.0, 0.5), 1e-3)
    p = lem.Plan(o, 2.0 / n, method="krylov", core=c, halo=h, dry_run=True)
    boxes, gather, scatter = p.maps()
    want = P.uniform_boxes(ndim, n, c, h)
    assert np.array_equal(boxes, np.array(want, dtype=np.int32))
    G, S = _oracle_maps(boxes, ndim, n)
    assert np.array_equal(gather, G.astype(np.int32))
    assert np.array_equal(scatter, S.astype(np.int32))


@pytest.mark.parametrize("work,c,tol", [("1d", 64, 1e-8), ("1d", 64, 1e-6), ("2d", 16, 1e-8),
                                        ("2d", 32, 1e-6)])
def test_decay_bound_halo_matches_oracle(work, c, tol):
    p = L.workload_1d() if work == "1d" else L.workload_2d_ensemble(n=256, n_states=1)
    W = op.from_problem(p)
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, core=c, halo=0, halo_min=4,
                    halo_max=64, halo_tol=tol, dry_run=True)
    boxes, _, _ = plan.maps()
    h = int(boxes[0, 4])
    co = H.block_coefficients(W, P.Box(*map(int, boxes[0])), p.ndim)
    assert H.accepts(co, p.ndim, tol, 4, h, H.growth_factor(W))


def test_uneven_variable_partition_tiles_and_halos():
    p = L.workload_2d_variable(n=256)
    W = op.from_problem(p)
    G = H.growth_factor(W)
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, core=0, halo=0, halo_min=4,
                    halo_max=16, halo_tol=1e-8, dry_run=True)
    boxes, gather, scatter = plan.maps()
    Go, So = _oracle_maps(boxes, 2, p.n)
    assert np.array_equal(gather, Go.astype(np.int32))
    assert np.array_equal(scatter, So.astype(np.int32))
    assert set(np.unique(boxes[:, 2])) <= {16, 32, 64}
    info = plan.query()
    clamped = 0
    for b in boxes:
        box = P.Box(*map(int, b))
        co = H.block_coefficients(W, box, 2)
        if box.h == 16 and H.eps(co, 16, 2, G) > 1e-8:
            clamped += 1
            continue
        assert H.accepts(co, 2, 1e-8, 4, box.h, G), box
    assert clamped == info["halo_clamped"]


def test_invalid_arguments_are_reported():
    o = lem.Operator(2, 64, 1 / 64, (1.0, 0.5), 1e-3)
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, 2 / 64, core=24, halo=4, dry_run=True)  # core does not divide n
    assert e.value.status == 1
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, 2 / 64, core=32, halo=16, dry_run=True)  # 32 + 32 >= 64
    assert e.value.status == 1
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, -1.0, core=16, halo=4, dry_run=True)
    assert e.value.status == 1
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, 2 / 64, method="krylov", precision="fp32", core=16, dry_run=True)
    assert e.value.status == 6
    with pytest.raises(lem.LemError) as e:
        lem.Plan(lem.Operator(1, 64, 1 / 64, (1.0, 0), 1e-3), 2 / 64, core=0, dry_run=True,
                 method="dense")
    assert e.value.status == 6  # uneven cores are a 2D Krylov feature
    with pytest.raises(lem.LemError) as e:
        lem.Plan(o, 2 / 64, core=16, halo=4, krylov_m_max=60, dry_run=True)
    assert e.value.status == 1
    for tile in (-2, 8):  # apply launch shapes are -1 (default) or 0..7
        with pytest.raises(lem.LemError) as e:
            lem.Plan(o, 2 / 64, method="dense", core=16, halo=4, n_states=64, tile=tile,
                     dry_run=True)
        assert e.value.status == 1
    # Krylov boxes hold at most 9216 points, one fewer with a forcing (the
    # augmented coordinate), and dimensions up to 40; the checks precede any
    # device work
    big = lem.Operator(2, 256, 1 / 256, (1.0, 0.5), 1e-3)
    lem.Plan(big, 2 / 256, method="krylov", core=64, halo=16, krylov_m_max=40, dry_run=True)
    with pytest.raises(lem.LemError) as e:
        lem.Plan(big, 2 / 256, method="krylov", core=64, halo=17, dry_run=True)
    assert e.value.status == 6 and "9216" in str(e.value)
    with pytest.raises(lem.LemError) as e:
        lem.Plan(big, 2 / 256, method="krylov", core=64, halo=8, krylov_m_max=41, dry_run=True)
    assert e.value.status == 1
    g = np.ones((256 * 256, 1))
    forced = lem.Operator(2, 256, 1 / 256, (1.0, 0.5), 1e-3, forcing=g)
    lem.Plan(forced, 2 / 256, method="krylov", core=64, halo=15, dry_run=True)
    with pytest.raises(lem.LemError) as e:
        lem.Plan(forced, 2 / 256, method="krylov", core=64, halo=16, dry_run=True)
    assert e.value.status == 6 and "9215" in str(e.value)


def test_dry_plan_cannot_step_and_reports_sizes():
    o = lem.Operator(1, 1024, 1 / 1024, (1.0, 0.0), 1e-3)
    p = lem.Plan(o, 4 / 1024, core=64, halo=16, dry_run=True)
    q = p.query()
    assert q["n_blocks"] == 16 and q["n_loc_total"] == 16 * 96 and q["n_loc_max"] == 96
    lib = lem.load()
    st = lib.lem_step(p._h, ctypes.c_void_p(8), ctypes.c_void_p(8 + 1 << 20), 1, None)
    assert st == 1
    p.close()
    assert lib.lem_plan_destroy(None) == 0


@pytest.mark.parametrize("height", [1.0, 0.25])
def test_vortex_faces_partition_and_halos_match_oracle(height):
    """Face velocities (and an anisotropic dy): the host planner's per-block
    decay-bound halos are accepted by the oracle's rule on the same weights."""
    p = L.workload_2d_vortex(n=128, n_states=1, courant=2.0)
    if height != 1.0:
        p.vel_faces = L.vortex_faces(p.n, height=height)
        p.dy = p.dx * height
    W = op.from_problem(p)
    G = H.growth_factor(W)
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, core=16, halo=0, halo_min=2,
                    halo_max=24, halo_tol=1e-8, dry_run=True)
    boxes, gather, scatter = plan.maps()
    Go, So = _oracle_maps(boxes, 2, p.n)
    assert np.array_equal(gather, Go.astype(np.int32))
    assert np.array_equal(scatter, So.astype(np.int32))
    info = plan.query()
    for b in boxes:
        box = P.Box(*map(int, b))
        co = H.block_coefficients(W, box, 2)
        if box.h == 24 and H.eps(co, 24, 2, G) > 1e-8:
            continue
        assert H.accepts(co, 2, 1e-8, 2, box.h, G), box
    assert info["halo_min"] < info["halo_max"]  # the vortex is slow near its centre


def test_face_velocity_errors():
    n = 16
    F = L.vortex_faces(n)
    with pytest.raises(lem.LemError):
        lem.Plan(lem.Operator(2, n, 1 / n, (1.0, 0.0), 1e-3, vel_faces=F), 1 / n, core=8, halo=2,
                 dry_run=True)  # vel must be zero with face velocities
    with pytest.raises(lem.LemError):
        lem.Plan(lem.Operator(2, n, 1 / n, (0.0, 0.0), 1e-3, vel_faces=F), 1 / n, method="dense",
                 core=0, halo=2, dry_run=True)  # stored blocks need a uniform core
    with pytest.raises(lem.LemError):
        lem.Plan(lem.Operator(2, n, 1 / n, (0.0, 0.0), 1e-3, vel_faces=F), 1 / n, method="dense",
                 precision="bf16x3", core=8, halo=2, n_states=64, dry_run=True)


def test_column_partition_maps_and_halos_match_oracle():
    # 64 rows: every column box stays within the 4096 points of a Krylov box
    p = L.workload_2d_columns(n=64, n_states=1)
    W = op.from_problem(p)
    G = H.growth_factor(W)
    plan = lem.Plan(lem.Operator.from_problem(p), p.dt, core=16, halo=0, halo_min=2,
                    halo_max=24, halo_tol=1e-8, columns=True, dry_run=True)
    boxes, gather, scatter = plan.maps()
    assert boxes.shape == (4, 5) and np.all(boxes[:, 3] == 64) and np.all(boxes[:, 1] == 0)
    Go, So = _oracle_maps(boxes, 2, p.n)
    assert np.array_equal(gather, Go.astype(np.int32))
    assert np.array_equal(scatter, So.astype(np.int32))
    for b in boxes:
        box = P.Box(*map(int, b))
        co = H.block_coefficients(W, box, 2)
        assert H.accepts(co, 2, 1e-8, 2, box.h, G, cut_y=False), box
    q = plan.query()
    assert q["n_loc_max"] == (16 + 2 * q["halo_max"]) * 64
    p128 = L.workload_2d_columns(n=128, n_states=1)
    with pytest.raises(lem.LemError) as e:  # column boxes above 4096 points are refused
        lem.Plan(lem.Operator.from_problem(p128), p128.dt, core=16, halo=10, columns=True,
                 dry_run=True)
    assert e.value.status == 6 and "4096" in str(e.value)
    with pytest.raises(lem.LemError):  # column-wise cores are a Krylov feature
        lem.Plan(lem.Operator.from_problem(p), p.dt, method="dense", core=16, halo=4,
                 columns=True, dry_run=True)


def test_static_global_expmv_refuses_oversize_before_device_work():
    # the allocation-free global action checks its work space against the
    # 64 MiB static scratch before touching the device (no GPU needed here)
    lib = lem.load()
    o = lem.Operator(2, 1024, 1 / 1024, (1.0, 0.5), 1e-3)._c()
    st = lib.lem_global_expmv_static(ctypes.byref(o), 1e-3, None, None, 1, 1e-13, 40, None)
    assert st == 5 and "64 MiB" in lib.lem_last_error().decode()
    st = lib.lem_global_expmv_static(None, 1e-3, None, None, 1, 1e-13, 40, None)
    assert st == 1
