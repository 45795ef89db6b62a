"""Serving scheduler on the host (dry-run servers: no device memory, no
kernels): admission order, memory budget, slot reuse, limits, errors."""
import numpy as np
import pytest

import lem_inputs as L
import paper_1505_02248_amd as lem


def op2d(n, nu=1e-3):
    return lem.Operator(2, n, 1.0 / n, (1.0, 0.5), nu)


def drain(s, limit=10000):
    for _ in range(limit):
        a, q = s.tick()
        if a == 0 and q == 0:
            return
    raise AssertionError("server did not drain")


def test_fifo_admission_and_max_active():
    s = lem.Server(hbm_budget=1 << 30, max_active=2, dry_run=True)
    ids = [s.submit(op2d(64), 1 / 64, k + 1, np.full(64 * 64, float(k))) for k in range(5)]
    a, q = s.tick()  # admits ids 0, 1; advances them one step -> id0 done
    assert (a, q) == (1, 3)
    assert s.poll(ids[0]) == "done" and s.poll(ids[1]) == "active"
    assert [s.poll(i) for i in ids[2:]] == ["queued"] * 3
    drain(s)
    for k, i in enumerate(ids):
        assert s.poll(i) == "done"
        info = s.request_info(i)
        assert info["steps_done"] == info["n_steps"] == k + 1
        assert info["t_submit_ms"] <= info["t_admit_ms"] <= info["t_done_ms"]
        assert np.array_equal(s.fetch(i), np.full(64 * 64, float(k)))  # dry run: unchanged
    with pytest.raises(lem.LemError) as e:
        s.poll(ids[0])
    assert e.value.status == 7


def test_budget_blocks_queue_head_until_memory_frees():
    per = 2 * 128 * 128 * 8  # two state buffers of a 128^2 request
    s = lem.Server(hbm_budget=per * 2 + 1024, max_active=8, dry_run=True)
    ids = [s.submit(op2d(128), 1 / 128, 3, np.zeros(128 * 128)) for _ in range(3)]
    a, q = s.tick()
    assert (a, q) == (2, 1)  # the third does not fit yet
    assert s.query()["bytes_in_use"] <= s.query()["bytes_budget"]
    s.tick(); s.tick()       # the first two finish on tick 3 and free their memory
    a, q = s.tick()
    assert s.poll(ids[2]) == "active" and q == 0
    drain(s)
    assert s.query()["bytes_in_use"] == 0 and s.query()["n_done"] == 3


def test_oversized_request_rejected_and_invalid_inputs():
    s = lem.Server(hbm_budget=1 << 20, max_active=4, dry_run=True)
    with pytest.raises(lem.LemError) as e:
        s.submit(op2d(512), 1 / 512, 5, np.zeros(512 * 512))  # 4 MiB of state > 1 MiB
    assert e.value.status == 5
    with pytest.raises(lem.LemError) as e:
        s.submit(op2d(64), -1.0, 5, np.zeros(64 * 64))
    assert e.value.status == 1
    with pytest.raises(lem.LemError) as e:
        s.submit(op2d(64), 1 / 64, 0, np.zeros(64 * 64))
    assert e.value.status == 1
    rid = s.submit(op2d(64), 1 / 64, 2, np.zeros(64 * 64))
    with pytest.raises(lem.LemError) as e:
        s.fetch(rid)  # not finished
    assert e.value.status == 1


def test_partition_choice_and_global_fallback():
    # constant coefficients: Kronecker-factored blocks whenever a core fits
    # (box side below n and at most 128); variable coefficients: Krylov boxes
    # within the overhead cap; neither: the global method
    s = lem.Server(hbm_budget=1 << 30, max_active=8, dry_run=True, max_overhead=4.0)
    small = s.submit(op2d(256, nu=1e-3), 2 / 256, 2, np.zeros(256 * 256))
    wide = s.submit(op2d(64, nu=1e-2), 4 / 64, 2, np.zeros(64 * 64))
    f = L.lognormal_field_2d(256, 16, median=2e-4)
    var = s.submit(lem.Operator(2, 256, 1 / 256, (1.0, 0.5), 0.0, nu_field=f), 1 / 256, 2,
                   np.zeros(256 * 256))
    f = L.lognormal_field_2d(64, 17, median=3e-2)
    varwide = s.submit(lem.Operator(2, 64, 1 / 64, (1.0, 0.5), 0.0, nu_field=f), 4 / 64, 2,
                       np.zeros(64 * 64))
    s.tick()
    i1, i2 = s.request_info(small), s.request_info(wide)
    i3, i4 = s.request_info(var), s.request_info(varwide)
    assert i1["method"] == "kronecker" and i1["core"] in (16, 32, 64) and i1["halo"] >= 4
    assert i1["core"] + 2 * i1["halo"] < 256
    assert i2["method"] == "kronecker" and i2["core"] + 2 * i2["halo"] < 64
    assert i3["method"] == "krylov" and i3["core"] in (16, 32, 64)
    assert (i3["core"] + 2 * i3["halo"]) ** 2 <= 4.0 * i3["core"] ** 2
    assert i4["method"] == "global" and i4["core"] == 0


def test_buffer_cap_decides_between_kronecker_and_global():
    # a stiff 512^2 request (nu dt / dx^2 about 20) has a decay-bound buffer
    # of about 45 points: a Kronecker box under the default cap of 56, the
    # global method under a cap of 32
    o = op2d(512, nu=1e-2)
    for cap, method in ((56, "kronecker"), (32, "global")):
        s = lem.Server(hbm_budget=1 << 30, max_active=8, dry_run=True, halo_max=cap)
        rid = s.submit(o, 4 / 512, 1, np.zeros(512 * 512))
        s.tick()
        info = s.request_info(rid)
        assert info["method"] == method, (cap, info)
        if method == "kronecker":
            assert 32 < info["halo"] <= cap
            assert info["core"] + 2 * info["halo"] <= 128
