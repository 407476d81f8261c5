"""The continuous-batching request server on the GPU, through the C ABI.

Each result must be the same alone and in a mix: the batched stage kernel
computes every element with the same arithmetic whatever else shares the
launch, so the comparison is bitwise.  Results are also held to the FP64
oracle (1e-5 relative L2, the FP32 target) at the server's own dt and step
count, and to the single-solve path."""

import time

import numpy as np
import pytest

import oracle
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _req_mesh(s, seed, disk=None):
    m = inputs.tri_grid(s, seed=seed, permute=True)
    if disk is not None:
        m.eps = inputs.disk_inclusion_eps(m, disk[0], disk[1])
        m.mu = np.ones(m.K)
    return m


# a small mix of uneven size, order and material
MIX = [
    # (grid s, seed, order, mode, disk, t_final)
    (12, 11, 5, (1, 2), ((0.1, 0.2), 0.4), 0.30),
    (20, 12, 3, (2, 1), None, 0.40),
    (9, 13, 7, (1, 1), ((-0.3, 0.0), 0.3), 0.25),
    (30, 14, 5, (3, 2), ((0.0, 0.0), 0.5), 0.20),
    (6, 15, 3, (1, 3), None, 0.50),
    (16, 16, 7, (2, 2), None, 0.15),
]


def _submit(srv, case, keep=True):
    s, seed, N, mode, disk, tf = case
    return srv.submit(_req_mesh(s, seed, disk), N, mode=mode, t_final=tf, keep_fields=keep)


def test_alone_vs_mix_bitwise_and_vs_oracle():
    alone = {}
    with dgw.Server(max_chunk_steps=16) as srv:
        for i, case in enumerate(MIX):
            res, q = srv.wait(_submit(srv, case), fields=True)
            assert res["status"] == "DGW_OK"
            alone[i] = (res, q)
    with dgw.Server(max_chunk_steps=16) as srv:
        # reversed submission order changes tile placement and grouping
        tickets = {i: _submit(srv, MIX[i]) for i in reversed(range(len(MIX)))}
        mix = {i: srv.wait(t, fields=True) for i, t in tickets.items()}
    for i in range(len(MIX)):
        ra, qa = alone[i]
        rm, qm = mix[i]
        assert rm["status"] == "DGW_OK"
        assert rm["steps"] == ra["steps"] and rm["dt"] == ra["dt"]
        assert np.array_equal(qa, qm), f"request {i}: alone and mixed results differ"
        assert rm["energy"] == ra["energy"]
    # the mixed requests overlapped on the device
    spans = sorted((mix[i][0]["t_start"], mix[i][0]["t_finish"]) for i in mix)
    assert any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))
    # every result against the FP64 oracle at the server's dt and step count
    for i, (s, seed, N, mode, disk, tf) in enumerate(MIX):
        m = _req_mesh(s, seed, disk)
        d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, N, eps=m.eps, mu=m.mu)
        op = oracle.Maxwell2D(d, 1.0)
        res, q = mix[i]
        q0 = oracle.cavity_mode_2d(d.x, d.y, 0.0, *mode)
        want = op.run(q0, res["dt"], res["steps"])
        err = rel(q, want)
        print(f"request {i}: s={s} N={N} K={m.K} steps={res['steps']} vs oracle {err:.2e}")
        assert err < 1e-5
        assert abs(res["energy"] / op.energy(q) - 1) < 1e-12
        if disk is None:
            assert abs(res["rel_l2_mode"] / op.rel_l2(q, oracle.cavity_mode_2d(d.x, d.y, tf, *mode)) - 1) < 1e-9
        else:
            assert np.isnan(res["rel_l2_mode"])


def test_server_matches_single_solve_path():
    s, seed, N, mode, disk, tf = MIX[0]
    m = _req_mesh(s, seed, disk)
    with dgw.Server() as srv:
        res, q = srv.wait(srv.submit(m, N, mode=mode, t_final=tf, keep_fields=True), fields=True)
    # the server's batched launches run the fused-operand kernel (kernel 2)
    with dgw.Solver(m, N, kernel=2) as sol:
        sol.set_cavity_mode(*mode)
        sol.advance_steps(res["steps"], res["dt"])
        want = sol.get_fields()
    err = rel(q, want)
    print(f"server vs single-solve kernel: {err:.2e}, bitwise {np.array_equal(q, want)}")
    assert np.array_equal(q, want)


def test_admission_by_footprint():
    a = _req_mesh(24, 21)
    b = _req_mesh(24, 22)
    fa = dgw.footprint(a, 5)
    # a budget for one request at a time: the second waits for the first
    with dgw.Server(hbm_budget_bytes=fa + fa // 2) as srv:
        ta = srv.submit(a, 5, mode=(1, 1), t_final=0.2)
        tb = srv.submit(b, 5, mode=(1, 2), t_final=0.2)
        with pytest.raises(dgw.DgwError) as ei:
            srv.submit(_req_mesh(40, 23), 5, t_final=0.1)
        assert ei.value.name == "DGW_ETOOBIG"
        ra, _ = srv.wait(ta)
        rb, _ = srv.wait(tb)
    assert ra["status"] == rb["status"] == "DGW_OK"
    assert ra["footprint_bytes"] == fa
    assert rb["t_admit"] >= ra["t_finish"] - 1e-3
    # one slot has the same effect
    with dgw.Server(max_slots=1) as srv:
        ta = srv.submit(a, 3, t_final=0.2)
        tb = srv.submit(b, 3, t_final=0.2)
        ra, _ = srv.wait(ta)
        rb, _ = srv.wait(tb)
    assert rb["t_admit"] >= ra["t_finish"] - 1e-3


def test_late_arrival_joins_running_batch():
    long_m = _req_mesh(128, 31)  # 32768 elements, N=7, ~9000 steps
    short_m = _req_mesh(10, 32)
    with dgw.Server(max_chunk_steps=8) as srv:
        tl = srv.submit(long_m, 7, mode=(2, 3), t_final=2.0)
        time.sleep(0.3)
        ts = srv.submit(short_m, 3, t_final=0.05)
        rs, _ = srv.wait(ts)
        rl, _ = srv.wait(tl)
    print(f"long: start {rl['t_start']:.3f} finish {rl['t_finish']:.3f}; "
          f"short: arrival {rs['t_arrival']:.3f} start {rs['t_start']:.3f} finish {rs['t_finish']:.3f}")
    assert rs["status"] == rl["status"] == "DGW_OK"
    assert rs["t_arrival"] > rl["t_start"]
    assert rs["t_finish"] < rl["t_finish"]  # it joined and left while the long one ran
    assert rl["rel_l2_mode"] < 1e-5


def test_cancel_and_destroy_in_flight():
    with dgw.Server(max_slots=1, max_chunk_steps=4) as srv:
        t1 = srv.submit(_req_mesh(96, 41), 7, t_final=2.0)  # ~18000 steps
        t2 = srv.submit(_req_mesh(8, 42), 3, t_final=0.1)
        srv.cancel(t2)  # still pending behind the one slot
        r2, _ = srv.wait(t2)
        assert r2["status"] == "DGW_ECANCELLED"
        time.sleep(0.2)
        srv.cancel(t1)  # running: leaves at the next chunk boundary
        r1, _ = srv.wait(t1)
        assert r1["status"] == "DGW_ECANCELLED"
        with pytest.raises(dgw.DgwError) as ei:
            srv.poll(t1)
        assert ei.value.name == "DGW_ENOTFOUND"
        t3 = srv.submit(_req_mesh(8, 43), 3, t_final=0.1)
        r3, _ = srv.wait(t3)
        assert r3["status"] == "DGW_OK"
        assert srv.stats()["completed"] == 1
    # destroy with requests queued and running returns and frees everything
    srv = dgw.Server(max_slots=2)
    for k in range(5):
        srv.submit(_req_mesh(32, 50 + k), 5, t_final=2.0)
    time.sleep(0.2)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 30


def test_serving_mix_small_requests_vs_oracle():
    """Requests of the seeded serving mix with s <= 32 (their full t_final,
    their disk inclusions) through the server, each against the FP64 oracle
    at the server's dt and step count."""
    reqs = [r for r in inputs.make_requests(256, seed=4) if r.s <= 32][:3]
    assert len(reqs) == 3
    with dgw.Server() as srv:
        tickets = [srv.submit(inputs.request_mesh(r), r.order, mode=r.mode, t_final=r.t_final, keep_fields=True)
                   for r in reqs]
        results = [srv.wait(t, fields=True) for t in tickets]
    for r, (res, q) in zip(reqs, results):
        assert res["status"] == "DGW_OK"
        m = inputs.request_mesh(r)
        d = oracle.Discretization2D(m.vx, m.vy, m.elem_verts, r.order, eps=m.eps, mu=m.mu)
        op = oracle.Maxwell2D(d, 1.0)
        want = op.run(oracle.cavity_mode_2d(d.x, d.y, 0.0, *r.mode), res["dt"], res["steps"])
        err = rel(q, want)
        print(f"mix request {r.index}: s={r.s} N={r.order} t_final={r.t_final:.3f} steps={res['steps']}: {err:.2e}")
        assert err < 1e-5
