"""Checkpoint/resume and failure isolation on the GPU, through the C ABI.

Resume.  The first stage of every LSRK step has a = 0, so the residual does
not carry information across steps: a solve continued from its fields alone
(read back to the host in FP64, set into a fresh solver) must give bitwise
the same result as the uninterrupted solve, T/2 + T/2 = T.

Isolation.  A request whose initial fields hold a NaN fails with
DGW_ENONFINITE; every other request sharing its batched launches finishes
with DGW_OK and bitwise the same fields as when it runs alone (elements of
different requests never read each other's data)."""

import numpy as np
import pytest

import oracle
from paper_1304_5546_amd import dgw, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,N,prec", [(2, 5, "fp32"), (2, 7, "fp32"), (2, 5, "split_bf16"),
                                         (2, 4, "split_fp16"), (2, 5, "fp64"), (3, 3, "fp32"),
                                         (3, 4, "split_bf16")])
def test_resume_from_fields_is_bitwise(dim, N, prec):
    if dim == 2:
        m, mode = inputs.tri_grid(24, seed=3, permute=True), (2, 1)
    else:
        m, mode = inputs.tet_grid(4, seed=3, permute=True), (1, 1, 1)
    with dgw.Solver(m, N, prec=prec) as a:
        a.set_cavity_mode(*mode)
        dt = a.cfl_dt()
        a.advance_steps(30, dt)
        q_half = a.get_fields()
        a.advance_steps(30, dt)
        q_full = a.get_fields()
    with dgw.Solver(m, N, prec=prec) as b:
        b.set_fields(q_half)
        b.advance_steps(30, dt)
        q_resumed = b.get_fields()
    with dgw.Solver(m, N, prec=prec) as c:
        c.set_cavity_mode(*mode)
        c.advance_steps(60, dt)
        q_straight = c.get_fields()
    assert np.array_equal(q_full, q_straight)
    assert np.array_equal(q_resumed, q_straight), "resumed solve differs from the uninterrupted one"


# (grid s, seed, order, mode, t_final); all eps = mu = 1
ISO_MIX = [
    (12, 21, 5, (1, 2), 0.30),
    (20, 22, 3, (2, 1), 0.25),
    (9, 23, 7, (1, 1), 0.20),
    (16, 24, 5, (2, 2), 0.25),
]


def _mesh(s, seed):
    return inputs.tri_grid(s, seed=seed, permute=True)


def test_nonfinite_request_is_isolated():
    alone = {}
    with dgw.Server(max_chunk_steps=8) as srv:
        for i, (s, seed, N, mode, tf) in enumerate(ISO_MIX):
            res, q = srv.wait(srv.submit(_mesh(s, seed), N, mode=mode, t_final=tf, keep_fields=True), fields=True)
            assert res["status"] == "DGW_OK"
            alone[i] = q
    # the poisoned request: same mesh and order as request 0, one NaN in Ez
    s, seed, N, mode, tf = ISO_MIX[0]
    m0 = _mesh(s, seed)
    d = oracle.Discretization2D(m0.vx, m0.vy, m0.elem_verts, N)
    q_bad = oracle.cavity_mode_2d(d.x, d.y, 0.0, *mode)
    q_bad[2, m0.K // 2, 3] = np.nan
    with dgw.Server(max_chunk_steps=8) as srv:
        bad = srv.submit(m0, N, q0=q_bad, t_final=tf, keep_fields=True)
        tickets = {i: srv.submit(_mesh(s, seed), Nn, mode=md, t_final=t, keep_fields=True)
                   for i, (s, seed, Nn, md, t) in enumerate(ISO_MIX)}
        rb, qb = srv.wait(bad, fields=True)
        mixed = {i: srv.wait(t, fields=True) for i, t in tickets.items()}
    print(f"poisoned request: {rb['status']}")
    assert rb["status"] == "DGW_ENONFINITE"
    for i, (res, q) in mixed.items():
        assert res["status"] == "DGW_OK", (i, res["status"])
        assert np.array_equal(q, alone[i]), f"request {i} changed next to a non-finite request"
