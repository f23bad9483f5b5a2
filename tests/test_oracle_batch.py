"""Semantics of the batched level step in the oracle: independent boxes with
fixed ghosts advanced with one level-wide time step and one substep count."""
import numpy as np

import oracle
from paper_2110_01792_amd import inputs


def test_batch_equals_boxes_run_alone_with_level_dt():
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=6, seed=11, edges=(8, 12))
    Ug0 = [u.copy() for u in Ugs]
    Ur0 = [None if u is None else u.copy() for u in Urs]
    st = oracle.batch_step(boxes, Ugs, Urs, hp["gamma"], hp["cfl"], p)
    # level dt is the minimum CFL step over boxes, shrunk to N_sub,max chat steps
    dts = [hp["cfl"] * min(b.dx) / oracle.hydro_max_signal(b, u, hp["gamma"]) for b, u in zip(boxes, Ug0)]
    dt_r = hp["cfl"] * min(boxes[0].dx) / p["chat"]
    n = int(np.ceil(min(dts) / dt_r))
    exp_dt = min(dts) if n <= p["nsub_max"] else p["nsub_max"] * dt_r
    assert abs(st["dt"] - exp_dt) <= 1e-15 * exp_dt
    assert st["nsub"] == min(n, p["nsub_max"])
    for b, g0, r0, g1, r1 in zip(boxes, Ug0, Ur0, Ugs, Urs):
        if r0 is None:
            oracle.hydro_step(b, g0, hp["gamma"], hp["cfl"], st["dt"])
            assert np.array_equal(g0, g1)
        else:
            oracle.hydro_step(b, g0, p["gamma"], hp["cfl"], st["dt"])
            for _ in range(st["nsub"]):
                oracle.rad_transport_substep(b, r0, g0, p, st["dt"] / st["nsub"])
                oracle.exchange_all(b, g0, r0, p, st["dt"] / st["nsub"])
            assert np.array_equal(g0, g1) and np.array_equal(r0, r1)


def test_fixed_ghosts_are_held():
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=3, seed=12, edges=(8,))
    ghosts = []
    for b, u in zip(boxes, Ugs):
        m = np.ones(u.shape[1:], bool)
        m[b.interior()[1:]] = False
        ghosts.append((m, u[:, m].copy()))
    oracle.batch_step(boxes, Ugs, Urs, hp["gamma"], hp["cfl"], p)
    for (m, g0), u in zip(ghosts, Ugs):
        assert np.array_equal(u[:, m], g0)
