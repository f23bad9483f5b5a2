"""GPU parity of the radiation and radiation-hydrodynamics path (HIP library
through its C ABI) against the FP64 oracle on the same seeded inputs.
Bar: relative L-infinity per variable <= 1e-10 (FP64)."""
import numpy as np
import pytest

import oracle
from paper_2110_01792_amd import binding as qb
from paper_2110_01792_amd import inputs
from tests.gpu_util import dev, host, padded_view, rel_linf, worst_cell

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = qb.Context(0)
    yield c
    c.close()


def gpu_rhd(ctx, b, Ug, Ur, p, nsteps=1):
    G, R = dev(Ug), dev(Ur)
    ctx.fill_ghosts(b, G)
    ctx.fill_ghosts(b, R)
    rp = qb.rad_params(p)
    for _ in range(nsteps):
        ctx.rhd_step(b, G, R, rp)
    st = ctx.sync_status()
    return host(G), host(R), st


def oracle_rhd(b, Ug, Ur, p, nsteps=1):
    G, R = Ug.copy(), Ur.copy()
    for _ in range(nsteps):
        st = oracle.rhd_step(b, G, R, p)
    return G, R, st


def check_pair(g, o, b, what):
    for name, x, y in (("gas", g[0], o[0]), ("rad", g[1], o[1])):
        e = rel_linf(x, y, b)
        assert np.all(e <= TOL), (what, name, e, worst_cell(x, y, b))


@pytest.mark.parametrize("n", [32, (40, 36, 20)])
def test_rhd_small_and_ragged(ctx, n):
    """RHD workload (log-normal density, independent gas/radiation
    temperatures, chat = 10 max c_s): one step = hydro + 10 substeps."""
    nn = n if isinstance(n, int) else max(n)
    b0, Ug, Ur, p = inputs.rhd_lognormal(n=nn)
    if not isinstance(n, int):
        b = inputs.make_box(n)
        g = 4
        sl = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        G0 = np.zeros((5,) + b.shape)
        R0 = np.zeros((4,) + b.shape)
        G0[sl] = Ug[sl]
        R0[sl] = Ur[sl]
        Ug, Ur = G0, R0
    else:
        b = b0
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, p, 2)
    og, orr, ost = oracle_rhd(b, Ug, Ur, p, 2)
    assert st == qb.QK_OK
    check_pair((gg, gr), (og, orr), b, f"n={n}")


def test_rhd_plm(ctx):
    """PLM for hydro and radiation (the reconstruction of the paper's RHD
    performance runs)."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=32, seed=17)
    q = dict(p, recon=1)
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, q, 2)
    og, orr, _ = oracle_rhd(b, Ug, Ur, q, 2)
    assert st == qb.QK_OK
    check_pair((gg, gr), (og, orr), b, "plm")


def test_rhd_128(ctx):
    """The RHD workload at 128^3, one step, compared everywhere."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=128)
    oracle.set_threads(0)
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, p, 1)
    og, orr, _ = oracle_rhd(b, Ug, Ur, p, 1)
    assert st == qb.QK_OK
    check_pair((gg, gr), (og, orr), b, "128^3")


def test_rhd_256_full_size(ctx):
    """The RHD workload at full size (256^3), one step, compared everywhere."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=256)
    oracle.set_threads(0)
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, p, 1)
    assert st == qb.QK_OK
    og, orr, _ = oracle_rhd(b, Ug, Ur, p, 1)
    check_pair((gg, gr), (og, orr), b, "256^3")


def test_substep_count_and_dt(ctx):
    """Section 2.2.4 substep cap: N = 10 on the RHD workload's initial state
    (the reduced speed of light is 10 times its largest sound speed); the dt
    the device takes equals the oracle's."""
    torch = pytest.importorskip("torch")
    b, Ug, Ur, p = inputs.rhd_lognormal(n=32)
    G = dev(Ug)
    ctx.fill_ghosts(b, G)
    nsub = torch.zeros(1, dtype=torch.int32, device="cuda")
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = ctx.compute_dt(b, G, hp=qb.hydro_params(p["gamma"], p["cfl"]), rp=qb.rad_params(p), dt_dev=dtd,
                        nsub_dev=nsub)
    assert int(nsub.item()) == 10
    og, orr, st = oracle_rhd(b, Ug, Ur, p, 1)
    assert abs(dt - st["dt"]) <= 1e-15 * st["dt"]


def test_optically_thick_faces_and_eddington(ctx):
    """Optical-depth factor active (tau_face ~ 2-10, Levermore closure) and the
    Eddington closure, with a smooth sub-luminal flux field: GPU matches the
    oracle."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=24, seed=13)
    z, y, x = inputs.cell_centres(b)
    I = b.interior()
    E = Ur[(0,) + I[1:]]
    for d, ph in enumerate((0.3, 1.1, 2.0)):
        Ur[(1 + d,) + I[1:]] = 0.2 * p["c"] * E * np.sin(2 * np.pi * (x + 2 * y + 3 * z) + ph) / np.sqrt(3)
    for closure, kap in ((0, 100.0), (1, 2.0)):
        q = dict(p, kappa_P=kap, kappa_R=kap, closure=closure)
        gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, q, 1)
        og, orr, ost = oracle_rhd(b, Ug, Ur, q, 1)
        assert st == qb.QK_OK and ost["neg_cells"] == 0 and ost["newton_fail"] == 0
        check_pair((gg, gr), (og, orr), b, f"closure={closure} kappa={kap}")


def test_rad_step_with_host_dt_matches_oracle_substeps(ctx):
    """quokka_rad_step with a host dt: N = ceil(dt/dt_r) substeps of transport +
    coupling, equal to the oracle's substep sequence."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=20, seed=21)
    o_g, o_r = Ug.copy(), Ur.copy()
    oracle.fill_ghosts(b, o_g)
    oracle.fill_ghosts(b, o_r)
    dt_r = p["cfl"] * min(b.dx) / p["chat"]
    dt = 3.5 * dt_r
    G, R = dev(o_g), dev(o_r)
    ctx.rad_step(b, G, R, qb.rad_params(p), dt=dt)
    assert ctx.sync_status() == qb.QK_OK
    for _ in range(4):
        oracle.rad_transport_substep(b, o_r, o_g, p, dt / 4)
        oracle.exchange_all(b, o_g, o_r, p, dt / 4)
        oracle.fill_ghosts(b, o_g)
        oracle.fill_ghosts(b, o_r)
    check_pair((host(G), host(R)), (o_g, o_r), b, "host dt")


def test_linear_exchange_closed_form_on_gpu(ctx):
    """Uniform box (no transport), C_v = alpha T^3: after N substeps
    D = a_r T^4 - E_r equals D0 / (1 + lambda dt/N)^N (Section 3.2.3 set-up in
    dimensionless form)."""
    b = inputs.make_box(8)
    p = inputs.rad_params(chat=50.0, eos=1, alpha_cv=4.0, kappa_P=20.0, kappa_R=20.0)
    Ug = np.zeros((5,) + b.shape)
    Ur = np.zeros((4,) + b.shape)
    I = b.interior()
    Eg0, Er0, rho = 0.5, 3.0, 1.0
    Ug[I] = np.array([rho, 0, 0, 0, Eg0])[:, None, None, None]
    Ur[I] = np.array([Er0, 0, 0, 0])[:, None, None, None]
    G, R = dev(Ug), dev(Ur)
    ctx.fill_ghosts(b, G)
    ctx.fill_ghosts(b, R)
    ctx.newton_iter_max()  # reset the counter
    dt = 5 * p["cfl"] * min(b.dx) / p["chat"]
    ctx.rad_step(b, G, R, qb.rad_params(p), dt=dt)
    assert ctx.sync_status() == qb.QK_OK
    g, r = host(G), host(R)
    lam = rho * p["kappa_P"] * (4 * p["a_r"] * p["c"] / p["alpha_cv"] + p["chat"])
    D0 = 4 * p["a_r"] / p["alpha_cv"] * Eg0 - Er0
    D = 4 * p["a_r"] / p["alpha_cv"] * g[4][I[1:]] - r[0][I[1:]]
    assert np.allclose(D, D0 / (1 + lam * dt / 5) ** 5, rtol=1e-11, atol=1e-13)
    assert ctx.newton_iter_max() == 1


def test_newton_failure_is_reported(ctx):
    b, Ug, Ur, p = inputs.rhd_lognormal(n=12, seed=2)
    q = dict(p, newton_max_iter=1, newton_tol=1e-15)
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, q, 1)
    assert st == qb.QK_ENEWTON
    assert ctx.sync_status() == qb.QK_OK


def test_rhd_deterministic(ctx):
    b, Ug, Ur, p = inputs.rhd_lognormal(n=32, seed=7)
    a = gpu_rhd(ctx, b, Ug, Ur, p, 1)
    c = gpu_rhd(ctx, b, Ug, Ur, p, 1)
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])


def test_rhd_with_radiation_source_matches_oracle(ctx):
    """The optional source term of Section 2.2.3 (S = dt_sub j per cell, a
    seeded non-negative rate array in the box layout) through quokka_rhd_step
    against the oracle's RHD step with the same rate."""
    torch = pytest.importorskip("torch")
    b, Ug, Ur, p = inputs.rhd_lognormal(n=24, seed=41)
    rng = np.random.default_rng(42)
    j = np.zeros(b.shape)
    j[b.interior()[1:]] = rng.uniform(0.0, 200.0, size=(b.n[2], b.n[1], b.n[0]))
    G, R = dev(Ug), dev(Ur)
    ctx.fill_ghosts(b, G)
    ctx.fill_ghosts(b, R)
    J = dev(j)
    rp = qb.rad_params(p, source=J)
    for _ in range(2):
        ctx.rhd_step(b, G, R, rp)
    assert ctx.sync_status() == qb.QK_OK
    ps = dict(p, source=j)
    oG, oR, _ = oracle_rhd(b, Ug, Ur, ps, nsteps=2)
    check_pair((host(G), host(R)), (oG, oR), b, "source")
    # the source changed the result
    nG, nR, _ = oracle_rhd(b, Ug, Ur, p, nsteps=2)
    assert np.max(np.abs(nR[0] - oR[0])) > 1e-3 * np.max(np.abs(oR[0]))


def test_batch_rejects_radiation_source(ctx):
    torch = pytest.importorskip("torch")
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=2, seed=43, edges=(8,))
    G = [dev(u) for u in Ugs]
    R = [None if u is None else dev(u) for u in Urs]
    J = torch.zeros(boxes[0].shape, dtype=torch.float64, device="cuda")
    with pytest.raises(qb.QuokkaError) as e:
        ctx.batch_step(boxes, G, R, qb.hydro_params(hp["gamma"], hp["cfl"]), qb.rad_params(p, source=J))
    assert e.value.status == qb.QK_EINVAL


def test_rad_pressure_tube_matches_oracle(ctx):
    """Optically thick column (radiation pressure tube, tau_cell ~ 100, cgs
    magnitudes, Dirichlet ends): five RHD steps on the GPU against the oracle."""
    b, Ug, Ur, p, ref = inputs.rad_pressure_tube()
    g, r, st = gpu_rhd(ctx, b, Ug, Ur, p, nsteps=5)
    assert st == qb.QK_OK
    og, orr, _ = oracle_rhd(b, Ug, Ur, p, nsteps=5)
    check_pair((g, r), (og, orr), b, "tube")


@pytest.mark.parametrize("closure", [1, 2])
def test_rhd_other_closures(ctx, closure):
    """Eddington and Minerbo closures through the same kernels (the closure is
    one device function of f)."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=24, seed=44)
    rng = np.random.default_rng(45)
    # give the radiation a flux so that the closure matters
    I = b.interior()
    Ur[(slice(1, 4),) + I[1:]] = rng.uniform(-0.3, 0.3, size=(3, b.n[2], b.n[1], b.n[0])) * p["c"] * Ur[(0,) + I[1:]]
    p = dict(p, closure=closure)
    g, r, st = gpu_rhd(ctx, b, Ug, Ur, p)
    assert st == qb.QK_OK
    og, orr, _ = oracle_rhd(b, Ug, Ur, p)
    check_pair((g, r), (og, orr), b, f"closure {closure}")


@pytest.mark.parametrize("closure", [0, 2])
def test_rhd_streaming_states_take_the_fallback(ctx, closure):
    """Reduced fluxes up to |f| = 0.97 in random directions, and 1 % of cells
    at |f| = 1.03: reconstructed face states pass |f| = 1, so faces fall back
    to the cell averages, and some of those averages still have |f| > 1 (the
    closure then takes min(|f|, 1)).  One RHD step (10 substeps) against the
    oracle.  (Eddington's closure cannot carry such streaming states: the
    oracle itself reaches negative energies there.)"""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=24, seed=46)
    rng = np.random.default_rng(47)
    I = b.interior()
    shape = (b.n[2], b.n[1], b.n[0])
    d = rng.normal(size=(3,) + shape)
    d /= np.linalg.norm(d, axis=0)
    mag = rng.uniform(0.0, 0.97, size=shape)
    mag[rng.uniform(size=shape) < 0.01] = 1.03
    Ur[(slice(1, 4),) + I[1:]] = d * mag * p["c"] * Ur[(0,) + I[1:]]
    p = dict(p, closure=closure)
    g, r, st = gpu_rhd(ctx, b, Ug, Ur, p)
    assert st == qb.QK_OK
    og, orr, ost = oracle_rhd(b, Ug, Ur, p)
    assert ost["neg_cells"] == 0 and ost["newton_fail"] == 0
    check_pair((g, r), (og, orr), b, f"streaming, closure {closure}")


def test_rhd_padded_layout_equals_contiguous_bitwise(ctx):
    """Gas and radiation states in one padded layout (shared pitches) give the
    bits of the contiguous layout over an RHD step; states of one box in
    different layouts are refused on the host."""
    b, Ug, Ur, p = inputs.rhd_lognormal(n=20, seed=43)
    rp = qb.rad_params(p)
    G, R = dev(Ug), dev(Ur)
    bg, PG = padded_view(dev(Ug))
    br, PR = padded_view(dev(Ur))
    for g, r in ((G, R), (PG, PR)):
        ctx.fill_ghosts(b, g)
        ctx.fill_ghosts(b, r)
        ctx.rhd_step(b, g, r, rp)
    assert ctx.sync_status() == qb.QK_OK
    assert np.array_equal(host(G), host(PG.contiguous()))
    assert np.array_equal(host(R), host(PR.contiguous()))
    with pytest.raises(ValueError):
        ctx.rhd_step(b, G, PR, rp)


# ------------------------------------- causality rule of the optical-depth correction
def _oracle_rhd_counting(b, Ug, Ur, p, nsteps):
    G, R = Ug.copy(), Ur.copy()
    causal = 0
    for _ in range(nsteps):
        st = oracle.rhd_step(b, G, R, p)
        assert st["neg_cells"] == 0 and st["newton_fail"] == 0
        causal += st["causal_cells"]
    return G, R, causal


@pytest.mark.parametrize("n,nsteps", [((32, 1, 1), 3), ((24, 12, 8), 2), ((40, 20, 12), 1)])
def test_causality_rule_matches_oracle(ctx, n, nsteps):
    """Section 2.2.2: a beam (|f| = 0.99) enters an optically thick slab
    (tau_cell 100 beside 0.01, curved surface in 3-D), so thick faces sit
    beside streaming ones and the corrected update gives |F| > c E_r at the
    slab's surface.  The oracle switches the correction off there (its count
    of such cells is > 0); the GPU matches it after whole RHD steps, in 1-D,
    in 3-D and on a box spanning several tiles with partial ones."""
    b, Ug, Ur, p = inputs.rad_thick_streaming(n=n)
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, p, nsteps)
    assert st == qb.QK_OK
    og, orr, causal = _oracle_rhd_counting(b, Ug, Ur, p, nsteps)
    assert causal > 0
    check_pair((gg, gr), (og, orr), b, f"causality rule n={n}")
    # without the correction the result differs (the rule's cells matter)
    ng, nr, _ = oracle_rhd(b, Ug, Ur, dict(p, tau_correction=0), nsteps)
    assert np.max(np.abs(nr[0] - orr[0])) > 1e-6 * np.max(np.abs(orr[0]))


def test_causality_rule_periodic_box(ctx):
    """The same slab in a box periodic on every face: the radiation stages
    skip the ghost fills between stages and read cells outside the box at
    their periodic images, the fix-up included; the beam leaving at x = 1
    re-enters at x = 0, so thick and streaming cells also meet across the
    periodic boundary."""
    b0, Ug, Ur, p = inputs.rad_thick_streaming(n=(24, 12, 8))
    b = inputs.Box(b0.n, b0.ng, b0.dx, ((inputs.PERIODIC, inputs.PERIODIC),) * 3)
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, p, 2)
    assert st == qb.QK_OK
    og, orr, causal = _oracle_rhd_counting(b, Ug, Ur, p, 2)
    assert causal > 0
    check_pair((gg, gr), (og, orr), b, "causality rule, periodic box")


@pytest.mark.parametrize("n", [(4, 5, 6), (6, 4, 4)])
def test_rhd_ghost_images_on_small_boxes(ctx, n):
    """The RHD workload on periodic boxes with an extent of exactly 4: the
    radiation stages read the periodic images of a 3-deep halo and skip
    the fills between stages; two steps against the oracle."""
    b0, Ug0, Ur0, p = inputs.rhd_lognormal(n=max(n))
    b = inputs.make_box(n)
    g = b.ng
    sl = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
    Ug, Ur = np.zeros((5,) + b.shape), np.zeros((4,) + b.shape)
    Ug[sl], Ur[sl] = Ug0[sl], Ur0[sl]
    gg, gr, st = gpu_rhd(ctx, b, Ug, Ur, p, 2)
    assert st == qb.QK_OK
    og, orr, _ = oracle_rhd(b, Ug, Ur, p, 2)
    check_pair((gg, gr), (og, orr), b, f"rhd small box {n}")


def test_causality_rule_mixed_precision_stays_causal_and_positive(ctx):
    """The FP32 path on the thick slab: the rule keeps it positive and close
    to the FP64 oracle (normalised L1 per variable within 1e-3 on this
    discontinuous slab; the 1e-5 bar is for smooth workloads)."""
    torch = pytest.importorskip("torch")
    b, Ug, Ur, p = inputs.rad_thick_streaming(n=(24, 12, 8))
    G, R = dev(Ug, torch.float32), dev(Ur, torch.float32)
    ctx.fill_ghosts(b, G)
    ctx.fill_ghosts(b, R)
    ctx.rhd_step(b, G, R, qb.rad_params(p))
    assert ctx.sync_status() == qb.QK_OK
    og, orr, causal = _oracle_rhd_counting(b, host(dev(Ug, torch.float32)), host(dev(Ur, torch.float32)), p, 1)
    from tests.gpu_util import norm_l1
    assert np.all(norm_l1(host(R), orr, b) < 1e-3), norm_l1(host(R), orr, b)
    assert np.all(norm_l1(host(G), og, b) < 1e-3), norm_l1(host(G), og, b)


def test_causality_rule_in_batched_level(ctx):
    """The rule inside the batched level step: two slab boxes with fixed ghost
    cells (filled beforehand) and one hydro-only box, three level steps (one
    capture, two graph replays), against the oracle's level step."""
    torch = pytest.importorskip("torch")
    boxes, Gs, Rs = [], [], []
    for n, seed in (((24, 12, 8), 9), ((16, 16, 8), 19)):
        b, Ug, Ur, p = inputs.rad_thick_streaming(n=n, seed=seed)
        oracle.fill_ghosts(b, Ug)
        oracle.fill_ghosts(b, Ur)
        boxes.append(b._replace(bc=((inputs.FIXED, inputs.FIXED),) * 3))
        Gs.append(Ug)
        Rs.append(Ur)
    hb, hU, _ = inputs.hydro_smooth(n=16)
    oracle.fill_ghosts(hb, hU)
    boxes.append(hb._replace(bc=((inputs.FIXED, inputs.FIXED),) * 3))
    Gs.append(hU)
    Rs.append(None)
    hp = {"gamma": p["gamma"], "cfl": p["cfl"]}
    G = [dev(u) for u in Gs]
    R = [None if u is None else dev(u) for u in Rs]
    oG = [u.copy() for u in Gs]
    oR = [None if u is None else u.copy() for u in Rs]
    causal = 0
    for s in range(3):
        ctx.batch_step(boxes, G, R, qb.hydro_params(hp["gamma"], hp["cfl"]), qb.rad_params(p))
        st = oracle.batch_step(boxes, oG, oR, hp["gamma"], hp["cfl"], p)
        causal += st["causal_cells"]
        for k, b in enumerate(boxes):
            e = rel_linf(host(G[k]), oG[k], b)
            assert np.all(e <= TOL), (s, k, "gas", e)
            if oR[k] is not None:
                e = rel_linf(host(R[k]), oR[k], b)
                assert np.all(e <= TOL), (s, k, "rad", e, worst_cell(host(R[k]), oR[k], b))
    assert ctx.sync_status() == qb.QK_OK
    assert causal > 0


def test_rad_pressure_tube_whole_column_within_paper_bound(ctx):
    """Section 3.3.1: over one sound-crossing time (CFL 0.4, 128 cells,
    tau_cell ~ 100) the GPU keeps gas and radiation temperatures within the
    paper's 0.2 per cent of the ODE steady state over the whole column
    (Dirichlet ends hold rho, v and T; the radiation flux in the ghost cells is
    extrapolated), with T_rad = T_gas; and it stays within 1e-9 of the oracle
    run with the same step sizes."""
    torch = pytest.importorskip("torch")
    b, Ug, Ur, p, ref = inputs.rad_pressure_tube()
    G, R = dev(Ug), dev(Ur)
    ctx.fill_ghosts(b, G)
    ctx.fill_ghosts(b, R)
    rp = qb.rad_params(p)
    hp = qb.hydro_params(p["gamma"], p["cfl"], p["recon"])
    oG, oR = Ug.copy(), Ur.copy()
    t, tend = 0.0, ref["t_end"]
    dt_r = p["cfl"] * b.dx[0] / p["chat"]
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    nsub = torch.zeros(1, dtype=torch.int32, device="cuda")
    while t < tend * (1 - 1e-12):
        oracle.fill_ghosts(b, oG)
        sig = oracle.hydro_max_signal(b, oG, p["gamma"])
        dt = min(p["cfl"] * b.dx[0] / sig, tend - t)
        nn = max(1, int(np.ceil(dt / dt_r)))
        if nn > p["nsub_max"]:  # the substep cap shrinks the step (Section 2.2.4)
            nn = p["nsub_max"]
            dt = nn * dt_r
        dtd.fill_(dt)
        nsub.fill_(nn)
        ctx.hydro_step(b, G, hp, dt_dev=dtd)
        ctx.rad_step(b, G, R, rp, dt_dev=dtd, nsub_dev=nsub)
        st = oracle.rhd_step(b, oG, oR, p, dt=dt)
        assert st["dt"] == dt and st["nsub"] == nn
        t += dt
    assert ctx.sync_status() == qb.QK_OK
    g, r = host(G), host(R)
    n, gi = b.n[0], b.ng
    rho = g[0, gi, gi, gi:gi + n]
    Tg = (g[4, gi, gi, gi:gi + n] - 0.5 * g[1, gi, gi, gi:gi + n] ** 2 / rho) * (p["gamma"] - 1) / rho
    Tr = (r[0, gi, gi, gi:gi + n] / p["a_r"]) ** 0.25
    T = ref["T"][gi:gi + n]
    assert np.max(np.abs(Tg / T - 1)) < 2e-3
    assert np.max(np.abs(Tr / T - 1)) < 2e-3
    assert np.max(np.abs(Tg - Tr) / T) < 1e-5
    for name, x, y in (("gas", g, oG), ("rad", r, oR)):
        e = rel_linf(x, y, b)
        assert np.all(e <= 1e-9), (name, e)


@pytest.mark.parametrize("var,tau", [(0, 4.0), (1, 4.0), (0, 100.0), (1, 100.0)])
def test_grid_scale_modes_with_the_optical_depth_factor(ctx, var, tau):
    """The checkerboard states on which the oracle's optical-depth factor is
    pinned (only the scaled HLL dissipation acts on them): one radiation
    substep (transport and coupling, kappa_P = 0) on the GPU against the
    oracle, and the transported amplitude ratio against its closed form."""
    from tests.test_oracle_rad import _uniform_slab
    n = 16
    b, Ug, p = _uniform_slab(n, tau)
    c, ch = p["c"], p["chat"]
    g = b.ng
    sgn = (-1.0) ** np.arange(-g, n + g)
    Ur = np.zeros((4,) + b.shape)
    Ur[0] = 1.0
    if var == 0:
        Ur[0] = (1.0 + 0.01 * sgn)[None, None, :]
    else:
        Ur[1] = (0.1 * c * sgn)[None, None, :]
    oracle.fill_ghosts(b, Ug)
    oracle.fill_ghosts(b, Ur)
    dt = p["cfl"] * b.dx[0] / ch
    G, R = dev(Ug), dev(Ur)
    ctx.rad_step(b, G, R, qb.rad_params(p), dt=dt)
    assert ctx.sync_status() == qb.QK_OK
    oG, oR = Ug.copy(), Ur.copy()
    oracle.rad_transport_substep(b, oR, oG, p, dt)
    oracle.exchange_all(b, oG, oR, p, dt)
    oracle.fill_ghosts(b, oG)
    oracle.fill_ghosts(b, oR)
    check_pair((host(G), host(R)), (oG, oR), b, f"checkerboard var={var} tau={tau}")
    if var == 0:  # E: the coupling leaves it (F = 0, kappa_P = 0)
        z = 2.0 * min(1.0, 1.0 / tau) * (ch / np.sqrt(3.0)) * dt / b.dx[0]
        a0 = Ur[0, g, g, g:g + n] - 1.0
        a1 = host(R)[0, g, g, g:g + n] - 1.0
        np.testing.assert_allclose(a1, (1.0 - z + 0.5 * z * z) * a0, rtol=1e-10, atol=1e-15)
