"""GPU parity of the AMR level-synchronisation operations (refinement ratio
2) against the oracle: flux registers recorded by the fused stage kernel,
average-down, prolongation with time interpolation, reflux, and the two-level
step built from them (FP64 <= 1e-10 relative, conservation to round-off)."""
import numpy as np
import pytest

import oracle
from paper_2110_01792_amd import binding as qb
from paper_2110_01792_amd import inputs
from tests.amr_runs import (composite_totals, composite_totals_n, coarse_totals, coarse_totals_n, region_size,
                            two_level_rad_step, two_level_step)
from tests.gpu_util import dev, host, rel_linf
from tests.test_oracle_amr import OracleAMR

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = qb.Context(0)
    yield c
    c.close()


class GpuAMR:
    """The GPU entry points with the oracle driver's signatures."""

    def __init__(self, ctx):
        import torch
        self.ctx, self.torch = ctx, torch

    def copy(self, U):
        return U.clone()

    def zeros(self, n):
        return self.torch.zeros(n, dtype=self.torch.float64, device="cuda")

    def fill_ghosts(self, b, U):
        self.ctx.fill_ghosts(b, U)

    def max_signal(self, b, U, gamma):
        hp = qb.hydro_params(gamma, 1.0)
        dt = self.ctx.compute_dt(b, U, hp=hp)  # dt = 1.0 * min(dx) / s_max
        return min(b.dx) / dt

    def hydro_step_reg(self, b, U, gamma, cfl, dt, lo, hi, reg):
        self.ctx.hydro_step_reg(b, U, qb.hydro_params(gamma, cfl), lo, hi, reg, dt=dt)

    def prolong(self, cb, U0, U1, alpha, fb, Uf, off, interior=False, nvar=5):
        self.ctx.prolong(cb, U0, U1, alpha, fb, Uf, off, nvar=nvar, interior=interior)

    def average_down(self, fb, Uf, cb, Uc, off, nvar=5):
        self.ctx.average_down(fb, Uf, cb, Uc, off, nvar=nvar)

    def reflux(self, cb, Uc, lo, hi, reg_c, fb, reg_f, nvar=5):
        self.ctx.reflux(cb, Uc, lo, hi, reg_c, fb, reg_f, nvar=nvar)

    def rad_step_reg(self, b, Ug, Ur, p, dt, lo, hi, reg):
        self.ctx.rad_step_reg(b, Ug, Ur, qb.rad_params(p), lo, hi, reg, dt)


def test_register_matches_oracle(ctx):
    """Registers over an interior region and over the whole box (its boundary
    faces), both RK stages, on a 24 x 20 x 28 box (partial tiles, several
    z chunks)."""
    b = inputs.make_box((24, 20, 28))
    _, U, p = inputs.hydro_smooth(n=28, seed=62)
    g = 4
    U0 = np.zeros((5,) + b.shape)
    U0[b.interior()] = U[:, g:g + 28, g:g + 20, g:g + 24]
    for lo, hi in (((3, 5, 4), (19, 12, 21)), ((0, 0, 0), b.n)):
        ro = np.zeros(region_size(lo, hi))
        Uo = U0.copy()
        oracle.hydro_step_reg(b, Uo, p["gamma"], p["cfl"], 2e-3, lo, hi, ro)
        Ud = dev(U0)
        ctx.fill_ghosts(b, Ud)
        rd = GpuAMR(ctx).zeros(region_size(lo, hi))
        ctx.hydro_step_reg(b, Ud, qb.hydro_params(p["gamma"], p["cfl"]), lo, hi, rd, dt=2e-3)
        assert ctx.sync_status() == qb.QK_OK
        e = np.abs(host(rd) - ro).max() / np.abs(ro).max()
        assert e <= TOL, (lo, hi, e)
        assert np.all(rel_linf(host(Ud), Uo, b) <= TOL)


def test_prolong_and_average_down_match_oracle(ctx):
    cb, Uc, fb, Uf, off, p = inputs.two_level()
    oracle.fill_ghosts(cb, Uc)
    U1 = Uc * 1.1
    for interior in (False, True):
        fo = Uf.copy()
        oracle.prolong(cb, Uc, U1, 0.3, fb, fo, off, interior=interior)
        fd = dev(Uf)
        ctx.prolong(cb, dev(Uc), dev(U1), 0.3, fb, fd, off, interior=interior)
        assert np.array_equal(host(fd), fo)
    co = Uc.copy()
    oracle.average_down(fb, Uf, cb, co, off)
    cd = dev(Uc)
    ctx.average_down(fb, dev(Uf), cb, cd, off)
    assert np.array_equal(host(cd), co)


@pytest.mark.parametrize("n,m,off", [(16, 16, (4, 4, 4)), (64, 72, (10, 14, 20))], ids=["16", "64_multi_tile"])
def test_two_level_step_matches_oracle_and_conserves(ctx, n, m, off):
    """Two coarse steps of the two-level scheme (coarse step, two fine steps
    with ghosts from the coarse level in space and time, average-down,
    reflux) on the GPU against the oracle, and the composite totals kept to
    round-off.  The larger case spans several stage tiles and z-chunks on
    both levels, with a footprint that cuts through tiles."""
    cb, Uc, fb, Uf, off, p = inputs.two_level(n=n, m=m, off=off)
    oracle.average_down(fb, Uf, cb, Uc, off)
    t0 = composite_totals(cb, Uc, fb, Uf, off)
    Cd, Fd = dev(Uc), dev(Uf)
    Co, Fo = Uc.copy(), Uf.copy()
    A = GpuAMR(ctx)
    for _ in range(2):
        two_level_step(A, cb, Cd, fb, Fd, off, p["gamma"], p["cfl"])
        two_level_step(OracleAMR, cb, Co, fb, Fo, off, p["gamma"], p["cfl"])
        assert ctx.sync_status() == qb.QK_OK
        assert np.all(rel_linf(host(Cd), Co, cb) <= TOL)
        assert np.all(rel_linf(host(Fd), Fo, fb) <= TOL)
    t1 = coarse_totals(cb, host(Cd))
    assert np.all(np.abs(t1 - t0) / np.abs(t0).max() < 1e-14)


@pytest.mark.parametrize("n,m,off", [(16, 16, (4, 4, 4)), (48, 40, (6, 10, 14))], ids=["16", "48_multi_tile"])
def test_radiation_two_level_step_matches_oracle_and_conserves(ctx, n, m, off):
    """Radiation on two levels (transport only, kappa = 0): registers of every
    substep's stages, prolongation and average-down of 4 variables, reflux;
    GPU against the oracle and the totals of E_r and F kept to round-off."""
    cb, Gc, Rc, fb, Gf, Rf, off, hp, p = inputs.two_level(n=n, m=m, off=off, rad=True)
    oracle.average_down(fb, Rf, cb, Rc, off, nvar=4)
    oracle.average_down(fb, Gf, cb, Gc, off, nvar=5)
    t0 = composite_totals_n(cb, Rc, fb, Rf, off)
    d = [dev(x) for x in (Gc, Rc, Gf, Rf)]
    o = [x.copy() for x in (Gc, Rc, Gf, Rf)]
    A = GpuAMR(ctx)
    for _ in range(2):
        two_level_rad_step(A, cb, d[0], d[1], fb, d[2], d[3], off, p)
        two_level_rad_step(OracleAMR, cb, o[0], o[1], fb, o[2], o[3], off, p)
        assert ctx.sync_status() == qb.QK_OK
        for x, y, b in zip(d, o, (cb, cb, fb, fb)):
            assert np.all(rel_linf(host(x), y, b) <= TOL)
    t1 = coarse_totals_n(cb, host(d[1]))
    assert np.all(np.abs(t1 - t0) / np.abs(t0[0]) < 1e-13)


def test_amr_argument_errors(ctx):
    torch = pytest.importorskip("torch")
    cb, Uc, fb, Uf, off, p = inputs.two_level()
    Cd, Fd = dev(Uc), dev(Uf)
    with pytest.raises(qb.QuokkaError) as e:
        ctx.average_down(fb, Fd, cb, Cd, (10, 4, 4))  # footprint leaves the coarse interior
    assert e.value.status == qb.QK_EINVAL
    reg = torch.zeros(region_size((0, 0, 0), (4, 4, 40)), dtype=torch.float64, device="cuda")
    with pytest.raises(qb.QuokkaError) as e:
        ctx.hydro_step_reg(cb, Cd, qb.hydro_params(p["gamma"], p["cfl"]), (0, 0, 0), (4, 4, 40), reg, dt=1e-3)
    assert e.value.status == qb.QK_EINVAL


def test_amr_operations_in_fp32(ctx):
    """Mixed-precision (FP32) state through prolongation and average-down
    (FP64 arithmetic inside, one FP32 rounding on store) against the FP64
    oracle on the same FP32-rounded data."""
    torch = pytest.importorskip("torch")
    cb, Uc, fb, Uf, off, p = inputs.two_level()
    oracle.fill_ghosts(cb, Uc)
    Uc = inputs.to_f32_and_back(Uc)
    Uf = inputs.to_f32_and_back(Uf)
    fo = Uf.copy()
    oracle.prolong(cb, Uc, Uc, 0.0, fb, fo, off, interior=True)
    fd = dev(Uf, torch.float32)
    cd = dev(Uc, torch.float32)
    ctx.prolong(cb, cd, cd, 0.0, fb, fd, off, interior=True)
    assert np.all(rel_linf(host(fd), fo, fb) <= 2e-7)
    co = Uc.copy()
    oracle.average_down(fb, Uf, cb, co, off)
    cd = dev(Uc, torch.float32)
    ctx.average_down(fb, dev(Uf, torch.float32), cb, cd, off)
    assert np.all(rel_linf(host(cd), co, cb) <= 2e-7)
