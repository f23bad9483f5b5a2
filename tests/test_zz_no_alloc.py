"""quokka_hydro_step_noalloc (the step for callers that cannot allocate) gives
the bits of quokka_hydro_step on the same input, through the C ABI, on two
calls in a row whose second box is smaller than the first (the static scratch
keeps the first call's contents), in FP64 and FP32; boxes beyond its limit
are refused on the host."""
import numpy as np
import pytest

from paper_2110_01792_amd import binding as qb
from paper_2110_01792_amd import inputs
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _smooth_box(n, dtype, seed):
    b, U, p = inputs.hydro_smooth(n=max(n) if not isinstance(n, int) else n, seed=seed)
    if not isinstance(n, int):
        b2 = inputs.make_box(n)
        g = b.ng
        V = np.ones((5,) + b2.shape)
        sl = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        V[sl] = U[sl]
        b, U = b2, V
    return b, dev(U, dtype), p


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_step_equals_allocating_step_on_two_calls(prec):
    torch = pytest.importorskip("torch")
    dtype = torch.float64 if prec == "f64" else torch.float32
    ctx = qb.Context(0)
    try:
        for n, seed in ((128 if prec == "f64" else 160, 71), ((40, 36, 20), 72)):
            b, U, p = _smooth_box(n, dtype, seed)
            ctx.fill_ghosts(b, U)
            hp = qb.hydro_params(p["gamma"], p["cfl"])
            A, B = U.clone(), U.clone()
            dta = torch.zeros(1, dtype=torch.float64, device="cuda")
            dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
            for _ in range(2):  # CFL dt from the state, next dt fused
                ctx.hydro_step(b, A, hp, dt_next_dev=dta)
                ctx.hydro_step_noalloc(b, B, hp, dt_next_dev=dtb)
            assert ctx.sync_status() == qb.QK_OK
            a, c = host(A), host(B)
            assert np.array_equal(a, c), (n, prec, np.max(np.abs(a - c)))
            assert dta.item() == dtb.item() and dta.item() > 0
            assert not np.array_equal(a, host(U))  # the step did something
    finally:
        ctx.close()


def test_noalloc_step_refuses_boxes_beyond_its_scratch():
    torch = pytest.importorskip("torch")
    ctx = qb.Context(0)
    try:
        b, U, p = _smooth_box(136, torch.float64, 73)  # 144^3 x 48 B > 128 MiB
        with pytest.raises(qb.QuokkaError) as e:
            ctx.hydro_step_noalloc(b, U, qb.hydro_params(p["gamma"], p["cfl"]))
        assert e.value.status == qb.QK_EINVAL
        assert "no-allocation" in str(e.value)
    finally:
        ctx.close()
