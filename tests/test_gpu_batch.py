"""GPU parity of the batched level step (persistent kernels over a (box,
tile) work list, replayed as a HIP graph) against the oracle's level step."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2110_01792_amd import binding as qb
from paper_2110_01792_amd import inputs
from tests.gpu_util import dev, host, norm_l1, rel_linf, worst_cell

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = qb.Context(0)
    yield c
    c.close()


def run_gpu(ctx, boxes, Ugs, Urs, hp, p, nsteps=1, dtype=None, check=None):
    torch = pytest.importorskip("torch")
    dtype = dtype or torch.float64
    G = [dev(u, dtype) for u in Ugs]
    R = [None if u is None else dev(u, dtype) for u in Urs]
    rp = qb.rad_params(p)
    dts = []
    for s in range(nsteps):
        dts.append(ctx.batch_step(boxes, G, R, qb.hydro_params(hp["gamma"], hp["cfl"]), rp))
        if check is not None:
            check(s, [host(g) for g in G], [None if r is None else host(r) for r in R])
    assert ctx.sync_status() == qb.QK_OK
    return [host(g) for g in G], [None if r is None else host(r) for r in R], dts


def compare(boxes, gG, gR, oG, oR, tol=TOL, what=""):
    for k, b in enumerate(boxes):
        e = rel_linf(gG[k], oG[k], b)
        assert np.all(e <= tol), (what, "gas", k, b.n, e, worst_cell(gG[k], oG[k], b))
        if oR[k] is not None:
            e = rel_linf(gR[k], oR[k], b)
            assert np.all(e <= tol), (what, "rad", k, b.n, e, worst_cell(gR[k], oR[k], b))


def test_batch_small_level_matches_oracle_over_graph_replays(ctx):
    """12 uneven boxes (edges 8..24, half with radiation): three level steps,
    i.e. one capture and two replays, each compared with the oracle."""
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=12, seed=31, edges=(8, 16, 24))
    oG = [u.copy() for u in Ugs]
    oR = [None if u is None else u.copy() for u in Urs]
    odts = []

    def check(s, gG, gR):
        st = oracle.batch_step(boxes, oG, oR, hp["gamma"], hp["cfl"], p)
        odts.append(st["dt"])
        compare(boxes, gG, gR, oG, oR, what=f"step {s}")

    gG, gR, dts = run_gpu(ctx, boxes, Ugs, Urs, hp, p, nsteps=3, check=check)
    for a, b in zip(dts, odts):
        assert abs(a - b) <= 1e-14 * b
    tile, zc, _ = ctx.batch_config()
    assert tile in (8, 14, 16) and zc >= 1


def test_batch_hydro_only_equals_single_box_runs_bitwise(ctx):
    """A batched box and the same box advanced alone with the level dt give the
    same bits (same per-tile device code, fixed ghosts read in place)."""
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=8, seed=32, edges=(8, 24, 40), rad_fraction=0.0)
    gG, gR, dts = run_gpu(ctx, boxes, Ugs, Urs, hp, p, nsteps=1)
    hpp = qb.hydro_params(hp["gamma"], hp["cfl"])
    for k, b in enumerate(boxes):
        U = dev(Ugs[k])
        ctx.hydro_step(b, U, hpp, dt=dts[0])
        assert np.array_equal(host(U), gG[k]), (k, b.n)


def test_batch_plm_equals_single_box_runs_bitwise(ctx):
    """PLM (reconstruction 1) through the batched level: each box equals the
    same box advanced alone with the level dt."""
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=6, seed=35, edges=(8, 16, 24), rad_fraction=0.0)
    G = [dev(u) for u in Ugs]
    hpp = qb.hydro_params(hp["gamma"], hp["cfl"], recon=1)
    dt = ctx.batch_step(boxes, G, [None] * len(boxes), hpp, qb.rad_params(p))
    assert ctx.sync_status() == qb.QK_OK
    for k, b in enumerate(boxes):
        U = dev(Ugs[k])
        ctx.hydro_step(b, U, hpp, dt=dt)
        assert np.array_equal(host(U), host(G[k])), (k, b.n)


def test_batch_full_level_sampled_against_oracle(ctx):
    """The benchmark's batched level at full size (600 boxes, edges
    {8..64}, half RHD): every box advanced on the GPU in one graph; a sample
    of boxes advanced by the oracle alone with the level dt and N_sub."""
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=600, seed=5)
    gG, gR, dts = run_gpu(ctx, boxes, Ugs, Urs, hp, p, nsteps=1)
    # level dt and substep count from the oracle's definitions
    sig = [oracle.hydro_max_signal(b, u, p["gamma"] if r is not None else hp["gamma"])
           for b, u, r in zip(boxes, Ugs, Urs)]
    dt = min(hp["cfl"] * min(b.dx) / s for b, s in zip(boxes, sig))
    dt_r = p["cfl"] * min(boxes[0].dx) / p["chat"]
    n = int(np.ceil(dt / dt_r))
    if n > p["nsub_max"]:
        n, dt = p["nsub_max"], p["nsub_max"] * dt_r
    assert abs(dts[0] - dt) <= 1e-14 * dt
    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(len(boxes), size=12, replace=False).tolist() + [int(np.argmax(
        [b.ncells for b in boxes]))])
    for k in sample:
        b, g, r = boxes[k], Ugs[k].copy(), None if Urs[k] is None else Urs[k].copy()
        oracle.hydro_step(b, g, p["gamma"] if r is not None else hp["gamma"], hp["cfl"], dt)
        if r is not None:
            for _ in range(n):
                oracle.rad_transport_substep(b, r, g, p, dt / n)
                oracle.exchange_all(b, g, r, p, dt / n)
        compare([b], [gG[k]], [gR[k]], [g], [r], what=f"box {k}")


def test_batch_mixed_precision_error(ctx):
    """FP32 state and flux arithmetic (FP64 internal energy, exchange and stage
    sums) against the FP64 oracle started from the same FP32-rounded data:
    per-variable normalised L1 within 1e-5, except the radiation flux, held to
    2e-5.  F starts at zero and after two steps is a small field driven by
    differences of E_r, so the FP32 rounding of the stored E_r dominates its
    error (the same floor as on the 256^3 RHD workload)."""
    torch = pytest.importorskip("torch")
    boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=10, seed=33, edges=(8, 16, 24))
    Ugs = [inputs.to_f32_and_back(u) for u in Ugs]
    Urs = [None if u is None else inputs.to_f32_and_back(u) for u in Urs]
    gG, gR, _ = run_gpu(ctx, boxes, Ugs, Urs, hp, p, nsteps=2, dtype=torch.float32)
    oG = [u.copy() for u in Ugs]
    oR = [None if u is None else u.copy() for u in Urs]
    for _ in range(2):
        oracle.batch_step(boxes, oG, oR, hp["gamma"], hp["cfl"], p)
    for k, b in enumerate(boxes):
        # per variable, sum |g - o| / sum |o| (momenta and F included)
        eg = norm_l1(gG[k], oG[k], b)
        assert np.all(eg <= 1e-5), (k, eg)
        if oR[k] is not None:
            er = norm_l1(gR[k], oR[k], b)
            assert er[0] <= 1e-5 and np.all(er[1:] <= 2e-5), (k, er)


def test_batch_alternating_lists_on_side_streams(ctx):
    """Two box lists stepped alternately on two non-default streams with no
    host synchronisation between calls: every call re-plans (the cached graph
    belongs to the other list) while the previous replay may still run, and a
    call on the other stream must wait for it.  After five calls each level
    equals the oracle's level steps."""
    torch = pytest.importorskip("torch")
    levels = []
    for seed, nbox, edges in ((41, 9, (8, 16, 24)), (42, 6, (8, 16))):
        boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=nbox, seed=seed, edges=edges)
        levels.append(dict(boxes=boxes, p=p, hp=hp, G=[dev(u) for u in Ugs],
                           R=[None if u is None else dev(u) for u in Urs],
                           oG=[u.copy() for u in Ugs], oR=[None if u is None else u.copy() for u in Urs]))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    order = [(0, 0), (1, 0), (0, 1), (1, 1), (0, 0)]
    for lv, si in order:
        L, s = levels[lv], streams[si]
        with torch.cuda.stream(s):
            ctx.batch_step(L["boxes"], L["G"], L["R"], qb.hydro_params(L["hp"]["gamma"], L["hp"]["cfl"]),
                           qb.rad_params(L["p"]), host_dt=False, stream=s.cuda_stream)
        oracle.batch_step(L["boxes"], L["oG"], L["oR"], L["hp"]["gamma"], L["hp"]["cfl"], L["p"])
    for s in streams:
        s.synchronize()
    assert ctx.sync_status() == qb.QK_OK
    for lv, L in enumerate(levels):
        compare(L["boxes"], [host(g) for g in L["G"]], [None if r is None else host(r) for r in L["R"]],
                L["oG"], L["oR"], what=f"level {lv}")


def test_batch_autotune_cache_file(tmp_path):
    """The autotuner writes its choice to the JSON file named by QK_TUNE_CACHE
    and a new context reads it back."""
    path = tmp_path / "tune.json"
    os.environ["QK_TUNE_CACHE"] = str(path)
    try:
        boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=5, seed=34, edges=(8, 16))
        c1 = qb.Context(0)
        run_gpu(c1, boxes, Ugs, Urs, hp, p)
        t1 = c1.batch_config()
        c1.close()
        data = json.loads(path.read_text())
        assert len(data["quokka_batch_autotune"]) == 1
        c2 = qb.Context(0)
        run_gpu(c2, boxes, Ugs, Urs, hp, p)
        t2 = c2.batch_config()
        c2.close()
        assert t1[:2] == t2[:2] and t2[2] == 0.0  # read from the file, not re-tuned
    finally:
        del os.environ["QK_TUNE_CACHE"]


@pytest.mark.parametrize("tile", [8, 14, 16])
def test_every_tile_family(tile, tmp_path):
    """Each tile family (8 x 8, 16 x 14 with split buffers, 16 x 16), forced
    through the autotuner's cache file: a level step of hydro and RHD boxes
    matches the oracle's level step, and every hydro-only box equals the same
    box advanced alone with the level dt, bit for bit."""
    path = tmp_path / "tune.json"
    os.environ["QK_TUNE_CACHE"] = str(path)
    try:
        boxes, Ugs, Urs, p, hp = inputs.batch_level(nbox=8, seed=36, edges=(8, 16, 24, 40))
        c0 = qb.Context(0)
        run_gpu(c0, boxes, Ugs, Urs, hp, p)  # tunes once and writes the signature's key
        c0.close()
        entry = json.loads(path.read_text())["quokka_batch_autotune"][0]
        path.write_text(json.dumps({"quokka_batch_autotune": [dict(entry, tile=tile, zc=16)]}))
        c = qb.Context(0)
        gG, gR, dts = run_gpu(c, boxes, Ugs, Urs, hp, p)
        assert c.batch_config()[:2] == (tile, 16)
        oG = [u.copy() for u in Ugs]
        oR = [None if u is None else u.copy() for u in Urs]
        st = oracle.batch_step(boxes, oG, oR, hp["gamma"], hp["cfl"], p)
        assert abs(dts[0] - st["dt"]) <= 1e-14 * st["dt"]
        compare(boxes, gG, gR, oG, oR, what=f"tile {tile}")
        hpp = qb.hydro_params(hp["gamma"], hp["cfl"])
        for k, b in enumerate(boxes):
            if Urs[k] is None:
                U = dev(Ugs[k])
                c.hydro_step(b, U, hpp, dt=dts[0])
                assert np.array_equal(host(U), gG[k]), (tile, k, b.n)
        c.close()
    finally:
        del os.environ["QK_TUNE_CACHE"]


def test_batch_rejects_non_fixed_ghosts(ctx):
    torch = pytest.importorskip("torch")
    b = inputs.make_box(8)
    U = torch.zeros((5,) + b.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(qb.QuokkaError) as e:
        ctx.batch_step([b], [U], [None], qb.hydro_params(1.4, 0.3), None)
    assert e.value.status == qb.QK_EINVAL
