"""FP64 parity: the HIP path through the C ABI against the CPU oracle.

Both sides get the same host FP64 arrays from the shared input module.  The
bar (stated for FP64 results after 1000 steps): max relative error 1e-11 in
rho and T (pointwise) and in u (normalised by max |u| of the oracle, since u
vanishes in places).  The arithmetic differs only in rounding order and FMA
contraction, so the two agree to a few ulp per step.
"""

import numpy as np
import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _gpu():
    from paper_1709_04400_amd import lbpc
    return lbpc


def _errors(a, b):
    (r1, ux1, uy1, T1), (r2, ux2, uy2, T2) = a, b
    umax = max(np.abs(ux2).max(), np.abs(uy2).max(), 1e-300)
    return dict(
        rho=float(np.max(np.abs(r1 - r2) / np.abs(r2))),
        T=float(np.max(np.abs(T1 - T2) / np.abs(T2))),
        u=float(max(np.abs(ux1 - ux2).max(), np.abs(uy1 - uy2).max()) / umax))


def run_pair(cfg, fields, steps, chunks=1):
    print(f"\n[parity] {cfg['nx']}x{cfg['ny']} bc={cfg['bc']} "
          f"prec={cfg['precision']} steps={steps}", flush=True)
    o = O.Oracle(cfg)
    o.init_fields(**fields)
    g = _gpu().Simulation(cfg)
    g.init_fields(fields["rho"], fields["ux"], fields["uy"], fields["T"])
    errs = []
    per = steps // chunks
    for _ in range(chunks):
        o.step(per)
        g.step(per)
        errs.append(_errors(g.rho_u_T(), o.rho_u_T()))
    g.close()
    print(f"[parity] errors {errs[-1]}", flush=True)
    return errs


def _assert_ok(errs, tol=TOL):
    for e in errs:
        assert e["rho"] < tol and e["T"] < tol and e["u"] < tol, e


def test_init_matches_oracle_exactly_at_step0():
    cfg, fl = I.static_droplet(40, 36, 10.0)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    g = _gpu().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    e = _errors(g.rho_u_T(), o.rho_u_T())
    g.close()
    assert e["rho"] < 1e-15 and e["T"] < 1e-15, e


def test_static_droplet_1000_steps():
    """Static droplet: 100 x 100 periodic, R = 25, 1000 steps."""
    cfg, fl = I.static_droplet(100, 100, 25.0)
    _assert_ok(run_pair(cfg, fl, 1000, chunks=4))


def test_evaporation_cut_open_sides():
    """128 x 128 cut of the evaporation case: four open fixed-T sides."""
    cfg, fl = I.evaporation(128, 128 / 6.0, 1.1)
    _assert_ok(run_pair(cfg, fl, 1000, chunks=2))


def test_bubble_cut_walls_hot_spot_gravity():
    """128 x 128 cut of the boiling case: periodic x, walls in y, hot spot,
    buoyancy, lambda = rho c_V chi."""
    cfg, fl = I.bubble(nx=128, ny=128, pool=96, hot_width=14, g=3e-5)
    _assert_ok(run_pair(cfg, fl, 1000, chunks=2))


def test_random_distinct_rates():
    """Every MRT rate distinct and off 1, so no moment path is masked."""
    sf, sg = I.random_rates(18)
    sg[5] = sg[3]
    cfg, fl = I.static_droplet(64, 64, 16.0)
    cfg.update(s_f=sf, s_g=sg, gx=2e-5, gy=-1e-5)
    _assert_ok(run_pair(cfg, fl, 1000, chunks=2))


def test_compromised_model():
    cfg, fl = I.static_droplet(64, 48, 14.0)
    cfg.update(thermal_model=I.THERMAL_COMPROMISED,
               bc=[I.BC_WALL, I.BC_WALL, I.BC_OPEN, I.BC_OPEN],
               T_bc=[1.05 * I.T_SAT, 1.02 * I.T_SAT, 1.1 * I.T_SAT,
                     1.0 * I.T_SAT])
    _assert_ok(run_pair(cfg, fl, 400))


@pytest.mark.parametrize("tile_h", [16, 37])
def test_ragged_tiles_many_blocks(monkeypatch, tile_h):
    """nx = 300 needs two strips of 252 columns (ragged second strip); small
    row runs give many blocks with ragged last runs."""
    monkeypatch.setenv("LBPC_TILE_H", str(tile_h))
    cfg, fl = I.evaporation(300, 40.0, 1.1)
    cfg.update(ny=150, bc=[I.BC_PERIODIC, I.BC_PERIODIC, I.BC_WALL, I.BC_OPEN],
               hot_x0=120, hot_x1=180, T_hot=1.15 * I.T_SAT, gy=-2e-5)
    fl = I.droplet_fields(300, 150, 40.0)
    _assert_ok(run_pair(cfg, fl, 200))


def test_save_load_roundtrip_matches_uninterrupted():
    cfg, fl = I.bubble(nx=64, ny=64, pool=40, hot_width=8)
    g = _gpu().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(30)
    st = g.save_state()
    g.step(20)
    ref = g.rho_u_T()
    g2 = _gpu().Simulation(cfg)
    g2.load_state(st)
    g2.step(20)
    out = g2.rho_u_T()
    for a, b in zip(ref, out):
        assert np.array_equal(a, b)
    # the saved state is the oracle's canonical state
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(30)
    ost = o.get_state()
    n = cfg["nx"] * cfg["ny"]
    f = st[:9 * n * 8].view(np.float64).reshape(9, cfg["ny"], cfg["nx"])
    assert np.max(np.abs(f - ost["f"])) < 1e-12
    g.close()
    g2.close()


DIAG_KEYS = ("mass", "sum_T", "sum_rhocvT", "liquid_area", "radius",
             "max_speed")


@pytest.mark.parametrize("case", ["open", "walls_tiled", "bgk"])
def test_diag_matches_oracle(case):
    """The no-store diagnostic pass (lbpc_get_diag) and the diagnostic step
    (lbpc_step_diag) against the oracle's sums at the same level; sum S0 of
    the step from a level is the oracle's S0 sum of that step."""
    if case == "open":
        cfg, fl = I.evaporation(96, 20.0, 1.1)
    elif case == "walls_tiled":
        cfg, fl = I.bubble(nx=96, ny=80, pool=50, hot_width=10, g=3e-5)
    else:
        cfg, fl = I.static_droplet(72, 64, 15.0)
        cfg.update(thermal_model=I.THERMAL_IMPROVED_BGK, gy=-2e-5)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    g = _gpu().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    o.step(100)
    g.step(100)
    do, dg = o.diag(), g.diag()
    ds = g.step_diag(3)          # level 100, then on to 103
    o.step(1)
    do1 = o.diag()               # its sum_S0: the step 100 -> 101
    o.step(2)
    dend, gend = o.diag(), g.diag()
    g.close()
    for k in DIAG_KEYS:
        assert np.isclose(dg[k], do[k], rtol=1e-11, atol=1e-14), k
        assert dg[k] == ds[k], k     # same reduction, same order
        assert np.isclose(gend[k], dend[k], rtol=1e-11, atol=1e-14), k
    assert dg["radius_count"] == do["radius_count"] == ds["radius_count"]
    assert np.isclose(dg["sum_S0"], do1["sum_S0"], rtol=1e-9, atol=1e-15)
    assert ds["sum_S0"] == dg["sum_S0"]
    assert dg["step"] == ds["step"] == 100 and gend["step"] == 103
    assert not dg["nonfinite"] and not ds["nonfinite"]


def test_diag_is_deterministic_and_budget_closes():
    """Two runs give bitwise the same diagnostics; on a periodic lattice
    sum T of the next level is sum T + sum S0 (Eq. 46: the collision changes
    the zeroth thermal moment by S0 only, streaming permutes)."""
    cfg, fl = I.static_droplet(128, 96, 20.0)
    cfg.update(gy=-1e-5, s_g=[1.0, 1.2, 0.9, 1.1, 1.3, 1.1, 0.8, 1.05, 0.95])
    runs = []
    for _ in range(2):
        g = _gpu().Simulation(cfg)
        g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
        g.step(7)
        runs.append([g.step_diag(1) for _ in range(4)])
        g.close()
    assert runs[0] == runs[1]
    for a, b in zip(runs[0], runs[0][1:]):
        assert np.isclose(b["sum_T"], a["sum_T"] + a["sum_S0"], rtol=1e-13,
                          atol=1e-13)


@pytest.mark.parametrize("which", ["periodic", "walls"])
def test_autotune_and_tiles_leave_results_unchanged(which):
    """Tile shape is a schedule, not arithmetic: any shape and a mid-run
    autotune give bitwise the same fields."""
    cfg, fl = I.static_droplet(100, 100, 25.0)
    if which == "walls":
        cfg.update(bc=[I.BC_WALL] * 4, T_bc=[1.1 * I.T_SAT] * 4)
    ref = _gpu().Simulation(cfg)
    ref.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    ref.step(40)
    out = ref.rho_u_T()
    ref.close()
    g = _gpu().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.set_tiles(64, 7)
    g.step(9)
    g.set_tiles(512, 11)
    g.step(6)
    res = g.autotune(steps=2)
    assert res["block_width"] in (64, 128, 256, 512) and res["rows"] >= 4
    g.step(25)
    for a, b in zip(g.rho_u_T(), out):
        assert np.array_equal(a, b)
    g.close()


@pytest.mark.parametrize("prec", [I.FP64, I.FP16_LOCAL])
@pytest.mark.parametrize("which", ["periodic", "walls"])
def test_graph_replay_equals_eager(monkeypatch, which, prec):
    """Steady steps replayed from the captured two-step graph match launches
    one by one, bitwise, through odd step counts, reads, a tile change, an
    autotune and a save / load (FP64, and the node-referenced FP16 form with
    its rest and reference arrays)."""
    cfg, fl = I.bubble(nx=200, ny=96, pool=60, hot_width=16, g=3e-5,
                       precision=prec)
    if which == "periodic":
        cfg["bc"] = [I.BC_PERIODIC] * 4
    sims = []
    for graph in ("0", "1"):
        monkeypatch.setenv("LBPC_GRAPH", graph)
        g = _gpu().Simulation(cfg)
        g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
        sims.append(g)
    eager, graph = sims
    st = None
    for k, chunk in enumerate((1, 4, 3, 6, 2, 5, 8)):
        for g in sims:
            g.step(chunk)
        for x, y in zip(eager.rho_u_T(), graph.rho_u_T()):
            assert np.array_equal(x, y), (chunk, k)
        if k == 2:
            for g in sims:
                g.set_tiles(128, 20)
        if k == 3:
            for g in sims:
                g.autotune(1)
        if k == 4:
            st = graph.save_state()
    graph.load_state(st)
    eager.load_state(st)
    for g in sims:
        g.step(9)
    for x, y in zip(eager.rho_u_T(), graph.rho_u_T()):
        assert np.array_equal(x, y)
    for g in sims:
        g.close()


def test_diagnostics_log(tmp_path):
    """run(): diagnostics every K steps as records and JSON lines; mass is
    conserved on a periodic lattice and sum T follows the oracle."""
    import json
    cfg, fl = I.static_droplet(64, 48, 12.0)
    g = _gpu().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    m0 = g.diag()["mass"]
    path = tmp_path / "diag.jsonl"
    recs = g.run(100, 30, log=str(path))
    g.close()
    assert [r["step"] for r in recs] == [30, 60, 90, 100]
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert lines == recs
    assert max(abs(r["mass"] - m0) / m0 for r in recs) < 1e-12
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(100)
    assert np.isclose(recs[-1]["sum_T"], o.diag()["sum_T"], rtol=1e-12)
    b = _gpu().Batch([cfg, I.heated_droplet(40, 8.0, 1.1)[0]])
    b.init_fields(0, fl["rho"], fl["ux"], fl["uy"], fl["T"])
    f1 = I.heated_droplet(40, 8.0, 1.1)[1]
    b.init_fields(1, f1["rho"], f1["ux"], f1["uy"], f1["T"])
    brec = b.run(50, 25)
    b.close()
    assert [(r["lattice"], r["step"]) for r in brec] == \
        [(0, 25), (1, 25), (0, 50), (1, 50)]
