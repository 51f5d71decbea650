"""The batched form: many lattices of uneven size in one persistent launch per
step, hipGraph-captured steps and the tile autotuner, through the C ABI."""

import numpy as np
import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I

pytestmark = pytest.mark.gpu


def _lb():
    from paper_1709_04400_amd import lbpc
    return lbpc


def _mixed_fp64():
    """Lattices of different sizes, sides and models."""
    out = []
    c, f = I.static_droplet(72, 60, 14.0)
    out.append((c, f))
    c, f = I.evaporation(96, 19.0, 1.15)
    out.append((c, f))
    c, f = I.bubble(nx=80, ny=64, pool=44, hot_width=10, g=3e-5)
    out.append((c, f))
    c, f = I.static_droplet(40, 90, 10.0)
    c.update(bc=[I.BC_WALL, I.BC_WALL, I.BC_OPEN, I.BC_OPEN],
             T_bc=[1.05 * I.T_SAT, 1.0 * I.T_SAT, 1.1 * I.T_SAT, I.T_SAT],
             thermal_model=I.THERMAL_COMPROMISED)
    out.append((c, f))
    return out


def _batch(cases, **tiles):
    b = _lb().Batch([c for c, _ in cases])
    for k, (_, f) in enumerate(cases):
        b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    if tiles:
        b.set_tiles(tiles["bw"], tiles["rows"])
    return b


@pytest.mark.parametrize("bw,rows", [(256, 32), (64, 13)])
def test_every_lattice_matches_the_oracle(bw, rows):
    cases = _mixed_fp64()
    print(f"\n[batch] fp64 mixed, tiles {bw}x{rows}", flush=True)
    b = _batch(cases, bw=bw, rows=rows)
    b.step(201)   # odd: graph pairs plus one eager step
    for k, (cfg, f) in enumerate(cases):
        o = O.Oracle(cfg)
        o.init_fields(**f)
        o.step(201)
        (r1, ux1, uy1, T1), (r2, ux2, uy2, T2) = b.rho_u_T(k), o.rho_u_T()
        umax = max(np.abs(ux2).max(), np.abs(uy2).max())
        assert np.max(np.abs(r1 - r2) / r2) < 1e-11, k
        assert np.max(np.abs(T1 - T2) / T2) < 1e-11, k
        assert max(np.abs(ux1 - ux2).max(), np.abs(uy1 - uy2).max()) \
            < 1e-11 * umax, k
    b.close()


@pytest.mark.parametrize("prec", [I.FP32, I.FP32_SHIFTED, I.FP16_SHIFTED,
                                  I.FP16_LOCAL])
def test_batch_equals_single_handles_bitwise(prec):
    """Every lattice of a batch is bitwise the same lattice run alone (the
    arithmetic of a node does not depend on the tiling), in each storage form
    whose (f, g) pairs and rest arrays the batch lays out per lattice."""
    print(f"\n[batch] batch vs single handles precision={prec}", flush=True)
    cases = I.batch_cases(count=5, seed=11, precision=prec)
    b = _batch(cases)
    b.step(60)
    for k, (cfg, f) in enumerate(cases):
        s = _lb().Simulation(cfg)
        s.init_fields(f["rho"], f["ux"], f["uy"], f["T"])
        s.step(60)
        for x, y in zip(s.rho_u_T(), b.rho_u_T(k)):
            assert np.array_equal(x, y), k
        s.close()
    b.close()


def test_graph_replay_equals_eager(monkeypatch):
    """Replays of the captured two-step graph, interleaved with eager steps
    and synchronising reads, match a batch that never uses graphs."""
    cases = I.batch_cases(count=6, seed=5, precision=I.FP32_SHIFTED)
    monkeypatch.setenv("LBPC_BATCH_GRAPH", "0")
    eager = _batch(cases)
    monkeypatch.setenv("LBPC_BATCH_GRAPH", "1")
    graph = _batch(cases)
    for chunk in (1, 4, 3, 6, 2, 5):   # graph pairs with eager odd steps
        eager.step(chunk)
        graph.step(chunk)
        for k in range(len(cases)):
            for x, y in zip(eager.rho_u_T(k), graph.rho_u_T(k)):
                assert np.array_equal(x, y), (chunk, k)
    eager.close()
    graph.close()


def test_autotune_picks_a_shape_and_leaves_the_state():
    """Tuning before the first step and again mid-run (steady state) changes
    nothing in the results."""
    cases = I.batch_cases(count=6, seed=8, precision=I.FP32)
    tuned = _batch(cases)
    res = tuned.autotune(steps=2)
    assert res["block_width"] in (64, 128, 256) and res["rows"] >= 4
    assert res["ms_per_step"] > 0
    plain = _batch(cases)
    tuned.step(17)
    plain.step(17)
    res2 = tuned.autotune(steps=2)
    assert res2["ms_per_step"] > 0
    tuned.step(13)
    plain.step(13)
    for k in range(len(cases)):
        for x, y in zip(tuned.rho_u_T(k), plain.rho_u_T(k)):
            assert np.array_equal(x, y), k
    tuned.close()
    plain.close()


def test_diag_per_lattice():
    cases = _mixed_fp64()[:2]
    b = _batch(cases)
    b.step(50)
    for k, (cfg, f) in enumerate(cases):
        o = O.Oracle(cfg)
        o.init_fields(**f)
        o.step(50)
        do, db = o.diag(), b.diag(k)
        assert np.isclose(db["mass"], do["mass"], rtol=1e-12)
        assert np.isclose(db["sum_T"], do["sum_T"], rtol=1e-12)
        assert np.isclose(db["liquid_area"], do["liquid_area"], rtol=1e-11)
        assert np.isclose(db["max_speed"], do["max_speed"], rtol=1e-10)
        assert db["step"] == 50
    # the diagnostic step gives every lattice's record of the same level,
    # bitwise the no-store pass's (same kernel, same reduction order)
    before = [b.diag(k) for k in range(len(cases))]
    recs = b.step_diag(2)
    assert recs == before
    for k in range(len(cases)):
        assert recs[k]["step"] == 50 and b.diag(k)["step"] == 52
    b.close()


def test_batch_sweep_sample_runs_clean():
    """A slice of the 256-lattice sweep (same seed and draws): finite after
    500 steps, and the mass of each open lattice within 10 % of its start."""
    cases = I.batch_cases(count=256, seed=1709, precision=I.FP32)[:24]
    b = _batch(cases)
    m0 = [b.diag(k)["mass"] for k in range(len(cases))]
    b.step(500)
    for k in range(len(cases)):
        d = b.diag(k)
        assert not d["nonfinite"]
        assert abs(d["mass"] - m0[k]) / m0[k] < 0.1
    b.close()
