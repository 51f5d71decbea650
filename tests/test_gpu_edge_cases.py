"""Edge cases of the step on the GPU, each against the oracle: the smallest
lattices the library accepts (4 nodes on a side, where the two-node halo of a
tile wraps onto the lattice itself or meets both walls of an axis at once),
thin lattices (one tile row or one strip, ragged), every kind of side on
them, a hot spot and wetting on a 4 x 4 box, the reduced-precision forms
there, n = 0 steps, and a batch that mixes the smallest lattices with a
larger one."""
import numpy as np
import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I
from test_gpu_parity import TOL, _errors

pytestmark = pytest.mark.gpu

P, W, OP = I.BC_PERIODIC, I.BC_WALL, I.BC_OPEN
SIDES = {"periodic": [P] * 4, "walls": [W] * 4, "y_walls": [P, P, W, W],
         "x_walls": [W, W, P, P], "wall_open": [P, P, W, OP]}


def _lb():
    from paper_1709_04400_amd import lbpc
    return lbpc


# Velocities on these lattices stay near 1e-6, so a velocity difference is
# judged against the rounding of j = sum_a e_a f_a (about 1e-16 absolute,
# whatever |v| is) with a floor of 1e-14 on top of the relative tolerance;
# rho and T keep the relative one.
U_FLOOR = 1e-14


def _check(a, b, tol=TOL):
    (r1, ux1, uy1, T1), (r2, ux2, uy2, T2) = a, b
    e_rho = float(np.max(np.abs(r1 - r2) / r2))
    e_T = float(np.max(np.abs(T1 - T2) / T2))
    umax = max(np.abs(ux2).max(), np.abs(uy2).max())
    du = max(np.abs(ux1 - ux2).max(), np.abs(uy1 - uy2).max())
    assert e_rho < tol and e_T < tol and du < tol * umax + U_FLOOR, \
        (e_rho, e_T, du, umax)


def _run_pair(cfg, fl, steps, chunks=2):
    print(f"\n[edge] {cfg['nx']}x{cfg['ny']} bc={cfg['bc']} steps={steps}",
          flush=True)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    g = _lb().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    for _ in range(chunks):
        o.step(steps // chunks)
        g.step(steps // chunks)
        _check(g.rho_u_T(), o.rho_u_T())
    g.close()


def _cut(nx, ny, sides, precision=I.FP64):
    """The spinodal recipe (seeded noise on rho and T) cut to nx x ny."""
    cfg, fl = I.spinodal(max(nx, ny), precision=precision)
    fl = {k: np.ascontiguousarray(v[:ny, :nx]) for k, v in fl.items()}
    cfg.update(nx=nx, ny=ny, bc=list(SIDES[sides]))
    return cfg, fl


@pytest.mark.parametrize("sides", list(SIDES))
@pytest.mark.parametrize("shape", [(4, 4), (4, 37), (37, 4), (5, 6)])
def test_smallest_and_thin_lattices(shape, sides):
    cfg, fl = _cut(*shape, sides)
    _run_pair(cfg, fl, 60)


def test_smallest_box_hot_spot_wetting_variable_conductivity():
    cfg, fl = _cut(4, 4, "walls")
    cfg.update(hot_x0=1, hot_x1=3, T_hot=1.1 * I.T_SAT, wet_amp=0.1,
               wet_shift=0.05, lambda_mode=I.LAMBDA_RHO_CV_CHI,
               chi=I.CHI_BUBBLE)
    _run_pair(cfg, fl, 60)


# the short-run bounds of the other reduced-precision parity tests
SHORT = {I.FP32: 3e-5, I.FP32_SHIFTED: 3e-5, I.FP16_SHIFTED: 2e-2,
         I.FP16_LOCAL: 2e-3}


@pytest.mark.parametrize("prec", [I.FP32, I.FP32_SHIFTED, I.FP16_SHIFTED,
                                  I.FP16_LOCAL])
@pytest.mark.parametrize("sides", ["periodic", "walls"])
def test_smallest_lattice_reduced_precision(prec, sides):
    cfg, fl = _cut(4, 4, sides)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(60)
    g = _lb().Simulation(dict(cfg, precision=prec))
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(60)
    e = _errors(g.rho_u_T(), o.rho_u_T())
    g.close()
    assert e["rho"] < SHORT[prec] and e["T"] < SHORT[prec], e


def test_memory_probe_leaves_the_state_and_refuses_narrow_tiles():
    """lbpc_memory_probe times the step's memory schedule on the periodic
    kernel's default block widths and leaves the state as it was; on 64- or
    128-thread tiles (no probe kernel is built for them) and on a walled
    lattice it reports LBPC_ERR_UNSUPPORTED."""
    lb = _lb()
    cfg, fl = I.static_droplet(300, 40, 10.0)
    for prec in (I.FP64, I.FP16_LOCAL):
        g = lb.Simulation(dict(cfg, precision=prec))
        g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
        g.step(3)
        s0 = g.save_state()
        assert g.memory_probe(2) > 0.0
        assert np.array_equal(g.save_state(), s0)
        for bw in (64, 128):
            g.set_tiles(bw, 8)
            with pytest.raises(lb.LbpcError) as e:
                g.memory_probe(2)
            assert e.value.status == lb.ERR_UNSUPPORTED
        g.close()
    w = lb.Simulation(dict(cfg, bc=[I.BC_WALL] * 4))
    w.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    with pytest.raises(lb.LbpcError) as e:
        w.memory_probe(2)
    assert e.value.status == lb.ERR_UNSUPPORTED
    w.close()


def test_zero_steps_change_nothing():
    """lbpc_step with n = 0 (and lbpc_batch_step) leaves state, history and
    step count as they were, and the run continues bitwise as if it had not
    been called."""
    lb = _lb()
    cfg, fl = I.static_droplet(40, 36, 10.0)
    runs = []
    for zero in (False, True):
        g = lb.Simulation(cfg)
        g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
        g.step(3)
        if zero:
            s0, k0 = g.save_state(), g.diag()["step"]
            g.step(0)
            assert np.array_equal(g.save_state(), s0)
            assert g.diag()["step"] == k0 == 3
        g.step(4)
        runs.append(g.save_state())
        g.close()
    assert np.array_equal(runs[0], runs[1])

    b = lb.Batch([cfg, I.heated_droplet(32, 8.0, 1.1)[0]])
    b.init_fields(0, fl["rho"], fl["ux"], fl["uy"], fl["T"])
    f1 = I.heated_droplet(32, 8.0, 1.1)[1]
    b.init_fields(1, f1["rho"], f1["ux"], f1["uy"], f1["T"])
    b.step(2)
    before = [b.rho_u_T(k) for k in range(2)]
    b.step(0)
    for k in range(2):
        for x, y in zip(before[k], b.rho_u_T(k)):
            assert np.array_equal(x, y)
    b.close()


def test_batch_mixing_smallest_and_larger_lattices():
    """The persistent batch launch with 4 x 4 and thin lattices beside a
    130 x 130 walled droplet: every lattice matches its own oracle run."""
    cases = [_cut(4, 4, "periodic"), _cut(4, 4, "walls"),
             _cut(5, 6, "wall_open"), _cut(37, 4, "x_walls"),
             _cut(4, 37, "y_walls"), I.heated_droplet(130, 30.0, 1.1)]
    b = _lb().Batch([c for c, _ in cases])
    for k, (_, f) in enumerate(cases):
        b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    b.step(60)
    for k, (cfg, f) in enumerate(cases):
        o = O.Oracle(cfg)
        o.init_fields(**f)
        o.step(60)
        print(f"[edge] batch lattice {k}", flush=True)
        _check(b.rho_u_T(k), o.rho_u_T())
    b.close()


def _with_env(env, fn):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("prec", [I.FP64, I.FP32, I.FP16_SHIFTED,
                                  I.FP16_LOCAL])
def test_shorter_runs_in_the_x_edge_strips(prec):
    """Strips holding walls on the x sides with their own run height (13
    rows against 24 elsewhere, 128-thread blocks: 3 strips, so runs of
    different heights meet along both strip boundaries) on a walled
    boiling cut with a hot spot: the same result as the oracle.  FP64 and
    the FP16 forms take the separate height; the FP32 forms keep one for
    every strip."""
    cfg, fl = _cut(300, 200, "walls")
    cfg.update(hot_x0=140, hot_x1=160, T_hot=1.1 * I.T_SAT,
               lambda_mode=I.LAMBDA_RHO_CV_CHI, chi=I.CHI_BUBBLE,
               precision=prec)
    o = O.Oracle(dict(cfg, precision=I.FP64))
    o.init_fields(**fl)
    o.step(60)
    g = _with_env({"LBPC_TILE_BW": 128, "LBPC_TILE_H": 24,
                   "LBPC_TILE_HE": 13}, lambda: _lb().Simulation(cfg))
    edge = 24 if prec in (I.FP32, I.FP32_SHIFTED) else 13
    assert g.tiles() == {"block_width": 128, "rows": 24, "rows_edge": edge}
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(60)
    if prec == I.FP64:
        _check(g.rho_u_T(), o.rho_u_T())
    else:
        e = _errors(g.rho_u_T(), o.rho_u_T())
        assert e["rho"] < SHORT[prec] and e["T"] < SHORT[prec], e
    g.close()


def test_default_tiles_on_a_wide_walled_lattice():
    """1530 x 1100 FP64 walled on all sides with its default tiles (four
    512-thread strips, runs sized to fill whole waves): five steps agree with
    the oracle over the whole lattice."""
    cfg, fl = _cut(1530, 1100, "walls")
    g = _lb().Simulation(cfg)
    t = g.tiles()
    print(f"\n[edge] default tiles {t}", flush=True)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(5)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(5)
    _check(g.rho_u_T(), o.rho_u_T())
    g.close()


@pytest.mark.parametrize("prec", [I.FP32, I.FP32_SHIFTED, I.FP16_SHIFTED,
                                  I.FP16_LOCAL])
@pytest.mark.parametrize("bc", [[OP, OP, W, W], [OP] * 4])
def test_open_x_sides_reduced_precision(prec, bc):
    """The FP32 forms' short edge path for rows away from the y sides also
    serves open x sides (fixed temperature, velocity kept): an evaporating
    droplet with open x sides, 200 steps against the oracle within the
    short-run bounds of the reduced-precision forms."""
    cfg, fl = I.evaporation(96, 16.0, 1.1)
    cfg.update(bc=list(bc))
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(200)
    g = _lb().Simulation(dict(cfg, precision=prec))
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(200)
    e = _errors(g.rho_u_T(), o.rho_u_T())
    g.close()
    assert e["rho"] < SHORT[prec] and e["T"] < SHORT[prec], e
