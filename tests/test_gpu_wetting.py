"""GPU parity of the wall-wetting rule (virtual density of the wall ghosts in
the interaction force) against the oracle, through the C ABI: the readback
path at step 0, the fused step on hydrophobic and hydrophilic walls, walls on
all sides with corners and a hot spot, a bottom wall under an open top (the
heated-surface set-up), a batch mixing wetting and neutral lattices, and the
reduced-precision forms."""
import json

import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I
from test_gpu_parity import TOL, _assert_ok, _errors, run_pair

pytestmark = pytest.mark.gpu


def _lb():
    from paper_1709_04400_amd import lbpc
    return lbpc


def test_wetting_readback_at_step0():
    """v = (j + F/2)/rho at the initial state uses the readback kernels'
    force, with the wall ghosts' psi of the virtual density."""
    cfg, fl = I.sessile_droplet(48, 32, 10.0, wet_amp=0.2, wet_shift=0.3)
    cfg["bc"] = [I.BC_WALL] * 4
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    g = _lb().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    e = _errors(g.rho_u_T(), o.rho_u_T())
    g.close()
    assert e["rho"] < 1e-14 and e["T"] < 1e-14 and e["u"] < 1e-12, e


def test_sessile_hydrophobic():
    cfg, fl = I.sessile_droplet(80, 40, 13.0, wet_amp=I.WET_AMP_108)
    _assert_ok(run_pair(cfg, fl, 600, chunks=2))


def test_walls_all_sides_hydrophilic_hot_spot():
    cfg, fl = I.sessile_droplet(64, 64, 14.0, wet_amp=I.WET_AMP_45)
    cfg.update(bc=[I.BC_WALL] * 4, hot_x0=28, hot_x1=36,
               T_hot=1.1 * I.T_SAT, lambda_mode=I.LAMBDA_RHO_CV_CHI,
               chi=I.CHI_BUBBLE)
    _assert_ok(run_pair(cfg, fl, 400, chunks=2))


@pytest.mark.parametrize("model", [I.THERMAL_IMPROVED, I.THERMAL_COMPROMISED,
                                   I.THERMAL_GONG_CHENG])
def test_heated_surface_cut(model):
    """The heated-surface set-up (bottom wall at 0.875 Tc, open top,
    periodic x, lambda = rho c_V chi) on a 96 x 48 cut, its wall at about
    108 degrees."""
    cfg, fl = I.heated_surface(model, nx=96, ny=48, radius=14.0,
                               wet_amp=I.WET_AMP_108)
    _assert_ok(run_pair(cfg, fl, 400, chunks=2))


def test_wetting_in_a_batch():
    cases = [I.sessile_droplet(64, 40, 12.0, wet_amp=I.WET_AMP_108),
             I.heated_droplet(48, 10.0, 1.1),
             I.heated_surface(I.THERMAL_GONG_CHENG, nx=72, ny=40,
                              radius=11.0, wet_amp=I.WET_AMP_108),
             I.sessile_droplet(56, 56, 12.0, wet_amp=I.WET_AMP_45)]
    b = _lb().Batch([c for c, _ in cases])
    for k, (_, f) in enumerate(cases):
        b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    b.step(301)
    for k, (cfg, f) in enumerate(cases):
        o = O.Oracle(cfg)
        o.init_fields(**f)
        o.step(301)
        e = _errors(b.rho_u_T(k), o.rho_u_T())
        assert e["rho"] < TOL and e["T"] < TOL and e["u"] < TOL, (k, e)
    b.close()


# bounds about three times the errors measured when they were set
WET_SHORT = {I.FP32: 3e-5, I.FP32_SHIFTED: 3e-5, I.FP16_SHIFTED: 2e-2,
             I.FP16_LOCAL: 2e-3}


@pytest.mark.parametrize("prec", [I.FP32, I.FP32_SHIFTED, I.FP16_SHIFTED,
                                  I.FP16_LOCAL])
def test_wetting_reduced_precision_short_run(prec):
    cfg, fl = I.heated_surface(nx=96, ny=48, radius=14.0,
                               wet_amp=I.WET_AMP_108)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(200)
    cfg["precision"] = prec
    g = _lb().Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(200)
    e = _errors(g.rho_u_T(), o.rho_u_T())
    g.close()
    print("\n[precision] " + json.dumps({"result": "wetting_short_run",
                                          "precision": prec, **e}), flush=True)
    assert e["rho"] < WET_SHORT[prec] and e["T"] < WET_SHORT[prec], e
