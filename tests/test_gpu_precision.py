"""Reduced-precision storage forms against FP64: the error stated per result.

FP32 (storage and arithmetic), FP32 deviations from the rest equilibrium,
FP16 deviations from one reference and FP16 deviations from node-local
references (both with FP32 arithmetic), on the workloads' own geometries:
  * a short run against the CPU oracle;
  * coexistence densities of a flat film (T = 0.86 Tc, 24000 steps);
  * the droplet-radius history of the evaporation case (300 x 300, open
    fixed-T sides at 1.1 T_sat, 20000 steps, radius every 500 steps);
  * the bubble departure time on the boiling geometry (400 x 800, hot spot,
    g = 3e-5), run until the first departure.
The long runs use the GPU FP64 path as the reference (it matches the oracle
to 1e-11, see test_gpu_parity.py).  Each test prints one "[precision]" JSON
line with the measured errors; the bounds asserted are about three times the
errors measured when the bounds were set.
"""
import json

import numpy as np
import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I

pytestmark = pytest.mark.gpu
NAMES = {I.FP64: "FP64", I.FP32: "FP32", I.FP32_SHIFTED: "FP32_SHIFTED",
         I.FP16_SHIFTED: "FP16_SHIFTED", I.FP16_LOCAL: "FP16_LOCAL"}
REDUCED = [I.FP32, I.FP32_SHIFTED, I.FP16_SHIFTED, I.FP16_LOCAL]


def _sim(cfg):
    from paper_1709_04400_amd import lbpc
    return lbpc.Simulation(cfg)


def _report(name, payload):
    print("\n[precision] " + json.dumps({"result": name, **payload}),
          flush=True)


# bounds: (FP32, FP32_SHIFTED, FP16_SHIFTED, FP16_LOCAL)
SHORT_BOUNDS = {"rho": (2e-5, 2e-5, 2e-2, 1e-3), "T": (2e-5, 2e-5, 2e-2, 1e-4),
                "u": (3e-3, 3e-3, 0.5, 8e-3)}


@pytest.mark.parametrize("prec", REDUCED)
def test_short_run_against_oracle(prec):
    cfg, fl = I.static_droplet(64, 64, 16.0)
    cfg.update(gy=-2e-5)
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    o.step(200)
    cfg["precision"] = prec
    g = _sim(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(200)
    (r1, ux1, uy1, T1), (r2, ux2, uy2, T2) = g.rho_u_T(), o.rho_u_T()
    g.close()
    umax = max(np.abs(ux2).max(), np.abs(uy2).max())
    err = dict(rho=float(np.max(np.abs(r1 - r2) / r2)),
               T=float(np.max(np.abs(T1 - T2) / T2)),
               u=float(max(np.abs(ux1 - ux2).max(),
                           np.abs(uy1 - uy2).max()) / umax))
    _report("short_run_vs_oracle", {"precision": NAMES[prec], **err})
    k = REDUCED.index(prec)
    for q in ("rho", "T", "u"):
        assert err[q] < SHORT_BOUNDS[q][k], (q, err)


def _film(prec, steps=24000):
    ny, nx = 256, 16
    cfg = I.base_config(nx, ny, precision=prec)
    y = np.mgrid[0:ny, 0:nx][0].astype(float)
    rho = I.tanh_profile(np.abs(y - 127.5) - 64, 5.0, I.RHO_L, I.RHO_V)
    z = np.zeros((ny, nx))
    g = _sim(cfg)
    g.init_fields(rho, z, z, np.full((ny, nx), I.T_SAT))
    m0 = g.diag()["mass"]
    g.step(steps)
    r, _, _, T = g.rho_u_T()
    d = g.diag()
    g.close()
    return dict(rho_l=float(r[ny // 2].mean()), rho_v=float(r[0].mean()),
                T_l=float(T[ny // 2].mean()), mass_drift=(d["mass"] - m0) / m0)


def test_coexistence_densities():
    ref = _film(I.FP64)
    # FP64: the known pseudopotential deviation from the Maxwell values (the
    # temperature of the coupled film drifts slightly from 0.86 Tc)
    assert abs(ref["rho_l"] - I.RHO_L) / I.RHO_L < 0.01
    assert abs(ref["rho_v"] - I.RHO_V) / I.RHO_V < 0.06
    assert abs(ref["mass_drift"]) < 1e-11
    out = {"FP64": ref}

    def errs(r, base):
        return dict(rho_l=abs(r["rho_l"] - base["rho_l"]) / base["rho_l"],
                    rho_v=abs(r["rho_v"] - base["rho_v"]) / base["rho_v"],
                    mass_drift=abs(r["mass_drift"]))

    for prec in (I.FP32, I.FP32_SHIFTED):
        e = errs(_film(prec), ref)
        out[NAMES[prec]] = e
        assert e["rho_l"] < 1.5e-4 and e["rho_v"] < 1e-3 and \
            e["mass_drift"] < 1e-3, (NAMES[prec], e)
    # FP16 deviations: binary16 moving populations, FP32 rest populations
    # that absorb the eight others' rounding errors, so biased rounding does
    # not drain the liquid (a single FP16 reference had the film inverted by
    # 24000 steps)
    r24 = _film(I.FP16_SHIFTED)
    e24 = errs(r24, ref)
    out["FP16_SHIFTED"] = dict(e24, film_intact_24000=r24["rho_l"] > 3.0)
    # node-local references: binary16 holds only the velocity and
    # non-equilibrium parts of the populations
    rl = _film(I.FP16_LOCAL)
    el = errs(rl, ref)
    out["FP16_LOCAL"] = el
    _report("coexistence_film", out)
    assert r24["rho_l"] > 3.0, r24
    assert e24["rho_l"] < 3e-3 and e24["rho_v"] < 3e-3 and \
        e24["mass_drift"] < 3e-3, e24
    assert el["rho_l"] < 4e-4 and el["rho_v"] < 1e-3 and \
        el["mass_drift"] < 1e-3, el


def _radius_history(prec):
    cfg, fl = I.evaporation(300, 50.0, 1.1, precision=prec)
    g = _sim(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    hist = []
    for k in range(41):
        d = g.diag()
        assert not d["nonfinite"]
        hist.append(d["radius"])
        if k < 40:
            g.step(500)
    g.close()
    return np.array(hist)


def test_droplet_radius_history():
    ref = _radius_history(I.FP64)
    out = {"FP64_R0": ref[0], "FP64_R20000": ref[-1]}
    bounds = {I.FP32: 1e-4, I.FP32_SHIFTED: 1e-4, I.FP16_SHIFTED: 1e-3,
              I.FP16_LOCAL: 4e-4}
    for prec in REDUCED:
        h = _radius_history(prec)
        err = float(np.max(np.abs(h - ref) / ref))
        out[NAMES[prec]] = {"max_rel_err": err, "R20000": h[-1]}
        assert err < bounds[prec], (NAMES[prec], err)
    _report("radius_history_evaporation_300", out)


def _departure(prec, max_steps=80000, every=500):
    """First step at which the largest vapour region below the initial pool
    surface no longer touches the wall row y = 0 (regions reaching row 599,
    i.e. the vapour above the pool, do not count)."""
    from scipy import ndimage
    cfg, fl = I.bubble(precision=prec)
    g = _sim(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    half = 0.5 * (I.RHO_L + I.RHO_V)
    seen = False
    step = None
    largest = 0.0     # largest attached vapour region seen (nodes)
    for k in range(max_steps // every):
        g.step(every)
        r = g.rho_u_T()[0]
        vap = r[:600] < half
        lab, n = ndimage.label(vap)
        if n == 0:
            continue
        sizes = ndimage.sum(vap, lab, range(1, n + 1))
        for c in np.unique(lab[-1]):
            if c:
                sizes[c - 1] = 0
        if sizes.max() == 0:
            continue
        big = int(np.argmax(sizes)) + 1
        touches = bool((lab[0] == big).any())
        if touches:
            largest = max(largest, float(sizes[big - 1]))
        if touches and sizes[big - 1] > 200:
            seen = True
        if seen and not touches:
            step = (k + 1) * every
            break
    g.close()
    return step, largest


def test_bubble_departure_time():
    """FP32, FP32 deviations and FP16 deviations from node-local references
    depart within 5 % of the FP64 step.  FP16 deviations from one reference:
    no departure within 80000 steps (FP64: 66000) when this bound was set --
    the binary16 quantisation of the liquid populations (~7e-4 relative)
    changes nucleation on the hot spot -- so for that form the result is
    stated (step, largest attached bubble), not bounded; its run must stay
    finite (a non-finite field fails the readback)."""
    ref, _ = _departure(I.FP64)
    assert ref is not None, "FP64 bubble did not depart"
    out = {"FP64": ref}
    for prec in (I.FP32, I.FP32_SHIFTED, I.FP16_SHIFTED, I.FP16_LOCAL):
        s, largest = _departure(prec)
        out[NAMES[prec]] = {"step": s, "largest_attached": largest,
                            "rel_err": None if s is None else
                            abs(s - ref) / ref}
    _report("bubble_departure_step", out)
    for name in ("FP32", "FP32_SHIFTED", "FP16_LOCAL"):
        assert out[name]["step"] is not None, name
        assert out[name]["rel_err"] < 0.05, (name, out[name])
