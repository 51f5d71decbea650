"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 4096 x 4096 periodic spinodal lattice, default tiles, one launch
per step.  The oracle cannot step 1.7e7 nodes in a test, so the check is
local.  One step's outputs at a node depend on the state within three nodes
(the pull, then the interaction force one node further, then the divergence
of v in the thermal source one node further still), so a window of the GPU
state cut out with a margin of four, stepped once by the oracle as a small
periodic lattice, reproduces the GPU's next state in its interior exactly
(up to rounding).  Windows sit on strip, row-run and lattice boundaries of
the FP64 and FP32 tilings and on the periodic wrap; the whole lattice is
checked against a property that holds at any size (mass conservation)."""
import numpy as np
import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I

pytestmark = pytest.mark.gpu

N = 4096
WIN, MARGIN = 24, 4
# window centres: strip boundaries of 241-column (FP64) and 252-column (FP32)
# strips, boundaries of 35-row runs, the lattice corner (periodic wrap), the
# last strip and run, and the middle
CENTRES = [(0, 0), (241, 35), (252, 70), (4095, 4095), (3856, 4095),
           (4032, 2100), (2048, 2047), (1205, 1260)]
# max relative error of rho and T in the window interiors, and of f and g
# (relative to their largest magnitude) for FP64; the reduced-precision
# bounds (and the mass-drift bounds below) are about three times the errors
# measured when they were set (FP64 6.5e-16; FP32 1.4e-7, FP32 deviations
# 1.5e-7, FP16 deviations 2.2e-4; mass drift 1e-15, 9e-9, 9e-9, 7.8e-7)
TOL = {I.FP64: 1e-12, I.FP32: 5e-7, I.FP32_SHIFTED: 5e-7,
       I.FP16_SHIFTED: 7e-4, I.FP16_LOCAL: 7e-6}
MASS = {I.FP64: 1e-12, I.FP32: 3e-8, I.FP32_SHIFTED: 3e-8,
        I.FP16_SHIFTED: 3e-6, I.FP16_LOCAL: 3e-8}


def _split(state):
    w = state.view(np.float64)
    n = N * N
    f = w[:9 * n].reshape(9, N, N)
    g = w[9 * n:18 * n].reshape(9, N, N)
    phi = w[18 * n:19 * n].reshape(N, N)
    meta = w[19 * n:19 * n + 3]
    return f, g, phi, int(meta[:1].view(np.int64)[0]), float(meta[1]), \
        int(meta[2:3].view(np.int64)[0])


def _window(a, cx, cy):
    ys = (np.arange(cy - WIN // 2, cy + WIN // 2)) % N
    xs = (np.arange(cx - WIN // 2, cx + WIN // 2)) % N
    return a[..., ys[:, None], xs[None, :]]


@pytest.mark.parametrize("prec", [I.FP64, I.FP32, I.FP32_SHIFTED,
                                  I.FP16_SHIFTED, I.FP16_LOCAL])
def test_spinodal_4096_one_step_in_windows(prec):
    from paper_1709_04400_amd import lbpc
    cfg, fl = I.spinodal(N, precision=prec)
    g = lbpc.Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    del fl
    g.step(20)
    m0 = g.diag()["mass"]
    s0 = g.save_state()
    g.step(1)
    s1 = g.save_state()
    m1 = g.diag()["mass"]
    g.close()
    print(f"\n[fullsize] prec={prec} mass drift {abs(m1 - m0) / m0:.2e}",
          flush=True)
    assert abs(m1 - m0) <= MASS[prec] * m0

    f0, g0, p0, valid, rho_ave, step = _split(s0)
    f1, g1, _, _, _, _ = _split(s1)
    ocfg = dict(cfg, nx=WIN, ny=WIN, precision=I.FP64)
    inner = slice(MARGIN, WIN - MARGIN)
    worst = 0.0
    for cx, cy in CENTRES:
        o = O.Oracle(ocfg)
        o.set_state({"f": _window(f0, cx, cy), "g": _window(g0, cx, cy),
                     "phi_prev": _window(p0, cx, cy), "phi_valid": valid,
                     "rho_ave": rho_ave, "step": step})
        o.step(1)
        st = o.get_state()
        fo = st["f"].reshape(9, WIN, WIN)[:, inner, inner]
        go = st["g"].reshape(9, WIN, WIN)[:, inner, inner]
        fg = _window(f1, cx, cy)[:, inner, inner]
        gg = _window(g1, cx, cy)[:, inner, inner]
        e_rho = np.abs(fg.sum(0) - fo.sum(0)).max() / np.abs(fo.sum(0)).min()
        e_T = np.abs(gg.sum(0) - go.sum(0)).max() / np.abs(go.sum(0)).min()
        worst = max(worst, e_rho, e_T)
        assert e_rho < TOL[prec] and e_T < TOL[prec], (cx, cy, e_rho, e_T)
        if prec == I.FP64:
            assert np.abs(fg - fo).max() < TOL[prec] * np.abs(fo).max()
            assert np.abs(gg - go).max() < TOL[prec] * np.abs(go).max()
    print(f"[fullsize] prec={prec} worst window error {worst:.2e}",
          flush=True)


# FP32 and FP16 with node-local references: about three times the error
# measured when the bound was set (FP64 3.5e-15, FP32 1.67e-6, FP16
# node-local 1.04e-4)
BATCH_TOL = {I.FP64: 1e-11, I.FP32: 5e-6, I.FP16_LOCAL: 3e-4}


@pytest.mark.parametrize("prec", [I.FP64, I.FP32, I.FP16_LOCAL])
def test_full_sweep_batch_sampled_lattices(prec):
    """The batched workload at its full size: all 256 lattices of the seeded
    sweep (2.5e7 nodes) in one persistent launch per step with autotuned
    tiles, as bench.py runs it; after 20 steps the smallest, the largest and
    four other lattices are compared whole with the oracle."""
    from paper_1709_04400_amd import lbpc
    cases = I.batch_cases(count=256, seed=1709, precision=prec)
    b = lbpc.Batch([c for c, _ in cases])
    for k, (_, f) in enumerate(cases):
        b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    b.autotune(2)
    b.step(20)
    sizes = [c["nx"] * c["ny"] for c, _ in cases]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 101,
                   163, 255})
    worst = 0.0
    for k in pick:
        cfg, f = cases[k]
        o = O.Oracle(dict(cfg, precision=I.FP64))
        o.init_fields(**f)
        o.step(20)
        (r1, ux1, uy1, T1), (r2, ux2, uy2, T2) = b.rho_u_T(k), o.rho_u_T()
        e = max(np.max(np.abs(r1 - r2) / r2), np.max(np.abs(T1 - T2) / T2))
        worst = max(worst, e)
        assert e < BATCH_TOL[prec], (k, cfg["nx"], e)
    b.close()
    print(f"\n[fullsize] batch prec={prec} lattices {pick} worst {worst:.2e}",
          flush=True)


def _cut_window(a, x0, y0):
    return a[..., y0:y0 + WIN, x0:x0 + WIN]


@pytest.mark.parametrize("prec", [I.FP64, I.FP32, I.FP32_SHIFTED,
                                  I.FP16_SHIFTED, I.FP16_LOCAL])
def test_walled_4096_in_windows(prec):
    """The 4096 x 4096 spinodal walled on all four sides.  FP64 with the two
    x-edge strips on 137-row runs and the others on 147-row runs (one wave);
    the FP32 forms with their default tiles (their edge waves take the short
    x-side path in rows away from the y sides).  After 20 steps one more GPU
    step is compared in windows: at each wall (the oracle window keeps that
    wall; a cut side gets a wall or the periodic pair and is excluded with
    the dependence margin), at a corner, and where an edge strip's run
    boundary (y = 1918) and an interior strip's (y = 1911) meet across a
    strip boundary (x = 456).  FP64 compares f and g, every form rho and T,
    within the bounds of the periodic test."""
    import os
    from paper_1709_04400_amd import lbpc
    W_, P_ = I.BC_WALL, I.BC_PERIODIC
    cfg, fl = I.spinodal(N, precision=prec)
    cfg["bc"] = [W_] * 4
    env = ({"LBPC_TILE_BW": "512", "LBPC_TILE_H": "147",
            "LBPC_TILE_HE": "137"} if prec == I.FP64 else {})
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        g = lbpc.Simulation(cfg)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    if prec == I.FP64:
        assert g.tiles() == {"block_width": 512, "rows": 147,
                             "rows_edge": 137}
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    del fl
    g.step(20)
    s0 = g.save_state()
    g.step(1)
    s1 = g.save_state()
    g.close()
    f0, g0, p0, valid, rho_ave, step = _split(s0)
    f1, g1, _, _, _, _ = _split(s1)
    # (x0, y0) of each window; which window sides are the lattice's walls
    wins = [(0, 399), (N - WIN, 1200), (2000, 0), (2000, N - WIN), (0, 0),
            (444, 1903)]
    worst = 0.0
    for x0, y0 in wins:
        real = [x0 == 0, x0 + WIN == N, y0 == 0, y0 + WIN == N]
        bx = W_ if real[0] or real[1] else P_
        by = W_ if real[2] or real[3] else P_
        ocfg = dict(cfg, nx=WIN, ny=WIN, bc=[bx, bx, by, by],
                    precision=I.FP64)
        o = O.Oracle(ocfg)
        o.set_state({"f": _cut_window(f0, x0, y0),
                     "g": _cut_window(g0, x0, y0),
                     "phi_prev": _cut_window(p0, x0, y0),
                     "phi_valid": valid, "rho_ave": rho_ave, "step": step})
        o.step(1)
        st = o.get_state()
        xs = slice(0 if real[0] else MARGIN, WIN if real[1] else WIN - MARGIN)
        ys = slice(0 if real[2] else MARGIN, WIN if real[3] else WIN - MARGIN)
        fo = st["f"].reshape(9, WIN, WIN)[:, ys, xs]
        go = st["g"].reshape(9, WIN, WIN)[:, ys, xs]
        fg = _cut_window(f1, x0, y0)[:, ys, xs]
        gg = _cut_window(g1, x0, y0)[:, ys, xs]
        e_rho = np.abs(fg.sum(0) - fo.sum(0)).max() / np.abs(fo.sum(0)).min()
        e_T = np.abs(gg.sum(0) - go.sum(0)).max() / np.abs(go.sum(0)).min()
        worst = max(worst, e_rho, e_T)
        assert e_rho < TOL[prec] and e_T < TOL[prec], (x0, y0, e_rho, e_T)
        if prec == I.FP64:
            e_f = np.abs(fg - fo).max() / np.abs(fo).max()
            e_g = np.abs(gg - go).max() / np.abs(go).max()
            worst = max(worst, e_f, e_g)
            assert e_f < TOL[prec] and e_g < TOL[prec], (x0, y0, e_f, e_g)
    print(f"\n[fullsize] walled prec={prec} worst window error {worst:.2e}",
          flush=True)


def test_16384_fp64_offsets_beyond_2_31_elements():
    """The largest lattice here: 16384 x 16384 FP64 (2.7e8 nodes, 86 GiB of
    workspace), whose f and g buffers hold 2.4e9 elements, so rows above
    y = 14563 sit at element offsets past 2^31.  Two GPU steps from the
    seeded spinodal state; rho, u and T then match, in windows, the oracle
    stepping the same initial state cut out with a margin of 8 (two steps
    reach 3 nodes each, the readback of v one more).  Windows in the top
    rows, at the periodic corner and in the middle."""
    import torch
    from paper_1709_04400_amd import lbpc
    n, win, margin = 16384, 32, 8
    cfg, fl = I.spinodal(n, precision=I.FP64)
    need = lbpc.lbpc_workspace_bytes(cfg)
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory")
    g = lbpc.Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(2)
    out = g.rho_u_T()
    g.close()
    del g
    worst = 0.0
    for cx, cy in [(100, n - 5), (n // 2, n - 700), (0, 0), (n - 1, n - 1),
                   (8000, 8000)]:
        ys = (np.arange(cy - win // 2, cy + win // 2)) % n
        xs = (np.arange(cx - win // 2, cx + win // 2)) % n
        cut = {k: np.ascontiguousarray(v[ys[:, None], xs[None, :]])
               for k, v in fl.items()}
        o = O.Oracle(dict(cfg, nx=win, ny=win))
        o.init_fields(**cut)
        o.step(2)
        ref = o.rho_u_T()
        inner = slice(margin, win - margin)
        for k, (a, b) in enumerate(zip(out, ref)):
            ga = a[ys[:, None], xs[None, :]][inner, inner]
            rb = b[inner, inner]
            scale = np.abs(rb).max() if k in (1, 2) else np.abs(rb).min()
            e = np.abs(ga - rb).max() / scale
            worst = max(worst, e)
            assert e < 1e-12, (cx, cy, k, e)
    print(f"\n[fullsize] 16384^2 FP64 worst window error {worst:.2e}",
          flush=True)


def _split_hist(state, nh):
    """Saved state with nh history arrays after f and g (phi, then for the
    BGK form T v_x and T v_y of the previous step)."""
    w = state.view(np.float64)
    n = N * N
    f = w[:9 * n].reshape(9, N, N)
    g = w[9 * n:18 * n].reshape(9, N, N)
    hist = w[18 * n:(18 + nh) * n].reshape(nh, N, N)
    meta = w[(18 + nh) * n:(18 + nh) * n + 3]
    return f, g, hist, int(meta[:1].view(np.int64)[0]), float(meta[1]), \
        int(meta[2:3].view(np.int64)[0])


@pytest.mark.parametrize("model", [I.THERMAL_GONG_CHENG,
                                   I.THERMAL_IMPROVED_BGK])
def test_spinodal_4096_other_models_in_windows(model):
    """The Gong-Cheng model and the BGK form of the improved model at the
    benchmark's full size, FP64, in the launch configuration bench.py times
    for them: 20 steps, then one more GPU step compared in the windows of
    the improved model's test (the BGK form's T v history travels with the
    window)."""
    from paper_1709_04400_amd import lbpc
    cfg, fl = I.spinodal(N, precision=I.FP64)
    cfg["thermal_model"] = model
    nh = 3 if model == I.THERMAL_IMPROVED_BGK else 1
    g = lbpc.Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    del fl
    g.step(20)
    s0 = g.save_state()
    g.step(1)
    s1 = g.save_state()
    g.close()
    f0, g0, h0, valid, rho_ave, step = _split_hist(s0, nh)
    f1, g1, _, _, _, _ = _split_hist(s1, nh)
    ocfg = dict(cfg, nx=WIN, ny=WIN)
    inner = slice(MARGIN, WIN - MARGIN)
    worst = 0.0
    for cx, cy in CENTRES:
        st0 = {"f": _window(f0, cx, cy), "g": _window(g0, cx, cy),
               "phi_prev": _window(h0[0], cx, cy), "phi_valid": valid,
               "rho_ave": rho_ave, "step": step}
        if nh == 3:
            st0["tv_prev"] = np.ascontiguousarray(_window(h0[1:3], cx, cy))
        o = O.Oracle(ocfg)
        o.set_state(st0)
        o.step(1)
        st = o.get_state()
        fo = st["f"].reshape(9, WIN, WIN)[:, inner, inner]
        go = st["g"].reshape(9, WIN, WIN)[:, inner, inner]
        fg = _window(f1, cx, cy)[:, inner, inner]
        gg = _window(g1, cx, cy)[:, inner, inner]
        e_f = np.abs(fg - fo).max() / np.abs(fo).max()
        e_g = np.abs(gg - go).max() / np.abs(go).max()
        worst = max(worst, e_f, e_g)
        assert e_f < TOL[I.FP64] and e_g < TOL[I.FP64], (cx, cy, e_f, e_g)
    print(f"\n[fullsize] model {model} worst window error {worst:.2e}",
          flush=True)


def _spinodal_2000(prec):
    from paper_1709_04400_amd import lbpc
    cfg, fl = I.spinodal(N, precision=prec)
    g = lbpc.Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    del fl
    d0 = g.diag()
    g.step(2000)
    d = g.diag()
    r = g.rho_u_T()[0]
    g.close()
    assert not d["nonfinite"]
    return dict(mass_drift=(d["mass"] - d0["mass"]) / d0["mass"],
                sum_T_change=(d["sum_T"] - d0["sum_T"]) / d0["sum_T"],
                liquid_fraction=float(
                    (r > 0.5 * (I.RHO_L + I.RHO_V)).mean()))


def test_spinodal_4096_2000_steps_global_results():
    """The benchmark workload run as its configuration states: 2000 steps
    of the 4096 x 4096 spinodal in every storage form.  Decomposition is
    chaotic, so the forms are compared on global results against FP64: the
    mass drift, the change of sum T (the thermal source moves it by 3.5 %)
    and the liquid fraction.  Bounds are about three times the errors
    measured when they were set (mass drift FP32 1.8e-5, FP32 deviations
    1.9e-5, FP16 deviations 5.0e-5, node-local 2.4e-5; liquid fraction
    within 2e-5 of FP64, 1.3e-4 for FP16 deviations)."""
    import json
    ref = _spinodal_2000(I.FP64)
    assert abs(ref["mass_drift"]) < 1e-11, ref
    out = {"FP64": ref}
    bounds = {I.FP32: (6e-5, 6e-5), I.FP32_SHIFTED: (6e-5, 6e-5),
              I.FP16_SHIFTED: (1.5e-4, 4e-4), I.FP16_LOCAL: (8e-5, 6e-5)}
    for prec, (bm, bl) in bounds.items():
        r = _spinodal_2000(prec)
        out[str(prec)] = r
        assert abs(r["mass_drift"]) < bm, (prec, r)
        assert abs(r["liquid_fraction"] - ref["liquid_fraction"]) < bl, \
            (prec, r, ref)
        assert abs(r["sum_T_change"] - ref["sum_T_change"]) < 1e-4, \
            (prec, r, ref)
    print("\n[fullsize] spinodal 2000 steps " + json.dumps(out), flush=True)


def _sweep_5000(prec):
    from paper_1709_04400_amd import lbpc
    cases = I.batch_cases(count=256, seed=1709, precision=prec)
    b = lbpc.Batch([c for c, _ in cases])
    for k, (_, f) in enumerate(cases):
        b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    d0 = [b.diag(k) for k in range(len(cases))]
    b.autotune(2)
    b.step(5000)
    d1 = [b.diag(k) for k in range(len(cases))]
    b.close()
    assert not any(d["nonfinite"] for d in d1), prec
    return (np.array([(a["mass"] - z["mass"]) / z["mass"]
                      for a, z in zip(d1, d0)]),
            np.array([a["liquid_area"] for a in d1]))


def test_full_sweep_batch_5000_steps():
    """The batched workload as its configuration states: all 256 lattices,
    5000 steps, one persistent launch per step with autotuned tiles.  Every
    lattice stays finite; FP64 conserves each lattice's mass to 1e-11; FP32
    storage and FP16 storage with node-local references conserve it to
    2e-4 and keep each lattice's liquid area within 3e-4 of FP64's
    (measured when the bounds were set: mass 5.0e-5 and 5.8e-5, area 7.4e-5
    and 8.5e-5)."""
    import json
    m64, a64 = _sweep_5000(I.FP64)
    assert np.abs(m64).max() < 1e-11
    out = {}
    for prec in (I.FP32, I.FP16_LOCAL):
        m, a = _sweep_5000(prec)
        out[str(prec)] = dict(mass=float(np.abs(m).max()),
                              area=float((np.abs(a - a64) / a64).max()))
        assert out[str(prec)]["mass"] < 2e-4, (prec, out)
        assert out[str(prec)]["area"] < 3e-4, (prec, out)
    print("\n[fullsize] batch 5000 steps " + json.dumps(out), flush=True)
