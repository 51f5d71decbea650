"""lbpc_get_diag_noalloc against lbpc_get_diag, through the C ABI.

The no-allocation variant runs the same no-store diagnostic pass and final
reduction with its tile records in the library's static device scratch; its
results must equal those of lbpc_get_diag bitwise.  Two calls in a row on
different handles, the second on a smaller lattice (fewer tile records than
the first left in the shared scratch), and the limit on the tile count.
"""
import numpy as np
import pytest

from paper_1709_04400_amd import inputs as I

pytestmark = pytest.mark.gpu


def _sim(cfg, fl, steps):
    from paper_1709_04400_amd import lbpc
    g = lbpc.Simulation(cfg)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    g.step(steps)
    return g


def test_noalloc_diag_equals_get_diag_twice():
    cases = [
        # 512 x 384 walled boiling cut (tile-list path), 64-wide strips
        (I.bubble(nx=512, ny=384, pool=250, hot_width=30, g=3e-5), 40,
         (64, 8)),
        # then a smaller periodic droplet (periodic path, default tiles)
        (I.static_droplet(96, 80, 20.0), 25, None),
    ]
    for (cfg, fl), steps, tiles in cases:
        print(f"\n[noalloc] {cfg['nx']}x{cfg['ny']} tiles={tiles}",
              flush=True)
        g = _sim(cfg, fl, steps)
        if tiles:
            g.set_tiles(*tiles)
        ref = g.diag()
        got = g.diag_noalloc()
        again = g.diag()
        g.close()
        assert got == ref, (got, ref)
        assert again == ref
        assert got["step"] == steps and not got["nonfinite"]
        assert np.isfinite(got["mass"]) and got["mass"] > 0


def test_noalloc_diag_rejects_more_tiles_than_its_scratch():
    from paper_1709_04400_amd import lbpc
    cfg, fl = I.spinodal(n=64, precision=I.FP16_SHIFTED)
    nx, ny = 8192, 2048
    cfg.update(nx=nx, ny=ny)
    rng = np.random.default_rng(3)
    rho = 0.5 * (I.RHO_L + I.RHO_V) * (1 + rng.uniform(-0.01, 0.01, (ny, nx)))
    z = np.zeros((ny, nx))
    g = lbpc.Simulation(cfg)
    g.init_fields(rho, z, z, np.full((ny, nx), I.T_SAT))
    g.set_tiles(64, 4)           # 137 strips x 512 runs = 70144 tiles
    with pytest.raises(lbpc.LbpcError) as e:
        g.diag_noalloc()
    assert e.value.status == lbpc.ERR_UNSUPPORTED
    g.set_tiles(256, 64)         # 17 x 32 tiles: fits
    assert g.diag_noalloc() == g.diag()
    g.close()
