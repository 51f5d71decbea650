"""The step kernels of one lattice agree bit for bit: the periodic kernel
(with, for the FP16 forms under an MRT thermal model, their instantiations
that compile out the Gong-Cheng and BGK-form branches) against the tile-list
kernel with every branch compiled in, on the same periodic lattice; and the
tile-list kernel launched with one block per tile against the same kernel
with one block per resident slot walking the list (LBPC_PERSISTENT=1)."""
import os

import numpy as np
import pytest

from paper_1709_04400_amd import inputs as I
from test_gpu_edge_cases import _cut

pytestmark = pytest.mark.gpu


def _lb():
    from paper_1709_04400_amd import lbpc
    return lbpc


@pytest.mark.parametrize("prec,model", [(I.FP64, I.THERMAL_IMPROVED),
                                        (I.FP32, I.THERMAL_IMPROVED),
                                        (I.FP32_SHIFTED, I.THERMAL_IMPROVED),
                                        (I.FP16_SHIFTED, I.THERMAL_IMPROVED),
                                        (I.FP16_SHIFTED, I.THERMAL_GONG_CHENG),
                                        (I.FP16_LOCAL, I.THERMAL_IMPROVED),
                                        (I.FP16_LOCAL, I.THERMAL_GONG_CHENG)])
def test_periodic_kernel_equals_tile_list_kernel(prec, model):
    """The periodic step kernel (for the FP16 form under an MRT thermal
    model, its instantiation without the Gong-Cheng and BGK branches) and
    the tile-list kernel (LBPC_FORCE_TILED=1, every branch compiled in) give
    the same state on a periodic lattice, bit for bit."""
    print(f"\n[paths] periodic vs tile-list precision={prec} model={model}",
          flush=True)
    cfg, fl = _cut(61, 47, "periodic", precision=prec)
    cfg["thermal_model"] = model
    old = os.environ.get("LBPC_FORCE_TILED")
    os.environ["LBPC_FORCE_TILED"] = "1"
    try:
        tiled = _lb().Simulation(cfg)
    finally:
        if old is None:
            os.environ.pop("LBPC_FORCE_TILED", None)
        else:
            os.environ["LBPC_FORCE_TILED"] = old
    plain = _lb().Simulation(cfg)
    for s in (plain, tiled):
        s.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
        s.step(25)
    assert np.array_equal(plain.save_state(), tiled.save_state())
    plain.close()
    tiled.close()


@pytest.mark.parametrize("prec", [I.FP64, I.FP32, I.FP16_SHIFTED,
                                  I.FP16_LOCAL])
def test_persistent_walk_equals_one_block_per_tile(prec):
    """A walled 1000 x 800 lattice on 64 x 4 tiles (17 strips x 200 runs =
    3400 tiles, more than the resident slots -- at most 12 one-wave blocks
    per CU -- so blocks of the persistent launch walk several) steps to the
    same state bit for bit with one block per tile and with
    LBPC_PERSISTENT=1."""
    print(f"\n[paths] persistent tile walk precision={prec}", flush=True)
    cfg, _ = I.evaporation(800, 100.0, 1.1, precision=prec)
    cfg.update(nx=1000, bc=[I.BC_WALL] * 4)
    fl = I.droplet_fields(1000, 800, 100.0)
    runs = []
    for persistent in (False, True):
        old = os.environ.get("LBPC_PERSISTENT")
        if persistent:
            os.environ["LBPC_PERSISTENT"] = "1"
        try:
            s = _lb().Simulation(cfg)
            s.set_tiles(64, 4)
            s.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
            s.step(6)
            runs.append(s.save_state())
            s.close()
        finally:
            if old is None:
                os.environ.pop("LBPC_PERSISTENT", None)
            else:
                os.environ["LBPC_PERSISTENT"] = old
    assert np.array_equal(runs[0], runs[1])
