"""The step kernels of one lattice agree bit for bit: the periodic kernel
(with, for the FP16 form under an MRT thermal model, its instantiation that
compiles out the Gong-Cheng and BGK-form branches) against the tile-list
kernel with every branch compiled in, on the same periodic lattice."""
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
