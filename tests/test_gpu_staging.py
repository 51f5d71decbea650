"""Chunked host transfers on the GPU: initial fields, field readback and
checkpoints pass through a staging scratch of a few rows (LBPC_STAGE_NODES=1
leaves three rows per field: readback bands of one row, init chunks of under
four rows, checkpoint chunks of fifteen).  Every value must equal, bit for
bit, the one a handle staging the whole lattice at once gives: the per-node
kernels are the same, only the chunking differs.  A checkpoint loaded
through the row staging resumes the run bit for bit (the node-referenced
FP16 form: as the same checkpoint loaded whole, since its references are
not in the canonical state).  One case is also checked against the
oracle."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1709_04400_amd import inputs as I
from test_gpu_edge_cases import _check, _cut

pytestmark = pytest.mark.gpu


def _lb():
    from paper_1709_04400_amd import lbpc
    return lbpc


def _make(cls, arg, stage):
    """A handle (or batch) created with LBPC_STAGE_NODES = stage (None: the
    default staging, which holds these small lattices whole)."""
    old = os.environ.get("LBPC_STAGE_NODES")
    if stage is None:
        os.environ.pop("LBPC_STAGE_NODES", None)
    else:
        os.environ["LBPC_STAGE_NODES"] = str(stage)
    try:
        return cls(arg)
    finally:
        if old is None:
            os.environ.pop("LBPC_STAGE_NODES", None)
        else:
            os.environ["LBPC_STAGE_NODES"] = old


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


CASES = [(37, 23, "periodic", I.FP64), (37, 23, "walls", I.FP64),
         (29, 31, "wall_open", I.FP64), (4, 37, "y_walls", I.FP64),
         (37, 4, "x_walls", I.FP64), (33, 21, "walls", I.FP32),
         (33, 21, "periodic", I.FP32_SHIFTED),
         (33, 21, "wall_open", I.FP16_SHIFTED),
         (33, 21, "wall_open", I.FP16_LOCAL), (29, 31, "walls", I.FP16_LOCAL),
         (37, 23, "periodic", I.FP16_LOCAL)]


@pytest.mark.parametrize("nx,ny,sides,prec", CASES)
def test_staged_transfers_equal_whole_lattice_transfers(nx, ny, sides, prec):
    print(f"\n[staging] {nx}x{ny} {sides} precision={prec}", flush=True)
    cfg, fl = _cut(nx, ny, sides, precision=prec)
    whole = _make(_lb().Simulation, cfg, None)
    rows = _make(_lb().Simulation, cfg, 1)
    for s in (whole, rows):
        s.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    _same(rows.rho_u_T(), whole.rho_u_T())
    for s in (whole, rows):
        s.step(7)
    _same(rows.rho_u_T(), whole.rho_u_T())
    st = whole.save_state()
    assert np.array_equal(rows.save_state(), st)
    rows.load_state(st)
    if prec == I.FP16_LOCAL:
        # the node-local references are not part of the canonical
        # checkpoint: a load stores each value against a reference taken
        # from its node's rest populations, so the resumed run equals the
        # same checkpoint loaded through whole-lattice staging bit for bit,
        # and the uninterrupted run to the binary16 rounding of that one
        # re-encoding
        loaded = _make(_lb().Simulation, cfg, None)
        loaded.load_state(st)
        for s in (whole, rows, loaded):
            s.step(5)
        _same(rows.rho_u_T(), loaded.rho_u_T())
        assert np.array_equal(rows.save_state(), loaded.save_state())
        # (rho, ux, uy, T); the velocity is a small difference of
        # populations, so it carries the rounding of the deviations most
        for x, y, b in zip(rows.rho_u_T(), whole.rho_u_T(),
                           (1e-5, 3e-3, 3e-3, 1e-5)):
            e = np.abs(x - y).max() / np.abs(y).max()
            print(f"[staging] resumed vs uninterrupted: {e:.2e}", flush=True)
            assert e <= b
        loaded.close()
    else:
        # a checkpoint loaded through the row staging resumes identically
        for s in (whole, rows):
            s.step(5)
        _same(rows.rho_u_T(), whole.rho_u_T())
        assert np.array_equal(rows.save_state(), whole.save_state())
    whole.close()
    rows.close()


def test_staged_readback_matches_oracle():
    cfg, fl = _cut(41, 27, "wall_open")
    o = O.Oracle(cfg)
    o.init_fields(**fl)
    g = _make(_lb().Simulation, cfg, 1)
    g.init_fields(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    o.step(20)
    g.step(20)
    _check(g.rho_u_T(), o.rho_u_T())
    g.close()


def test_batch_staged_transfers_equal_whole_lattice_transfers():
    cases = [_cut(4, 4, "periodic"), _cut(37, 23, "walls"),
             _cut(5, 6, "wall_open"), _cut(29, 9, "y_walls")]
    cfgs = [c for c, _ in cases]
    whole = _make(_lb().Batch, cfgs, None)
    rows = _make(_lb().Batch, cfgs, 1)
    for b in (whole, rows):
        for k, (_, f) in enumerate(cases):
            b.init_fields(k, f["rho"], f["ux"], f["uy"], f["T"])
    for k in range(len(cases)):
        _same(rows.rho_u_T(k), whole.rho_u_T(k))
    for b in (whole, rows):
        b.step(9)
    for k in range(len(cases)):
        print(f"[staging] batch lattice {k}", flush=True)
        _same(rows.rho_u_T(k), whole.rho_u_T(k))
    whole.close()
    rows.close()
