"""The Python binding rejects, before any library call, the arguments the C
ABI cannot check: host tensors, a dtype other than the call's, buffers too
small for the sizes the call implies.  Runs without a GPU (stub operator and
model objects; the library is never reached)."""
import types

import pytest
import torch

from paper_1406_7042_amd import yeerom as Y


def _op(field_len=60, dim=2, n=4):
    return types.SimpleNamespace(field_len=field_len, handle=None, dim=dim, nx=n, ny=n, nz=1,
                                 ne_slots=1, len=20)


class _Rom:
    def __init__(self, q1=5, q2=6, nsrc=1, nprb=2):
        self._i = dict(q1=q1, q2=q2, nsrc=nsrc, nprb=nprb)
        self.handle = None

    def info(self):
        return dict(self._i)


SRC = [[(2, 1, 1, 0, 1.0)]]
PRB = [[(2, 2, 2, 0, 1.0)], [(2, 1, 2, 0, 1.0)]]


def test_fdtd_step_checks():
    op = _op()
    f64 = torch.zeros(60, dtype=torch.float64)
    u = torch.zeros((10, 1), dtype=torch.float64)
    y = torch.zeros((10, 2), dtype=torch.float64)
    with pytest.raises(ValueError, match="exactly 60"):
        Y.fdtd_step(op, 1e-12, 10, torch.zeros(59, dtype=torch.float64), SRC, u, PRB, y)
    with pytest.raises(ValueError, match="dtype"):
        Y.fdtd_step(op, 1e-12, 10, f64, SRC, u.float(), PRB, y)
    with pytest.raises(ValueError, match="at least 10"):
        Y.fdtd_step(op, 1e-12, 10, f64, SRC, u[:9], PRB, y)
    with pytest.raises(ValueError, match="at least 20"):
        Y.fdtd_step(op, 1e-12, 10, f64, SRC, u, PRB, y[:9])
    with pytest.raises(ValueError, match="required"):
        Y.fdtd_step(op, 1e-12, 10, f64, SRC, None, PRB, y)
    with pytest.raises(ValueError, match="contiguous"):
        Y.fdtd_step(op, 1e-12, 10, torch.zeros((60, 2), dtype=torch.float64)[:, 0], SRC, u, PRB, y)
    with pytest.raises(ValueError, match="CUDA"):
        Y.fdtd_step(op, 1e-12, 10, f64, SRC, u, PRB, y)
    with pytest.raises(TypeError):
        Y.fdtd_step(op, 1e-12, 10, torch.zeros(60, dtype=torch.int32), SRC, u, PRB, y)


def test_fdtd_adjoint_checks():
    op = _op()
    u = torch.zeros((10, 1), dtype=torch.float32)
    g = torch.zeros((10, 2), dtype=torch.float32)
    with pytest.raises(ValueError, match="probe"):
        Y.fdtd_adjoint(op, 1e-12, 10, SRC, u, None, g)
    with pytest.raises(ValueError, match="at least 20"):
        Y.fdtd_adjoint(op, 1e-12, 10, SRC, u, PRB, g[:5])
    with pytest.raises(ValueError, match="dtype"):
        Y.fdtd_adjoint(op, 1e-12, 10, SRC, u.double(), PRB, g)
    with pytest.raises(ValueError, match="CUDA"):
        Y.fdtd_adjoint(op, 1e-12, 10, SRC, u, PRB, g)


def test_rom_step_checks():
    r = _Rom()
    u = torch.zeros((8, 1), dtype=torch.float32)
    y = torch.zeros((8, 2), dtype=torch.float32)
    st = torch.zeros(11, dtype=torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        Y.rom_step([r], 1e-12, 8, [u.double()], ys=[y])
    with pytest.raises(ValueError, match="at least 8"):
        Y.rom_step([r], 1e-12, 8, [u[:7]], ys=[y])
    with pytest.raises(ValueError, match="at least 16"):
        Y.rom_step([r], 1e-12, 8, [u], ys=[y[:7]])
    with pytest.raises(ValueError, match="exactly 11"):
        Y.rom_step([r], 1e-12, 8, [u], ys=[y], states=[st[:10]])
    with pytest.raises(ValueError, match="per model"):
        Y.rom_step([r, r], 1e-12, 8, [u], ys=[y, y])
    with pytest.raises(ValueError, match="CUDA"):
        Y.rom_step([r], 1e-12, 8, [u], ys=[y], states=[st])


def test_rom_lift_and_adjoint_checks():
    r = _Rom()
    op = _op()
    with pytest.raises(ValueError, match="entries"):
        Y.rom_lift(op, r, torch.zeros((2, 10), dtype=torch.float64))
    with pytest.raises(ValueError, match="exactly 120"):
        Y.rom_lift(op, r, torch.zeros((2, 11), dtype=torch.float64),
                   fields=torch.zeros(119, dtype=torch.float64))
    with pytest.raises(ValueError, match="CUDA"):
        Y.rom_lift(op, r, torch.zeros((2, 11), dtype=torch.float64),
                   fields=torch.zeros(120, dtype=torch.float64))
    u = torch.zeros((6, 1), dtype=torch.float64)
    g = torch.zeros((6, 2), dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        Y.rom_adjoint(r, 1e-12, 6, u.float(), g)
    with pytest.raises(ValueError, match="at least 12"):
        Y.rom_adjoint(r, 1e-12, 6, u, g[:5])
    with pytest.raises(ValueError, match="CUDA"):
        Y.rom_adjoint(r, 1e-12, 6, u, g)


def test_schur_apply_checks():
    op = _op()
    with pytest.raises(ValueError, match="complex"):
        Y.schur_apply(op, 1e-12, 1.1, torch.zeros((2, 20), dtype=torch.float64))
    with pytest.raises(ValueError, match="complex"):
        Y.schur_apply(op, 1e-12, 1.1, torch.zeros((2, 19), dtype=torch.complex128))
    with pytest.raises(ValueError, match="CUDA"):
        Y.schur_apply(op, 1e-12, 1.1, torch.zeros((2, 20), dtype=torch.complex128))
