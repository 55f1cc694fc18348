"""Shared helpers of the GPU parity tests: run the HIP library through its C
ABI and the FP64 oracle on the same seeded inputs, and compare them."""
import numpy as np
import torch

import oracle as O
from paper_1110_0740_amd import ctu, inputs as I

DEV = torch.device("cuda:0")


def _scales(r, ch, physics):
    """Per-variable denominators of the parity norms (r: 9 x ncell oracle).

    MHD: every conserved variable is measured against its own magnitude,
    sum|ref_q| for the L1 norm and max|ref_q| for the per-cell bound; only
    psi, which starts at zero and is driven by c_h div B, is measured against
    its natural scale c_h |B| / 3 where that is larger.  RMHD: the workload's
    resting background makes the momentum and field components vanish over
    large regions, so they are measured against their natural scales where
    larger: momentum against E + D (|m| <= E + D), each B component against
    |B| / 3, psi against c_h |B| / 3."""
    l1 = np.abs(r).sum(axis=1)
    mx = np.abs(r).max(axis=1)
    bmag = np.sqrt((r[5:8] ** 2).sum(axis=0))
    if physics == "rmhd":
        ms = np.abs(r[4]) + np.abs(r[0])
        for q in (1, 2, 3):
            l1[q] = max(l1[q], ms.sum())
            mx[q] = max(mx[q], ms.max())
        for q in (5, 6, 7):
            l1[q] = max(l1[q], bmag.sum() / 3.0)
            mx[q] = max(mx[q], bmag.max() / 3.0)
    l1[8] = max(l1[8], ch * bmag.sum() / 3.0)
    mx[8] = max(mx[8], ch * bmag.max() / 3.0)
    return np.maximum(l1, 1e-300), np.maximum(mx, 1e-300)


def l1rel(got, ref, ng, dim, ch=1.0, physics="mhd"):
    """Per-variable relative L1 over interior cells, sum|got - ref| / S_q
    (S_q from _scales)."""
    g = I.interior(got, ng, dim).reshape(9, -1).astype(np.float64)
    r = I.interior(ref, ng, dim).reshape(9, -1)
    return np.abs(g - r).sum(axis=1) / _scales(r, ch, physics)[0]


def cellrel(got, ref, ng, dim, ch=1.0, physics="mhd"):
    """Per-variable largest single-cell difference over interior cells,
    max|got - ref| / M_q (M_q = max|ref_q|, natural scales as in _scales)."""
    g = I.interior(got, ng, dim).reshape(9, -1).astype(np.float64)
    r = I.interior(ref, ng, dim).reshape(9, -1)
    return np.abs(g - r).max(axis=1) / _scales(r, ch, physics)[1]


# per-cell bounds beside the L1 tolerances: one step from identical inputs
CELL64 = 1e-10
CELL32 = 1e-4


def cell_tol(tol):
    """Per-cell bound that goes with an L1 tolerance (FP64 or FP32 scale)."""
    return CELL64 if tol < 1e-9 else CELL32


def assert_parity(got, ref, ng, dim, ch, tol, physics="mhd", ctol=None, what=""):
    """L1 per variable <= tol and every cell within the per-cell bound."""
    e = l1rel(got, ref, ng, dim, ch, physics)
    c = cellrel(got, ref, ng, dim, ch, physics)
    ctol = cell_tol(tol) if ctol is None else ctol
    assert e.max() <= tol, (what, "L1", e)
    assert c.max() <= ctol, (what, "cell", c)
    return e, c


def oracle_opts(dim, dx, gamma, **kw):
    return O.make_opts(dim=dim, dx=dx, gamma=gamma, **kw)


def gpu_opts(dim, dx, gamma, precision="fp64", **kw):
    return ctu.make_opts(dim=dim, dx=dx, gamma=gamma, precision=precision, **kw)


def single_box_plan(gopts, shape_interior, ng, regfaces=None):
    n = tuple(shape_interior) + (1,) * (3 - len(shape_interior))
    return ctu.Plan(gopts, [((0, 0, 0), n, 0, 0)], ng, regfaces=regfaces)


def tdtype(precision):
    return torch.float32 if precision == "fp32" else torch.float64


class GpuStepper:
    """Holds device buffers for repeated steps of one plan."""

    def __init__(self, plan, shape, precision, nreg=0):
        self.plan = plan
        self.shape = shape
        self.dt = tdtype(precision)
        self.Uin = torch.zeros(int(np.prod(shape)), dtype=self.dt, device=DEV)
        self.Uout = torch.zeros_like(self.Uin)
        self.params = torch.zeros(2, dtype=torch.float64, device=DEV)
        self.rate = torch.zeros(1, dtype=torch.float64, device=DEV)
        self.dpp = torch.zeros(1, dtype=torch.float64, device=DEV)
        self.fails = torch.zeros(5, dtype=torch.int32, device=DEV)
        self.reg = torch.zeros(max(1, nreg) * 9, dtype=torch.float64, device=DEV) if nreg else None

    def step(self, U, dt, ch, L0=None):
        self.Uin.copy_(torch.from_numpy(np.ascontiguousarray(U).reshape(-1)).to(self.dt))
        self.Uout.copy_(self.Uin)
        self.params.copy_(torch.tensor([dt, ch], dtype=torch.float64))
        L0d = None
        if L0 is not None:
            L0d = torch.from_numpy(np.ascontiguousarray(L0).reshape(-1)).to(self.dt).to(DEV)
        self.plan.step(self.Uin, self.Uout, self.params, self.rate, L0=L0d, reg=self.reg, dpp=self.dpp,
                       fails=self.fails)
        torch.cuda.synchronize()
        out = self.Uout.cpu().numpy().astype(np.float64).reshape(self.shape)
        return out, float(self.rate.item()), float(self.dpp.item()), self.fails.cpu().tolist()
