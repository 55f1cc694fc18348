"""Shared helpers of the GPU parity tests: run the HIP library through its C
ABI and the FP64 oracle on the same seeded inputs, and compare them."""
import numpy as np
import torch

import oracle as O
from paper_1110_0740_amd import ctu, inputs as I

DEV = torch.device("cuda:0")


def l1rel(got, ref, ng, dim, ch=1.0, physics="mhd"):
    """Per-variable relative L1 over interior cells, sum|got - ref| / S_q.

    S_q = sum|ref_q|, except for variables that can vanish identically over a
    region, which are measured against their natural scale instead:
    momentum components against sum sqrt(2 rho E) (MHD, |m|^2 <= 2 rho E) or
    sum (E + D) (RMHD, |m| <= E + D); each B component against sum|B|/3;
    psi against c_h sum|B|/3."""
    g = I.interior(got, ng, dim).reshape(9, -1).astype(np.float64)
    r = I.interior(ref, ng, dim).reshape(9, -1)
    num = np.abs(g - r).sum(axis=1)
    den = np.abs(r).sum(axis=1)
    if physics == "rmhd":
        mscale = (np.abs(r[4]) + np.abs(r[0])).sum()
    else:
        mscale = np.sqrt(2.0 * np.abs(r[0]) * np.abs(r[4])).sum()
    bscale = np.sqrt((r[5:8] ** 2).sum(axis=0)).sum() / 3.0
    for q in (1, 2, 3):
        den[q] = max(den[q], mscale)
    for q in (5, 6, 7):
        den[q] = max(den[q], bscale)
    den[8] = max(den[8], ch * bscale)
    return num / np.maximum(den, 1e-300)


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
