"""Host-side argument checks of the Python binding: a buffer with the wrong
dtype, too few elements, a non-contiguous layout, aliased input and output,
or one that is not on the plan's GPU is refused before any C call (the
kernels size their ranges from the plan, not from the tensors)."""
import pytest
import torch

from paper_1110_0740_amd import ctu


class HostPlan(ctu.Plan):
    """A Plan whose C handle is never created: only the checks run."""

    def __init__(self, precision="fp32", state_elems=9 * 100, nslots=2, cooling=False):
        self.opts = ctu.make_opts(precision=precision, cooling=cooling)
        self.device = 0
        self.nslots = nslots
        self._se = state_elems
        self._h = None

    @property
    def state_elems(self):
        return self._se


def _bufs(dt=torch.float32, n=900):
    return dict(U_in=torch.zeros(n, dtype=dt), U_out=torch.zeros(n, dtype=dt),
                params=torch.zeros(2, dtype=torch.float64), rate=torch.zeros(1, dtype=torch.float64),
                reg=torch.zeros(18, dtype=torch.float64))


def _step(p, b, **kw):
    b = dict(b, **kw)
    p.step(b["U_in"], b["U_out"], b["params"], b["rate"], reg=b["reg"], L0=b.get("L0"), fails=b.get("fails"))


def test_dtype_must_match_the_plan_precision():
    with pytest.raises(ValueError, match="U_in must be torch.float32"):
        _step(HostPlan("fp32"), _bufs(torch.float64))
    with pytest.raises(ValueError, match="U_in must be torch.float64"):
        _step(HostPlan("fp64"), _bufs(torch.float32))
    with pytest.raises(ValueError, match="fails must be torch.int32"):
        _step(HostPlan(), _bufs(), fails=torch.zeros(5, dtype=torch.int64))


def test_short_buffers_are_refused():
    b = _bufs()
    with pytest.raises(ValueError, match="U_out needs at least 900"):
        _step(HostPlan(), b, U_out=torch.zeros(899))
    with pytest.raises(ValueError, match="reg needs at least 18"):
        _step(HostPlan(), b, reg=torch.zeros(17, dtype=torch.float64))
    with pytest.raises(ValueError, match="params needs at least 2"):
        _step(HostPlan(), b, params=torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError, match="cool_L0 needs at least 100"):
        _step(HostPlan(cooling=True), b, L0=torch.zeros(99))


def test_required_buffers_and_aliasing():
    b = _bufs()
    with pytest.raises(ValueError, match="reg is required"):
        _step(HostPlan(), b, reg=None)
    with pytest.raises(ValueError, match="cool_L0 is required"):
        _step(HostPlan(cooling=True), b)
    with pytest.raises(ValueError, match="alias"):
        _step(HostPlan(), b, U_out=b["U_in"])
    with pytest.raises(ValueError, match="contiguous"):
        _step(HostPlan(), b, U_in=torch.zeros(1800)[::2])


def test_host_tensors_are_refused():
    with pytest.raises(ValueError, match="CUDA tensor"):
        _step(HostPlan(), _bufs())


def test_plan_exposes_its_sizes_and_releases_its_handle():
    for name in ("state_elems", "workspace_bytes", "dtype"):
        assert isinstance(getattr(ctu.Plan, name), property), name
    for name in ("__del__", "step", "step_static", "graph_capture", "autotune", "set_shape", "reflux"):
        assert callable(getattr(ctu.Plan, name)), name
    assert HostPlan("fp64").dtype == torch.float64 and HostPlan("fp32").dtype == torch.float32
