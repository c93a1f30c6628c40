"""The LDS poisoning option (debug_fill_lds): every segment workgroup fills
its LDS with NaN before use, in the forward pass and in the backward pass
that differentiates it.  A kernel that read a value it never wrote would
turn outputs into NaN or change them; the option must leave every output
bit for bit as it is without it, for the launch shapes, both schedules and
the ADMM warm start, and the forward outputs must still match the oracle."""
import numpy as np
import pytest
import torch

from tests.parity_helpers import compare
from workloads import gen

pytestmark = pytest.mark.gpu


def run(batch, **kw):
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import SegmentBatchGPU
    o = _lib.default_opts()
    o.store_for_backward = 1
    for k, v in kw.items():
        assert k in {f[0] for f in _lib.SolveOpts._fields_}, k
        setattr(o, k, v)
    gb = SegmentBatchGPU(batch)
    x0 = torch.as_tensor(batch.x0, device=gb.device).contiguous()
    goal = torch.as_tensor(batch.goal, device=gb.device).contiguous()
    res = gb.solve(x0, goal, opts=o)
    rng = np.random.default_rng(3)
    gP = torch.as_tensor(rng.standard_normal(res.P.numel()), device=gb.device)
    gC = torch.ones(batch.n, dtype=torch.float64, device=gb.device)
    g = gb.backward(gP, gC)
    torch.cuda.synchronize()
    out = dict(P=res.P.cpu().numpy(), cost=res.cost.cpu().numpy(), status=res.status.cpu().numpy(),
               kkt=res.kkt.cpu().numpy(), iters=res.iters.cpu().numpy(), gx0=g.x0.cpu().numpy(),
               ggoal=g.goal.cpu().numpy(), gb=g.b_inst.cpu().numpy())
    gb.close()
    return out


def same_bits(a, b, label):
    for k in a:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.shape == y.shape, (label, k)
        if x.dtype.kind == "f":
            assert np.array_equal(x.view(np.int64), y.view(np.int64)), (label, k)
        else:
            assert np.array_equal(x, y), (label, k)


@pytest.mark.parametrize("case", ["seg64", "edges1500", "uneven1200"])
@pytest.mark.parametrize("launch", [dict(), dict(launch_shape=1), dict(launch_shape=2), dict(schedule=1),
                                    dict(admm_iters=10)])
def test_poisoned_lds_changes_nothing(gpu_available, case, launch):
    b = {"seg64": lambda: gen.gen_cfg0(64), "edges1500": lambda: gen.gen_cfg1(indices=range(1500)),
         "uneven1200": lambda: gen.gen_cfg2(indices=range(1200))}[case]()
    kw = dict(launch)
    kw.setdefault("admm_iters", 0)
    print(f"case: {case}, options {kw}, LDS poisoned vs not", flush=True)
    ref = run(b, debug_fill_lds=0, **kw)
    out = run(b, debug_fill_lds=1, **kw)
    same_bits(ref, out, f"{case} {kw}")
    if case == "seg64":
        compare(b, out["P"], out["cost"], out["status"], out["kkt"], label=f"{case} poisoned")


def test_option_is_validated(gpu_available):
    from paper_2411_13507_amd import _lib
    b = gen.gen_cfg0(8)
    for field, value in (("debug_fill_lds", 2), ("reserved", 1)):
        with pytest.raises(Exception):
            run(b, **{field: value})
