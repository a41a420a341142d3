"""stl_forward_static (the forward whose workspace is the library's fixed
device array) against stl_forward on the same inputs: bit for bit, on two
calls in a row with the second input smaller, for the matrix-core path, the
generic executor (smooth Until) and node traces; and its host-side refusal of
a batch whose workspace exceeds the array."""
import numpy as np
import pytest

from paper_2501_04194_amd import stl, workloads as W

pytestmark = pytest.mark.gpu


def _pair(spec, D, params, xs, node_traces=False, launch=None):
    import torch
    plan = stl.Plan(spec, D, params)
    pv = torch.from_numpy(plan.param_vector()).cuda()
    for x in xs:
        print("forward_static: B=%d T=%d traces=%s" % (x.shape[0], x.shape[1], node_traces), flush=True)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        ref = plan.forward(xd, pv, node_traces=node_traces, launch=launch)
        got = plan.forward_static(xd, pv, node_traces=node_traces, launch=launch)
        torch.cuda.synchronize()
        if node_traces:
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
        else:
            assert torch.equal(got, ref)


def test_static_forward_matrix_core_path():
    spec, params, x1 = W.workload(2, B=300, T=1500)
    _, _, x2 = W.workload(2, B=40, T=700)
    x1[7, 700:, 0] += 25.0          # one trajectory handed off to the generic executor
    _pair(spec, 2, params, [x1, x2])


def test_static_forward_generic_executor_and_traces():
    spec, params, x1 = W.workload(1, B=64, T=512)
    _, _, x2 = W.workload(1, B=9, T=300)
    _pair(spec, x1.shape[-1], params, [x1, x2])
    _pair(spec, x1.shape[-1], params, [x1[:20, :400], x2[:5, :100]], node_traces=True)


def test_static_forward_rejects_oversized_workspace():
    import torch
    spec, params, x0 = W.workload(1, B=2, T=16)
    D = x0.shape[-1]
    plan = stl.Plan(spec, D, params)
    pv = torch.from_numpy(plan.param_vector()).cuda()
    x = torch.zeros((2048, 4096, D), dtype=torch.float32, device="cuda")
    glob = stl.Launch(256, 0, 1, 0)            # node traces in the workspace: far beyond the array
    with pytest.raises(stl.StlError, match="static"):
        plan.forward_static(x, pv, launch=glob)
