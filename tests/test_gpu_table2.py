"""GPU parity of the Table II formula suite (phi_1 .. phi_6: invariance,
stabilization, strict ordering, sequenced visits, sequenced visit +
stabilization, regions in any order) with synthetic linear predicates, hard
and smooth, against the FP64 oracle, through the C ABI.  The hard variants
are also compared bit for bit: the oracle's temporal part run on the GPU's
own float32 predicate traces must give the GPU's float32 node traces."""
import numpy as np
import pytest

import oracle
from gpu_util import Gpu, assert_close, check_formula
from paper_2501_04194_amd import workloads as W

pytestmark = pytest.mark.gpu


def _kinds(spec):
    out = []

    def walk(f):
        for k in ("child", "left", "right"):
            if k in f:
                walk(f[k])
        for c in f.get("children", []):
            walk(c)
        out.append(f["op"])
    walk(spec)
    return out


@pytest.mark.parametrize("smooth", [False, True])
@pytest.mark.parametrize("name", ["phi1", "phi2", "phi3", "phi4", "phi5", "phi6"])
def test_table2_formula(name, smooth):
    spec = W.table2_formulas(smooth=smooth)[name]
    for T in (64, 333):
        x = W.random_walks(50 + T, 8, T, 2, 0.1)
        # smooth And over an empty-window sentinel and finite values rounds to
        # 1e6 in fp64 but only to within a few float32 ulps of it
        check_formula(spec, x, what="%s %s T=%d" % (name, "smooth" if smooth else "hard", T),
                      exact_sentinels=not smooth)


@pytest.mark.parametrize("name", ["phi1", "phi2", "phi3", "phi4", "phi5", "phi6"])
def test_table2_hard_bitexact(name):
    spec = W.table2_formulas(smooth=False)[name]
    kinds = _kinds(spec)
    leaves = [i for i, k in enumerate(kinds) if k in ("linear", "norm")]
    for T in (64, 333):
        x = W.random_walks(50 + T, 8, T, 2, 0.1)
        g = Gpu(spec, 2)
        root, traces = g.fwd(x, traces=True)
        _, ref_tr = oracle.forward(spec, x, all_nodes=True)
        for i in leaves:
            assert_close(traces[i], ref_tr[i], what="%s pred %d" % (name, i))
        lt = {i: traces[i].astype(np.float64) for i in leaves}
        mine_root, mine = oracle.forward(spec, x, leaf_traces=lt, all_nodes=True)
        assert np.array_equal(root, mine_root.astype(np.float32)), "%s T=%d root not bit-exact" % (name, T)
        for i in range(len(kinds)):
            if i not in leaves:
                assert np.array_equal(traces[i], mine[i].astype(np.float32)), "%s T=%d node %d" % (name, T, i)
