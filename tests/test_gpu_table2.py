"""GPU parity of the Table II formula suite (phi_1 .. phi_6: invariance,
stabilization, strict ordering, sequenced visits, sequenced visit +
stabilization, regions in any order) with synthetic linear predicates, hard
and smooth, against the FP64 oracle, through the C ABI."""
import pytest

from gpu_util import check_formula
from paper_2501_04194_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("smooth", [False, True])
@pytest.mark.parametrize("name", ["phi1", "phi2", "phi3", "phi4", "phi5", "phi6"])
def test_table2_formula(name, smooth):
    spec = W.table2_formulas(smooth=smooth)[name]
    for T in (64, 333):
        x = W.random_walks(50 + T, 8, T, 2, 0.1)
        check_formula(spec, x, what="%s %s T=%d" % (name, "smooth" if smooth else "hard", T))
