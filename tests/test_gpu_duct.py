"""The duct experiment of Sec. 5.1 on the GPU path (FP64): the improved
equilibrium keeps the transverse velocity at rounding level; the standard one
shows spurious currents that converge at second order for Lambda^2 = 4/25 and
at fourth order for Lambda^2 = 1/12, with the smallest error at 1/12."""
import json

import pytest

pytestmark = pytest.mark.gpu

SIZES = [25, 45, 65, 95, 135]   # within the paper's range 15 ... 135


def _run(lam2, eq, sizes=SIZES):
    from paper_1803_04937_amd.experiments import duct_spurious_current
    return [duct_spurious_current(D, lam2, eq) for D in sizes]


@pytest.mark.parametrize("lam2,order,tol", [(4 / 25, 2.0, 0.25), (1 / 12, 4.0, 0.4)],
                         ids=["4/25", "1/12"])
def test_standard_spurious_current_order(lam2, order, tol):
    from paper_1803_04937_amd.experiments import convergence_order
    rows = _run(lam2, "standard")
    got = convergence_order(rows)
    print("\nduct standard", json.dumps({"lambda2": lam2, "order": got,
                                         "ratios": [(r["D"], r["ratio"]) for r in rows]}))
    for r in rows:
        assert r["last_chunk_rel_change"] < 1e-6
    # measured on MI355X: -2.08 (4/25) and -3.81 (1/12)
    assert abs(-got - order) < tol, got


@pytest.mark.parametrize("lam2", [4 / 25, 1 / 12], ids=["4/25", "1/12"])
def test_improved_has_no_spurious_current(lam2):
    rows = _run(lam2, "improved")
    print("\nduct improved", json.dumps({"lambda2": lam2,
                                         "ratios": [(r["D"], r["ratio"]) for r in rows]}))
    for r in rows:   # measured: 8e-16 ... 1.2e-14
        assert r["ratio"] < 1e-13, r


def test_standard_error_is_smallest_at_lambda2_one_twelfth():
    from paper_1803_04937_amd.experiments import duct_spurious_current
    lams = [0.02, 0.04, 0.06, 1 / 12, 0.1, 0.12, 0.16]
    ratios = [duct_spurious_current(65, l2, "standard")["ratio"] for l2 in lams]
    print("\nduct lambda sweep D=65", json.dumps(list(zip(lams, ratios))))
    assert min(range(len(lams)), key=lambda i: ratios[i]) == lams.index(1 / 12)
