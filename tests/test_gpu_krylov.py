"""The CG's convergence test runs on the device after every iteration and the
host reads its flags only every check_every iterations: the solution, the
compliance and the iteration count must not depend on check_every (bitwise),
for one load case and for four load cases solved column by column."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _solve(p, every, block_cg):
    import paper_1909_13585_amd as mlb
    c = mlb.Context(p["nel"], mg_levels=3, eig_level=2, precision=mlb.MLB_MIXED)
    c.set_opts(check_every=every, block_cg=block_cg)
    c.set_bc(p["fixed"])
    c.set_loads(p["F"])
    c.set_density(p["x"])
    U, J, si = c.solve_static(tol=1e-9, max_it=2000)
    c.close()
    return U, J, si


@pytest.mark.parametrize("case", ["column_2d", "box_3d_four_cases"])
def test_results_do_not_depend_on_check_every(case):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    if case == "column_2d":
        p = W.column_2d_small()
    else:
        p = W.box_3d_four_cases(nel=(32, 8, 8))
    print(f"case {case}", flush=True)
    ref = _solve(p, 1, 2)
    for every in (3, 8, 50):
        U, J, si = _solve(p, every, 2)
        print(f"check_every {every}: {si['iterations']} iterations (reference {ref[2]['iterations']})")
        assert si["iterations"] == ref[2]["iterations"]
        assert np.array_equal(U, ref[0]) and np.array_equal(J, ref[1])
        assert si["true_rel_residual"] == ref[2]["true_rel_residual"]
