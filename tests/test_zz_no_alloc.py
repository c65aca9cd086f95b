"""The allocation-free L2 error (igamg_l2_error_noalloc) against the
allocating entry point (igamg_l2_error): both run the same kernels in the
same fixed summation order, so the values must agree (the bar is 1e-14
relative; identical bits are expected).  Two calls in a row on the shared
device scratch, the second on a smaller problem, so that a value left in
the scratch by the first call cannot leak into the second."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solved(cfg_elems, p, dim=2):
    from paper_1902_01818_amd import igamg
    if dim == 2:
        corners = workloads.config("c1")["corners"]
    else:
        corners = workloads.config("c3", 8)["corners"]
    elems = np.full((corners.shape[0], dim), cfg_elems, dtype=np.int32)
    conforming = dim == 2
    sv = igamg.Solver(corners, elems, p, 5.0, conforming=conforming,
                      smoother="scms" if conforming else "hybrid",
                      tau=0.5 if conforming else 0.25, delta=0.12 if conforming else 0.1)
    f = sv.load_manufactured()
    u, info = sv.solve(f, tol=1e-12, maxit=200)
    return sv, u


@pytest.mark.parametrize("first,second", [((64, 3, 2), (16, 2, 2)), ((12, 3, 3), (8, 2, 2))])
def test_noalloc_l2_error_matches_allocating(first, second):
    for ne, p, dim in (first, second):
        print("noalloc L2 error: dim %d, %d elements per patch direction, p %d" % (dim, ne, p),
              flush=True)
        sv, u = _solved(ne, p, dim)
        ref = sv.l2_error(u)
        got = sv.l2_error_noalloc(u)
        again = sv.l2_error_noalloc(u)
        sv.close()
        assert np.isfinite(ref) and ref > 0
        assert abs(got - ref) <= 1e-14 * ref, (got, ref)
        assert got == again
        # the value is the discretization error: small at these sizes
        assert ref < 1e-2
