"""The allocation-free binding (dd_bind_static_workspace), through the C ABI:
for callers that cannot allocate device memory, the workspace is the
library's static device array.  Two problems bound in a row, the second
smaller, each factored and solved on the array and compared with the same
problem on a caller-owned workspace (dd_bind_workspace): the kernels are the
same, so the solutions agree bit for bit (beyond the 1e-10 / 1e-9 gates).
The first context is refused once the second owns the array, and a problem
larger than the array is refused."""
import numpy as np
import pytest

from tests.conftest import cached_case
from tests.test_gpu_parity import DEV, _rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _vals(c):
    return torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV)


def _solve(s, c):
    s.factor(_vals(c))
    u = s.solve(_rhs(c))
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_static_workspace_matches_caller_workspace(precision):
    from paper_2002_05019_amd.binding import STATIC_WORKSPACE_BYTES, DDError, Solver
    big, small = cached_case("cube12"), cached_case("cube6")
    print(f"[no-alloc] {precision}: cube12 then cube6 on the static array", flush=True)
    s1 = Solver.from_case(big, precision=precision, max_rhs=8)
    assert s1.workspace_bytes <= STATIC_WORKSPACE_BYTES
    s1.bind_static(DEV)
    u1 = _solve(s1, big)
    r1 = _solve(Solver.from_case(big, precision=precision, max_rhs=8).bind(DEV), big)
    assert np.array_equal(u1, r1)
    s2 = Solver.from_case(small, precision=precision, max_rhs=8)
    assert s2.workspace_bytes < s1.workspace_bytes
    s2.bind_static(DEV)
    u2 = _solve(s2, small)
    r2 = _solve(Solver.from_case(small, precision=precision, max_rhs=8).bind(DEV), small)
    assert np.array_equal(u2, r2)
    # the array now holds the second context's tables and factors
    with pytest.raises(DDError) as e:
        s1.solve(_rhs(big))
    assert e.value.status == -4   # DD_ERR_STATE
    # rebinding makes the first context usable again
    s1.bind_static(DEV)
    assert np.array_equal(_solve(s1, big), r1)


def test_static_workspace_refuses_large_problems():
    from paper_2002_05019_amd.binding import STATIC_WORKSPACE_BYTES, DDError, Solver
    c = cached_case("cube16")
    s = Solver.from_case(c)
    assert s.workspace_bytes > STATIC_WORKSPACE_BYTES
    with pytest.raises(DDError) as e:
        s.bind_static(DEV)
    assert e.value.status == -5   # DD_ERR_NOMEM
