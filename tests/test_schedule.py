"""Host check of the factorisation's stream schedule (no GPU).

The factorisation overlaps its latency-bound pivot chain with the trailing
update on a side stream.  ``verify_schedule`` replays the plan's fork / join points and fails
``dd_setup`` if two launches that those leave unordered touch the same front
data with at least one write.  It also checks the memory plan: fronts share
one arena, each alive from its own level to its parent's (which gathers its
update block), so the full matrices of fronts alive at the same level must be
disjoint, and the stored factors must not overlap each other."""
import pytest

from paper_2002_05019_amd.binding import Solver
from tests.conftest import cached_case


@pytest.mark.parametrize("name", ["cube12", "cube16", "cube18u", "cube24"])
@pytest.mark.parametrize("tiles", [None, [64] * 5, [128] * 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_side_streams_touch_disjoint_data(name, tiles, precision):
    Solver.from_case(cached_case(name), precision=precision, schur_tile=tiles, verify_schedule=True)


def test_uneven_batch_schedule():
    """Uneven fronts of the 216-domain workload in one batch (partial pivot
    tiles everywhere, fronts ending in different outer blocks)."""
    Solver.from_case(cached_case("cube64j"), precision="fp32_refine", verify_schedule=True)

