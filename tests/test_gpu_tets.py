"""GPU parity on unstructured tetrahedral meshes split by the project's graph
partitioner (section III: the paper's models are unstructured meshes of a
dielectric sphere and of antenna arrays).  Irregular domains with many
neighbours give a denser auxiliary matrix than box decompositions; the
orderings run with the DoF coordinates and graph-only (no coordinates).
FP64 against the oracle's serial DD solve (solution, multipliers,
interface inverses: 1e-10); FP32 + refinement: the undecomposed residual
and the error against the oracle within 1e-9."""
import numpy as np
import pytest

import oracle
from tests.test_gpu_parity import DEV, _colerr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_CASES, _REF = {}, {}


def _case(name):
    from paper_2002_05019_amd.tetmesh import make_tet_case
    if name not in _CASES:
        _CASES[name] = make_tet_case(name)
        _REF[name] = oracle.serial_dd(_CASES[name])
    return _CASES[name], _REF[name]


def _solve(c, precision, coords, **kw):
    from paper_2002_05019_amd.binding import Solver
    s = Solver.from_case(c, precision=precision, coordinates=coords, **kw).bind(DEV)
    s.factor(torch.from_numpy(np.concatenate([d.K.data for d in c.domains])).to(DEV))
    u, lam = s.solve(torch.from_numpy(c.torn_rhs()).to(DEV), return_lam=True)
    torch.cuda.synchronize()
    return s, u.cpu().numpy(), lam.cpu().numpy()


@pytest.mark.parametrize("coords", [True, False])
@pytest.mark.parametrize("name", ["tet8", "tet12s", "tet16"])
def test_tet_fp64(name, coords):
    c, ref = _case(name)
    print(f"[tet] {name} fp64 coords={coords}: {c.n_global} unknowns, {c.n_dom} domains", flush=True)
    s, u, lam = _solve(c, "fp64", coords)
    eu, el = _colerr(u, ref["u"]), _colerr(lam, ref["lam"])
    print(f"[tet] {name} fp64 coords={coords}: u {eu:.2e} lam {el:.2e}", flush=True)
    assert s.last_status == 0 and s.info()["n_perturbed"] == 0
    assert eu < 1e-10 and el < 1e-10
    for i in (0, c.n_dom - 1):
        X = s.interface_inverse(i).cpu().numpy()
        R = ref["S_inv"][i]
        assert np.abs(X - R).max() / np.abs(R).max() < 1e-10


@pytest.mark.parametrize("name", ["tet12s", "tet16"])
def test_tet_mixed(name):
    c, ref = _case(name)
    print(f"[tet] {name} fp32+refine graph-only", flush=True)
    s, u, _ = _solve(c, "fp32_refine", False)
    gr = oracle.global_residual(c, u).max()
    eu = _colerr(u, ref["u"])
    print(f"[tet] {name} mixed: iters {s.info()['refine_iters']} resid {gr:.2e} err {eu:.2e}", flush=True)
    assert s.last_status == 0
    assert gr <= 1e-9 and eu <= 1e-9
