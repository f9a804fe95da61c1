"""The committed Schur-update traffic record (no GPU): ``bench.py`` reports it
only for the kernel source, tile policy and launch count it was measured on,
and ``--gpus`` above 1 is refused."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _record():
    with open(os.path.join(ROOT, "profiles", "schur_update_cube48_traffic.json")) as fh:
        return json.load(fh)


def _current_record(tmp_path):
    """The committed record re-keyed to the current kernel source."""
    import hashlib
    rec = _record()
    with open(os.path.join(ROOT, "paper_2002_05019_amd", "csrc", "kernels.hip"), "rb") as fh:
        rec["kernels_hip_sha256"] = hashlib.sha256(fh.read()).hexdigest()
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    return rec, str(path)


def test_record_reported_for_its_plan(tmp_path):
    rec, path = _current_record(tmp_path)
    got = bench.recorded_traffic("cube48", rec["schur_tile_by_front_size"], rec["launches_per_factorization"], path=path)
    assert got == rec["bytes_per_launch"] > 0


def test_record_refused_for_other_plans(tmp_path):
    rec, path = _current_record(tmp_path)
    tiles = rec["schur_tile_by_front_size"]
    per = rec["launches_per_factorization"]
    assert rec["launches"] == 2 * per   # the counter run's two factorisations
    assert bench.recorded_traffic("cube48", tiles, per + 1, path=path) is None
    assert bench.recorded_traffic("cube48", tiles, rec["launches"], path=path) is None
    assert bench.recorded_traffic("cube48", [128] * len(tiles), per, path=path) is None
    assert bench.recorded_traffic("no_such_workload", tiles, per) is None
    stale = dict(rec, kernels_hip_sha256="0" * 64)
    (tmp_path / "stale.json").write_text(json.dumps(stale))
    assert bench.recorded_traffic("cube48", tiles, per, path=str(tmp_path / "stale.json")) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr), r.stdout + r.stderr


def test_global_direct_model():
    """The footprint model of the undecomposed sparse direct factor that the
    memory record compares against: every non-PEC edge (3 n (n-1)^2 of an n^3
    PEC cube) is eliminated exactly once, the 6^3 and 48^3 figures are the
    closed-form recursion's (4.44e6 flop; 2.21e8 factor entries = 3.54 GB in
    complex FP64, 2.46e12 flop), and SuperLU's own ordering of the same
    matrix lands in the same range (nnz(L + U) / 2 against the model's
    symmetric factor)."""
    import scipy.sparse.linalg as spl

    from tests.conftest import cached_case
    for n in (4, 6, 12, 24, 48):
        assert bench.global_direct_model(n)["eliminated"] == 3 * n * (n - 1) ** 2
    m6 = bench.global_direct_model(6)
    assert abs(m6["fma"] * 8 - 4.4394e6) < 1e3
    m48 = bench.global_direct_model(48)
    assert m48["nnz"] == 221021208
    assert abs(m48["fma"] * 8 / 2.4607e12 - 1) < 1e-3
    for name, n in (("cube12", 12), ("cube16", 16)):
        A = cached_case(name).A.tocsc()
        lu = spl.splu(A)
        ratio = (lu.L.nnz + lu.U.nnz) / 2 / bench.global_direct_model(n)["nnz"]
        print(f"[model] {name}: SuperLU nnz(L+U)/2 over the model's nnz(L): {ratio:.2f}")
        assert 0.5 < ratio < 4
