"""The host planner (symbolic analysis, schedule, workspace layout, and the
checks of the stream schedule and the layout) built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on valid and malformed problems (no GPU).

`tests/planner_check.cpp` reads problem files written here, builds the plan in
both precisions with the schedule and layout checks, checks that the schedule
check refuses plans with planted conflicts, and expects malformed problems to
be refused by the validator; any sanitizer report aborts it."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from tests.conftest import cached_case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_05019_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "planner_check.cpp"), os.path.join(CSRC, "symbolic.cpp"),
           os.path.join(CSRC, "schedule_check.cpp")]
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _write(path, doms, n_mult, imap, xyz=None, valid=True):
    """doms: list of (n, rowptr int64, colind int32); imap: (ptr, dof, mult, sign)."""
    with open(path, "wb") as f:
        f.write(struct.pack("<iqii", len(doms), int(n_mult), 0 if xyz is None else 1, 1 if valid else 0))
        for n, rp, ci in doms:
            f.write(struct.pack("<iq", int(n), int(rp[-1])))
            f.write(np.ascontiguousarray(rp, np.int64).tobytes())
            f.write(np.ascontiguousarray(ci, np.int32).tobytes())
        ptr, dof, mult, sign = imap
        f.write(np.ascontiguousarray(ptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(dof, np.int32).tobytes())
        f.write(np.ascontiguousarray(mult, np.int64).tobytes())
        f.write(np.ascontiguousarray(sign, np.int8).tobytes())
        if xyz is not None:
            f.write(np.ascontiguousarray(xyz, np.float32).tobytes())


def _dump_case(path, c, coordinates=True, valid=True, mutate=None):
    doms = [(d.n, d.K.indptr.astype(np.int64).copy(), d.K.indices.astype(np.int32).copy()) for d in c.domains]
    imap = [np.asarray(c.imap_ptr, np.int64).copy(), np.asarray(c.imap_dof, np.int32).copy(),
            np.asarray(c.imap_mult, np.int64).copy(), np.asarray(c.imap_sign, np.int8).copy()]
    if mutate:
        mutate(doms, imap)
    xyz = np.concatenate([d.xyz for d in c.domains]) if coordinates else None
    _write(path, doms, c.n_mult, imap, xyz, valid)


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("planner")
    probe = d / "probe.cpp"
    probe.write_text("int main() { return 0; }\n")
    if subprocess.run([gxx, *FLAGS, str(probe), "-o", str(d / "probe")], capture_output=True).returncode:
        pytest.skip("sanitizer runtimes not available")
    exe = d / "planner_check"
    r = subprocess.run([gxx, *FLAGS, f"-I{CSRC}", *SOURCES, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe, d


def _run(exe, files):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), *map(str, files)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    if r.returncode != 0 and "LeakSanitizer has encountered a fatal error" in r.stderr:
        # leak checking needs ptrace, which some sandboxes forbid: rerun without it
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
        r = subprocess.run([str(exe), *map(str, files)], capture_output=True, text=True, env=env, timeout=600)
        print(r.stdout[-3000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_planner_valid_problems(planner):
    exe, d = planner
    files = []
    for name, coords in [("cube6", True), ("cube12", True), ("cube18u", True), ("cube16", False)]:
        f = d / f"{name}_{int(coords)}.bin"
        _dump_case(f, cached_case(name), coordinates=coords)
        files.append(f)
    from paper_2002_05019_amd.tetmesh import make_tet_case
    f = d / "tet8.bin"
    _dump_case(f, make_tet_case("tet8"), coordinates=False)
    files.append(f)
    # one domain, no interface
    one = cached_case("cube6", cuts=((0, 6), (0, 6), (0, 6)))
    f = d / "one.bin"
    _dump_case(f, one)
    files.append(f)
    out = _run(exe, files)
    assert out.count("factor launches") == 2 * len(files)
    # the schedule check refuses plans with planted conflicts
    assert out.count("planted conflicts caught") == len(files), out


def test_planner_refuses_malformed_problems(planner):
    exe, d = planner
    c = cached_case("cube6")

    def col_out_of_range(doms, imap):
        doms[1][2][5] = doms[1][0] + 3

    def unsorted_row(doms, imap):
        rp, ci = doms[0][1], doms[0][2]
        r = int(np.argmax(np.diff(rp) >= 3))
        ci[rp[r]], ci[rp[r] + 1] = ci[rp[r] + 1], ci[rp[r]]

    def rowptr_decreasing(doms, imap):
        doms[2][1][3] = doms[2][1][4] + 1

    def bad_sign(doms, imap):
        imap[3][0] = 2

    def mult_out_of_range(doms, imap):
        imap[2][1] = c.n_mult + 7

    def dof_out_of_range(doms, imap):
        imap[1][2] = -1

    files = []
    for k, m in enumerate([col_out_of_range, unsorted_row, rowptr_decreasing, bad_sign, mult_out_of_range,
                           dof_out_of_range]):
        f = d / f"bad{k}.bin"
        _dump_case(f, c, valid=False, mutate=m)
        files.append(f)
    out = _run(exe, files)
    assert out.count("refused") == len(files)
