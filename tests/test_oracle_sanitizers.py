"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

tests/oracle_sanitize_driver.c calls every exported function of
oracle/ctrex_oracle.c once on small seeded inputs (plain and warped
projections with a view list that repeats a view, both backprojectors, the
ellipsoid indicator, voxel points, the cylindrical pair with a pose).  Built
with -fsanitize=address,undefined and no recovery, any out-of-bounds access,
use after free, leak, signed overflow or misaligned access ends the run with
an error.  Its outputs must equal those of the ordinary build (same
arithmetic: no OpenMP, no contraction, so the same sums in the same order up
to the backprojection's thread partition, compared at 1e-12).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NP, NS, NU, NV = 3, 2, 24, 20
SHAPE = (9, 12, 10)            # (nz, ny, nx)
CYL = (6, 16, 9, 1.5, 1.0)     # (n_r, n_phi, n_z, dr, dz)
VIEWS = [2, 0, 2, 1]


def _gcc_has_sanitizers(tmp):
    src = os.path.join(tmp, "probe.c")
    with open(src, "w") as f:
        f.write("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", src, "-o",
                        os.path.join(tmp, "probe")], capture_output=True)
    return r.returncode == 0


def _inputs(rng):
    P = synth.circular_cone(NP, NU, NV, 40.0, 80.0, 1.0, n_sub=NS, arc=2.0,
                            det_offset_u=0.4)
    vol = rng.uniform(0.0, 1.0, SHAPE)
    sino = rng.normal(size=(NP, NV, NU))
    U = rng.normal(0.0, 0.6, (4, 4, 4, 3))
    tau = rng.uniform(-0.5, 0.5, (NP, NS))
    Q = np.diag([1 / 9.0, 1 / 16.0, 1 / 6.0])
    centre = np.array([4.3, 5.1, 3.9])           # (x, y, z) index coordinates
    a = 0.3
    pose = np.array([[np.cos(a), -np.sin(a), 0.0, 0.4],
                     [np.sin(a), np.cos(a), 0.0, -0.2],
                     [0.0, 0.0, 1.0, 0.3]])
    cvol = rng.uniform(0.0, 1.0, (CYL[2], CYL[1], CYL[0]))
    ijk = np.array([[0, 0, 0], [9, 11, 8], [4, 6, 3], [1, 10, 7], [8, 2, 5]], np.int32)
    return P, vol, sino, U, tau, Q, centre, pose, cvol, ijk


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    tmp = str(tmp_path)
    if shutil.which("gcc") is None or not _gcc_has_sanitizers(tmp):
        pytest.skip("gcc with the sanitizer runtimes is not available")
    rng = np.random.default_rng(20)
    P, vol, sino, U, tau, Q, centre, pose, cvol, ijk = _inputs(rng)
    for name, arr in (("P", P), ("vol", vol), ("sino", sino), ("U", U), ("tau", tau),
                      ("Q", Q), ("centre", centre), ("pose", pose), ("cvol", cvol)):
        np.ascontiguousarray(arr, np.float64).tofile(os.path.join(tmp, name + ".bin"))
    ijk.tofile(os.path.join(tmp, "ijk.bin"))

    exe = os.path.join(tmp, "driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "ctrex_oracle.c"), "-lm", "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, tmp], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"

    def out(name, shape, dtype=np.float64):
        return np.fromfile(os.path.join(tmp, name), dtype=dtype).reshape(shape)

    def close(a, b):
        return np.linalg.norm(a - b) <= 1e-12 * max(np.linalg.norm(b), 1e-300)

    shape = SHAPE
    y, n0 = oracle.forward(P, shape, NU, NV, vol, 0.5, return_count=True)
    assert close(out("fwd.bin", (NP, NV, NU)), y)
    yw, n1 = oracle.forward(P, shape, NU, NV, vol, 0.7, views=VIEWS, U=U, tau=tau,
                            return_count=True)
    assert close(out("fwd_warp.bin", (4, NV, NU)), yw)
    assert close(out("back.bin", shape), oracle.back(P, shape, NU, NV, sino, 0.5))
    assert close(out("back_warp.bin", shape),
                 oracle.back(P, shape, NU, NV, sino, 0.7, views=VIEWS[:3], U=U, tau=tau))
    assert close(out("indicator.bin", (NP, NV, NU)),
                 oracle.forward_indicator(P, shape, NU, NV, Q, centre, 0.5))
    assert close(out("back_voxel.bin", shape), oracle.back_voxel(P, shape, NU, NV, sino))
    assert close(out("points.bin", (5,)),
                 oracle.back_voxel_points(P, shape, NU, NV, sino, ijk, views=VIEWS[:3]))
    yc, n2 = oracle.forward_cyl(P, CYL, NU, NV, cvol, 0.5, pose=pose, return_count=True)
    assert close(out("fwd_cyl.bin", (NP, NV, NU)), yc)
    assert close(out("back_cyl.bin", cvol.shape),
                 oracle.back_voxel_cyl(P, CYL, NU, NV, sino, pose=pose))
    assert out("counts.bin", (3,), np.int64).tolist() == [n0, n1, n2]
